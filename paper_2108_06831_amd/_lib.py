"""ctypes binding of libtnq.so: the C ABI of include/tn.h, same names.

Argument marshalling only -- every step of the contraction runs in the HIP
library.  There is no fallback: if libtnq.so is missing the import of the
binding fails.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# TNQ_LIB selects another build of the same library (the host-sanitizer build)
LIB_PATH = os.environ.get("TNQ_LIB") or os.path.join(_HERE, "libtnq.so")

TN_OK, TN_EINVAL, TN_ENOMEM, TN_ELIMIT, TN_EDEVICE, TN_EUNSUPPORTED = range(6)
STATUS_NAMES = {0: "TN_OK", 1: "TN_EINVAL", 2: "TN_ENOMEM", 3: "TN_ELIMIT", 4: "TN_EDEVICE", 5: "TN_EUNSUPPORTED"}
TN_PREC_C64, TN_PREC_BF16X3, TN_PREC_Q3_28 = 0, 1, 2
TN_OUT_STATEVECTOR, TN_OUT_AMPLITUDES = 0, 1
TN_PATH_GREEDY, TN_PATH_SEQUENTIAL, TN_PATH_RANDOM, TN_PATH_SEARCH = 0, 1, 2, 3
TN_FUSE_2Q = 1
TN_FUSE_SPLIT = 2
TN_MAX_RANK = 64

GATE_KIND = {name: i + 1 for i, name in enumerate(
    ["H", "X", "Y", "Z", "S", "T", "SX", "SY", "SW", "RX", "RY", "RZ", "U3", "MIXER",
     "CZ", "CNOT", "SWAP", "CPHASE", "ZZPHASE", "MATRIX1", "MATRIX2"])}


class tn_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q", ctypes.c_int32 * 2), ("angle", ctypes.c_double * 3),
                ("param", ctypes.c_int32 * 3), ("matrix", ctypes.POINTER(ctypes.c_double))]


class tn_observable(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("z_mask", ctypes.POINTER(ctypes.c_uint64)),
                ("coeff", ctypes.POINTER(ctypes.c_double))]


class tn_plan_opts(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("max_log2_intermediate", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("trials", ctypes.c_int32), ("max_slice_bits", ctypes.c_int32)]


class tn_path_stats(ctypes.Structure):
    _fields_ = [("flops", ctypes.c_double), ("bytes", ctypes.c_double), ("max_intermediate_elems", ctypes.c_double),
                ("large_step_flops", ctypes.c_double), ("plan_seconds", ctypes.c_double),
                ("modeled_seconds", ctypes.c_double),
                ("n_steps", ctypes.c_int32), ("n_permutes", ctypes.c_int32), ("n_gemm_steps", ctypes.c_int32),
                ("n_skinny_steps", ctypes.c_int32), ("n_small_steps", ctypes.c_int32),
                ("n_small_lists", ctypes.c_int32), ("n_sweep_steps", ctypes.c_int32),
                ("n_sweep_passes", ctypes.c_int32), ("n_product_launches", ctypes.c_int32),
                ("n_slice_bits", ctypes.c_int32), ("n_sweep_gate_runs", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TNError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


EXPORTS = [
    "tn_build_network", "tn_network_destroy", "tn_network_info", "tn_network_tensor", "tn_network_output",
    "tn_network_values", "tn_plan_path", "tn_path_destroy", "tn_path_pairs", "tn_path_slices", "tn_path_step", "tn_workspace_bytes",
    "tn_contract_path", "tn_amplitudes", "tn_expectation_workspace_bytes", "tn_expectation",
    "tn_backward_workspace_bytes", "tn_backward", "tn_contract_pair_workspace_bytes", "tn_contract_pair",
    "tn_last_error", "tn_version", "tn_profile_enable", "tn_profile_read", "tn_profile_reset", "tn_autotune",
    "tn_path_gemm_config", "tn_graph_begin", "tn_graph_end", "tn_graph_launch", "tn_graph_destroy",
    "tn_profile_select", "tn_contract_path_noalloc",
]

KERNEL_KINDS = ["materialize", "skinny", "permute", "gemm", "reduce", "copy", "adjoint", "interp", "sweep",
                "gemm_large"]


class tn_tune_report(ctypes.Structure):
    _fields_ = [("n_products", ctypes.c_int32), ("n_changed", ctypes.c_int32), ("seconds_before", ctypes.c_double),
                ("seconds_after", ctypes.c_double)]


class tn_kernel_profile(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("launches", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


def _declare(lib):
    P = ctypes.c_void_p
    i32, i64, u64, sz, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
    st = ctypes.c_int
    lib.tn_build_network.argtypes = [i32, P, i32, i32, i32, i64, i32, ctypes.POINTER(P)]
    lib.tn_build_network.restype = st
    lib.tn_network_destroy.argtypes = [P]
    lib.tn_network_destroy.restype = None
    lib.tn_network_info.argtypes = [P, P, P, P, P]
    lib.tn_network_info.restype = st
    lib.tn_network_tensor.argtypes = [P, i32, P, P, P]
    lib.tn_network_tensor.restype = st
    lib.tn_network_output.argtypes = [P, P, P]
    lib.tn_network_output.restype = st
    lib.tn_network_values.argtypes = [P, P, P, P, i64]
    lib.tn_network_values.restype = st
    lib.tn_plan_path.argtypes = [P, P, ctypes.POINTER(P), P]
    lib.tn_plan_path.restype = st
    lib.tn_path_destroy.argtypes = [P]
    lib.tn_path_destroy.restype = None
    lib.tn_path_pairs.argtypes = [P, P, P, i32]
    lib.tn_path_pairs.restype = st
    lib.tn_path_slices.argtypes = [P, P, P, i32]
    lib.tn_path_slices.restype = st
    lib.tn_path_step.argtypes = [P, i32, P, P, P, P]
    lib.tn_path_step.restype = st
    lib.tn_workspace_bytes.argtypes = [P, P, i32]
    lib.tn_workspace_bytes.restype = sz
    lib.tn_contract_path.argtypes = [P, i32, P, P, P, i32, P, sz, P]
    lib.tn_contract_path.restype = st
    lib.tn_contract_path_noalloc.argtypes = [P, i32, P, P, P, i32, P]
    lib.tn_contract_path_noalloc.restype = st
    lib.tn_amplitudes.argtypes = [P, i32, P, P, P, P, i64, P, sz, P]
    lib.tn_amplitudes.restype = st
    lib.tn_expectation_workspace_bytes.argtypes = [P, P, i32, i32]
    lib.tn_expectation_workspace_bytes.restype = sz
    lib.tn_expectation.argtypes = [P, i32, P, P, i32, P, i32, P, P, sz, P]
    lib.tn_expectation.restype = st
    lib.tn_backward_workspace_bytes.argtypes = [P, P, i32]
    lib.tn_backward_workspace_bytes.restype = sz
    lib.tn_backward.argtypes = [P, i32, P, P, P, i32, P, P, P, sz, P, P]
    lib.tn_backward.restype = st
    lib.tn_contract_pair_workspace_bytes.argtypes = [i32, P, P, i32, P, P, i32, P]
    lib.tn_contract_pair_workspace_bytes.restype = sz
    lib.tn_contract_pair.argtypes = [P, i32, P, i32, P, P, P, i32, P, P, P, i32, P, P, sz]
    lib.tn_contract_pair.restype = st
    lib.tn_last_error.argtypes = []
    lib.tn_last_error.restype = ctypes.c_char_p
    lib.tn_version.argtypes = []
    lib.tn_version.restype = ctypes.c_char_p
    lib.tn_profile_enable.argtypes = [i32]
    lib.tn_profile_enable.restype = st
    lib.tn_profile_read.argtypes = [P, i32]
    lib.tn_profile_read.restype = i32
    lib.tn_profile_reset.argtypes = []
    lib.tn_profile_reset.restype = None
    lib.tn_profile_select.argtypes = [ctypes.c_uint32]
    lib.tn_profile_select.restype = st
    lib.tn_autotune.argtypes = [P, i32, P, P, P, i32, P, sz, i32, P]
    lib.tn_autotune.restype = st
    lib.tn_path_gemm_config.argtypes = [P, i32, i32, P, P, P, i32]
    lib.tn_path_gemm_config.restype = st
    lib.tn_graph_begin.argtypes = [P]
    lib.tn_graph_begin.restype = st
    lib.tn_graph_end.argtypes = [P, ctypes.POINTER(P)]
    lib.tn_graph_end.restype = st
    lib.tn_graph_launch.argtypes = [P, P]
    lib.tn_graph_launch.restype = st
    lib.tn_graph_destroy.argtypes = [P]
    lib.tn_graph_destroy.restype = None
    del i64, u64, dbl


_lib = None


def lib():
    """The loaded libtnq.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2108_06831_amd.build.build()")
        # torch ships its own HIP runtime under the same soname as the system one this library
        # links; whichever is loaded first serves both.  torch goes first, so that the runtime
        # torch initialises the GPU with is the one the library's calls reach (loading the library
        # first left its HIP calls without a device once torch had started).
        import torch  # noqa: F401
        l = ctypes.CDLL(LIB_PATH)
        _declare(l)
        _lib = l
    return _lib


def check(status: int):
    if status != TN_OK:
        raise TNError(status, lib().tn_last_error().decode())
