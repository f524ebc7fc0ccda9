"""Tensor-network quantum-circuit contraction on MI355X (gfx950).

Python front end of libtnq.so (C ABI in include/tn.h).  PyTorch supplies device
memory and the stream; every contraction step runs in the library's HIP
kernels.

    net  = Network.from_circuit(circ)                  # circuit -> tensor network
    path = net.plan()                                  # greedy contraction order
    psi  = contract_path(net, path)                    # complex64 [batch, 2^n]
    amps = amplitudes(net, path, bits)                 # <b|U|0>
    e    = expectation([net], [path], [params], [obs]) # <psi|D|psi>, FP64 accumulation
    e    = Expectation.apply(params, net, path, obs)   # differentiable (adjoint method)
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (TN_FUSE_2Q, TN_OUT_AMPLITUDES, TN_OUT_STATEVECTOR, TN_PATH_GREEDY, TN_PATH_RANDOM,
                   TN_PATH_SEARCH, TN_PATH_SEQUENTIAL, TN_PREC_BF16X3, TN_PREC_C64, TN_PREC_Q3_28, TNError, check,
                   lib)

__all__ = ["Network", "Path", "contract_path", "amplitudes", "expectation", "backward", "contract_pair", "autotune",
           "Expectation", "Graph", "Observable", "TNError", "tn_build_network", "tn_plan_path", "tn_contract_pair",
           "tn_contract_path", "tn_contract_path_noalloc", "tn_amplitudes", "tn_expectation", "tn_backward"]

PRECISION = {"c64": TN_PREC_C64, "bf16x3": TN_PREC_BF16X3, "q3.28": TN_PREC_Q3_28}
PATH_KIND = {"greedy": TN_PATH_GREEDY, "sequential": TN_PATH_SEQUENTIAL, "random": TN_PATH_RANDOM,
             "search": TN_PATH_SEARCH}


def _prec(p) -> int:
    return PRECISION[p] if isinstance(p, str) else int(p)


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# gates
# ---------------------------------------------------------------------------
def gates_from_circuit(circ, matrices=None):
    """tn_gate array from a workloads.Circuit (kinds by name; parameter
    references kept).  ``matrices`` maps gate index -> explicit matrix."""
    n = len(circ.gates)
    arr = (_lib.tn_gate * max(n, 1))()
    keep = []
    for i, g in enumerate(circ.gates):
        G = arr[i]
        if matrices and i in matrices:
            m = np.ascontiguousarray(np.asarray(matrices[i], dtype=np.complex128)).view(np.float64)
            keep.append(m)
            G.kind = _lib.GATE_KIND["MATRIX2" if m.size == 32 else "MATRIX1"]
            G.matrix = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            G.kind = _lib.GATE_KIND[g.kind]
            G.matrix = None
        G.q[0] = g.qubits[0]
        G.q[1] = g.qubits[1] if len(g.qubits) > 1 else -1
        for j in range(3):
            G.angle[j] = g.angles[j] if j < len(g.angles) else 0.0
            G.param[j] = g.params[j] if j < len(g.params) else -1
    return arr, n, keep


class Observable:
    """Diagonal observable sum_t c_t prod_{q in mask_t} Z_q (mask bit n-1-q = qubit q)."""

    def __init__(self, masks, coeffs):
        self.masks = np.ascontiguousarray(masks, dtype=np.uint64)
        self.coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        self.c = _lib.tn_observable(len(self.masks), self.masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    self.coeffs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


# ---------------------------------------------------------------------------
# network and path handles
# ---------------------------------------------------------------------------
class Network:
    def __init__(self, handle: ctypes.c_void_p, n_qubits: int, n_params: int, output_kind: int, n_bitstrings: int):
        self.handle = handle
        self.n_qubits = n_qubits
        self.n_params = n_params
        self.output_kind = output_kind
        self.n_bitstrings = n_bitstrings

    @classmethod
    def from_circuit(cls, circ, output: str = "statevector", n_bitstrings: int = 0, fuse=False,
                     matrices=None):
        """fuse: False, "dense" (one 4x4 tensor per fused block) or "split" / True
        (operator-Schmidt halves where the two-qubit gate allows)."""
        arr, n, _keep = gates_from_circuit(circ, matrices)
        kind = TN_OUT_STATEVECTOR if output == "statevector" else TN_OUT_AMPLITUDES
        flags = 0
        if fuse:
            flags = _lib.TN_FUSE_2Q | (0 if fuse == "dense" else _lib.TN_FUSE_SPLIT)
        return tn_build_network(circ.n_qubits, arr, n, circ.n_params, kind, n_bitstrings, flags)

    def __del__(self):
        try:
            if self.handle:
                lib().tn_network_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def info(self):
        a = [ctypes.c_int32() for _ in range(4)]
        check(lib().tn_network_info(self.handle, *[ctypes.byref(x) for x in a]))
        return {"n_tensors": a[0].value, "n_modes": a[1].value, "n_qubits": a[2].value, "n_output_modes": a[3].value}

    def tensor(self, t: int):
        rank = ctypes.c_int32()
        modes = (ctypes.c_int32 * _lib.TN_MAX_RANK)()
        ext = (ctypes.c_int64 * _lib.TN_MAX_RANK)()
        check(lib().tn_network_tensor(self.handle, t, ctypes.byref(rank), modes, ext))
        return list(modes[: rank.value]), list(ext[: rank.value])

    def output(self):
        k = self.info()["n_output_modes"]
        modes = (ctypes.c_int32 * max(k, 1))()
        ext = (ctypes.c_int64 * max(k, 1))()
        check(lib().tn_network_output(self.handle, modes, ext))
        return list(modes[:k]), list(ext[:k])

    def values(self, params=None, bitstrings=None):
        """FP64 host values of the input tensors (list of complex128 arrays)."""
        info = self.info()
        shapes = [self.tensor(t) for t in range(info["n_tensors"])]
        total = sum(int(np.prod(e)) if e else 1 for _, e in shapes)
        out = np.zeros(2 * total, dtype=np.float64)
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        b = None if bitstrings is None else np.ascontiguousarray(bitstrings, dtype=np.uint64)
        check(lib().tn_network_values(self.handle, None if p is None else p.ctypes.data_as(ctypes.c_void_p),
                                      None if b is None else b.ctypes.data_as(ctypes.c_void_p),
                                      out.ctypes.data_as(ctypes.c_void_p), out.size))
        vals, off = [], 0
        c = out.view(np.complex128)
        for _, e in shapes:
            sz = int(np.prod(e)) if e else 1
            vals.append(c[off: off + sz].reshape(e))
            off += sz
        return vals

    def plan(self, kind: str = "greedy", max_log2_intermediate: int = 0, seed: int = 0, trials: int = 0,
             max_slice_bits: int = 0) -> "Path":
        return tn_plan_path(self, kind, max_log2_intermediate, seed, trials, max_slice_bits)


class Path:
    def __init__(self, handle, net: Network, stats: dict):
        self.handle = handle
        self.net = net
        self.stats = stats

    def __del__(self):
        try:
            if self.handle:
                lib().tn_path_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def pairs(self):
        n = ctypes.c_int32()
        check(lib().tn_path_pairs(self.handle, ctypes.byref(n), None, 0))
        arr = (ctypes.c_int32 * max(2 * n.value, 1))()
        check(lib().tn_path_pairs(self.handle, ctypes.byref(n), arr, 2 * n.value))
        return [(arr[2 * i], arr[2 * i + 1]) for i in range(n.value)]

    def slices(self):
        """Sliced bond modes (slice sigma fixes them to sigma's bits, mode by mode, low bits first)."""
        n = ctypes.c_int32()
        check(lib().tn_path_slices(self.handle, ctypes.byref(n), None, 0))
        arr = (ctypes.c_int32 * max(n.value, 1))()
        check(lib().tn_path_slices(self.handle, ctypes.byref(n), arr, n.value))
        return list(arr[: n.value])

    def step(self, s: int):
        rank = ctypes.c_int32()
        modes = (ctypes.c_int32 * _lib.TN_MAX_RANK)()
        bmnk = (ctypes.c_int64 * 4)()
        kind = ctypes.c_int32()
        check(lib().tn_path_step(self.handle, s, ctypes.byref(rank), modes, bmnk, ctypes.byref(kind)))
        return {"modes": list(modes[: rank.value]), "bmnk": tuple(bmnk),
                "kind": ["skinny", "gemm", "small"][kind.value]}

    def gemm_config(self, s: int, precision="c64"):
        """(tile, split, transposed) launch shape of matrix-product step s."""
        t, sp, tr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().tn_path_gemm_config(self.handle, s, _prec(precision), ctypes.byref(t), ctypes.byref(sp),
                                        ctypes.byref(tr), 0))
        return t.value, sp.value, tr.value

    def set_gemm_config(self, s: int, tile: int, split: int, transposed: int = 0, precision="c64"):
        t, sp, tr = ctypes.c_int32(tile), ctypes.c_int32(split), ctypes.c_int32(transposed)
        check(lib().tn_path_gemm_config(self.handle, s, _prec(precision), ctypes.byref(t), ctypes.byref(sp),
                                        ctypes.byref(tr), 1))

    def gemm_configs(self, precision="c64"):
        """{step: (tile, split, transposed)} for every matrix-product step (e.g. to cache tuned shapes)."""
        out = {}
        for s in range(self.stats["n_steps"]):
            if self.step(s)["kind"] == "gemm":
                try:
                    out[s] = self.gemm_config(s, precision)
                except TNError:
                    pass
        return out

    def workspace_bytes(self, batch: int = 1) -> int:
        return int(lib().tn_workspace_bytes(self.net.handle, self.handle, batch))


# ---------------------------------------------------------------------------
# C ABI, same names
# ---------------------------------------------------------------------------
def tn_build_network(n_qubits, gates, n_gates, n_params, output_kind, n_bitstrings, flags) -> Network:
    h = ctypes.c_void_p()
    check(lib().tn_build_network(n_qubits, gates, n_gates, n_params, output_kind, n_bitstrings, flags,
                                 ctypes.byref(h)))
    return Network(h, n_qubits, n_params, output_kind, n_bitstrings)


def tn_plan_path(net: Network, kind="greedy", max_log2_intermediate: int = 0, seed: int = 0, trials: int = 0,
                 max_slice_bits: int = 0) -> Path:
    opts = _lib.tn_plan_opts(PATH_KIND[kind] if isinstance(kind, str) else int(kind), max_log2_intermediate, seed,
                             trials, max_slice_bits)
    h = ctypes.c_void_p()
    st = _lib.tn_path_stats()
    check(lib().tn_plan_path(net.handle, ctypes.byref(opts), ctypes.byref(h), ctypes.byref(st)))
    return Path(h, net, st.as_dict())


def tn_contract_path(stream, precision, net, path, params_dev, batch, workspace, workspace_bytes, out_dev):
    check(lib().tn_contract_path(stream, precision, net.handle, path.handle, params_dev, batch, workspace,
                                 workspace_bytes, out_dev))


def tn_contract_path_noalloc(stream, precision, net, path, params_dev, batch, out_dev):
    check(lib().tn_contract_path_noalloc(stream, precision, net.handle, path.handle, params_dev, batch, out_dev))


def tn_amplitudes(stream, precision, net, path, params_dev, bits_dev, count, workspace, workspace_bytes, out_dev):
    check(lib().tn_amplitudes(stream, precision, net.handle, path.handle, params_dev, bits_dev, count, workspace,
                              workspace_bytes, out_dev))


def tn_expectation(stream, precision, nets, paths, n, params_ptrs, batch, obs_arr, workspace, workspace_bytes,
                   out_dev):
    check(lib().tn_expectation(stream, precision, nets, paths, n, params_ptrs, batch, obs_arr, workspace,
                               workspace_bytes, out_dev))


def tn_backward(stream, precision, net, path, params_dev, batch, obs, grad_out_dev, workspace, workspace_bytes,
                value_dev, grad_dev):
    check(lib().tn_backward(stream, precision, net.handle, path.handle, params_dev, batch, obs, grad_out_dev,
                            workspace, workspace_bytes, value_dev, grad_dev))


def tn_contract_pair(stream, precision, a, rank_a, modes_a, ext_a, b, rank_b, modes_b, ext_b, c, rank_c, modes_c,
                     workspace, workspace_bytes):
    check(lib().tn_contract_pair(stream, precision, a, rank_a, modes_a, ext_a, b, rank_b, modes_b, ext_b, c, rank_c,
                                 modes_c, workspace, workspace_bytes))


# ---------------------------------------------------------------------------
# torch-level helpers
# ---------------------------------------------------------------------------
def _params_tensor(net: Network, params, batch: int, device):
    torch = _torch()
    if net.n_params == 0:
        return None
    if params is None:
        raise ValueError("this network reads parameters")
    p = torch.as_tensor(params, dtype=torch.float64, device=device).reshape(batch, net.n_params).contiguous()
    return p


def contract_path(net: Network, path: Path, params=None, batch: int = 1, precision="c64", device="cuda",
                  out=None, workspace=None, stream=None):
    """Full statevector(s), complex64 [batch, 2^n], qubit 0 = most significant bit."""
    torch = _torch()
    p = _params_tensor(net, params, batch, device)
    if out is None:
        out = torch.empty(batch, 1 << net.n_qubits, dtype=torch.complex64, device=device)
    nbytes = path.workspace_bytes(batch)
    ws = workspace if workspace is not None else _workspace(nbytes, device)
    tn_contract_path(_stream_handle(stream), _prec(precision), net, path, _ptr(p), batch, _ptr(ws), ws.numel(),
                     _ptr(out))
    return out


def autotune(net: Network, path: Path, params=None, batch: int = 1, precision="c64", reps: int = 5, device="cuda",
             workspace=None, stream=None) -> dict:
    """Times the candidate launch shapes of every matrix-product step of `path`
    on the GPU and keeps the fastest (see tn_autotune).  Returns the report."""
    p = _params_tensor(net, params, batch, device)
    nbytes = path.workspace_bytes(batch)
    ws = workspace if workspace is not None else _workspace(nbytes, device)
    rep = _lib.tn_tune_report()
    check(lib().tn_autotune(_stream_handle(stream), _prec(precision), net.handle, path.handle, _ptr(p), batch,
                            _ptr(ws), ws.numel(), reps, ctypes.byref(rep)))
    return {"n_products": rep.n_products, "n_changed": rep.n_changed, "seconds_before": rep.seconds_before,
            "seconds_after": rep.seconds_after}


def amplitudes(net: Network, path: Path, bitstrings, params=None, precision="c64", device="cuda", out=None,
               workspace=None, stream=None):
    """<b|U|0> for each bitstring (qubit q in bit n-1-q), complex64 [count]."""
    torch = _torch()
    bits = torch.as_tensor(np.asarray(bitstrings, dtype=np.uint64).view(np.int64), device=device) \
        if not torch.is_tensor(bitstrings) else bitstrings.to(device)
    count = bits.numel()
    p = _params_tensor(net, params, 1, device)
    if out is None:
        out = torch.empty(count, dtype=torch.complex64, device=device)
    ws = workspace if workspace is not None else _workspace(path.workspace_bytes(1), device)
    tn_amplitudes(_stream_handle(stream), _prec(precision), net, path, _ptr(p), _ptr(bits), count, _ptr(ws),
                  ws.numel(), _ptr(out))
    return out


def expectation(nets: Sequence[Network], paths: Sequence[Path], params: Sequence, observables: Sequence[Observable],
                batch: int = 1, precision="c64", device="cuda", workspace=None, stream=None, out=None):
    """<psi_c|D_c|psi_c> for each circuit c and parameter vector: float64 [n_circuits, batch]."""
    torch = _torch()
    n = len(nets)
    net_arr = (ctypes.c_void_p * n)(*[x.handle.value for x in nets])
    path_arr = (ctypes.c_void_p * n)(*[x.handle.value for x in paths])
    ptensors = [_params_tensor(nt, pr, batch, device) for nt, pr in zip(nets, params)]
    pptr = (ctypes.c_void_p * n)(*[(t.data_ptr() if t is not None else None) for t in ptensors])
    obs_arr = (_lib.tn_observable * n)(*[o.c for o in observables])
    nbytes = lib().tn_expectation_workspace_bytes(net_arr, path_arr, n, batch)
    ws = workspace if workspace is not None and workspace.numel() >= nbytes else _workspace(nbytes, device)
    if out is None:
        out = torch.empty(n, batch, dtype=torch.float64, device=device)
    tn_expectation(_stream_handle(stream), _prec(precision), net_arr, path_arr, n, pptr, batch, obs_arr, _ptr(ws),
                   ws.numel(), _ptr(out))
    return out


def backward(net: Network, path: Path, params, obs: Observable, batch: int = 1, grad_out=None, precision="c64",
             device="cuda", workspace=None, stream=None):
    """Value E (float64 [batch]) and adjoint gradient dL/dtheta (float64 [batch, n_params])."""
    torch = _torch()
    p = _params_tensor(net, params, batch, device)
    nbytes = int(lib().tn_backward_workspace_bytes(net.handle, path.handle, batch))
    ws = workspace if workspace is not None and workspace.numel() >= nbytes else _workspace(nbytes, device)
    value = torch.empty(batch, dtype=torch.float64, device=device)
    grad = torch.empty(batch, max(net.n_params, 1), dtype=torch.float64, device=device)
    go = None if grad_out is None else torch.as_tensor(grad_out, dtype=torch.float64, device=device).contiguous()
    tn_backward(_stream_handle(stream), _prec(precision), net, path, _ptr(p), batch, ctypes.byref(obs.c), _ptr(go),
                _ptr(ws), ws.numel(), _ptr(value), _ptr(grad))
    return value, grad[:, : net.n_params]


def contract_pair(a, modes_a, b, modes_b, modes_c, precision="c64", stream=None):
    """C = sum over contracted modes of A * B (complex64 torch tensors on the GPU)."""
    torch = _torch()
    ma = (ctypes.c_int32 * max(len(modes_a), 1))(*modes_a)
    mb = (ctypes.c_int32 * max(len(modes_b), 1))(*modes_b)
    mc = (ctypes.c_int32 * max(len(modes_c), 1))(*modes_c)
    ea = (ctypes.c_int64 * max(len(modes_a), 1))(*a.shape)
    eb = (ctypes.c_int64 * max(len(modes_b), 1))(*b.shape)
    ext = dict(zip(modes_a, a.shape))
    ext.update(zip(modes_b, b.shape))
    shape_c = [ext[m] for m in modes_c]
    a = a.contiguous()
    b = b.contiguous()
    c = torch.empty(shape_c, dtype=torch.complex64, device=a.device)
    nbytes = lib().tn_contract_pair_workspace_bytes(len(modes_a), ma, ea, len(modes_b), mb, eb, len(modes_c), mc)
    ws = _workspace(nbytes, a.device)
    tn_contract_pair(_stream_handle(stream), _prec(precision), _ptr(a), len(modes_a), ma, ea, _ptr(b), len(modes_b),
                     mb, eb, _ptr(c), len(modes_c), mc, _ptr(ws), ws.numel())
    return c


def _make_expectation_function():
    torch = _torch()

    class Expectation(torch.autograd.Function):
        """E(theta) = <psi(theta)|D|psi(theta)> of one circuit, differentiable in
        theta.  params: [n_params] (gives a 0-d value) or [batch, n_params]
        (gives [batch]).  The forward pass evaluates the value only
        (tn_expectation); the backward pass runs the adjoint sweep
        (tn_backward) with dL/dE as its output weights.  Nothing but params is
        kept between the two: the backward pass contracts the network again
        instead of holding the state (recomputation in place of stored
        intermediates)."""

        @staticmethod
        def forward(ctx, params, net, path, obs, precision="c64"):
            if net.n_params < 1 or params.dim() not in (1, 2) or params.shape[-1] != net.n_params:
                raise ValueError("params must be [n_params] or [batch, n_params] of a parametric network")
            flat = params.detach().to(torch.float64).reshape(-1, net.n_params).contiguous()
            batch = flat.shape[0]
            value = expectation([net], [path], [flat], [obs], batch=batch, precision=precision,
                                device=params.device)[0]
            ctx.save_for_backward(flat)
            ctx.meta = (net, path, obs, precision, tuple(params.shape), params.dtype)
            return value.reshape(()) if params.dim() == 1 else value

        @staticmethod
        def backward(ctx, grad_value):
            (flat,) = ctx.saved_tensors
            net, path, obs, precision, shape, dtype = ctx.meta
            if not ctx.needs_input_grad[0]:
                return None, None, None, None, None
            batch = flat.shape[0]
            go = grad_value.detach().to(torch.float64).reshape(-1).expand(batch).contiguous()
            _, grad = backward(net, path, flat, obs, batch=batch, grad_out=go, precision=precision,
                               device=flat.device)
            return grad.reshape(shape).to(dtype), None, None, None, None

    return Expectation


class _LazyExpectation:
    _cls = None

    def __getattr__(self, name):
        if _LazyExpectation._cls is None:
            _LazyExpectation._cls = _make_expectation_function()
        return getattr(_LazyExpectation._cls, name)


Expectation = _LazyExpectation()


# ---------------------------------------------------------------------------
# HIP graphs
# ---------------------------------------------------------------------------
class Graph:
    """A recording of library calls replayed as one HIP graph launch.

        g = Graph(stream)            # a torch.cuda.Stream (not the null stream)
        with g.capture():
            expectation(..., workspace=ws, out=out, stream=stream)
        g.launch()                   # replays every kernel of the calls above

    Buffers (params, workspace, outputs) must be allocated before the capture
    and are reused by every launch; run the calls once before capturing so
    the library's device-side tables exist."""

    def __init__(self, stream):
        self.stream = stream
        self.handle = None

    def capture(self):
        import contextlib

        @contextlib.contextmanager
        def _cap():
            if self.handle is not None:
                raise TNError(1, "graph already captured")
            check(lib().tn_graph_begin(ctypes.c_void_p(self.stream.cuda_stream)))
            try:
                yield self
            finally:
                h = ctypes.c_void_p()
                check(lib().tn_graph_end(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
                self.handle = h

        return _cap()

    def launch(self):
        check(lib().tn_graph_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)))

    def __del__(self):
        try:
            if self.handle:
                lib().tn_graph_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


# ---------------------------------------------------------------------------
# kernel timing
# ---------------------------------------------------------------------------
def profile_enable(on: bool = True):
    check(lib().tn_profile_enable(1 if on else 0))


def profile_select(kinds=None):
    """Time only these kernel kinds (names from profile_read; None = all)."""
    mask = 0xFFFFFFFF if kinds is None else sum(1 << _lib.KERNEL_KINDS.index(k) for k in kinds)
    check(lib().tn_profile_select(mask))


def profile_reset():
    lib().tn_profile_reset()


def profile_read():
    """{kernel kind: {launches, seconds, bytes, flops}} for the launches recorded
    since the last read (synchronises on the recorded events)."""
    arr = (_lib.tn_kernel_profile * 16)()
    n = lib().tn_profile_read(arr, 16)
    return {_lib.KERNEL_KINDS[arr[i].kind]: {"launches": arr[i].launches, "seconds": arr[i].seconds,
                                             "bytes": arr[i].bytes, "flops": arr[i].flops} for i in range(n)}
