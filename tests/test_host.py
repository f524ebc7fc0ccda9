"""Host-side logic of libtnq.so, CPU only: the exported C ABI, the circuit ->
network builder, the greedy planner and the compiled program's semantics
(checked by executing planned paths in FP64 on the CPU against the oracle)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads
from paper_2108_06831_amd import Network, Observable, TNError, _lib
from tests import pathexec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "tn.h")).read()
    declared = set(re.findall(r"\b(tn_[a-z_0-9]+)\s*\(", header))
    lib = _lib.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTS) == declared
    assert lib.tn_version().decode().startswith("tnq")


def test_network_structure_config0():
    circ = workloads.config0()
    net = Network.from_circuit(circ)
    info = net.info()
    # 10 |0> vectors + 80 U3 (dense, new output legs) + 36 CZ (diagonal: hyper-indices)
    assert info["n_tensors"] == 10 + 80 + 36
    assert info["n_modes"] == 10 + 80
    ranks = [len(net.tensor(t)[0]) for t in range(info["n_tensors"])]
    assert ranks.count(1) == 10 and ranks.count(2) == 80 + 36


def test_network_structure_config1_fused():
    net = Network.from_circuit(workloads.config1(), fuse="dense")
    info = net.info()
    assert info["n_tensors"] == 24 + 184
    assert all(len(net.tensor(t)[0]) == 4 for t in range(24, 24 + 184))
    # split form: every CZ block becomes two 3-leg halves [bond, out, in] sharing a bond of extent 2
    net = Network.from_circuit(workloads.config1(), fuse="split")
    assert net.info()["n_tensors"] == 24 + 2 * 184
    for t in range(24, 24 + 2 * 184, 2):
        (ma, ea), (mb, eb) = net.tensor(t), net.tensor(t + 1)
        assert ea == eb == [2, 2, 2] and ma[0] == mb[0]


@pytest.mark.parametrize("fuse", ["dense", "split"])
def test_fused_networks_match_oracle(fuse):
    rng = np.random.default_rng(77)
    kinds = ["U3", "RX", "RZ", "H", "SX", "CZ", "CNOT", "CPHASE", "ZZPHASE", "SWAP"]
    for trial in range(6):
        circ = workloads.random_circuit(6, 50, rng, kinds=kinds)
        net = Network.from_circuit(circ, fuse=fuse)
        for kind in ("greedy", "search"):
            got = pathexec.execute(net, net.plan(kind, trials=8)).reshape(-1)
            assert np.max(np.abs(got - oracle.statevector(circ))) < 1e-12


def test_small_steps_come_first_and_form_independent_lists():
    net = Network.from_circuit(workloads.config1(), fuse=True)
    path = net.plan("search", trials=8)
    st = path.stats
    assert st["n_small_steps"] > 0 and st["n_small_lists"] >= 1
    kinds = [path.step(s)["kind"] for s in range(st["n_steps"])]
    assert kinds[: st["n_small_steps"]] == ["small"] * st["n_small_steps"]
    assert "small" not in kinds[st["n_small_steps"]:]


def test_amplitude_network_has_projectors():
    circ, bits = workloads.config2(rows=2, cols=3, depth=4, n_bitstrings=100)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=100)
    modes, ext = net.output()
    assert len(modes) == 1 and ext == [128]
    n_t = net.info()["n_tensors"]
    for t in range(n_t - 6, n_t):
        m, e = net.tensor(t)
        assert e == [128, 2] and m[0] == modes[0]


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("fuse", [False, True])
def test_greedy_path_matches_oracle_random(seed, fuse):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(2, 8))
    circ = workloads.random_circuit(n, 25, rng)
    net = Network.from_circuit(circ, fuse=fuse)
    path = net.plan()
    got = pathexec.execute(net, path).reshape(-1)
    want = oracle.statevector(circ)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("kind", ["greedy", "sequential", "random"])
def test_path_independence_config0(kind):
    """Contraction is associative: every order gives the same state (Sec. 2.2.3)."""
    circ = workloads.config0()
    net = Network.from_circuit(circ)
    want = oracle.statevector(circ)
    for seed in range(3 if kind == "random" else 1):
        path = net.plan(kind, seed=seed)
        got = pathexec.execute(net, path).reshape(-1)
        assert np.max(np.abs(got - want)) < 1e-12


def test_fused_config0_matches_oracle():
    circ = workloads.config0()
    net = Network.from_circuit(circ, fuse=True)
    got = pathexec.execute(net, net.plan()).reshape(-1)
    assert np.max(np.abs(got - oracle.statevector(circ))) < 1e-12


def test_parametric_network_values_match_oracle():
    circ, params, (masks, coeffs) = workloads.config4(n=6, layers=2, batch=3)
    net = Network.from_circuit(circ)
    path = net.plan()
    for b in range(3):
        got = pathexec.execute(net, path, params=params[b]).reshape(-1)
        want = oracle.statevector(circ, params[b])
        assert np.max(np.abs(got - want)) < 1e-12


def test_qaoa_network_values_match_oracle():
    inst = workloads.config3(n_circuits=2, sizes=(8,))
    for it in inst:
        net = Network.from_circuit(it.circuit)
        got = pathexec.execute(net, net.plan(), params=it.params).reshape(-1)
        want = oracle.statevector(it.circuit, it.params)
        assert np.max(np.abs(got - want)) < 1e-12


def test_amplitude_path_matches_oracle():
    circ, bits = workloads.config2(rows=3, cols=3, depth=6, n_bitstrings=50)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=50)
    path = net.plan()
    got = pathexec.execute(net, path, bitstrings=bits)[:50]
    psi = oracle.statevector(circ)
    want = oracle.amplitudes(psi, circ.n_qubits, bits)
    assert np.max(np.abs(got - want)) < 1e-12


def test_greedy_is_deterministic():
    circ = workloads.config1()
    a = Network.from_circuit(circ, fuse=True).plan().pairs()
    b = Network.from_circuit(circ, fuse=True).plan().pairs()
    assert a == b


def test_plan_stats_and_step_views():
    net = Network.from_circuit(workloads.config0())
    path = net.plan()
    st = path.stats
    assert st["n_steps"] == net.info()["n_tensors"] - 1
    assert st["max_intermediate_elems"] == 1024  # the statevector is the largest tensor
    assert st["n_skinny_steps"] + st["n_gemm_steps"] + st["n_small_steps"] == st["n_steps"]
    tot = 0.0
    for s in range(st["n_steps"]):
        b, m, n, k = path.step(s)["bmnk"]
        tot += 8.0 * b * m * n * k
    assert tot == pytest.approx(st["flops"])
    assert path.workspace_bytes(1) >= 8 * 1024


def test_config_plan_sizes():
    """Largest intermediates the greedy order reaches on the workloads."""
    p1 = Network.from_circuit(workloads.config1(), fuse=True).plan()
    assert p1.stats["max_intermediate_elems"] <= 2 ** 26
    circ, params, _ = workloads.config4()
    p4 = Network.from_circuit(circ).plan()
    assert p4.stats["max_intermediate_elems"] >= 2 ** 20


def test_gate_passes_are_planned_on_the_pass_workloads():
    """The fused gate passes (paper Sec. 3's streaming of gates over a large
    state) take the whole gate chains of the ansatz and of a 26-qubit QAOA
    circuit: the pass planner checks its own reordering of diagonal gates
    and would leave a chain to the per-step kernels if that check failed."""
    circ, params, _ = workloads.config4()
    p4 = Network.from_circuit(circ).plan("sequential")
    assert p4.stats["n_sweep_passes"] == 8
    assert p4.stats["n_sweep_steps"] >= 590
    # most dense one-qubit gates (RY on every qubit of every layer) run in straight-line runs
    assert p4.stats["n_sweep_gate_runs"] >= 25
    inst = [it for it in workloads.config3() if it.circuit.n_qubits == 26][0]
    p3 = Network.from_circuit(inst.circuit).plan("sequential")
    assert 9 <= p3.stats["n_sweep_passes"] <= 11
    assert p3.stats["n_sweep_steps"] >= 280
    assert p3.stats["n_sweep_gate_runs"] >= 18   # the mixers' RX gates
    # small states take the full 2^12-element chunk too: few, launch-bound passes
    inst16 = [it for it in workloads.config3() if it.circuit.n_qubits == 16][0]
    p16 = Network.from_circuit(inst16.circuit).plan("sequential")
    assert p16.stats["n_sweep_passes"] <= 5


def test_invalid_inputs_are_rejected():
    c = workloads.Circuit(3, [workloads.Gate("CZ", (0, 1))])
    c.gates[0].qubits = (0, 0)
    with pytest.raises(TNError) as e:
        Network.from_circuit(c)
    assert e.value.status == _lib.TN_EINVAL
    c.gates[0].qubits = (0, 5)
    with pytest.raises(TNError):
        Network.from_circuit(c)
    c2 = workloads.Circuit(2, [workloads.Gate("RX", (0,), (0.1,), (3,))], n_params=2)
    with pytest.raises(TNError):
        Network.from_circuit(c2)


def test_intermediate_cap_gives_elimit():
    net = Network.from_circuit(workloads.config0())
    with pytest.raises(TNError) as e:
        net.plan(max_log2_intermediate=8)
    assert e.value.status == _lib.TN_ELIMIT


def test_workspace_too_small_gives_enomem_before_any_device_call():
    net = Network.from_circuit(workloads.config0())
    path = net.plan()
    fake = ctypes.c_void_p(0x1000)
    st = _lib.lib().tn_contract_path(None, 0, net.handle, path.handle, None, 1, fake, 16, fake)
    assert st == _lib.TN_ENOMEM


def test_contract_pair_argument_checks():
    lib = _lib.lib()
    ma = (ctypes.c_int32 * 2)(0, 1)
    ea = (ctypes.c_int64 * 2)(4, 4)
    mb = (ctypes.c_int32 * 2)(1, 2)
    eb = (ctypes.c_int64 * 2)(3, 4)  # extent mismatch on the shared mode
    mc = (ctypes.c_int32 * 2)(0, 2)
    assert lib.tn_contract_pair_workspace_bytes(2, ma, ea, 2, mb, eb, 2, mc) == 0
    eb2 = (ctypes.c_int64 * 2)(4, 4)
    assert lib.tn_contract_pair_workspace_bytes(2, ma, ea, 2, mb, eb2, 2, mc) > 0
    mc_bad = (ctypes.c_int32 * 1)(0)  # mode 2 of B only must be in C
    assert lib.tn_contract_pair_workspace_bytes(2, ma, ea, 2, mb, eb2, 1, mc_bad) == 0


def test_observable_marshalling():
    masks, coeffs = workloads.maxcut_observable(4, [(0, 1), (2, 3)])
    o = Observable(masks, coeffs)
    assert o.c.n_terms == 3


@pytest.mark.parametrize("shapes", [
    ([1, 1], [1, 1], [0, 2]),          # M = N = K = 1
    ([], [2, 2], [1, 2]),              # scalar times a matrix (no shared mode)
    ([2], [2, 4], [2]),                # vector-matrix, summed mode
    ([4, 4], [4, 4], [0, 1, 2]),       # batch mode shared by both and kept
])
def test_contract_pair_plans_tiny_shapes(shapes):
    """Planning a single pairwise contraction (no device call): operands that
    are not gate tensors of a network, including extent-1 and rank-0 ones."""
    ea, eb, mc = shapes
    lib = _lib.lib()
    ma = list(range(len(ea)))
    mb = [1, 2][: len(eb)] if len(ea) != 0 else [1, 2]
    if shapes[2] == [0, 1, 2]:
        ma, mb = [0, 1], [1, 2]
    if len(ea) == 1:
        ma, mb = [1], [1, 2]
    arr = lambda t, v: (t * max(len(v), 1))(*v)
    n = lib.tn_contract_pair_workspace_bytes(len(ma), arr(ctypes.c_int32, ma), arr(ctypes.c_int64, ea), len(mb),
                                             arr(ctypes.c_int32, mb), arr(ctypes.c_int64, eb), len(mc),
                                             arr(ctypes.c_int32, mc))
    assert n > 0, _lib.lib().tn_last_error()


def test_gemm_launch_shape_get_set():
    """Launch shapes of product steps: defaults are valid, invalid shapes are refused."""
    from paper_2108_06831_amd import TNError
    circ = workloads.brickwork(16, 12, np.random.default_rng(5))
    path = Network.from_circuit(circ).plan(kind="greedy")
    shapes = path.gemm_configs()
    assert shapes
    for s, (tile, split, tr) in shapes.items():
        b, m, n, k = path.step(s)["bmnk"]
        assert 0 <= tile <= 6 and split in (1, 2, 4, 8) and k % split == 0 and tr == 0
        if tile == 4:
            assert k <= 1024 and split == 1
        with pytest.raises(TNError):
            path.set_gemm_config(s, 9, 1)
        with pytest.raises(TNError):
            path.set_gemm_config(s, 5, 1, 0, "bf16x3")  # the 3M tiles are FP32 only
        with pytest.raises(TNError):
            path.set_gemm_config(s, 0, 3)
        with pytest.raises(TNError):
            path.set_gemm_config(s, 0, 1, 2)
        path.set_gemm_config(s, 0, 1, 1, "bf16x3")
        assert path.gemm_config(s, "bf16x3") == (0, 1, 1)
        assert path.gemm_config(s) == (tile, split, tr)  # the other precision is untouched
    non_gemm = next(s for s in range(path.stats["n_steps"]) if s not in shapes)
    with pytest.raises(TNError):
        path.gemm_config(non_gemm)


def test_grouped_launch_plan():
    """Planning places independent per-output products next to each other so
    that they share launches: the 32-qubit amplitude network's batched outer
    products go from one launch each to a few grouped launches, and the
    statevector network's small products also group."""
    import workloads
    from paper_2108_06831_amd import Network
    circ, bits = workloads.config2()
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=len(bits))
    st = net.plan("greedy", max_log2_intermediate=28).stats
    n = st["n_gemm_steps"] + st["n_skinny_steps"]
    print(n, st["n_product_launches"])
    assert st["n_product_launches"] <= n // 2
    st1 = Network.from_circuit(workloads.config1(), fuse="split").plan("greedy").stats
    assert st1["n_product_launches"] < st1["n_gemm_steps"] + st1["n_skinny_steps"]


def test_fig31_grid_plans_and_small_paths_match_oracle():
    """The paper's test circuit (Fig. 3.1) over its whole grid, n in 2..28 and
    k in 2..14 (even): the greedy planner orders every statevector network and
    every network closed by <0...0| (and <1...1|), each in well under a second (Fig.
    4.1b's third-party greedy search took up to 728.6 s); the planned paths of
    the small ones, executed in FP64 on the host, equal the oracle."""
    import time
    worst = 0.0
    for n in range(2, 29, 2):
        for k in range(2, 15, 2):
            circ = workloads.paper_test_circuit(n, k)
            for output in ("statevector", "amplitudes"):
                net = Network.from_circuit(circ, output=output, n_bitstrings=2)
                t0 = time.perf_counter()
                path = net.plan("greedy")
                worst = max(worst, time.perf_counter() - t0)
                assert path.stats["n_steps"] == net.info()["n_tensors"] - 1
                if n <= 8 and k <= 6:
                    psi = oracle.statevector(circ)
                    if output == "statevector":
                        got = pathexec.execute(net, path).reshape(-1)
                        assert np.max(np.abs(got - psi)) < 1e-12
                    else:
                        bits = np.array([0, (1 << n) - 1], dtype=np.uint64)
                        got = pathexec.execute(net, path, bitstrings=bits).reshape(-1)
                        assert np.max(np.abs(got - psi[[0, -1]])) < 1e-12
    assert worst < 1.0


@pytest.mark.parametrize("case", ["grid3x4_cap10", "grid3x4_cap8", "brickwork12_dense", "hea10"])
def test_sliced_paths_sum_to_the_oracle(case):
    """Index slicing: a sum over a bond index equals the sum of the
    contractions with that index fixed to each value (eq. (2.2)).  The planned
    sliced path, executed slice by slice in FP64 on the CPU (fixing the
    sliced modes with np.take), must sum to the oracle's result, and every
    intermediate of the sliced program must fit the cap."""
    params = None
    if case.startswith("grid"):
        cap = int(case[-2:].lstrip("p"))
        circ, bits = workloads.config2(rows=3, cols=4, depth=8, n_bitstrings=64)
        net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=64)
        want = oracle.amplitudes(oracle.statevector(circ), circ.n_qubits, bits)
    elif case == "brickwork12_dense":
        cap, bits = 12, None
        circ = workloads.brickwork(12, 12, np.random.default_rng(5))
        net = Network.from_circuit(circ, fuse="dense")
        want = oracle.statevector(circ)
    else:
        cap, bits = 10, None
        circ, pb, _ = workloads.config4(n=10, layers=3, batch=1)
        params = pb[0]
        net = Network.from_circuit(circ)
        want = oracle.statevector(circ, params)
    assert net.plan().stats["max_intermediate_elems"] > 2 ** cap  # slicing is needed
    with pytest.raises(TNError) as e:
        net.plan(max_log2_intermediate=cap)
    assert e.value.status == _lib.TN_ELIMIT
    path = net.plan(max_log2_intermediate=cap, max_slice_bits=12)
    cut = path.slices()
    st = path.stats
    assert cut and st["n_slice_bits"] == len(cut)  # every mode here has extent 2
    assert st["max_intermediate_elems"] <= 2 ** cap
    out_modes, _ = net.output()
    assert not set(cut) & set(out_modes)
    for s in range(st["n_steps"]):
        assert not set(cut) & set(path.step(s)["modes"])
    got = pathexec.execute_sliced(net, path, params=params, bitstrings=bits).reshape(-1)[: want.size]
    assert np.max(np.abs(got - want)) < 1e-12


def test_slicing_options_and_limits():
    net = Network.from_circuit(workloads.config0())
    assert net.plan().slices() == [] and net.plan().stats["n_slice_bits"] == 0
    for bad in (-1, 17):
        with pytest.raises(TNError) as e:
            net.plan(max_slice_bits=bad)
        assert e.value.status == _lib.TN_EINVAL
    # an output intermediate cannot be sliced: a statevector never fits a cap below its own size
    with pytest.raises(TNError) as e:
        net.plan(max_log2_intermediate=8, max_slice_bits=16)
    assert e.value.status == _lib.TN_ELIMIT
    # too small a budget for the cap
    circ, bits = workloads.config2(rows=3, cols=4, depth=8, n_bitstrings=64)
    amp = Network.from_circuit(circ, output="amplitudes", n_bitstrings=64)
    with pytest.raises(TNError) as e:
        amp.plan(max_log2_intermediate=8, max_slice_bits=2)
    assert e.value.status == _lib.TN_ELIMIT
    # the sliced workspace holds the full inputs, the running sum and one slice's program
    p = amp.plan(max_log2_intermediate=10, max_slice_bits=12)
    assert p.workspace_bytes(1) < amp.plan().workspace_bytes(1)
