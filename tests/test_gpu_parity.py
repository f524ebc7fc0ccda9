"""Parity of the GPU contraction path with the FP64 oracle on the seeded
workloads (tolerances: 1e-5 normwise relative for complex64, 1e-3 for
BF16x3; scalars |e - e_ref| / max(|e_ref|, 1)).  GPU only."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

C64_TOL = 1e-5
BF16X3_TOL = 1e-3


def relerr(got, want):
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    want = np.asarray(want, dtype=np.complex128).reshape(-1)
    return np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)


def scalar_err(got, want):
    return abs(got - want) / max(abs(want), 1.0)


def statevector_gpu(circ, kind="greedy", fuse=False, precision="c64", params=None, batch=1):
    import torch
    from paper_2108_06831_amd import Network, contract_path
    net = Network.from_circuit(circ, fuse=fuse)
    path = net.plan(kind, trials=32)
    out = contract_path(net, path, params=params, batch=batch, precision=precision)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("kind", ["greedy", "sequential", "random", "search"])
@pytest.mark.parametrize("fuse", [False, "dense", "split"])
def test_config0_statevector(kind, fuse):
    circ = workloads.config0()
    print(f"config0 kind={kind} fuse={fuse}", flush=True)
    want = oracle.statevector(circ)
    got = statevector_gpu(circ, kind, fuse)[0]
    e = relerr(got, want)
    print(f"  rel err {e:.2e}", flush=True)
    assert e < C64_TOL


def test_config0_bf16x3():
    circ = workloads.config0()
    want = oracle.statevector(circ)
    e = relerr(statevector_gpu(circ, precision="bf16x3")[0], want)
    print(f"config0 bf16x3 rel err {e:.2e}", flush=True)
    assert e < BF16X3_TOL


@pytest.mark.parametrize("seed", range(6))
def test_random_circuits(seed):
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(1, 11))
    circ = workloads.random_circuit(n, 60, rng)
    print(f"random circuit seed={seed} n={n}", flush=True)
    for kind in ("greedy", "sequential", "search"):
        for fuse in (False, "dense", "split"):
            got = statevector_gpu(circ, kind, fuse)[0]
            assert relerr(got, oracle.statevector(circ)) < C64_TOL


def test_edge_cases():
    from workloads import Circuit, Gate
    # no gates: |0...0>
    got = statevector_gpu(Circuit(3, []), "greedy")[0]
    assert relerr(got, np.eye(8)[0]) < 1e-7
    # one qubit, one gate
    c = Circuit(1, [Gate("H", (0,))])
    assert relerr(statevector_gpu(c)[0], oracle.statevector(c)) < C64_TOL
    # a qubit that no gate touches, and a qubit with diagonal gates only
    c = Circuit(4, [Gate("H", (0,)), Gate("CNOT", (0, 2)), Gate("Z", (3,)), Gate("RZ", (3,), (0.3,))])
    assert relerr(statevector_gpu(c)[0], oracle.statevector(c)) < C64_TOL


def test_ghz_and_qft_closed_forms():
    n = 12
    c = workloads.Circuit(n, [workloads.Gate("H", (0,))] + [workloads.Gate("CNOT", (q, q + 1)) for q in range(n - 1)])
    got = statevector_gpu(c)[0]
    want = np.zeros(1 << n, complex)
    want[0] = want[-1] = 2 ** -0.5
    assert relerr(got, want) < C64_TOL


_C1_REF = {}


def config1_reference():
    if "psi" not in _C1_REF:
        _C1_REF["psi"] = oracle.statevector(workloads.config1())
    return _C1_REF["psi"]


@pytest.mark.parametrize("kind,fuse,precision,tol", [
    ("search", "split", "c64", C64_TOL), ("search", "split", "bf16x3", BF16X3_TOL),
    ("greedy", "dense", "c64", C64_TOL), ("sequential", "split", "c64", C64_TOL),
    ("sequential", "dense", "c64", C64_TOL), ("sequential", "dense", "bf16x3", BF16X3_TOL),
    ("search", "dense", "c64", C64_TOL)])
def test_config1_full_statevector(kind, fuse, precision, tol):
    """24 qubits, depth 16, 2-qubit fusion: the full 2^24 state."""
    circ = workloads.config1()
    print(f"config1 {kind} {fuse} {precision}: oracle ...", flush=True)
    want = config1_reference()
    print("config1: gpu ...", flush=True)
    got = statevector_gpu(circ, kind, fuse=fuse, precision=precision)[0]
    e = relerr(got, want)
    print(f"config1 {kind} {fuse} {precision} rel err {e:.3e} max abs {np.max(np.abs(got - want)):.2e}", flush=True)
    assert e < tol


@pytest.mark.parametrize("rows,cols,depth", [(2, 3, 4), (3, 3, 8), (4, 4, 12), (4, 6, 12)])
def test_config2_amplitudes_small_grids(rows, cols, depth):
    import torch
    from paper_2108_06831_amd import Network, amplitudes
    circ, bits = workloads.config2(rows, cols, depth, n_bitstrings=4096)
    print(f"config2 grid {rows}x{cols} depth {depth}", flush=True)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=4096)
    path = net.plan("greedy", max_log2_intermediate=30)
    got = amplitudes(net, path, bits).cpu().numpy()
    want = oracle.amplitudes(oracle.statevector(circ), circ.n_qubits, bits)
    e = relerr(got, want)
    print(f"  rel err {e:.2e}", flush=True)
    assert e < C64_TOL


def test_config3_expectations_subset():
    import torch
    from paper_2108_06831_amd import Network, Observable, expectation
    inst = workloads.config3()[:12]
    inst = [it for it in inst if it.circuit.n_qubits <= 20][:6]
    nets, paths, params, obs, want = [], [], [], [], []
    for it in inst:
        net = Network.from_circuit(it.circuit)
        nets.append(net)
        paths.append(net.plan("sequential"))
        params.append(it.params)
        m, c = workloads.maxcut_observable(it.circuit.n_qubits, it.edges)
        obs.append(Observable(m, c))
        want.append(oracle.circuit_expectation(it.circuit, it.params, m, c))
    got = expectation(nets, paths, params, obs).cpu().numpy()[:, 0]
    for g, w in zip(got, want):
        assert scalar_err(g, w) < C64_TOL
    # beta = 0: <C> = |E|/2 exactly
    it = inst[0]
    p0 = it.params.copy()
    p0[4:] = 0
    m, c = workloads.maxcut_observable(it.circuit.n_qubits, it.edges)
    g0 = expectation([nets[0]], [paths[0]], [p0], [Observable(m, c)]).cpu().numpy()[0, 0]
    assert abs(g0 - len(it.edges) / 2) < 1e-5 * len(it.edges)


def test_config4_gradients_small():
    import torch
    from paper_2108_06831_amd import Network, Observable, backward
    circ, params, (m, c) = workloads.config4(n=8, layers=3, batch=4)
    net = Network.from_circuit(circ)
    path = net.plan("sequential")
    value, grad = backward(net, path, params, Observable(m, c), batch=4)
    value, grad = value.cpu().numpy(), grad.cpu().numpy()
    for b in range(4):
        want_e = oracle.circuit_expectation(circ, params[b], m, c)
        assert scalar_err(value[b], want_e) < C64_TOL
        g = oracle.param_shift_gradient(circ, params[b], m, c)
        e = np.linalg.norm(grad[b] - g) / np.linalg.norm(g)
        print(f"  batch {b}: grad rel err {e:.2e}", flush=True)
        assert e < C64_TOL


def test_config2_full_size_orders_agree():
    """32-qubit grid, 4096 amplitudes: the FP64 state (64 GiB) is out of the
    oracle's reach here, so the full-size check is a property of the method:
    two different contraction orders give the same amplitudes (Sec. 2.2.3)."""
    from paper_2108_06831_amd import Network, amplitudes
    circ, bits = workloads.config2()
    # three genuinely different contractions: the unfused network (largest
    # intermediate 2^22), and the two-qubit-fused networks in dense and split
    # form (intermediates up to 2^27 and 2^28 elements)
    runs = []
    for fuse in (False, "dense", "split"):
        net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=4096, fuse=fuse)
        path = net.plan("search", max_log2_intermediate=28, trials=64, seed=7)
        print(f"  fuse={fuse}: {path.stats['flops']:.3e} flops, largest intermediate "
              f"2^{int(np.log2(path.stats['max_intermediate_elems']))}", flush=True)
        runs.append(amplitudes(net, path, bits).cpu().numpy())
    a1, a2, a3 = runs
    e12, e13 = relerr(a1, a2), relerr(a1, a3)
    print(f"config2 full: order agreement {e12:.2e} {e13:.2e}; mean 2^n|a|^2 = "
          f"{np.mean(np.abs(a1) ** 2) * 2 ** 32:.3f}", flush=True)
    assert e12 < 2 * C64_TOL and e13 < 2 * C64_TOL
    # Porter-Thomas: for a random circuit E[2^n |a|^2] = 1 (loose statistical sanity, 4096 samples)
    assert 0.8 < np.mean(np.abs(a1) ** 2) * 2 ** 32 < 1.2


def test_config3_full_batch():
    """All 512 QAOA circuits in one call: the oracle on a sample spanning every
    size, beta = 0 (<C> = |E|/2) on all 512, and the p = 1 closed form on the
    same 512 graphs."""
    from paper_2108_06831_amd import Network, Observable, expectation
    from tests.test_oracle import qaoa_p1_closed_form
    inst = workloads.config3()
    nets = [Network.from_circuit(it.circuit) for it in inst]
    paths = [nt.plan("sequential") for nt in nets]
    obs = [Observable(*workloads.maxcut_observable(it.circuit.n_qubits, it.edges)) for it in inst]
    got = expectation(nets, paths, [it.params for it in inst], obs).cpu().numpy()[:, 0]
    sample = []
    for n in (16, 18, 20, 22, 24, 26):
        sample += [i for i, it in enumerate(inst) if it.circuit.n_qubits == n][:1]
    for i in sample:
        it = inst[i]
        m, c = workloads.maxcut_observable(it.circuit.n_qubits, it.edges)
        want = oracle.circuit_expectation(it.circuit, it.params, m, c)
        print(f"  circuit {i} n={it.circuit.n_qubits}: {got[i]:.8f} vs {want:.8f}", flush=True)
        assert scalar_err(got[i], want) < C64_TOL
    p0 = [np.concatenate([it.params[:4], np.zeros(4)]) for it in inst]
    g0 = expectation(nets, paths, p0, obs).cpu().numpy()[:, 0]
    for it, g in zip(inst, g0):
        assert scalar_err(g, len(it.edges) / 2) < C64_TOL
    p1 = [workloads.qaoa_circuit(it.circuit.n_qubits, it.edges, 1) for it in inst]
    nets1 = [Network.from_circuit(c) for c in p1]
    paths1 = [nt.plan("sequential") for nt in nets1]
    prm1 = [np.array([it.params[0], it.params[4]]) for it in inst]
    g1 = expectation(nets1, paths1, prm1, obs).cpu().numpy()[:, 0]
    worst = 0.0
    for it, g, pr in zip(inst, g1, prm1):
        want = qaoa_p1_closed_form(it.circuit.n_qubits, it.edges, pr[0], pr[1])
        worst = max(worst, scalar_err(g, want))
    print(f"  p=1 closed form, worst error over 512 circuits {worst:.2e}", flush=True)
    assert worst < C64_TOL


def test_config4_full_gradients():
    """20 qubits, 10 layers, 64 parameter vectors: adjoint gradients against
    the oracle's exact parameter shift on sampled angles of vectors 0 and 63,
    and against central differences (h = 1e-3, FD = g sin(h)/h exactly)."""
    from paper_2108_06831_amd import Network, Observable, backward
    circ, params, (m, c) = workloads.config4()
    net = Network.from_circuit(circ)
    path = net.plan("sequential")
    value, grad = backward(net, path, params, Observable(m, c), batch=64)
    value, grad = value.cpu().numpy(), grad.cpu().numpy()
    rng = np.random.default_rng(99)
    which = sorted(rng.choice(circ.n_params, size=8, replace=False).tolist())
    for b in (0, 63):
        want_e = oracle.circuit_expectation(circ, params[b], m, c)
        assert scalar_err(value[b], want_e) < C64_TOL
        g = oracle.param_shift_gradient(circ, params[b], m, c, which=which)
        e = np.linalg.norm(grad[b, which] - g[which]) / np.linalg.norm(g[which])
        print(f"  vector {b}: value err {scalar_err(value[b], want_e):.2e}, grad rel err {e:.2e}", flush=True)
        assert e < C64_TOL
    h = 1e-3
    fd = oracle.finite_difference_gradient(circ, params[0], m, c, h=h, which=which[:4])
    e = np.linalg.norm(grad[0, which[:4]] - fd[which[:4]] / (np.sin(h) / h)) / np.linalg.norm(fd[which[:4]])
    print(f"  FD check rel err {e:.2e}", flush=True)
    assert e < C64_TOL


@pytest.mark.parametrize("n,seed", [(18, 0), (19, 1)])
def test_adjoint_passes_every_gate_kind(n, seed):
    """Adjoint gradients through the fused reverse-sweep passes (final tensor
    of 2^18 or more elements): random circuits with every gate kind, angles
    sharing parameters (product rule), a Z-string observable mixing one- and
    two-qubit terms; against the oracle's exact parameter shift."""
    from paper_2108_06831_amd import Network, Observable, backward, profile_enable, profile_read, profile_reset
    rng = np.random.default_rng(5150 + seed)
    circ = workloads.random_circuit(n, 120, rng, n_params=9)
    params = rng.uniform(0.0, 2.0 * np.pi, size=(2, circ.n_params))
    m, c = workloads.zz_ring_observable(n)
    m = np.concatenate([m, np.array([1 << (n - 1), 1 << 3], dtype=np.uint64)])
    c = np.concatenate([c, np.array([0.7, -1.3])])
    net = Network.from_circuit(circ)
    path = net.plan("sequential")
    profile_reset()
    profile_enable(True)
    value, grad = backward(net, path, params, Observable(m, c), batch=2)
    prof = profile_read()
    profile_enable(False)
    value, grad = value.cpu().numpy(), grad.cpu().numpy()
    n_sweep = sum(3 if (g.kind == "U3" and any(p >= 0 for p in g.params)) else 1 for g in circ.gates)
    print(f"n={n}: adjoint launches {prof['adjoint']['launches']} for {n_sweep} gates", flush=True)
    assert prof["adjoint"]["launches"] < n_sweep / 4
    for b in range(2):
        want_e = oracle.circuit_expectation(circ, params[b], m, c)
        assert scalar_err(value[b], want_e) < C64_TOL
        g = oracle.param_shift_gradient(circ, params[b], m, c)
        e = np.linalg.norm(grad[b] - g) / np.linalg.norm(g)
        print(f"  vector {b}: value err {scalar_err(value[b], want_e):.2e}, grad rel err {e:.2e}", flush=True)
        assert e < C64_TOL


def test_expectation_graph_replays():
    """Batched QAOA expectations captured in one HIP graph: every replay, with
    eager library work and synchronisations in between, equals the eager call;
    parameters updated in place between replays are picked up."""
    import torch
    from paper_2108_06831_amd import Graph, Network, Observable, expectation
    inst = [it for it in workloads.config3() if it.circuit.n_qubits in (16, 18)][:6]
    nets = [Network.from_circuit(it.circuit) for it in inst]
    paths = [nt.plan("sequential") for nt in nets]
    obs = [Observable(*workloads.maxcut_observable(it.circuit.n_qubits, it.edges)) for it in inst]
    stream = torch.cuda.Stream()
    params = [torch.as_tensor(it.params, device="cuda").reshape(1, -1).contiguous() for it in inst]
    out = torch.empty(len(inst), 1, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        eager = expectation(nets, paths, params, obs, stream=stream).clone()
        ws = torch.empty(1 << 26, dtype=torch.uint8, device="cuda")
    stream.synchronize()
    g = Graph(stream)
    with g.capture():
        expectation(nets, paths, params, obs, workspace=ws, out=out, stream=stream)
    for rep in range(3):
        out.fill_(0.0)
        torch.cuda.synchronize()
        g.launch()
        stream.synchronize()
        assert torch.equal(out, eager), rep
        # eager library work between replays
        other = expectation(nets[:2], paths[:2], params[:2], obs[:2])
        torch.cuda.synchronize()
        assert torch.equal(other, eager[:2])
    for p in params:
        p[0, 4:] = 0.0  # beta = 0: <C> = |E| / 2
    torch.cuda.synchronize()
    g.launch()
    stream.synchronize()
    for i, it in enumerate(inst):
        assert scalar_err(out[i, 0].item(), len(it.edges) / 2) < C64_TOL


@pytest.mark.parametrize("precision", ["c64", "bf16x3"])
def test_config2_full_size_sampled_amplitudes(precision):
    """32-qubit grid, all 4096 amplitudes on the GPU along the bench's order;
    24 of them, sampled, against the oracle's FP64 network contraction of each
    single amplitude."""
    from paper_2108_06831_amd import Network, amplitudes
    circ, bits = workloads.config2()
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=4096)
    path = net.plan("search", max_log2_intermediate=28, trials=256)
    got = amplitudes(net, path, bits, precision=precision).cpu().numpy()
    rng = np.random.default_rng(77)
    idx = sorted(rng.choice(4096, size=24, replace=False).tolist())
    want = np.array([oracle.single_amplitude(circ, int(bits[i])) for i in idx])
    err = relerr(got[idx], want)
    print(f"config2 {precision}: sampled amplitude rel err {err:.2e}", flush=True)
    assert err < (C64_TOL if precision == "c64" else BF16X3_TOL)


@pytest.mark.parametrize("precision,tol", [("c64", C64_TOL), ("bf16x3", BF16X3_TOL)])
def test_grouped_products(precision, tol):
    """Independent per-output products sharing launches (the batched outer
    products of a 4x6 grid's amplitude network): the launch count equals the
    planned one and is below the product count, results match the oracle, and
    moving one member to a matrix-core tile (which splits its group) changes
    nothing."""
    import torch
    from paper_2108_06831_amd import Network, amplitudes, profile_enable, profile_read, profile_reset, profile_select
    circ, bits = workloads.config2(4, 6, 12, n_bitstrings=4096)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=4096)
    path = net.plan("greedy", max_log2_intermediate=30)
    st = path.stats
    n_products = st["n_gemm_steps"] + st["n_skinny_steps"]
    print(f"products {n_products}, planned launches {st['n_product_launches']}", flush=True)
    assert st["n_product_launches"] < n_products
    want = oracle.amplitudes(oracle.statevector(circ), circ.n_qubits, bits)
    profile_reset()
    profile_select(["gemm", "skinny"])
    profile_enable(True)
    got = amplitudes(net, path, bits, precision=precision).cpu().numpy()
    prof = profile_read()
    profile_enable(False)
    profile_select(None)
    launches = sum(prof[k]["launches"] for k in ("gemm", "skinny") if k in prof)
    print(f"  launches {launches}, rel err {relerr(got, want):.2e}", flush=True)
    if precision == "c64":
        assert launches == st["n_product_launches"]
    assert relerr(got, want) < tol
    # a member of the first group on an MFMA tile: the group splits around it
    elem = [s for s, (t, sp, tr) in path.gemm_configs(precision).items() if t == 4]
    s = elem[len(elem) // 2]
    for tile in (3, 2, 1, 0):
        try:
            path.set_gemm_config(s, tile, 1, 0, precision)
            break
        except Exception:
            continue
    got2 = amplitudes(net, path, bits, precision=precision).cpu().numpy()
    torch.cuda.synchronize()
    assert relerr(got2, want) < tol


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_grouped_launches_random_grids(seed):
    """Random grid circuits (sizes, depths, bitstring batches and orders drawn
    from the seed), amplitudes on a batch index: the planner's grouping of
    per-output products (reordered steps, held-back buffers, shared launches)
    against the oracle, with the default shapes and after autotuning."""
    import torch
    from paper_2108_06831_amd import Network, amplitudes, autotune
    rng = np.random.default_rng(9100 + seed)
    rows, cols = [(4, 4), (3, 6), (4, 5), (4, 6)][seed]
    depth = int(rng.integers(8, 13))
    circ = workloads.grid_circuit(rows, cols, depth, rng, f"grid_{rows}x{cols}_d{depth}")
    nb = int(rng.choice([1024, 4096]))
    bits = workloads.random_bitstrings(circ.n_qubits, nb, rng)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=nb, fuse=["split", False][seed % 2])
    path = net.plan(["greedy", "search"][seed // 2], trials=64, seed=seed, max_log2_intermediate=30)
    st = path.stats
    n_products = st["n_gemm_steps"] + st["n_skinny_steps"]
    print(f"grid {rows}x{cols} depth {depth} batch {nb}: products {n_products}, "
          f"launches {st['n_product_launches']}", flush=True)
    assert st["n_product_launches"] < n_products  # some products share launches
    want = oracle.amplitudes(oracle.statevector(circ), circ.n_qubits, bits)
    got = amplitudes(net, path, bits).cpu().numpy()
    assert relerr(got, want) < C64_TOL
    autotune(net, path, reps=2)
    got = amplitudes(net, path, bits).cpu().numpy()
    torch.cuda.synchronize()
    assert relerr(got, want) < C64_TOL


@pytest.mark.parametrize("n,p,batch", [(18, 1, 1), (20, 2, 3)])
def test_product_state_outer_runs(n, p, batch):
    """|+> on every qubit, then QAOA layers (Sec. 3's circuits act on a
    product state): along the sequential order the state first grows one
    qubit at a time by outer products, which run as one launch; every
    amplitude of every parameter vector against the oracle."""
    rng = np.random.default_rng(500 + n)
    edges = workloads.random_regular_graph(n, 3, rng)
    circ = workloads.qaoa_circuit(n, edges, p)
    params = rng.uniform(0.0, np.pi, size=(batch, 2 * p))
    print(f"product-state circuit n={n} p={p} batch={batch}", flush=True)
    got = statevector_gpu(circ, "sequential", params=params, batch=batch)
    for b in range(batch):
        assert relerr(got[b], oracle.statevector(circ, params[b])) < C64_TOL
