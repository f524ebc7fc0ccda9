"""Pairwise contraction kernels through the C ABI (tn_contract_pair) against
the definition of a contraction (oracle.contract, FP64).  GPU only."""
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

C64_TOL = 1e-5
BF16X3_TOL = 1e-3


def relerr(got, want):
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    want = np.asarray(want, dtype=np.complex128).reshape(-1)
    return np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)


def crand(rng, shape):
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex64)


def run_pair(a, ma, b, mb, mc, precision="c64"):
    import torch
    from paper_2108_06831_amd import contract_pair
    ta = torch.from_numpy(a).cuda()
    tb = torch.from_numpy(b).cuda()
    c = contract_pair(ta, ma, tb, mb, mc, precision=precision)
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (2, 2, 2), (4, 4, 4), (32, 16, 2), (64, 64, 64), (128, 64, 16),
                                   (256, 128, 32), (512, 512, 512), (2, 1024, 2), (1024, 2, 4), (16, 256, 1024),
                                   (8, 8, 4096), (32, 32768, 4), (16, 1 << 20, 2), (4, 1 << 23, 1), (64, 64, 8192),
                                   (128, 64, 4096), (1, 4096, 256), (32, 64, 128), (1, 1, 1024)])
def test_matmul_eq22(M, N, K):
    """Z^i_j = M^i_k L^k_j (eq. (2.2)) through the matrix-product kernel."""
    print(f"matmul M={M} N={N} K={K}", flush=True)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A, B = crand(rng, (M, K)), crand(rng, (K, N))
    got = run_pair(A, [0, 1], B, [1, 2], [0, 2])
    assert relerr(got, oracle.contract(A, [0, 1], B, [1, 2], [0, 2])) < C64_TOL


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_matmul_operand_orientations(ta, tb):
    rng = np.random.default_rng(3)
    M, N, K = 128, 64, 256
    A = crand(rng, (K, M) if ta else (M, K))
    B = crand(rng, (N, K) if tb else (K, N))
    ma = [1, 0] if ta else [0, 1]
    mb = [2, 1] if tb else [1, 2]
    got = run_pair(A, ma, B, mb, [0, 2])
    assert relerr(got, oracle.contract(A, ma, B, mb, [0, 2])) < C64_TOL


def test_batched_matmul_block_diag():
    """Sec. 3's block-diagonal matrices: a batch mode shared by A, B and C."""
    rng = np.random.default_rng(4)
    A, B = crand(rng, (8, 64, 32)), crand(rng, (8, 32, 128))
    got = run_pair(A, [9, 0, 1], B, [9, 1, 2], [9, 0, 2])
    assert relerr(got, oracle.contract(A, [9, 0, 1], B, [9, 1, 2], [9, 0, 2])) < C64_TOL


def test_matvec_trace_outer():
    rng = np.random.default_rng(5)
    M, x = crand(rng, (256, 256)), crand(rng, (256,))
    assert relerr(run_pair(M, [0, 1], x, [1], [0]), M.astype(complex) @ x) < C64_TOL
    I = np.eye(256, dtype=np.complex64)
    assert relerr(run_pair(M, [0, 1], I, [1, 0], []), np.trace(M.astype(complex))) < C64_TOL
    L = crand(rng, (4, 8))
    got = run_pair(M[:16, :16].copy(), [0, 1], L, [2, 3], [0, 2, 1, 3]).reshape(64, 128)
    assert relerr(got, np.kron(M[:16, :16].astype(complex), L.astype(complex))) < C64_TOL


def random_bit_problem(rng, n_batch, n_m, n_n, n_k, big=None):
    """Random extent-2 modes in random orders for A, B and C."""
    modes = list(range(n_batch + n_m + n_n + n_k))
    rng.shuffle(modes)
    bt, mm, nn, kk = (modes[:n_batch], modes[n_batch:n_batch + n_m], modes[n_batch + n_m:n_batch + n_m + n_n],
                      modes[n_batch + n_m + n_n:])
    ma = list(bt + mm + kk)
    mb = list(bt + kk + nn)
    mc = list(bt + mm + nn)
    for l in (ma, mb, mc):
        rng.shuffle(l)
    A = crand(rng, (2,) * len(ma))
    B = crand(rng, (2,) * len(mb))
    return A, ma, B, mb, mc


@pytest.mark.parametrize("seed", range(12))
def test_random_mode_orders(seed):
    """Permute + product on random bit layouts (small and large operands)."""
    rng = np.random.default_rng(1000 + seed)
    shapes = [(0, 3, 8, 2), (1, 2, 10, 1), (0, 7, 7, 6), (2, 6, 5, 7), (0, 0, 12, 2), (1, 1, 1, 1),
              (0, 9, 9, 5), (3, 0, 9, 3), (0, 2, 14, 2), (0, 8, 0, 8), (2, 1, 12, 3), (0, 4, 11, 4)]
    nb, nm, nn, nk = shapes[seed]
    A, ma, B, mb, mc = random_bit_problem(rng, nb, nm, nn, nk)
    print(f"random layout seed={seed} b={nb} m={nm} n={nn} k={nk}", flush=True)
    got = run_pair(A, ma, B, mb, mc)
    assert relerr(got, oracle.contract(A, ma, B, mb, mc)) < C64_TOL


@pytest.mark.parametrize("seed", range(4))
def test_bf16x3_error_bound(seed):
    rng = np.random.default_rng(2000 + seed)
    A, ma, B, mb, mc = random_bit_problem(rng, 0, 7, 7, 6) if seed % 2 == 0 else random_bit_problem(rng, 0, 2, 14, 2)
    want = oracle.contract(A, ma, B, mb, mc)
    e_bf = relerr(run_pair(A, ma, B, mb, mc, "bf16x3"), want)
    e_32 = relerr(run_pair(A, ma, B, mb, mc, "c64"), want)
    print(f"bf16x3 rel err {e_bf:.3e}, c64 {e_32:.3e}", flush=True)
    assert e_bf < BF16X3_TOL
    assert e_32 < C64_TOL


def test_deterministic():
    rng = np.random.default_rng(7)
    A, ma, B, mb, mc = random_bit_problem(rng, 1, 8, 8, 6)
    x = run_pair(A, ma, B, mb, mc)
    y = run_pair(A, ma, B, mb, mc)
    assert np.array_equal(x, y)


def _bw16_path():
    import workloads
    from paper_2108_06831_amd import Network
    circ = workloads.brickwork(16, 12, np.random.default_rng(5))
    net = Network.from_circuit(circ)
    return circ, net, net.plan(kind="greedy")


@pytest.mark.parametrize("precision", ["c64", "bf16x3"])
def test_every_gemm_launch_shape(precision):
    """Every valid (tile, K split) launch shape of every product step of a
    16-qubit brickwork contraction gives the oracle's statevector."""
    import torch
    from paper_2108_06831_amd import TNError, contract_path
    circ, net, path = _bw16_path()
    want = oracle.statevector(circ)
    tol = C64_TOL if precision == "c64" else BF16X3_TOL
    shapes = path.gemm_configs(precision)
    assert shapes
    tried = 0
    for s, (t0, s0, o0) in shapes.items():
        for tr in (0, 1):
            for tile in range(9):
                for split in (1, 2, 4, 8):
                    try:
                        path.set_gemm_config(s, tile, split, tr, precision)
                    except TNError:
                        continue
                    print(f"step {s} bmnk {path.step(s)['bmnk']} tile {tile} split {split} transposed {tr} "
                          f"{precision}", flush=True)
                    got = contract_path(net, path, precision=precision)
                    torch.cuda.synchronize()
                    err = relerr(got.cpu().numpy()[0], want)
                    assert err < tol, (s, tile, split, tr, err)
                    tried += 1
        path.set_gemm_config(s, t0, s0, o0, precision)
    assert tried >= 8 * len(shapes)


def test_autotune_keeps_results():
    import torch
    from paper_2108_06831_amd import autotune, contract_path
    circ, net, path = _bw16_path()
    want = oracle.statevector(circ)
    rep = autotune(net, path, reps=3)
    print("autotune", rep, flush=True)
    assert rep["n_products"] == len(path.gemm_configs())
    assert rep["seconds_after"] <= rep["seconds_before"] * 1.0001
    got = contract_path(net, path)
    torch.cuda.synchronize()
    assert relerr(got.cpu().numpy()[0], want) < C64_TOL


def test_profile_counts_every_launch():
    """Kernel timing with runs of product launches sharing one event pair:
    every product launch (a launch may run several grouped products) is
    counted once and the products' algorithmic flops in full, whether all
    kinds or the products alone are timed, and the results are unchanged."""
    import torch
    from paper_2108_06831_amd import contract_path, profile_enable, profile_read, profile_reset, profile_select
    circ, net, path = _bw16_path()
    want = oracle.statevector(circ)
    n_gemm = len(path.gemm_configs())
    flops = sum(8.0 * np.prod(path.step(s)["bmnk"]) for s in path.gemm_configs())
    for kinds in (None, ["gemm"]):
        profile_reset()
        profile_select(kinds)
        profile_enable(True)
        got = contract_path(net, path)
        prof = profile_read()
        profile_enable(False)
        profile_select(None)
        print(kinds, {k: (v["launches"], round(v["seconds"] * 1e6, 1)) for k, v in prof.items()}, flush=True)
        assert prof["gemm"]["launches"] == path.stats["n_product_launches"] <= n_gemm
        assert prof["gemm"]["flops"] == pytest.approx(flops, rel=1e-12)
        assert prof["gemm"]["seconds"] > 0
        if kinds is not None:
            assert set(prof) <= {"gemm", "gemm_large"}
        torch.cuda.synchronize()
        assert relerr(got.cpu().numpy()[0], want) < C64_TOL


def test_wide_tile_offsets():
    """An 8 GiB operand whose top address bit is the result's lowest m bit:
    a tile's element offsets span more than 2^32 bytes, so the matrix-core
    kernel takes its full-pointer form.  Sampled outputs against the
    definition of the contraction (eq. (2.2))."""
    import torch
    from paper_2108_06831_amd import contract_pair
    print("wide tile offsets: A 2 x 2^20 x 512 (8 GiB), B 512 x 64", flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    A = torch.randn((2, 1 << 20, 512), dtype=torch.complex64, device="cuda", generator=gen)
    rng = np.random.default_rng(11)
    B = crand(rng, (512, 64))
    C = contract_pair(A, [0, 1, 2], torch.from_numpy(B).cuda(), [2, 3], [1, 3, 0])
    torch.cuda.synchronize()
    i0 = torch.as_tensor(rng.integers(0, 2, 96), device="cuda")
    i1 = torch.as_tensor(rng.integers(0, 1 << 20, 96), device="cuda")
    rows = A[i0, i1].cpu().numpy()
    got = C[i1, :, i0].cpu().numpy()
    del A, C
    torch.cuda.empty_cache()
    want = oracle.contract(rows, [0, 1], B, [1, 2], [0, 2])
    assert relerr(got, want) < C64_TOL


@pytest.mark.parametrize("grid", ["4x6", "4x8"])
def test_batch_packed_tile(grid):
    """The packed matrix-core tiles on every product step of a grid
    circuit's amplitude network that admits one: batch-packed (four batch
    items of at most 32 x 32 per workgroup) where it fits, else
    column-packed (M <= 32, four 32-column slices).  Ragged items (M, N in
    1..16) and sums of 1 to 256 terms on the 4x6 grid, against its
    statevector; whole 32 x 32 items with 8 and 32 terms on the 32-qubit
    grid, sampled amplitudes against the oracle's contraction of each."""
    import workloads
    from paper_2108_06831_amd import Network, TNError, amplitudes
    rows, cols = (4, 6) if grid == "4x6" else (4, 8)
    circ, bits = workloads.config2(rows, cols, 12, n_bitstrings=4096)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=4096)
    path = net.plan("search", max_log2_intermediate=28, trials=64, seed=1)
    packed, columns = [], []
    for s in path.gemm_configs():
        for tile, got in ((7, packed), (8, columns)):
            try:
                path.set_gemm_config(s, tile, 1, 0, "c64")
                got.append(path.step(s)["bmnk"])
                break
            except TNError:
                pass
    print(f"grid {grid}: batch-packed {sorted(set(packed))}, column-packed {sorted(set(columns))}", flush=True)
    assert packed and columns
    got = amplitudes(net, path, bits).cpu().numpy()
    if grid == "4x6":
        want = oracle.amplitudes(oracle.statevector(circ), circ.n_qubits, bits)
        assert relerr(got, want) < C64_TOL
    else:
        assert any(b[1] == 32 and b[2] == 32 for b in packed)
        idx = sorted(np.random.default_rng(78).choice(4096, size=8, replace=False).tolist())
        want = np.array([oracle.single_amplitude(circ, int(bits[i])) for i in idx])
        assert relerr(got[idx], want) < C64_TOL


def test_fresh_process_whose_first_call_is_the_library():
    """A process that builds and plans through the library before it touches
    torch: the binding loads torch's HIP runtime first, so both share it and
    the contraction runs (regression: the library loaded first found no
    device once torch had started its own runtime)."""
    import subprocess
    import sys
    code = (
        "import numpy as np, workloads, oracle\n"
        "from paper_2108_06831_amd import Network, contract_path\n"
        "c = workloads.config0(); net = Network.from_circuit(c); p = net.plan('greedy')\n"
        "got = contract_path(net, p).cpu().numpy()[0]; want = oracle.statevector(c)\n"
        "print('ERR', float(np.linalg.norm(got - want) / np.linalg.norm(want)))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=240)
    print(r.stdout[-500:], r.stderr[-500:], flush=True)
    assert r.returncode == 0
    err = float([ln for ln in r.stdout.splitlines() if ln.startswith("ERR")][0].split()[1])
    assert err < 1e-5
