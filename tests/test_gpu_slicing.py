"""Index slicing on the GPU: paths planned under a cap below the unsliced
largest intermediate, contracted slice by slice (each slice's inputs gathered
from the full input tensors, its program run, its result added to a running
sum), against the oracle.  A sum over a bond index is the sum of the
contractions with that index fixed (eq. (2.2)), so the sliced result is the
same quantity; only the rounding order differs.  GPU only."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

# complex64 products along orders of a few hundred steps: normwise relative
# error of a few 1e-7 per step's rounding, summed over at most 2^9 slices;
# 2e-5 leaves an order of magnitude of room (the same bound as the unsliced
# amplitude tests); BF16x3 carries about 16 mantissa bits per operand
TOL = {"c64": 2e-5, "bf16x3": 2e-4}


def rel(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


@pytest.mark.parametrize("cap,kind", [(16, "greedy"), (14, "search"), (12, "greedy")])
@pytest.mark.parametrize("precision", ["c64", "bf16x3"])
def test_sliced_amplitudes_match_oracle(cap, kind, precision):
    """4x6 grid of depth 12, 256 bitstrings; unsliced largest intermediate 2^22."""
    from paper_2108_06831_amd import Network, amplitudes
    circ, bits = workloads.config2(rows=4, cols=6, depth=12, n_bitstrings=256)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=len(bits))
    path = net.plan(kind, max_log2_intermediate=cap, max_slice_bits=16, trials=8)
    assert path.stats["n_slice_bits"] > 0 and path.stats["max_intermediate_elems"] <= 2 ** cap
    got = amplitudes(net, path, bits, precision=precision).cpu().numpy()
    want = oracle.amplitudes(oracle.statevector(circ), circ.n_qubits, bits)
    e = rel(got, want)
    print(f"  cap 2^{cap} {kind} {precision}: {2 ** path.stats['n_slice_bits']} slices, rel err {e:.2e}", flush=True)
    assert got.shape == want.shape and e < TOL[precision]


@pytest.mark.parametrize("fuse", [False, "dense"])
def test_sliced_statevector_batch_matches_oracle(fuse):
    """10-qubit HEA, 3 layers, three parameter vectors: every batch item's
    state from a path sliced under a cap of 2^10 (the state's own size)."""
    from paper_2108_06831_amd import Network, contract_path
    circ, params, _ = workloads.config4(n=10, layers=3, batch=3)
    net = Network.from_circuit(circ, fuse=fuse)
    path = net.plan("greedy", max_log2_intermediate=10, max_slice_bits=8)
    assert path.stats["n_slice_bits"] > 0
    got = contract_path(net, path, params=params, batch=3).cpu().numpy()
    for b in range(3):
        e = rel(got[b], oracle.statevector(circ, params[b]))
        print(f"  fuse={fuse} vector {b}: rel err {e:.2e}", flush=True)
        assert e < TOL["c64"]


def test_sliced_expectation_matches_oracle():
    from paper_2108_06831_amd import Network, Observable, expectation
    circ, params, (masks, coeffs) = workloads.config4(n=12, layers=4, batch=2)
    net = Network.from_circuit(circ)
    path = net.plan("greedy", max_log2_intermediate=12, max_slice_bits=8)
    assert path.stats["n_slice_bits"] > 0
    got = expectation([net], [path], [params], [Observable(masks, coeffs)], batch=2).cpu().numpy().reshape(-1)
    for b in range(2):
        want = oracle.circuit_expectation(circ, params[b], masks, coeffs)
        print(f"  vector {b}: {got[b]:.7f} vs {want:.7f}", flush=True)
        assert abs(got[b] - want) < 1e-4 * max(1.0, float(np.sum(np.abs(coeffs))))


def test_full_size_grid_sliced_amplitudes_sampled():
    """The 4x8 grid of depth 12 with 4096 bitstrings, sliced under a cap of
    2^20 (unsliced: 2^22): sampled amplitudes against the oracle's
    single-amplitude contraction."""
    from paper_2108_06831_amd import Network, amplitudes
    circ, bits = workloads.config2()
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=len(bits))
    path = net.plan("greedy", max_log2_intermediate=20, max_slice_bits=12)
    assert path.stats["n_slice_bits"] > 0
    got = amplitudes(net, path, bits).cpu().numpy()
    ref = amplitudes(net, net.plan("greedy"), bits).cpu().numpy()
    rng = np.random.default_rng(2003)
    idx = rng.choice(len(bits), size=6, replace=False)
    want = np.array([oracle.single_amplitude(circ, int(bits[i])) for i in idx])
    e = rel(got[idx], want)
    print(f"  {2 ** path.stats['n_slice_bits']} slices: sampled rel err {e:.2e}; "
          f"vs unsliced path {rel(got, ref):.2e}", flush=True)
    assert e < TOL["c64"] and rel(got, ref) < TOL["c64"]


def test_unsupported_calls_on_sliced_paths_are_refused():
    import torch
    from paper_2108_06831_amd import Network, Observable, TNError, _lib, autotune, backward, contract_path
    from paper_2108_06831_amd import tn_contract_path_noalloc, _ptr, _params_tensor, _stream_handle
    circ, params, (masks, coeffs) = workloads.config4(n=10, layers=3, batch=1)
    net = Network.from_circuit(circ)
    path = net.plan("greedy", max_log2_intermediate=10, max_slice_bits=8)
    assert path.stats["n_slice_bits"] > 0
    calls = [
        lambda: contract_path(net, path, params=params, precision="q3.28"),
        lambda: backward(net, path, params, Observable(masks, coeffs)),
        lambda: autotune(net, path, params=params),
    ]
    for call in calls:
        with pytest.raises(TNError) as ei:
            call()
        assert ei.value.status == _lib.TN_EUNSUPPORTED
    out = torch.empty((1, 2 ** 10), dtype=torch.complex64, device="cuda")
    p = _params_tensor(net, params, 1, "cuda")
    with pytest.raises(TNError) as ei:
        tn_contract_path_noalloc(_stream_handle(), _lib.TN_PREC_C64, net, path, _ptr(p), 1, _ptr(out))
    assert ei.value.status == _lib.TN_EUNSUPPORTED
