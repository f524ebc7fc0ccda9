"""The Q3.28 fixed-point mode (Sec. 3: the FPGA designs compute in 32-bit
fixed point with 28 fractional bits) on the GPU.

Along the sequential order of the unfused network every step applies one
gate to the state, so the GPU's fixed-point contraction performs exactly the
rounded products and saturating sums of the oracle's fixed-point gate-by-gate
sweep: the two agree bit for bit (integer work).  Along other orders the
rounding happens elsewhere; there the error against the FP64 oracle is
reported and held to a bound derived from the arithmetic.  GPU only."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def as_c64(raw):
    """Oracle Q3.28 state -> complex64 the way the library converts it (exact
    double, then rounded once to float32 per component)."""
    raw = np.asarray(raw, dtype=np.int64).reshape(-1, 2)
    out = np.empty(raw.shape[0], dtype=np.complex64)
    out.real = (raw[:, 0].astype(np.float64) / 2.0 ** 28).astype(np.float32)
    out.imag = (raw[:, 1].astype(np.float64) / 2.0 ** 28).astype(np.float32)
    return out


def gpu_state(circ, kind, fuse=False, params=None, batch=1):
    from paper_2108_06831_amd import Network, contract_path
    net = Network.from_circuit(circ, fuse=fuse)
    path = net.plan(kind, trials=16)
    return contract_path(net, path, params=params, batch=batch, precision="q3.28").cpu().numpy()


@pytest.mark.parametrize("case", ["config0", "random_all_kinds", "ghz14", "hea_batch"])
def test_sequential_order_bit_exact_with_oracle(case):
    if case == "config0":
        circ, params = workloads.config0(), None
    elif case == "random_all_kinds":
        circ, params = workloads.random_circuit(12, 150, np.random.default_rng(2801)), None
    elif case == "ghz14":
        n = 14
        circ = workloads.Circuit(n, [workloads.Gate("H", (0,))] +
                                 [workloads.Gate("CNOT", (q, q + 1)) for q in range(n - 1)])
        params = None
    else:
        circ, params, _ = workloads.config4(n=10, layers=3, batch=3)
    batch = 1 if params is None else params.shape[0]
    got = gpu_state(circ, "sequential", params=params, batch=batch)
    for b in range(batch):
        want = as_c64(oracle.statevector_q328(circ, None if params is None else params[b]))
        diff = int(np.sum(got[b] != want))
        print(f"  {case} vector {b}: {diff} of {want.size} elements differ", flush=True)
        assert diff == 0


@pytest.mark.parametrize("kind,fuse", [("greedy", False), ("search", "split"), ("greedy", "dense")])
def test_other_orders_within_the_rounding_bound(kind, fuse):
    """Every step of any order adds at most one rounding (2^-29) per real
    product; for these small networks the state's normwise error against FP64
    stays far below 1e-4 (reported)."""
    for circ in (workloads.config0(), workloads.random_circuit(16, 200, np.random.default_rng(2802))):
        got = gpu_state(circ, kind, fuse)[0]
        want = oracle.statevector(circ)
        e = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        e_c64 = float(np.linalg.norm(gpu_c64(circ, kind, fuse) - want) / np.linalg.norm(want))
        print(f"  {circ.name} {kind}/{fuse}: Q3.28 rel err {e:.2e} (complex64 {e_c64:.2e})", flush=True)
        assert e < 1e-4


def gpu_c64(circ, kind, fuse):
    from paper_2108_06831_amd import Network, contract_path
    net = Network.from_circuit(circ, fuse=fuse)
    return contract_path(net, net.plan(kind, trials=16)).cpu().numpy()[0]


def test_amplitudes_q328():
    """Grid amplitudes (4x4, depth 10) through a closed network in fixed
    point, against the FP64 oracle."""
    from paper_2108_06831_amd import Network, amplitudes
    circ, bits = workloads.config2(rows=4, cols=4, depth=10, n_bitstrings=300)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=len(bits))
    path = net.plan("greedy")
    got = amplitudes(net, path, bits, precision="q3.28").cpu().numpy()
    want = oracle.amplitudes(oracle.statevector(circ), circ.n_qubits, bits)
    e = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    print(f"  300 amplitudes of the 4x4 grid: Q3.28 rel err {e:.2e}", flush=True)
    assert got.shape == (300,) and e < 1e-4


def test_unsupported_calls_are_refused():
    import torch
    from paper_2108_06831_amd import Network, Observable, TNError, _lib, expectation
    circ, params, (m, c) = workloads.config4(n=6, layers=1, batch=1)
    net = Network.from_circuit(circ)
    path = net.plan("sequential")
    with pytest.raises(TNError) as ei:
        expectation([net], [path], [params[0]], [Observable(m, c)], precision="q3.28")
    assert ei.value.status == _lib.TN_EUNSUPPORTED


def test_error_against_fp64_on_the_workloads():
    """The paper's robustness question (Sec. 2.3, Sec. 3): the error of the
    Q3.28 mode against the FP64 oracle beside complex64 and BF16x3, on the
    10- and 24-qubit brickwork statevectors and on sampled amplitudes of the
    4x8 grid (reported).  Along the sequential order every intermediate is a
    state of norm 1 and every step sums at most K = 4 products per output,
    each real product rounded once (at most 2^-29): a step adds an error
    vector of norm at most sqrt(2 * 2^n) * 2K * 2^-29 (values stay within
    modulus 1, so nothing saturates), and unitary steps do not grow earlier
    errors, so steps x that bound holds the whole run."""
    from paper_2108_06831_amd import Network, amplitudes, contract_path
    for name, circ in (("10-qubit brickwork", workloads.config0()), ("24-qubit brickwork", workloads.config1())):
        want = oracle.statevector(circ)
        net = Network.from_circuit(circ, fuse="dense")
        path = net.plan("sequential")
        errs = {}
        for prec in ("c64", "bf16x3", "q3.28"):
            got = contract_path(net, path, precision=prec).cpu().numpy()[0]
            errs[prec] = float(np.linalg.norm(got - want))
        bound = path.stats["n_steps"] * np.sqrt(2.0 * 2 ** circ.n_qubits) * 8 * 2.0 ** -29
        print(f"  {name}, sequential order: normwise error c64 {errs['c64']:.2e}, bf16x3 {errs['bf16x3']:.2e}, "
              f"q3.28 {errs['q3.28']:.2e} (bound {bound:.1e})", flush=True)
        # the final conversion to complex64 adds at most 2^-24 relative per component
        assert errs["q3.28"] < bound + 1e-6
    circ, bits = workloads.config2()
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=len(bits))
    path = net.plan("greedy")
    idx = np.random.default_rng(2004).choice(len(bits), size=4, replace=False)
    want = np.array([oracle.single_amplitude(circ, int(bits[i])) for i in idx])
    msg = []
    for prec in ("c64", "bf16x3", "q3.28"):
        try:
            got = amplitudes(net, path, bits, precision=prec).cpu().numpy()[idx]
        except Exception as e:  # a step beyond the fixed-point kernel's index limits
            msg.append(f"{prec}: {e}")
            continue
        msg.append(f"{prec} {float(np.linalg.norm(got - want) / np.linalg.norm(want)):.2e}")
    print("  4x8 grid, greedy order, 4 sampled amplitudes, relative error: " + ", ".join(msg), flush=True)
