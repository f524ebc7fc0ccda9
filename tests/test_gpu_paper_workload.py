"""The paper's own test circuit (Fig. 3.1, Sec. 3): n qubits, k rounds of
CNOT(2i -> 2i+1), RZ on every qubit, CZ(2i+1, 2i+2), RX on every qubit,
between layers of H.  Statevectors and the closed-network amplitude
<0...0|U|0...0> on the GPU against the FP64 oracle.  GPU only."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "bf16x3": 1e-3}


def relerr(got, want):
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    want = np.asarray(want, dtype=np.complex128).reshape(-1)
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


@pytest.mark.parametrize("n,k", [(2, 2), (3, 4), (6, 6), (10, 8), (14, 14), (20, 4), (22, 6)])
@pytest.mark.parametrize("kind", ["greedy", "search"])
def test_fig31_statevector(n, k, kind):
    from paper_2108_06831_amd import Network, contract_path
    circ = workloads.paper_test_circuit(n, k)
    net = Network.from_circuit(circ)
    path = net.plan(kind, trials=32)
    got = contract_path(net, path).cpu().numpy()[0]
    e = relerr(got, oracle.statevector(circ))
    print(f"  n={n} k={k} {kind}: rel err {e:.2e}", flush=True)
    assert e < TOL["c64"]


@pytest.mark.parametrize("n,k", [(2, 14), (8, 8), (12, 10), (16, 12), (22, 14)])
@pytest.mark.parametrize("precision", ["c64", "bf16x3"])
def test_fig31_zero_amplitude(n, k, precision):
    """<0...0|U|0...0>: the network closed by the all-zeros bra (Sec. 2.2.3),
    together with a few more bitstrings in the same batch."""
    from paper_2108_06831_amd import Network, amplitudes
    circ = workloads.paper_test_circuit(n, k)
    rng = np.random.default_rng(1000 * n + k)
    bits = np.concatenate([np.zeros(1, dtype=np.uint64),
                           rng.integers(0, 1 << n, size=7, dtype=np.uint64)])
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=len(bits))
    path = net.plan("greedy")
    got = amplitudes(net, path, bits, precision=precision).cpu().numpy()
    want = oracle.amplitudes(oracle.statevector(circ), n, bits)
    e = relerr(got, want)
    print(f"  n={n} k={k} {precision}: <0|U|0> = {got[0]:.6f} (oracle {want[0]:.6f}), batch rel err {e:.2e}",
          flush=True)
    assert e < TOL[precision]


@pytest.mark.parametrize("n,k", [(6, 4), (18, 8)])
def test_fig31_single_amplitude_network(n, k):
    """A network closed by one bitstring only (a batch index of extent 1)."""
    from paper_2108_06831_amd import Network, amplitudes
    circ = workloads.paper_test_circuit(n, k)
    net = Network.from_circuit(circ, output="amplitudes", n_bitstrings=1)
    path = net.plan("greedy")
    got = amplitudes(net, path, np.zeros(1, dtype=np.uint64)).cpu().numpy()
    want = oracle.statevector(circ)[0]
    print(f"  n={n} k={k}: {got[0]:.6f} vs {want:.6f}", flush=True)
    assert got.shape == (1,) and abs(got[0] - want) / max(abs(want), 1.0) < TOL["c64"]
