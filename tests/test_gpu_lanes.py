"""tn_expectation spreads the circuits of one call over stream lanes (the
caller's stream and three of the library's, each with its own workspace
slot).  Every circuit's result must equal the same circuit computed alone in
a one-circuit call (one lane), bit for bit: the same kernels on the same
inputs.  Mixed sizes, a sliced path and a parameter batch among them.  GPU only."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def test_lanes_match_single_circuit_calls():
    import torch
    from paper_2108_06831_amd import Network, Observable, expectation
    inst = [it for it in workloads.config3() if it.circuit.n_qubits <= 20][:7]
    nets = [Network.from_circuit(it.circuit) for it in inst]
    paths = [nt.plan("sequential") for nt in nets]
    obs = [Observable(*workloads.maxcut_observable(it.circuit.n_qubits, it.edges)) for it in inst]
    params = [it.params for it in inst]
    # a sliced hardware-efficient ansatz among the QAOA circuits
    circ, hp, (m, c) = workloads.config4(n=10, layers=3, batch=1)
    hnet = Network.from_circuit(circ)
    hpath = hnet.plan("greedy", max_log2_intermediate=10, max_slice_bits=8)
    assert hpath.stats["n_slice_bits"] > 0
    nets.insert(3, hnet)
    paths.insert(3, hpath)
    obs.insert(3, Observable(m, c))
    params.insert(3, hp[0])
    together = expectation(nets, paths, params, obs).cpu().numpy()[:, 0]
    alone = np.array([expectation([n], [p], [q], [o]).cpu().numpy()[0, 0]
                      for n, p, q, o in zip(nets, paths, params, obs)])
    print(f"  {len(nets)} circuits: max |together - alone| = {np.max(np.abs(together - alone)):.1e}", flush=True)
    assert np.array_equal(together, alone)
    want = oracle.circuit_expectation(circ, hp[0], m, c)
    assert abs(together[3] - want) < 1e-4 * max(1.0, float(np.sum(np.abs(c))))


def test_lanes_with_a_parameter_batch():
    from paper_2108_06831_amd import Network, Observable, expectation
    circ, params, (m, c) = workloads.config4(n=12, layers=2, batch=3)
    nets = [Network.from_circuit(circ) for _ in range(5)]
    paths = [nt.plan("sequential") for nt in nets]
    obs = [Observable(m, c) for _ in range(5)]
    got = expectation(nets, paths, [params] * 5, obs, batch=3).cpu().numpy()
    want = np.array([oracle.circuit_expectation(circ, params[b], m, c) for b in range(3)])
    for i in range(5):
        assert np.array_equal(got[i], got[0])
    assert np.max(np.abs(got[0] - want)) < 1e-4 * max(1.0, float(np.sum(np.abs(c))))
