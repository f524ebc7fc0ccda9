"""tn_contract_path_noalloc (workspace in the library's static device array)
against tn_contract_path (caller's workspace) on the same inputs: two calls
in a row, the second on a smaller network, each equal to the allocating
call element by element (the same kernels and launch shapes on the same
operands).  Also the argument checks that need no kernel.  GPU only."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _noalloc(net, path, params=None, batch=1):
    import torch
    from paper_2108_06831_amd import _lib, _ptr, _stream_handle, tn_contract_path_noalloc
    p = None if params is None else torch.as_tensor(params, dtype=torch.float64, device="cuda").reshape(
        batch, net.n_params).contiguous()
    out = torch.full((batch, 1 << net.n_qubits), float("nan"), dtype=torch.complex64, device="cuda")
    tn_contract_path_noalloc(_stream_handle(), _lib.TN_PREC_C64, net, path, _ptr(p), batch, _ptr(out))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_allocating_call_twice():
    import torch
    from paper_2108_06831_amd import Network, TNError, contract_path
    from paper_2108_06831_amd import _lib
    big = workloads.random_circuit(16, 160, np.random.default_rng(31))
    circ4, params4, _ = workloads.config4(n=12, layers=3, batch=3)
    cases = [(big, None, 1, "search"), (circ4, params4, 3, "sequential")]
    nets = [Network.from_circuit(c, fuse=(k == "search")) for c, _, _, k in cases]
    paths = [nt.plan(k, trials=16) for nt, (_, _, _, k) in zip(nets, cases)]
    assert paths[0].workspace_bytes(1) > paths[1].workspace_bytes(3)  # the second call is the smaller one
    # before any allocating call the device tables do not exist: refused, nothing launched
    with pytest.raises(TNError) as ei:
        _noalloc(nets[0], paths[0])
    assert ei.value.status == _lib.TN_EINVAL
    want = []
    for nt, pt, (c, prm, b, _) in zip(nets, paths, cases):
        want.append(contract_path(nt, pt, params=prm, batch=b).cpu().numpy())
    torch.cuda.synchronize()
    for nt, pt, (c, prm, b, _), w in zip(nets, paths, cases, want):
        got = _noalloc(nt, pt, prm, b)
        print(f"  {c.name}: batch {b}, workspace {pt.workspace_bytes(b)} bytes, "
              f"max |diff| {np.max(np.abs(got - w)):.1e}", flush=True)
        assert got.shape == w.shape and np.array_equal(got, w)


def test_noalloc_rejects_workspace_beyond_the_scratch():
    from paper_2108_06831_amd import Network, TNError, contract_path
    from paper_2108_06831_amd import _lib
    circ = workloads.random_circuit(23, 40, np.random.default_rng(32))
    net = Network.from_circuit(circ)
    path = net.plan("sequential")
    assert path.workspace_bytes(1) > (64 << 20)
    contract_path(net, path)  # creates the device tables
    with pytest.raises(TNError) as ei:
        _noalloc(net, path)
    assert ei.value.status == _lib.TN_ENOMEM
