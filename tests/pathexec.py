"""CPU FP64 executor of a planned path (a debugging aid for the host logic,
not the oracle): contracts the network's FP64 input tensors pair by pair
with numpy.einsum, following the library's SSA pairs and result-mode orders."""
import numpy as np


def _letters(modes, table):
    s = ""
    for m in modes:
        if m not in table:
            table[m] = chr(ord("a") + len(table)) if len(table) < 26 else chr(ord("A") + len(table) - 26)
        s += table[m]
    return s


def execute(net, path, params=None, bitstrings=None):
    vals = net.values(params, bitstrings)
    info = net.info()
    T = info["n_tensors"]
    tensors = {t: (vals[t], net.tensor(t)[0]) for t in range(T)}
    for s, (i, j) in enumerate(path.pairs()):
        (A, ma), (B, mb) = tensors.pop(i), tensors.pop(j)
        mc = path.step(s)["modes"]
        table = {}
        spec = f"{_letters(ma, table)},{_letters(mb, table)}->{_letters(mc, table)}"
        tensors[T + s] = (np.einsum(spec, A, B), mc)
    assert len(tensors) == 1
    (X, mx), = tensors.values()
    out_modes, _ = net.output()
    table = {}
    return np.einsum(f"{_letters(mx, table)}->{_letters(out_modes, table)}", X)
