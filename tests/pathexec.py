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


def execute_sliced(net, path, params=None, bitstrings=None):
    """The same for a sliced path: every slice fixes the sliced modes' indices
    (np.take on each tensor that holds them), contracts the remaining network
    along the path, and the slices' results are summed."""
    vals = net.values(params, bitstrings)
    info = net.info()
    T = info["n_tensors"]
    cut = path.slices()
    ext = {}
    for t in range(T):
        modes, exts = net.tensor(t)
        for m, e in zip(modes, exts):
            ext[m] = e
    total = None
    n_slices = int(np.prod([ext[m] for m in cut])) if cut else 1
    for sigma in range(n_slices):
        fixed, r = {}, sigma
        for m in cut:
            fixed[m] = r % ext[m]
            r //= ext[m]
        tensors = {}
        for t in range(T):
            X, modes = vals[t], list(net.tensor(t)[0])
            for m in cut:
                while m in modes:
                    ax = modes.index(m)
                    X = np.take(X, fixed[m], axis=ax)
                    modes.pop(ax)
            tensors[t] = (X, modes)
        for s, (i, j) in enumerate(path.pairs()):
            (A, ma), (B, mb) = tensors.pop(i), tensors.pop(j)
            mc = path.step(s)["modes"]
            table = {}
            spec = f"{_letters(ma, table)},{_letters(mb, table)}->{_letters(mc, table)}"
            tensors[T + s] = (np.einsum(spec, A, B), mc)
        (X, mx), = tensors.values()
        out_modes, _ = net.output()
        table = {}
        X = np.einsum(f"{_letters(mx, table)}->{_letters(out_modes, table)}", X)
        total = X if total is None else total + X
    return total
