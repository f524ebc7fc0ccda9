"""FP64 CPU oracle: the plain definition of what the GPU path computes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with ``paper_2108_06831_amd`` (neither imports the other); both read
circuits from the ``workloads`` package, which holds no simulation arithmetic.

* ``statevector``        gate-by-gate FP64 sweep from |0...0> (Sec. 2.1).
* ``dense_unitary``      the circuit's 2^n x 2^n matrix from element-wise
                         gate embeddings, n <= 10 (Sec. 2.1, Kronecker products).
* ``expectation``        <psi|D|psi> for diagonal Z-string observables.
* ``amplitudes``         <b|psi>: closing the network with basis states
                         (Sec. 2.2.3).
* ``param_shift_gradient`` exact derivative of an expectation with respect to
                         each parameter, by the two-term shift rule of gates
                         exp(-i theta G) whose generator G has two eigenvalues.
* ``contract``           the definition of a pairwise tensor contraction
                         (Sec. 2.2.1: a sum over shared indices, eq. (2.2)).
* ``statevector_q328``   the gate-by-gate sweep in Q3.28 fixed point (Sec. 3's
                         32-bit format with 28 fractional bits).
* ``single_amplitude``   <b|U|0...0> of a circuit too wide for a full FP64
                         state, by contracting its closed network (Sec. 2.2.2)
                         pairwise in FP64 along a plain greedy order.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

from workloads import Circuit, Gate, TWO_QUBIT

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")  # ORACLE_LIB: sanitizer build

KIND_ID = {"H": 0, "X": 1, "Y": 2, "Z": 3, "S": 4, "T": 5, "SX": 6, "SY": 7, "SW": 8,
           "RX": 9, "RY": 10, "RZ": 11, "U3": 12, "MIXER": 13,
           "CZ": 32, "CNOT": 33, "SWAP": 34, "CPHASE": 35, "ZZPHASE": 36}
MAT1, MAT2 = 64, 65

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from oracle.build import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.oracle_gate_matrix.argtypes = [ctypes.c_int, P, P]
    lib.oracle_gate_matrix.restype = ctypes.c_int
    lib.oracle_statevector.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    lib.oracle_statevector.restype = ctypes.c_int
    lib.oracle_dense_unitary.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    lib.oracle_dense_unitary.restype = ctypes.c_int
    lib.oracle_expectation_zstrings.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P]
    lib.oracle_expectation_zstrings.restype = ctypes.c_double
    lib.oracle_amplitudes.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P]
    lib.oracle_amplitudes.restype = None
    lib.oracle_statevector_q328.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    lib.oracle_statevector_q328.restype = ctypes.c_int
    lib.oracle_q328_mul.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.oracle_q328_mul.restype = ctypes.c_int32
    lib.oracle_q328_from_double.argtypes = [ctypes.c_double]
    lib.oracle_q328_from_double.restype = ctypes.c_int32
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def gate_matrix(kind: str, angles: Sequence[float] = ()) -> np.ndarray:
    """The gate's matrix (2x2 or 4x4 complex128)."""
    lib = _load()
    ang = np.zeros(3, dtype=np.float64)
    ang[: len(angles)] = angles
    d = 4 if kind in TWO_QUBIT else 2
    out = np.zeros(32, dtype=np.float64)
    if lib.oracle_gate_matrix(KIND_ID[kind], _ptr(ang), _ptr(out)) != 0:
        raise ValueError(kind)
    return out[: 2 * d * d].view(np.complex128).reshape(d, d).copy()


def _marshal(circ: Circuit, params: Optional[np.ndarray], matrices=None):
    g = len(circ.gates)
    kinds = np.zeros(g, dtype=np.int32)
    qubits = np.full(2 * g, -1, dtype=np.int32)
    angles = np.zeros(3 * g, dtype=np.float64)
    mats = np.zeros(32 * max(g, 1), dtype=np.float64)
    for i, gate in enumerate(circ.gates):
        kinds[i] = KIND_ID[gate.kind]
        qubits[2 * i: 2 * i + len(gate.qubits)] = gate.qubits
        a = circ.resolved_angles(gate, params)
        angles[3 * i: 3 * i + len(a)] = a
    if matrices:
        for i, m in matrices.items():
            m = np.asarray(m, dtype=np.complex128)
            kinds[i] = MAT2 if m.shape[0] == 4 else MAT1
            flat = m.reshape(-1).view(np.float64)
            mats[32 * i: 32 * i + flat.size] = flat
    return kinds, qubits, angles, mats


def statevector(circ: Circuit, params: Optional[np.ndarray] = None, matrices=None) -> np.ndarray:
    """FP64 state after the circuit, from |0...0>; complex128[2^n], qubit 0 = MSB.
    ``matrices`` optionally replaces gate i by an explicit matrix {i: U}."""
    lib = _load()
    n = circ.n_qubits
    kinds, qubits, angles, mats = _marshal(circ, params, matrices)
    psi = np.empty(2 << n, dtype=np.float64)
    rc = lib.oracle_statevector(n, len(circ.gates), _ptr(kinds), _ptr(qubits), _ptr(angles), _ptr(mats),
                                _ptr(psi))
    if rc != 0:
        raise ValueError("oracle_statevector rejected the circuit")
    return psi.view(np.complex128)


Q328_ONE = 1 << 28


def q328_mul(a: int, b: int) -> int:
    """Q3.28 product of two raw int32 values (rounded to nearest, ties to even; saturating)."""
    return int(_load().oracle_q328_mul(int(a), int(b)))


def q328_from_double(x: float) -> int:
    """The raw int32 Q3.28 value nearest to x (ties to even; saturating)."""
    return int(_load().oracle_q328_from_double(float(x)))


def statevector_q328(circ: Circuit, params: Optional[np.ndarray] = None) -> np.ndarray:
    """The gate-by-gate state in Q3.28 fixed point (Sec. 3's 32-bit format with
    28 fractional bits; reading: two's complement, products rounded to
    nearest-even, saturating sums): raw int32 array [2^n, 2] of (re, im)."""
    lib = _load()
    n = circ.n_qubits
    kinds, qubits, angles, mats = _marshal(circ, params, None)
    psi = np.empty((1 << n, 2), dtype=np.int32)
    rc = lib.oracle_statevector_q328(n, len(circ.gates), _ptr(kinds), _ptr(qubits), _ptr(angles), _ptr(mats),
                                     _ptr(psi))
    if rc != 0:
        raise ValueError("oracle_statevector_q328 rejected the circuit")
    return psi


def q328_to_complex(raw: np.ndarray) -> np.ndarray:
    """complex128 values of raw Q3.28 (re, im) pairs."""
    raw = np.asarray(raw, dtype=np.int64).reshape(-1, 2)
    return (raw[:, 0] + 1j * raw[:, 1]) / float(Q328_ONE)


def dense_unitary(circ: Circuit, params: Optional[np.ndarray] = None, matrices=None) -> np.ndarray:
    """The circuit's unitary (2^n x 2^n complex128), n <= 10."""
    lib = _load()
    n = circ.n_qubits
    kinds, qubits, angles, mats = _marshal(circ, params, matrices)
    U = np.empty(2 << (2 * n), dtype=np.float64)
    rc = lib.oracle_dense_unitary(n, len(circ.gates), _ptr(kinds), _ptr(qubits), _ptr(angles), _ptr(mats),
                                  _ptr(U))
    if rc != 0:
        raise ValueError("oracle_dense_unitary rejected the circuit")
    return U.view(np.complex128).reshape(1 << n, 1 << n)


def expectation(psi: np.ndarray, n: int, masks: np.ndarray, coeffs: np.ndarray) -> float:
    """<psi|D|psi> for D = sum_t c_t prod_{q in mask_t} Z_q."""
    lib = _load()
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    masks = np.ascontiguousarray(masks, dtype=np.uint64)
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    return float(lib.oracle_expectation_zstrings(n, _ptr(psi), len(masks), _ptr(masks), _ptr(coeffs)))


def amplitudes(psi: np.ndarray, n: int, bits: np.ndarray) -> np.ndarray:
    lib = _load()
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    out = np.empty(2 * len(bits), dtype=np.float64)
    lib.oracle_amplitudes(n, _ptr(psi), len(bits), _ptr(bits), _ptr(out))
    return out.view(np.complex128)


def circuit_expectation(circ: Circuit, params, masks, coeffs) -> float:
    psi = statevector(circ, params)
    return expectation(psi, circ.n_qubits, masks, coeffs)


# Two-term shift rules.  A gate exp(-i theta G) whose generator has two
# eigenvalues r apart gives E(theta) = A + B cos(r theta) + C sin(r theta), so
# dE/dtheta = r [E(theta + pi/(2r)) - E(theta - pi/(2r))] / 2.
#   RX/RY/RZ and every U3 angle: G = P/2 (r = 1);  ZZPHASE: G = (1 - ZZ)/2 (r = 1);
#   CPHASE: G = -|11><11| (r = 1);  MIXER: G = X (r = 2).
_SHIFT_R = {"RX": 1.0, "RY": 1.0, "RZ": 1.0, "U3": 1.0, "ZZPHASE": 1.0, "CPHASE": 1.0, "MIXER": 2.0}


def param_shift_gradient(circ: Circuit, params: np.ndarray, masks, coeffs,
                         which: Optional[Iterable[int]] = None) -> np.ndarray:
    """dE/dparams by the exact shift rule, summed over every gate occurrence
    that reads the parameter (product rule).  ``which`` limits the parameters
    evaluated; the others are returned as NaN."""
    params = np.asarray(params, dtype=np.float64)
    which = range(circ.n_params) if which is None else list(which)
    grad = np.full(circ.n_params, np.nan)
    uses = {}
    for gi, g in enumerate(circ.gates):
        for slot, p in enumerate(g.params):
            if p >= 0:
                uses.setdefault(p, []).append((gi, slot))
    for p in which:
        total = 0.0
        for gi, slot in uses.get(p, []):
            g = circ.gates[gi]
            r = _SHIFT_R[g.kind]
            s = np.pi / (2 * r)
            vals = []
            for sign in (+1.0, -1.0):
                gates = list(circ.gates)
                ang = list(circ.resolved_angles(g, params))
                ang[slot] += sign * s
                gates[gi] = Gate(g.kind, g.qubits, tuple(ang), (-1,) * len(ang))
                c2 = Circuit(circ.n_qubits, gates, circ.n_params, circ.name)
                vals.append(circuit_expectation(c2, params, masks, coeffs))
            total += r * (vals[0] - vals[1]) / 2.0
        grad[p] = total
    return grad


def finite_difference_gradient(circ: Circuit, params: np.ndarray, masks, coeffs, h: float = 1e-3,
                               which: Optional[Iterable[int]] = None) -> np.ndarray:
    """Central differences [E(theta + h) - E(theta - h)] / (2h) in FP64."""
    params = np.asarray(params, dtype=np.float64)
    which = range(circ.n_params) if which is None else list(which)
    grad = np.full(circ.n_params, np.nan)
    for p in which:
        pp = params.copy()
        pp[p] += h
        ep = circuit_expectation(circ, pp, masks, coeffs)
        pp[p] -= 2 * h
        em = circuit_expectation(circ, pp, masks, coeffs)
        grad[p] = (ep - em) / (2 * h)
    return grad


def contract(a: np.ndarray, modes_a: Sequence[int], b: np.ndarray, modes_b: Sequence[int],
             modes_c: Sequence[int]) -> np.ndarray:
    """Pairwise contraction by its definition (Sec. 2.2.1): the tensor product
    of A and B with every mode shared by A and B that is absent from C summed
    over (eq. (2.2)); a shared mode kept in C is a batch (hyper) mode, taken
    diagonally.  No conjugation (contraction is bilinear).  Modes are integer
    labels; arrays are complex, C-ordered over their mode lists."""
    letters = {}

    def lab(ms):
        out = ""
        for m in ms:
            if m not in letters:
                letters[m] = chr(ord("a") + len(letters)) if len(letters) < 26 else chr(ord("A") + len(letters) - 26)
            out += letters[m]
        return out

    spec = f"{lab(modes_a)},{lab(modes_b)}->{lab(modes_c)}"
    return np.einsum(spec, np.asarray(a, dtype=np.complex128), np.asarray(b, dtype=np.complex128))


def single_amplitude(circ: Circuit, bits: int, params: Optional[np.ndarray] = None, max_log2: int = 30) -> complex:
    """<b|U|0...0> (qubit 0 = most significant bit of ``bits``) by contracting
    the circuit's tensor network closed with |0> kets and the bra <b| (Sec.
    2.2.2, eq. (2.3)), every pairwise step a plain sum over the shared indices
    (eq. (2.2), numpy.tensordot) in complex128.  The order: repeatedly the pair
    of tensors sharing an index whose result is smallest relative to its
    operands (ties: smaller result, then earlier tensors).  Every index joins
    exactly two tensors (gates are dense matrices here, no hyper-indices)."""
    n = circ.n_qubits
    arrays, labels = [], []
    wire = list(range(n))
    nxt = n

    def add(a, labs):
        arrays.append(np.asarray(a, dtype=np.complex128))
        labels.append(list(labs))

    for q in range(n):
        add([1.0, 0.0], [q])
    for g in circ.gates:
        m = gate_matrix(g.kind, circ.resolved_angles(g, params))
        if len(g.qubits) == 1:
            q = g.qubits[0]
            add(m, [nxt, wire[q]])
            wire[q] = nxt
            nxt += 1
        else:
            a, b = g.qubits
            add(m.reshape(2, 2, 2, 2), [nxt, nxt + 1, wire[a], wire[b]])
            wire[a], wire[b] = nxt, nxt + 1
            nxt += 2
    for q in range(n):
        e = np.zeros(2)
        e[(bits >> (n - 1 - q)) & 1] = 1.0
        add(e, [wire[q]])
    live = set(range(len(arrays)))
    holders = {}
    for t, ls in enumerate(labels):
        for lb in ls:
            holders.setdefault(lb, []).append(t)
    scalars = []
    while True:
        best = None
        for lb, ts in holders.items():
            i, j = sorted(ts)
            shared = set(labels[i]) & set(labels[j])
            rc = len(labels[i]) + len(labels[j]) - 2 * len(shared)
            key = (rc - len(labels[i]) - len(labels[j]), rc, i, j)
            if best is None or key < best[0]:
                best = (key, i, j, shared)
        if best is None:
            break
        _, i, j, shared = best
        if best[0][1] > max_log2:
            raise MemoryError(f"intermediate of 2^{best[0][1]} elements")
        sh = sorted(shared)
        ai = [labels[i].index(x) for x in sh]
        aj = [labels[j].index(x) for x in sh]
        c = np.tensordot(arrays[i], arrays[j], axes=(ai, aj))
        lc = [x for x in labels[i] if x not in shared] + [x for x in labels[j] if x not in shared]
        for x in sh:
            del holders[x]
        k = len(arrays)
        arrays.append(c)
        labels.append(lc)
        for x in lc:
            holders[x] = [k if t in (i, j) else t for t in holders[x]]
        arrays[i] = arrays[j] = None
        live -= {i, j}
        live.add(k)
        if not lc:
            scalars.append(complex(c))
            live.discard(k)
    for t in live:  # tensors left without indices (a closed network reduces to scalars)
        scalars.append(complex(np.asarray(arrays[t]).reshape(())))
    return complex(np.prod(scalars))
