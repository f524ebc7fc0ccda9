"""Seeded synthetic circuit workloads.

This module only *describes* circuits: gate names, the qubits they act on,
their angles (float64) or the index of the parameter that supplies an angle,
bitstrings and graphs.  It holds no gate matrix and no simulation arithmetic,
so the FP64 oracle and the GPU library can both read the same inputs without
sharing any of the method's code.

Conventions (Sec. 2.1, eq. (2.3) of the paper): qubit 0 is the most
significant bit of a basis-state index, so a bitstring ``b`` stores qubit ``q``
in bit ``n-1-q``.

Gate vocabulary (names only; each consumer defines the matrices itself):

  1-qubit, fixed:      H, X, Y, Z, S, T, SX, SY, SW     (SX = sqrt(X), ...)
  1-qubit, angle(s):   RX, RY, RZ (1 angle), U3 (theta, phi, lambda),
                       MIXER (beta: exp(-i beta X))
  2-qubit, fixed:      CZ, CNOT (control first), SWAP
  2-qubit, angle:      CPHASE (lambda: diag(1,1,1,e^{i lambda})),
                       ZZPHASE (gamma: exp(-i gamma (1 - Z Z)/2))
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 2108068310

ONE_QUBIT = {"H", "X", "Y", "Z", "S", "T", "SX", "SY", "SW", "RX", "RY", "RZ", "U3", "MIXER"}
TWO_QUBIT = {"CZ", "CNOT", "SWAP", "CPHASE", "ZZPHASE"}
N_ANGLES = {"RX": 1, "RY": 1, "RZ": 1, "U3": 3, "MIXER": 1, "CPHASE": 1, "ZZPHASE": 1}


@dataclass
class Gate:
    kind: str
    qubits: Tuple[int, ...]
    angles: Tuple[float, ...] = ()
    params: Tuple[int, ...] = ()  # parameter index per angle, -1 = use ``angles``

    def __post_init__(self):
        na = N_ANGLES.get(self.kind, 0)
        if self.kind not in ONE_QUBIT and self.kind not in TWO_QUBIT:
            raise ValueError(f"unknown gate {self.kind}")
        want_q = 1 if self.kind in ONE_QUBIT else 2
        if len(self.qubits) != want_q:
            raise ValueError(f"{self.kind} acts on {want_q} qubit(s)")
        if not self.angles:
            self.angles = (0.0,) * na
        if not self.params:
            self.params = (-1,) * na
        if len(self.angles) != na or len(self.params) != na:
            raise ValueError(f"{self.kind} takes {na} angle(s)")
        self.qubits = tuple(int(q) for q in self.qubits)
        self.angles = tuple(float(a) for a in self.angles)
        self.params = tuple(int(p) for p in self.params)


@dataclass
class Circuit:
    n_qubits: int
    gates: List[Gate]
    n_params: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    def resolved_angles(self, gate: Gate, params: Optional[np.ndarray]) -> Tuple[float, ...]:
        """Angles of ``gate`` with parameter references looked up in ``params``."""
        out = []
        for a, p in zip(gate.angles, gate.params):
            out.append(float(params[p]) if p >= 0 else a)
        return tuple(out)


def _rng(config_index: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config_index)


# ---------------------------------------------------------------------------
# Brickwork (configs 0 and 1)
# ---------------------------------------------------------------------------
def brickwork(n: int, depth: int, rng: np.random.Generator, name: str = "") -> Circuit:
    """Layer l: U3 on every qubit (angles drawn in the order l, q, (theta, phi,
    lambda), uniform in [0, 2 pi)), then CZ on (2i, 2i+1) for even l or
    (2i+1, 2i+2) for odd l."""
    angles = rng.uniform(0.0, 2.0 * np.pi, size=(depth, n, 3))
    gates: List[Gate] = []
    for layer in range(depth):
        for q in range(n):
            gates.append(Gate("U3", (q,), tuple(angles[layer, q])))
        start = 0 if layer % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            gates.append(Gate("CZ", (a, a + 1)))
    return Circuit(n, gates, 0, name or f"brickwork_n{n}_d{depth}")


def config0() -> Circuit:
    """10-qubit brickwork, depth 8, full statevector."""
    return brickwork(10, 8, _rng(0), "config0_brickwork_n10_d8")


def config1() -> Circuit:
    """24-qubit brickwork, depth 16, full statevector with 2-qubit fusion."""
    return brickwork(24, 16, _rng(1), "config1_brickwork_n24_d16")


# ---------------------------------------------------------------------------
# Grid random circuit with batched amplitudes (config 2)
# ---------------------------------------------------------------------------
GRID_1Q = ("SX", "SY", "SW")


def grid_patterns(rows: int, cols: int):
    """The four CZ edge patterns on a rows x cols grid, qubit q = cols*r + c.
    A: horizontal edges with c even; B: horizontal with c odd;
    C: vertical with r even; D: vertical with r odd."""
    A = [(cols * r + c, cols * r + c + 1) for r in range(rows) for c in range(0, cols - 1, 2)]
    B = [(cols * r + c, cols * r + c + 1) for r in range(rows) for c in range(1, cols - 1, 2)]
    C = [(cols * r + c, cols * (r + 1) + c) for r in range(0, rows - 1, 2) for c in range(cols)]
    D = [(cols * r + c, cols * (r + 1) + c) for r in range(1, rows - 1, 2) for c in range(cols)]
    return [A, B, C, D]


def grid_circuit(rows: int, cols: int, depth: int, rng: np.random.Generator, name: str = ""):
    """Per layer: one of sqrt(X)/sqrt(Y)/sqrt(W) drawn uniformly per qubit,
    then the CZs of one of the four grid patterns drawn uniformly."""
    n = rows * cols
    pats = grid_patterns(rows, cols)
    gates: List[Gate] = []
    chosen = []
    for _ in range(depth):
        kinds = rng.integers(0, 3, size=n)
        p = int(rng.integers(0, 4))
        chosen.append("ABCD"[p])
        for q in range(n):
            gates.append(Gate(GRID_1Q[int(kinds[q])], (q,)))
        for a, b in pats[p]:
            gates.append(Gate("CZ", (a, b)))
    return Circuit(n, gates, 0, name or f"grid_{rows}x{cols}_d{depth}", {"patterns": "".join(chosen)})


def random_bitstrings(n: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """``count`` uniform n-bit strings (with replacement); qubit q in bit n-1-q."""
    hi = np.uint64(1) << np.uint64(n)
    return rng.integers(0, hi, size=count, dtype=np.uint64)


def config2(rows: int = 4, cols: int = 8, depth: int = 12, n_bitstrings: int = 4096):
    """32-qubit 4x8 grid, depth 12; 4096 bitstrings on an open batch index.
    Smaller grids from the same generator (e.g. 4x6) serve as oracle-parity cases."""
    rng = _rng(2)
    circ = grid_circuit(rows, cols, depth, rng, f"config2_grid_{rows}x{cols}_d{depth}")
    bits = random_bitstrings(circ.n_qubits, n_bitstrings, rng)
    return circ, bits


# ---------------------------------------------------------------------------
# Batched QAOA MaxCut (config 3)
# ---------------------------------------------------------------------------
def random_regular_graph(n: int, d: int, rng: np.random.Generator, max_tries: int = 10000):
    """Simple d-regular graph by the configuration model with rejection:
    pair a random shuffle of n*d stubs; reject on a self-loop or a repeated edge."""
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    for _ in range(max_tries):
        stubs = np.repeat(np.arange(n), d)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        ok = True
        seen = set()
        edges = []
        for u, v in pairs:
            u, v = int(u), int(v)
            if u == v:
                ok = False
                break
            e = (min(u, v), max(u, v))
            if e in seen:
                ok = False
                break
            seen.add(e)
            edges.append(e)
        if ok:
            return sorted(edges)
    raise RuntimeError("no simple regular graph found")


def qaoa_circuit(n: int, edges: Sequence[Tuple[int, int]], p: int, name: str = "") -> Circuit:
    """|+>^n (H on |0>), then p layers of the phase separator
    exp(-i gamma_l C) (one ZZPHASE per edge) and the mixer exp(-i beta_l X)
    on every qubit.  Parameters: [gamma_0..gamma_{p-1}, beta_0..beta_{p-1}]."""
    gates = [Gate("H", (q,)) for q in range(n)]
    for layer in range(p):
        for u, v in edges:
            gates.append(Gate("ZZPHASE", (u, v), (0.0,), (layer,)))
        for q in range(n):
            gates.append(Gate("MIXER", (q,), (0.0,), (p + layer,)))
    return Circuit(n, gates, 2 * p, name or f"qaoa_n{n}_p{p}", {"edges": list(edges)})


def maxcut_observable(n: int, edges: Sequence[Tuple[int, int]]):
    """C = sum_{(u,v)} (1 - Z_u Z_v)/2 as Z-strings: (masks, coeffs).
    A mask has bit (n-1-q) set for each qubit q in the string; mask 0 is the identity."""
    masks = [0]
    coeffs = [0.5 * len(edges)]
    for u, v in edges:
        masks.append((1 << (n - 1 - u)) | (1 << (n - 1 - v)))
        coeffs.append(-0.5)
    return np.array(masks, dtype=np.uint64), np.array(coeffs, dtype=np.float64)


@dataclass
class QAOAInstance:
    circuit: Circuit
    edges: List[Tuple[int, int]]
    params: np.ndarray  # [2p] = gammas then betas


def config3(n_circuits: int = 512, p: int = 4, sizes=(16, 18, 20, 22, 24, 26)) -> List[QAOAInstance]:
    """512 QAOA MaxCut circuits; n uniform in {16,...,26}; simple 3-regular graphs;
    gamma ~ U[0, pi), beta ~ U[0, pi/2) drawn per layer and per circuit."""
    rng = _rng(3)
    out = []
    for i in range(n_circuits):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        edges = random_regular_graph(n, 3, rng)
        gam = rng.uniform(0.0, np.pi, size=p)
        bet = rng.uniform(0.0, np.pi / 2, size=p)
        circ = qaoa_circuit(n, edges, p, f"config3_qaoa_{i}_n{n}")
        out.append(QAOAInstance(circ, edges, np.concatenate([gam, bet])))
    return out


# ---------------------------------------------------------------------------
# Hardware-efficient ansatz gradients (config 4)
# ---------------------------------------------------------------------------
def hea_circuit(n: int, layers: int, ring: bool = True, name: str = "") -> Circuit:
    """Per layer: RY(theta[2n l + 2q]) then RZ(theta[2n l + 2q + 1]) on each qubit
    (circuit order), then CZ(q, q+1 mod n) on the ring."""
    gates: List[Gate] = []
    for layer in range(layers):
        for q in range(n):
            gates.append(Gate("RY", (q,), (0.0,), (2 * n * layer + 2 * q,)))
            gates.append(Gate("RZ", (q,), (0.0,), (2 * n * layer + 2 * q + 1,)))
        last = n if ring else n - 1
        for q in range(last):
            gates.append(Gate("CZ", (q, (q + 1) % n)))
    return Circuit(n, gates, 2 * n * layers, name or f"hea_n{n}_l{layers}")


def zz_ring_observable(n: int, ring: bool = True):
    """sum_i Z_i Z_{i+1 mod n} as Z-strings (periodic: n terms)."""
    last = n if ring else n - 1
    masks = [(1 << (n - 1 - i)) | (1 << (n - 1 - ((i + 1) % n))) for i in range(last)]
    return np.array(masks, dtype=np.uint64), np.ones(last, dtype=np.float64)


def config4(n: int = 20, layers: int = 10, batch: int = 64):
    """20-qubit HEA, 10 layers, 64 parameter vectors with angles U[0, 2 pi)."""
    rng = _rng(4)
    circ = hea_circuit(n, layers, True, f"config4_hea_n{n}_l{layers}")
    params = rng.uniform(0.0, 2.0 * np.pi, size=(batch, circ.n_params))
    masks, coeffs = zz_ring_observable(n, True)
    return circ, params, (masks, coeffs)


# ---------------------------------------------------------------------------
# The paper's own test circuit (Fig. 3.1)
# ---------------------------------------------------------------------------
def paper_test_circuit(n: int, k: int, rng: Optional[np.random.Generator] = None) -> Circuit:
    """Fig. 3.1: H on all qubits; per round CNOT(2i -> 2i+1), RZ on all,
    CZ(2i+1, 2i+2), RX on all; H on all at the end.  Angles U[0, 2 pi)."""
    rng = rng if rng is not None else np.random.default_rng(SEED_BASE + 5)
    gates: List[Gate] = [Gate("H", (q,)) for q in range(n)]
    for _ in range(k):
        for a in range(0, n - 1, 2):
            gates.append(Gate("CNOT", (a, a + 1)))
        for q in range(n):
            gates.append(Gate("RZ", (q,), (float(rng.uniform(0, 2 * np.pi)),)))
        for a in range(1, n - 1, 2):
            gates.append(Gate("CZ", (a, a + 1)))
        for q in range(n):
            gates.append(Gate("RX", (q,), (float(rng.uniform(0, 2 * np.pi)),)))
    gates += [Gate("H", (q,)) for q in range(n)]
    return Circuit(n, gates, 0, f"paper_fig31_n{n}_k{k}")


# ---------------------------------------------------------------------------
# Random small circuits for property tests
# ---------------------------------------------------------------------------
def random_circuit(n: int, n_gates: int, rng: np.random.Generator, kinds=None, n_params: int = 0) -> Circuit:
    """Uniformly random gates from ``kinds`` on random qubits; angles U[0, 2 pi).
    With ``n_params`` > 0 every angle of a parametric gate references a random
    parameter index instead of a fixed value."""
    kinds = list(kinds or ["H", "X", "Y", "Z", "S", "T", "SX", "SY", "SW", "RX", "RY", "RZ", "U3",
                           "MIXER", "CZ", "CNOT", "SWAP", "CPHASE", "ZZPHASE"])
    if n < 2:
        kinds = [k for k in kinds if k in ONE_QUBIT]
    gates = []
    for _ in range(n_gates):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind in ONE_QUBIT:
            qs = (int(rng.integers(0, n)),)
        else:
            a, b = rng.choice(n, size=2, replace=False)
            qs = (int(a), int(b))
        na = N_ANGLES.get(kind, 0)
        ang = tuple(float(x) for x in rng.uniform(0, 2 * np.pi, size=na))
        if n_params > 0 and na:
            prm = tuple(int(x) for x in rng.integers(0, n_params, size=na))
        else:
            prm = (-1,) * na
        gates.append(Gate(kind, qs, ang, prm))
    return Circuit(n, gates, n_params, f"random_n{n}_g{n_gates}")
