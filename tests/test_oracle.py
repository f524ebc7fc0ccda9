"""Pins for the FP64 oracle: values the paper prints, closed forms, library
routines for special cases and brute force.  CPU only."""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads
from workloads import Circuit, Gate

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.diag([1.0, -1.0]).astype(complex)
I2 = np.eye(2, dtype=complex)
ALL_KINDS = ["H", "X", "Y", "Z", "S", "T", "SX", "SY", "SW", "RX", "RY", "RZ", "U3", "MIXER",
             "CZ", "CNOT", "SWAP", "CPHASE", "ZZPHASE"]


def C(n, gates):
    return Circuit(n, [Gate(*g) if isinstance(g, tuple) else g for g in gates])


def random_unitary(d, rng):
    a = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))


# ---------------------------------------------------------------------------
# Worked examples printed in the paper
# ---------------------------------------------------------------------------
def test_two_qubit_product_order(golden_dir):
    """Sec. 2.1: psi (x) phi = (a a', a b', b a', b b'), first factor = MSB."""
    rows = [l.split() for l in open(os.path.join(golden_dir, "paper_two_qubit_product.txt"))
            if l.strip() and not l.startswith("#")]
    rng = np.random.default_rng(1)
    a0, a1 = rng.uniform(0, 2 * np.pi, 3), rng.uniform(0, 2 * np.pi, 3)
    psi = oracle.statevector(C(1, [("U3", (0,), tuple(a0))]))
    phi = oracle.statevector(C(1, [("U3", (0,), tuple(a1))]))
    both = oracle.statevector(C(2, [("U3", (0,), tuple(a0)), ("U3", (1,), tuple(a1))]))
    val = {"alpha": psi[0], "beta": psi[1], "alpha'": phi[0], "beta'": phi[1]}
    for idx, f1, f2 in rows:
        assert abs(both[int(idx)] - val[f1] * val[f2]) < 1e-14


def test_kron_4x4_layout(golden_dir):
    """Sec. 2.1: the element-wise listing of U (x) V; U on qubit 0, V on qubit 1."""
    rows = [l.split() for l in open(os.path.join(golden_dir, "paper_kron_4x4.txt"))
            if l.strip() and not l.startswith("#")]
    rng = np.random.default_rng(2)
    U, V = random_unitary(2, rng), random_unitary(2, rng)
    got = oracle.dense_unitary(C(2, [("H", (0,)), ("H", (1,))]), matrices={0: U, 1: V})
    for r, row in enumerate(rows):
        for c, ent in enumerate(row):
            u, v = ent.split("*")
            want = U[int(u[1]), int(u[2])] * V[int(v[1]), int(v[2])]
            assert abs(got[r, c] - want) < 1e-14
    # the same 4x4 applied as one two-qubit gate on (0, 1) and on (1, 0)
    W = random_unitary(4, rng)
    g01 = oracle.dense_unitary(C(2, [("CZ", (0, 1))]), matrices={0: W})
    assert np.allclose(g01, W, atol=1e-14)
    g10 = oracle.dense_unitary(C(2, [("CZ", (1, 0))]), matrices={0: W})
    perm = [0, 2, 1, 3]  # swap the roles of the two bits
    assert np.allclose(g10, W[np.ix_(perm, perm)], atol=1e-14)


def test_bell_state(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "paper_bell.txt"))
            if l.strip() and not l.startswith("#")]
    psi = oracle.statevector(C(2, [("H", (0,)), ("CNOT", (0, 1))]))
    for idx, re, im in rows:
        assert abs(psi[int(idx)] - complex(float(re), float(im))) < 1e-15


def test_fig21_true_output(golden_dir):
    """Fig. 2.1 as drawn; its caption's output is not what the circuit gives."""
    gates, amps = [], {}
    for l in open(os.path.join(golden_dir, "paper_fig21.txt")):
        t = l.split()
        if not t or t[0].startswith("#"):
            continue
        if t[0] == "gate":
            gates.append((t[1], tuple(int(x) for x in t[2:])))
        else:
            amps[int(t[1])] = complex(float(t[2]), float(t[3]))
    psi = oracle.statevector(C(3, gates))
    for i, a in amps.items():
        assert abs(psi[i] - a) < 1e-15
    assert abs(psi[7]) < 1e-15  # not the GHZ state the caption claims


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
def test_ghz(n):
    gates = [("H", (0,))] + [("CNOT", (q, q + 1)) for q in range(n - 1)]
    psi = oracle.statevector(C(n, gates))
    want = np.zeros(1 << n, complex)
    want[0] = want[-1] = 2 ** -0.5
    assert np.max(np.abs(psi - want)) < 1e-15


def qft_circuit(n, x):
    gates = [("X", (q,)) for q in range(n) if (x >> (n - 1 - q)) & 1]
    for q in range(n):
        gates.append(("H", (q,)))
        for j in range(q + 1, n):
            gates.append(("CPHASE", (j, q), (2 * np.pi / 2 ** (j - q + 1),)))
    for q in range(n // 2):
        gates.append(("SWAP", (q, n - 1 - q)))
    return C(n, gates)


@pytest.mark.parametrize("n,x", [(3, 5), (5, 19), (7, 100), (10, 777)])
def test_qft_basis_state(n, x):
    """QFT|x> = 2^{-n/2} sum_y e^{2 pi i x y / 2^n} |y> (with the final swaps)."""
    psi = oracle.statevector(qft_circuit(n, x))
    y = np.arange(1 << n)
    want = np.exp(2j * np.pi * x * y / 2 ** n) / 2 ** (n / 2)
    assert np.max(np.abs(psi - want)) < 1e-13


def test_qft_without_swaps_is_bit_reversed():
    n, x = 6, 43
    c = qft_circuit(n, x)
    c.gates = [g for g in c.gates if g.kind != "SWAP"]
    psi = oracle.statevector(c)
    rev = np.array([int(format(y, f"0{n}b")[::-1], 2) for y in range(1 << n)])
    want = np.exp(2j * np.pi * x * rev / 2 ** n) / 2 ** (n / 2)
    assert np.max(np.abs(psi - want)) < 1e-13


# ---------------------------------------------------------------------------
# Gate definitions against library routines
# ---------------------------------------------------------------------------
def test_gates_against_matrix_exponentials():
    rng = np.random.default_rng(3)
    for t in rng.uniform(-7, 7, 5):
        for name, P in (("RX", X), ("RY", Y), ("RZ", Z)):
            assert np.allclose(oracle.gate_matrix(name, [t]), scipy.linalg.expm(-0.5j * t * P), atol=1e-14)
        assert np.allclose(oracle.gate_matrix("MIXER", [t]), scipy.linalg.expm(-1j * t * X), atol=1e-14)
        ZZ = np.kron(Z, Z)
        assert np.allclose(oracle.gate_matrix("ZZPHASE", [t]),
                           scipy.linalg.expm(-1j * t * (np.eye(4) - ZZ) / 2), atol=1e-14)
        P11 = np.diag([0, 0, 0, 1.0])
        assert np.allclose(oracle.gate_matrix("CPHASE", [t]), scipy.linalg.expm(1j * t * P11), atol=1e-14)


def test_gate_special_cases():
    H = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    assert np.allclose(oracle.gate_matrix("H"), H, atol=1e-15)
    assert np.allclose(oracle.gate_matrix("U3", [np.pi / 2, 0, np.pi]), H, atol=1e-15)
    for t in (0.3, 2.1, -1.2):
        assert np.allclose(oracle.gate_matrix("U3", [t, 0, 0]), oracle.gate_matrix("RY", [t]), atol=1e-15)
        assert np.allclose(oracle.gate_matrix("U3", [t, -np.pi / 2, np.pi / 2]), oracle.gate_matrix("RX", [t]),
                           atol=1e-15)
    # U3 = e^{i(phi+lam)/2} RZ(phi) RY(theta) RZ(lam)
    th, ph, la = 0.7, 1.9, -0.4
    rz = lambda a: oracle.gate_matrix("RZ", [a])
    want = np.exp(0.5j * (ph + la)) * rz(ph) @ oracle.gate_matrix("RY", [th]) @ rz(la)
    assert np.allclose(oracle.gate_matrix("U3", [th, ph, la]), want, atol=1e-14)
    W = (X + Y) / np.sqrt(2)
    for name, P in (("SX", X), ("SY", Y), ("SW", W)):
        s = oracle.gate_matrix(name)
        assert np.allclose(s @ s, P, atol=1e-15)
        assert np.allclose(s, scipy.linalg.sqrtm(P), atol=1e-12)  # principal root
    assert np.allclose(oracle.gate_matrix("S"), np.diag([1, 1j]))
    assert np.allclose(oracle.gate_matrix("T") @ oracle.gate_matrix("T"), oracle.gate_matrix("S"))
    P0, P1 = np.diag([1.0, 0]), np.diag([0, 1.0])
    assert np.allclose(oracle.gate_matrix("CNOT"), np.kron(P0, I2) + np.kron(P1, X))
    assert np.allclose(oracle.gate_matrix("CZ"), np.kron(P0, I2) + np.kron(P1, Z))
    sw = np.zeros((4, 4))
    for a in range(2):
        for b in range(2):
            sw[2 * b + a, 2 * a + b] = 1
    assert np.allclose(oracle.gate_matrix("SWAP"), sw)
    assert np.allclose(oracle.gate_matrix("X"), X) and np.allclose(oracle.gate_matrix("Y"), Y)
    assert np.allclose(oracle.gate_matrix("Z"), Z)


@pytest.mark.parametrize("kind", ALL_KINDS)
def test_gate_unitarity(kind):
    """U^dagger U = I (the paper's footnote definition of a unitary)."""
    rng = np.random.default_rng(4)
    for _ in range(4):
        u = oracle.gate_matrix(kind, rng.uniform(0, 2 * np.pi, 3))
        assert np.max(np.abs(u.conj().T @ u - np.eye(len(u)))) < 1e-14


# ---------------------------------------------------------------------------
# Brute force: the sweep against the independently built dense unitary
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_sweep_matches_dense_unitary(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 7))
    circ = workloads.random_circuit(n, 30, rng)
    U = oracle.dense_unitary(circ)
    assert np.max(np.abs(U.conj().T @ U - np.eye(1 << n))) < 1e-12
    psi = oracle.statevector(circ)
    assert np.max(np.abs(psi - U[:, 0])) < 1e-13
    assert abs(np.linalg.norm(psi) - 1) < 1e-13


def test_dense_unitary_one_qubit_gates_are_krons():
    """1-qubit gates embed as I (x) ... (x) U (x) ... (x) I (numpy.kron)."""
    rng = np.random.default_rng(5)
    n = 4
    for q in range(n):
        u = random_unitary(2, rng)
        got = oracle.dense_unitary(C(n, [("H", (q,))]), matrices={0: u})
        mats = [I2] * n
        mats[q] = u
        want = mats[0]
        for m in mats[1:]:
            want = np.kron(want, m)
        assert np.allclose(got, want, atol=1e-15)


def test_sweep_matches_kron_products():
    """A layer of 1-qubit gates on |0..0> is the Kronecker product of columns."""
    rng = np.random.default_rng(6)
    n = 7
    angs = rng.uniform(0, 2 * np.pi, (n, 3))
    psi = oracle.statevector(C(n, [("U3", (q,), tuple(angs[q])) for q in range(n)]))
    want = np.array([1.0 + 0j])
    for q in range(n):
        want = np.kron(want, oracle.gate_matrix("U3", angs[q])[:, 0])
    assert np.max(np.abs(psi - want)) < 1e-15


def test_two_qubit_gate_on_distant_qubits_brute_force():
    """psi'[x] = sum_y G[x, y] psi[y] with G's elements from the definition."""
    rng = np.random.default_rng(7)
    n = 5
    W = random_unitary(4, rng)
    pre = [("U3", (q,), tuple(rng.uniform(0, 6, 3))) for q in range(n)]
    psi0 = oracle.statevector(C(n, pre))
    for qa, qb in [(0, 4), (3, 1), (2, 3)]:
        psi = oracle.statevector(C(n, pre + [("CZ", (qa, qb))]), matrices={n: W})
        want = np.zeros_like(psi0)
        for x in range(1 << n):
            for y in range(1 << n):
                bits = lambda v, q: (v >> (n - 1 - q)) & 1
                if all(bits(x, q) == bits(y, q) for q in range(n) if q not in (qa, qb)):
                    want[x] += W[2 * bits(x, qa) + bits(x, qb), 2 * bits(y, qa) + bits(y, qb)] * psi0[y]
        assert np.max(np.abs(psi - want)) < 1e-14


def test_configs_are_unitary_and_normalised():
    psi = oracle.statevector(workloads.config0())
    assert abs(np.vdot(psi, psi).real - 1) < 1e-12


# ---------------------------------------------------------------------------
# Expectations, amplitudes, gradients
# ---------------------------------------------------------------------------
def test_expectation_brute_force():
    rng = np.random.default_rng(8)
    n = 6
    psi = oracle.statevector(workloads.random_circuit(n, 40, rng))
    masks = np.array([0, 0b100001, 0b011000, 0b111111, 0b000100], dtype=np.uint64)
    coeffs = rng.normal(size=5)
    D = np.zeros(1 << n)
    for x in range(1 << n):
        for m, c in zip(masks, coeffs):
            D[x] += c * (-1) ** bin(x & int(m)).count("1")
    want = np.sum(np.abs(psi) ** 2 * D)
    assert abs(oracle.expectation(psi, n, masks, coeffs) - want) < 1e-13
    # the same through the dense Kronecker form of the observable
    Dk = np.zeros((1 << n, 1 << n), complex)
    for m, c in zip(masks, coeffs):
        t = np.array([[1.0 + 0j]])
        for q in range(n):
            t = np.kron(t, Z if (int(m) >> (n - 1 - q)) & 1 else I2)
        Dk += c * t
    assert abs(np.vdot(psi, Dk @ psi).real - want) < 1e-13


def test_product_state_zz():
    """<Z_a Z_b> on a product state is <Z_a><Z_b> = cos(t_a) cos(t_b) for RY(t)|0>."""
    t = np.array([0.3, 1.1, 2.5, 0.9])
    n = 4
    psi = oracle.statevector(C(n, [("RY", (q,), (t[q],)) for q in range(n)]))
    for a, b in [(0, 1), (1, 3), (0, 3)]:
        m = np.array([(1 << (n - 1 - a)) | (1 << (n - 1 - b))], dtype=np.uint64)
        assert abs(oracle.expectation(psi, n, m, np.ones(1)) - np.cos(t[a]) * np.cos(t[b])) < 1e-15


def test_amplitudes_index_convention():
    n = 5
    psi = oracle.statevector(C(n, [("X", (0,)), ("X", (3,))]))  # |10010>
    bits = np.array([0b10010, 0b00000, 0b01001], dtype=np.uint64)
    a = oracle.amplitudes(psi, n, bits)
    assert np.allclose(a, [1, 0, 0])


def test_qaoa_beta_zero():
    """beta = 0: the phase separator is diagonal, so <C> = |E|/2 for any gamma."""
    inst = workloads.config3(n_circuits=3)
    for it in inst:
        prm = it.params.copy()
        prm[4:] = 0.0
        masks, coeffs = workloads.maxcut_observable(it.circuit.n_qubits, it.edges)
        e = oracle.circuit_expectation(it.circuit, prm, masks, coeffs)
        assert abs(e - len(it.edges) / 2) < 1e-12


def qaoa_p1_closed_form(n, edges, gamma, beta):
    """<C> at p = 1 (Wang, Hadfield, Jiang, Rieffel, PRA 97, 022304 (2018))."""
    nbr = {v: set() for v in range(n)}
    for u, v in edges:
        nbr[u].add(v)
        nbr[v].add(u)
    tot = 0.0
    for u, v in edges:
        du, dv = len(nbr[u]) - 1, len(nbr[v]) - 1
        f = len(nbr[u] & nbr[v])
        c = np.cos(gamma)
        tot += (0.5 + 0.25 * np.sin(4 * beta) * np.sin(gamma) * (c ** du + c ** dv)
                - 0.25 * np.sin(2 * beta) ** 2 * c ** (du + dv - 2 * f) * (1 - np.cos(2 * gamma) ** f))
    return tot


@pytest.mark.parametrize("n,seed", [(8, 0), (10, 1), (12, 2)])
def test_qaoa_p1_closed_form(n, seed):
    rng = np.random.default_rng(seed)
    edges = workloads.random_regular_graph(n, 3, rng)
    circ = workloads.qaoa_circuit(n, edges, 1)
    masks, coeffs = workloads.maxcut_observable(n, edges)
    for g, b in rng.uniform(0, 3, (3, 2)):
        e = oracle.circuit_expectation(circ, np.array([g, b]), masks, coeffs)
        assert abs(e - qaoa_p1_closed_form(n, edges, g, b)) < 1e-12


def test_param_shift_vs_finite_difference():
    """Each angle sits in one gate whose generator has eigenvalues +-1/2, so
    E(t) = A + B cos t + C sin t and the central difference is exactly
    g sin(h)/h."""
    circ = workloads.hea_circuit(6, 3)
    rng = np.random.default_rng(9)
    params = rng.uniform(0, 2 * np.pi, circ.n_params)
    masks, coeffs = workloads.zz_ring_observable(6)
    g = oracle.param_shift_gradient(circ, params, masks, coeffs)
    h = 1e-3
    fd = oracle.finite_difference_gradient(circ, params, masks, coeffs, h=h)
    assert np.max(np.abs(fd / (np.sin(h) / h) - g)) < 1e-9
    # a plausible slip (the shift applied to the wrong parameter) would not match
    assert np.max(np.abs(g)) > 1e-3


@pytest.mark.parametrize("kind", ["RX", "RY", "RZ", "U3", "CPHASE", "ZZPHASE", "MIXER"])
def test_param_shift_every_parametric_kind_vs_finite_difference(kind):
    """The shift rule of every parametric gate kind (each angle of a U3 on its
    own) against the derivative's definition: with every angle its own
    parameter, E is A + B cos(r t) + C sin(r t) in each parameter (r = 1, or
    2 for the mixer exp(-i t X)), so the central difference is exactly
    g sin(r h)/(r h).  Fixed gates of every kind around the parametric ones;
    the observable mixes one- and two-qubit Z strings."""
    n = 5
    rng = np.random.default_rng(4242 + ALL_KINDS.index(kind) if kind in ALL_KINDS else 4242)
    fixed = ["H", "X", "Y", "S", "T", "SX", "SY", "SW", "CZ", "CNOT", "SWAP"]
    na = workloads.N_ANGLES[kind]
    gates = [workloads.Gate("H", (q,)) for q in range(n)]
    n_par = 0
    for _ in range(6):  # random fixed gates, then one parametric gate
        gates += workloads.random_circuit(n, 5, rng, kinds=fixed).gates
        if kind in workloads.TWO_QUBIT:
            qs = tuple(int(q) for q in rng.choice(n, size=2, replace=False))
        else:
            qs = (int(rng.integers(0, n)),)
        gates.append(workloads.Gate(kind, qs, (0.0,) * na, tuple(range(n_par, n_par + na))))
        n_par += na
    # non-diagonal gates after the last parametric one, so that diagonal gates show in a Z observable
    gates += [workloads.Gate("SX", (q,)) for q in range(n)] + [workloads.Gate("CNOT", (q, q + 1)) for q in range(n - 1)]
    circ = workloads.Circuit(n, gates, n_par)
    params = rng.uniform(0, 2 * np.pi, n_par)
    masks, coeffs = workloads.zz_ring_observable(n)
    masks = np.concatenate([masks, np.array([1 << 4, 1 << 1, (1 << 4) | (1 << 2) | 1], dtype=np.uint64)])
    coeffs = np.concatenate([coeffs, np.array([0.8, -0.6, 1.1])])
    g = oracle.param_shift_gradient(circ, params, masks, coeffs)
    r = 2.0 if kind == "MIXER" else 1.0
    h = 1e-3
    fd = oracle.finite_difference_gradient(circ, params, masks, coeffs, h=h)
    assert np.max(np.abs(fd / (np.sin(r * h) / (r * h)) - g)) < 1e-9
    assert np.max(np.abs(g)) > 1e-2  # the circuit depends on its parameters


def test_param_shift_multi_occurrence_and_mixer():
    """QAOA: gamma feeds every edge and beta every mixer (shift pi/4)."""
    n = 6
    rng = np.random.default_rng(10)
    edges = workloads.random_regular_graph(n, 3, rng)
    circ = workloads.qaoa_circuit(n, edges, 2)
    masks, coeffs = workloads.maxcut_observable(n, edges)
    params = rng.uniform(0, 1.5, 4)
    g = oracle.param_shift_gradient(circ, params, masks, coeffs)
    fd = oracle.finite_difference_gradient(circ, params, masks, coeffs, h=1e-5)
    assert np.max(np.abs(g - fd)) < 1e-7


# ---------------------------------------------------------------------------
# Pairwise contraction by definition
# ---------------------------------------------------------------------------
def test_contract_trace_matvec_matmul_outer():
    """Sec. 2.2.1: trace, matrix-vector and matrix-matrix products (eq. (2.2))
    and the tensor product as contractions."""
    rng = np.random.default_rng(11)
    M = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    L = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    x = rng.normal(size=4) + 1j * rng.normal(size=4)
    # mat-vec y^i = M^i_j x^j
    y = oracle.contract(M, [0, 1], x, [1], [0])
    assert np.allclose(y, [sum(M[i, j] * x[j] for j in range(4)) for i in range(4)])
    # mat-mat Z^i_j = M^i_k L^k_j
    Zm = oracle.contract(M, [0, 1], L, [1, 2], [0, 2])
    assert np.allclose(Zm, M @ L)
    # trace as a contraction of M with the identity (a (1,1) tensor)
    tr = oracle.contract(M, [0, 1], np.eye(4), [1, 0], [])
    assert abs(tr - np.trace(M)) < 1e-12
    # tensor product: no shared mode, order adds up; Kronecker layout
    T = oracle.contract(M, [0, 1], L, [2, 3], [0, 2, 1, 3]).reshape(16, 12)
    assert np.allclose(T, np.kron(M, L))
    # no conjugation
    v = oracle.contract(x, [0], x, [0], [])
    assert abs(v - np.sum(x * x)) < 1e-12


def test_contract_batch_mode_brute_force():
    rng = np.random.default_rng(12)
    A = rng.normal(size=(3, 2, 4)) + 1j * rng.normal(size=(3, 2, 4))  # (b, m, k)
    B = rng.normal(size=(4, 3, 5)) + 1j * rng.normal(size=(4, 3, 5))  # (k, b, n)
    got = oracle.contract(A, [7, 1, 9], B, [9, 7, 4], [4, 7, 1])
    want = np.zeros((5, 3, 2), complex)
    for b in range(3):
        for m in range(2):
            for nn in range(5):
                for k in range(4):
                    want[nn, b, m] += A[b, m, k] * B[k, b, nn]
    assert np.allclose(got, want)


# ---------------------------------------------------------------------------
# single amplitudes by network contraction (the oracle for circuits too wide
# for a full FP64 state)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["brickwork", "random_all_kinds", "grid"])
def test_single_amplitude_matches_statevector(which):
    """Two independent FP64 algorithms (pairwise network contraction vs the
    gate-by-gate sweep) give the same amplitudes."""
    rng = np.random.default_rng(31)
    if which == "brickwork":
        circ = workloads.config0()
    elif which == "random_all_kinds":
        circ = workloads.random_circuit(11, 90, rng)
    else:
        circ = workloads.grid_circuit(3, 4, 8, rng)
    psi = oracle.statevector(circ)
    n = circ.n_qubits
    for b in [0, (1 << n) - 1] + [int(x) for x in rng.integers(0, 1 << n, size=12)]:
        a = oracle.single_amplitude(circ, b)
        assert abs(a - psi[b]) < 1e-12, (b, a, psi[b])


def test_single_amplitude_ghz_closed_form():
    """GHZ: <0...0|psi> = <1...1|psi> = 1/sqrt2, every other amplitude 0."""
    n = 9
    gates = [workloads.Gate("H", (0,), (), ())] + [workloads.Gate("CNOT", (q, q + 1), (), ()) for q in range(n - 1)]
    circ = workloads.Circuit(n, gates, 0, "ghz9")
    s = 1 / np.sqrt(2)
    assert abs(oracle.single_amplitude(circ, 0) - s) < 1e-14
    assert abs(oracle.single_amplitude(circ, (1 << n) - 1) - s) < 1e-14
    for b in (1, 2, 255, 256, 300):
        assert abs(oracle.single_amplitude(circ, b)) < 1e-14


def test_single_amplitude_planted_mistake_fails():
    """A reversed bit order (qubit 0 as the least significant bit) is caught."""
    rng = np.random.default_rng(5)
    circ = workloads.random_circuit(8, 40, rng)
    psi = oracle.statevector(circ)
    b = 0b10110001
    rev = int(f"{b:08b}"[::-1], 2)
    assert abs(oracle.single_amplitude(circ, b) - psi[b]) < 1e-12
    assert abs(oracle.single_amplitude(circ, rev) - psi[b]) > 1e-6


# ---------------------------------------------------------------------------
# Q3.28 fixed point (Sec. 3: 32-bit complex arithmetic, 28 bits behind the
# binary point; reading: two's complement, products rounded to nearest with
# ties to even, saturating sums)
# ---------------------------------------------------------------------------
def _rne_fraction(num, den):
    """Nearest integer to num/den, ties to even (Python's round on a Fraction)."""
    from fractions import Fraction
    return round(Fraction(num, den))


def _sat(v):
    return max(-(1 << 31), min((1 << 31) - 1, v))


def test_q328_multiply_against_exact_rationals():
    """The oracle's Q3.28 product equals the exact rational a b / 2^56 rounded
    to the nearest multiple of 2^-28 (ties to even) and saturated."""
    rng = np.random.default_rng(328)
    cases = [(int(a), int(b)) for a, b in rng.integers(-(1 << 31), 1 << 31, size=(2000, 2))]
    cases += [(int(a), int(b)) for a, b in rng.integers(-(1 << 29), 1 << 29, size=(2000, 2))]
    one = 1 << 28
    cases += [(one, one), (-one, one), (one >> 1, 3), (3, one >> 1), (-(one >> 1), 3), (5, one >> 1),
              (-(5), one >> 1), (1, 1), (-1, 1), (1 << 31 - 1, 1 << 31 - 1), (-(1 << 31), -(1 << 31)),
              (-(1 << 31), (1 << 31) - 1), (8 * one - 1, 8 * one - 1), (0, 12345)]
    ties = 0
    for a, b in cases:
        want = _sat(_rne_fraction(a * b, 1 << 28))
        if (a * b) % (1 << 28) == 1 << 27:
            ties += 1
        assert oracle.q328_mul(a, b) == want, (a, b)
    assert ties >= 4  # exact halves, both parities, were exercised


def test_q328_from_double_rounds_to_nearest_even():
    one = 1 << 28
    for x, want in [(1.0, one), (-1.0, -one), (0.5 / one, 0), (1.5 / one, 2), (2.5 / one, 2), (-2.5 / one, -2),
                    (1 / np.sqrt(2), 189812531), (8.0, (1 << 31) - 1), (-8.0, -(1 << 31)), (100.0, (1 << 31) - 1)]:
        assert oracle.q328_from_double(x) == want, x
    rng = np.random.default_rng(329)
    from fractions import Fraction
    for x in rng.uniform(-7.9, 7.9, 500):
        assert oracle.q328_from_double(x) == round(Fraction(x) * one)


def _q328_sweep_fractions(circ):
    """Brute force with exact rationals: the state as Python integers, every
    real product an exact rational rounded by round() (ties to even)."""
    n = circ.n_qubits
    one = 1 << 28
    psi = [[0, 0] for _ in range(1 << n)]
    psi[0][0] = one
    for g in circ.gates:
        u = oracle.gate_matrix(g.kind, circ.resolved_angles(g, None))
        from fractions import Fraction
        uq = [[(round(Fraction(v.real) * one), round(Fraction(v.imag) * one)) for v in row] for row in u]
        qs = list(g.qubits)
        pos = [n - 1 - q for q in qs]
        d = len(uq)
        new = [list(p) for p in psi]
        for x in range(1 << n):
            if any((x >> p) & 1 for p in pos):
                continue
            idx = []
            for v in range(d):
                bits = [(v >> (len(pos) - 1 - j)) & 1 for j in range(len(pos))]
                idx.append(x | sum(b << p for b, p in zip(bits, pos)))
            for r in range(d):
                re = im = 0
                for c in range(d):
                    (ur, ui), (pr, pi) = uq[r][c], psi[idx[c]]
                    m = lambda a, b: _sat(_rne_fraction(a * b, one))
                    re = _sat(re + _sat(m(ur, pr) - m(ui, pi)))
                    im = _sat(im + _sat(m(ur, pi) + m(ui, pr)))
                new[idx[r]] = [re, im]
        psi = new
    return np.array(psi, dtype=np.int64)


@pytest.mark.parametrize("seed", range(3))
def test_q328_sweep_brute_force_exact_rationals(seed):
    rng = np.random.default_rng(3280 + seed)
    circ = workloads.random_circuit(3, 14, rng)
    got = oracle.statevector_q328(circ).astype(np.int64)
    assert np.array_equal(got, _q328_sweep_fractions(circ))


def test_q328_permutation_circuits_are_exact():
    """X, CNOT, SWAP and CZ have entries 0 and +-1: every product is exact,
    so the fixed-point state equals the FP64 one exactly."""
    rng = np.random.default_rng(3290)
    circ = workloads.random_circuit(9, 80, rng, kinds=["X", "CNOT", "SWAP", "CZ", "Z"])
    want = oracle.statevector(circ)
    got = oracle.q328_to_complex(oracle.statevector_q328(circ))
    assert np.array_equal(got, want)


def test_q328_error_within_rounding_bound():
    """Against the FP64 sweep: each gate adds at most one rounding of 2^-29 per
    real product (plus the gate entries' own rounding, at most 2^-29 each),
    so over G gates of at most 4 terms per output the max-abs error stays
    below G * 16 * 2^-29 * (1 + 1); in practice far below (uncorrelated)."""
    for circ in (workloads.config0(), workloads.random_circuit(8, 120, np.random.default_rng(3300))):
        want = oracle.statevector(circ)
        got = oracle.q328_to_complex(oracle.statevector_q328(circ))
        G = len(circ.gates)
        err = np.max(np.abs(got - want))
        assert err < G * 32 * 2.0 ** -29
        assert err > 0  # rounding did happen
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-5
