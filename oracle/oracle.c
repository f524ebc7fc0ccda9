/*
 * FP64 CPU oracle for quantum-circuit simulation.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library.
 * It shares no code, header, table or helper with the GPU library.
 *
 * What it computes is the plain definition of the circuit's output, not the
 * tensor-network algorithm: because contraction is exact and associative
 * (Sec. 2.2.3), every contraction order of the network reaches the same
 * result as applying the gates one by one to the state vector (Sec. 2.1).
 *
 * Conventions
 *  - Basis-state index of |b_0 b_1 ... b_{n-1}> is sum_q b_q 2^{n-1-q}: the
 *    first tensor factor is the most significant bit (Sec. 2.1, the
 *    two-qubit Kronecker example; eq. (2.3)).
 *  - A gate acts on a column vector by matrix product, psi' = U psi, upper
 *    index = row = output (Sec. 2.1; Sec. 2.2.1, matrices as (1,1) tensors).
 *  - A two-qubit gate on (a, b) is U[2 o_a + o_b][2 i_a + i_b]: the first
 *    listed qubit is the more significant one, as in the paper's explicit
 *    4x4 Kronecker product U (x) V (Sec. 2.1).
 *  - Gate matrices: see oracle_gate_matrix.  The paper names H, CNOT, CZ, RZ
 *    and RX (Fig. 2.1, Fig. 3.1) without fixing their phases; the readings
 *    used here are listed with each gate.
 *
 * Complex numbers are stored as interleaved (re, im) doubles.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* gate ids used by this library only (the Python wrapper maps names) */
enum {
  OG_H = 0, OG_X, OG_Y, OG_Z, OG_S, OG_T, OG_SX, OG_SY, OG_SW,
  OG_RX, OG_RY, OG_RZ, OG_U3, OG_MIXER,
  OG_CZ = 32, OG_CNOT, OG_SWAP, OG_CPHASE, OG_ZZPHASE,
  OG_MAT1 = 64, OG_MAT2 = 65 /* explicit matrices passed by the caller */
};

typedef struct { double re, im; } cplx;

static cplx cmk(double r, double i) { cplx z = {r, i}; return z; }
static cplx cadd(cplx a, cplx b) { return cmk(a.re + b.re, a.im + b.im); }
static cplx cmul(cplx a, cplx b) { return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static cplx cexpi(double t) { return cmk(cos(t), sin(t)); }

int oracle_is_two_qubit(int kind) { return (kind >= 32 && kind < 64) || kind == OG_MAT2; }

/*
 * Matrix of a named gate, row-major, complex128 (2x2 or 4x4).
 *  H      = [[1,1],[1,-1]]/sqrt2            X, Y, Z: the Pauli matrices
 *  S      = diag(1, i)                      T = diag(1, e^{i pi/4})
 *  SX/SY/SW = principal square roots  ((1+i) I + (1-i) P)/2  of P = X, Y and
 *           W = (X+Y)/sqrt2 (each squares to P exactly)
 *  RX/RY/RZ(t) = exp(-i t P/2) = cos(t/2) I - i sin(t/2) P
 *  U3(t,f,l) = [[cos t/2, -e^{il} sin t/2], [e^{if} sin t/2, e^{i(f+l)} cos t/2]]
 *  MIXER(b) = exp(-i b X)   (QAOA mixer)
 *  CZ = diag(1,1,1,-1)      CNOT: control = first qubit      SWAP
 *  CPHASE(l) = diag(1,1,1,e^{il})
 *  ZZPHASE(g) = exp(-i g (1 - Z Z)/2) = diag(1, e^{-ig}, e^{-ig}, 1)  (QAOA phase separator)
 * Returns 0, or -1 for an unknown kind.
 */
int oracle_gate_matrix(int kind, const double *ang, double *out)
{
  cplx m[16];
  int d = oracle_is_two_qubit(kind) ? 4 : 2;
  for (int i = 0; i < 16; ++i) m[i] = cmk(0, 0);
  const double r2 = 1.0 / sqrt(2.0);
  switch (kind) {
  case OG_H: m[0] = cmk(r2, 0); m[1] = cmk(r2, 0); m[2] = cmk(r2, 0); m[3] = cmk(-r2, 0); break;
  case OG_X: m[1] = cmk(1, 0); m[2] = cmk(1, 0); break;
  case OG_Y: m[1] = cmk(0, -1); m[2] = cmk(0, 1); break;
  case OG_Z: m[0] = cmk(1, 0); m[3] = cmk(-1, 0); break;
  case OG_S: m[0] = cmk(1, 0); m[3] = cmk(0, 1); break;
  case OG_T: m[0] = cmk(1, 0); m[3] = cexpi(M_PI / 4); break;
  case OG_SX: case OG_SY: case OG_SW: {
    /* P for X, Y, W = (X+Y)/sqrt2, then ((1+i) I + (1-i) P)/2 */
    cplx p01, p10;
    if (kind == OG_SX) { p01 = cmk(1, 0); p10 = cmk(1, 0); }
    else if (kind == OG_SY) { p01 = cmk(0, -1); p10 = cmk(0, 1); }
    else { p01 = cmk(r2, -r2); p10 = cmk(r2, r2); }
    cplx a = cmk(0.5, 0.5), b = cmk(0.5, -0.5);
    m[0] = a; m[3] = a; m[1] = cmul(b, p01); m[2] = cmul(b, p10);
    break;
  }
  case OG_RX: { double c = cos(ang[0] / 2), s = sin(ang[0] / 2);
    m[0] = cmk(c, 0); m[3] = cmk(c, 0); m[1] = cmk(0, -s); m[2] = cmk(0, -s); break; }
  case OG_RY: { double c = cos(ang[0] / 2), s = sin(ang[0] / 2);
    m[0] = cmk(c, 0); m[3] = cmk(c, 0); m[1] = cmk(-s, 0); m[2] = cmk(s, 0); break; }
  case OG_RZ: m[0] = cexpi(-ang[0] / 2); m[3] = cexpi(ang[0] / 2); break;
  case OG_U3: { double c = cos(ang[0] / 2), s = sin(ang[0] / 2);
    m[0] = cmk(c, 0);
    m[1] = cmul(cmk(-s, 0), cexpi(ang[2]));
    m[2] = cmul(cmk(s, 0), cexpi(ang[1]));
    m[3] = cmul(cmk(c, 0), cexpi(ang[1] + ang[2]));
    break; }
  case OG_MIXER: { double c = cos(ang[0]), s = sin(ang[0]);
    m[0] = cmk(c, 0); m[3] = cmk(c, 0); m[1] = cmk(0, -s); m[2] = cmk(0, -s); break; }
  case OG_CZ: m[0] = m[5] = m[10] = cmk(1, 0); m[15] = cmk(-1, 0); break;
  case OG_CNOT: m[0] = m[5] = cmk(1, 0); m[11] = m[14] = cmk(1, 0); break;
  case OG_SWAP: m[0] = m[15] = cmk(1, 0); m[6] = m[9] = cmk(1, 0); break;
  case OG_CPHASE: m[0] = m[5] = m[10] = cmk(1, 0); m[15] = cexpi(ang[0]); break;
  case OG_ZZPHASE: m[0] = m[15] = cmk(1, 0); m[5] = m[10] = cexpi(-ang[0]); break;
  default: return -1;
  }
  for (int i = 0; i < d * d; ++i) { out[2 * i] = m[i].re; out[2 * i + 1] = m[i].im; }
  return 0;
}

/* the matrix of gate g: named, or taken from the caller's explicit matrices */
static int gate_mat(int kind, const double *ang, const double *mats, long g, cplx *m)
{
  double buf[32];
  if (kind == OG_MAT1 || kind == OG_MAT2) {
    int d = kind == OG_MAT2 ? 4 : 2;
    memcpy(buf, mats + 32 * g, sizeof(double) * 2 * d * d);
  } else if (oracle_gate_matrix(kind, ang, buf) != 0) {
    return -1;
  }
  for (int i = 0; i < 16; ++i) m[i] = cmk(buf[2 * i], buf[2 * i + 1]);
  return 0;
}

/* psi <- U psi on qubit q (bit n-1-q): pairs of amplitudes differing in that bit */
static void apply_1q(cplx *psi, int n, int q, const cplx *u)
{
  const int64_t stride = (int64_t)1 << (n - 1 - q);
  const int64_t half = (int64_t)1 << (n - 1);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < half; ++j) {
    int64_t lo = j & (stride - 1);
    int64_t i0 = ((j - lo) << 1) | lo;  /* insert a 0 bit at the gate's position */
    int64_t i1 = i0 | stride;
    cplx a0 = psi[i0], a1 = psi[i1];
    psi[i0] = cadd(cmul(u[0], a0), cmul(u[1], a1));
    psi[i1] = cadd(cmul(u[2], a0), cmul(u[3], a1));
  }
}

/* psi <- U psi on qubits (a, b); U[2 o_a + o_b][2 i_a + i_b] */
static void apply_2q(cplx *psi, int n, int qa, int qb, const cplx *u)
{
  const int pa = n - 1 - qa, pb = n - 1 - qb;
  const int plo = pa < pb ? pa : pb, phi = pa < pb ? pb : pa;
  const int64_t quarter = (int64_t)1 << (n - 2);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < quarter; ++j) {
    /* insert zero bits at plo then phi */
    int64_t lo = j & (((int64_t)1 << plo) - 1);
    int64_t t = ((j - lo) << 1) | lo;
    int64_t lo2 = t & (((int64_t)1 << phi) - 1);
    int64_t base = ((t - lo2) << 1) | lo2;
    int64_t idx[4];
    for (int v = 0; v < 4; ++v) {
      int ba = v >> 1, bb = v & 1;
      idx[v] = base | ((int64_t)ba << pa) | ((int64_t)bb << pb);
    }
    cplx in[4];
    for (int v = 0; v < 4; ++v) in[v] = psi[idx[v]];
    for (int r = 0; r < 4; ++r) {
      cplx acc = cmk(0, 0);
      for (int c = 0; c < 4; ++c) acc = cadd(acc, cmul(u[4 * r + c], in[c]));
      psi[idx[r]] = acc;
    }
  }
}

/*
 * Gate-by-gate state-vector simulation from |0...0> (Sec. 2.1: qubit states
 * evolve by unitary matrices applied in circuit order).
 *   kinds[g], qubits[2g..2g+1], angles[3g..3g+2]; mats[32g..] for OG_MAT*.
 *   psi_out: 2^n complex128, interleaved.
 * Returns 0, or -1 on a bad gate.
 */
int oracle_statevector(int n, int ngates, const int *kinds, const int *qubits, const double *angles,
                       const double *mats, double *psi_out)
{
  if (n < 1 || n > 40) return -1;
  cplx *psi = (cplx *)psi_out;
  const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < dim; ++i) psi[i] = cmk(0, 0);
  psi[0] = cmk(1, 0);
  for (int g = 0; g < ngates; ++g) {
    cplx u[16];
    if (gate_mat(kinds[g], angles + 3 * g, mats, g, u) != 0) return -1;
    int qa = qubits[2 * g], qb = qubits[2 * g + 1];
    if (qa < 0 || qa >= n) return -1;
    if (oracle_is_two_qubit(kinds[g])) {
      if (qb < 0 || qb >= n || qb == qa) return -1;
      apply_2q(psi, n, qa, qb, u);
    } else {
      apply_1q(psi, n, qa, u);
    }
  }
  return 0;
}

/*
 * The circuit's full 2^n x 2^n unitary, built independently of the sweep
 * above: each gate is embedded by its element-wise definition
 *   G[x][y] = U[(x_a x_b)][(y_a y_b)] if x and y agree on every other qubit,
 *   else 0
 * (for a 1-qubit gate this is I (x) ... (x) U (x) ... (x) I, Sec. 2.1), and
 * the embedded matrices are multiplied in circuit order, U = G_k ... G_1.
 * U_out: row-major complex128, n <= 10.  Returns 0 or -1.
 */
int oracle_dense_unitary(int n, int ngates, const int *kinds, const int *qubits, const double *angles,
                         const double *mats, double *U_out)
{
  if (n < 1 || n > 10) return -1;
  const int64_t D = (int64_t)1 << n;
  cplx *U = (cplx *)U_out;
  cplx *G = (cplx *)malloc(sizeof(cplx) * D * D);
  cplx *T = (cplx *)malloc(sizeof(cplx) * D * D);
  if (!G || !T) { free(G); free(T); return -1; }
  for (int64_t i = 0; i < D * D; ++i) U[i] = cmk(i / D == i % D ? 1 : 0, 0);
  for (int g = 0; g < ngates; ++g) {
    cplx u[16];
    if (gate_mat(kinds[g], angles + 3 * g, mats, g, u) != 0) { free(G); free(T); return -1; }
    int two = oracle_is_two_qubit(kinds[g]);
    int qa = qubits[2 * g], qb = two ? qubits[2 * g + 1] : -1;
    if (qa < 0 || qa >= n || (two && (qb < 0 || qb >= n || qb == qa))) { free(G); free(T); return -1; }
    int64_t mask = (int64_t)1 << (n - 1 - qa);
    if (two) mask |= (int64_t)1 << (n - 1 - qb);
    for (int64_t x = 0; x < D; ++x) {
      for (int64_t y = 0; y < D; ++y) {
        cplx v = cmk(0, 0);
        if ((x & ~mask) == (y & ~mask)) {
          int xa = (int)((x >> (n - 1 - qa)) & 1), ya = (int)((y >> (n - 1 - qa)) & 1);
          if (two) {
            int xb = (int)((x >> (n - 1 - qb)) & 1), yb = (int)((y >> (n - 1 - qb)) & 1);
            v = u[4 * (2 * xa + xb) + (2 * ya + yb)];
          } else {
            v = u[2 * xa + ya];
          }
        }
        G[x * D + y] = v;
      }
    }
    /* T = G U */
    for (int64_t i = 0; i < D; ++i)
      for (int64_t j = 0; j < D; ++j) {
        cplx acc = cmk(0, 0);
        for (int64_t k = 0; k < D; ++k) acc = cadd(acc, cmul(G[i * D + k], U[k * D + j]));
        T[i * D + j] = acc;
      }
    memcpy(U, T, sizeof(cplx) * D * D);
  }
  free(G);
  free(T);
  return 0;
}

/*
 * <psi|D|psi> = sum_x |psi_x|^2 D(x) for a diagonal observable written as
 * Z-strings, D(x) = sum_t c_t prod_{q in mask_t} (-1)^{x_q}, where mask_t has
 * bit n-1-q set for each qubit q of the string.  The bra conjugates psi,
 * so only |psi_x|^2 enters.
 */
double oracle_expectation_zstrings(int n, const double *psi_in, int nterms, const uint64_t *masks,
                                   const double *coeffs)
{
  const cplx *psi = (const cplx *)psi_in;
  const int64_t dim = (int64_t)1 << n;
  double total = 0.0;
#pragma omp parallel for reduction(+ : total) schedule(static)
  for (int64_t x = 0; x < dim; ++x) {
    double p = psi[x].re * psi[x].re + psi[x].im * psi[x].im;
    double d = 0.0;
    for (int t = 0; t < nterms; ++t) {
      int par = __builtin_popcountll((uint64_t)x & masks[t]) & 1;
      d += par ? -coeffs[t] : coeffs[t];
    }
    total += p * d;
  }
  return total;
}

/* amplitudes <b|psi> for each bitstring b (qubit q in bit n-1-q): psi[b] */
void oracle_amplitudes(int n, const double *psi, int64_t count, const uint64_t *bits, double *out)
{
  const uint64_t dim = (uint64_t)1 << n;
  for (int64_t s = 0; s < count; ++s) {
    uint64_t b = bits[s];
    if (b >= dim) { out[2 * s] = NAN; out[2 * s + 1] = NAN; continue; }
    out[2 * s] = psi[2 * b];
    out[2 * s + 1] = psi[2 * b + 1];
  }
}

/*
 * Fixed-point arithmetic of the paper's FPGA designs (Sec. 3: complex
 * arithmetic in 32-bit fixed point with 28 bits behind the binary point).
 * The paper leaves the sign/integer split and the rounding unstated; the
 * reading used here is two's-complement Q3.28 (value = raw / 2^28, raw an
 * int32), every real product rounded to the nearest Q3.28 value with ties to
 * even, every sum saturating at the int32 range.  A complex product is formed
 * from four rounded real products: (ar br - ai bi) + i (ar bi + ai br).
 */
static int32_t q_sat(int64_t v)
{
  if (v > INT32_MAX) return INT32_MAX;
  if (v < INT32_MIN) return INT32_MIN;
  return (int32_t)v;
}

/* x (a double) to the nearest Q3.28 value, ties to even (rint in the default rounding mode) */
int32_t oracle_q328_from_double(double x)
{
  double r = rint(x * 268435456.0);
  if (r > (double)INT32_MAX) return INT32_MAX;
  if (r < (double)INT32_MIN) return INT32_MIN;
  return (int32_t)r;
}

/* a * b: the exact product raw_a raw_b / 2^56 rounded to Q3.28, ties to even, saturated */
int32_t oracle_q328_mul(int32_t a, int32_t b)
{
  const int64_t p = (int64_t)a * (int64_t)b;
  int64_t q = p >> 28; /* floor (arithmetic shift) */
  const int64_t rem = p - q * ((int64_t)1 << 28); /* in [0, 2^28) */
  const int64_t half = (int64_t)1 << 27;
  if (rem > half || (rem == half && (q & 1))) q += 1;
  return q_sat(q);
}

typedef struct { int32_t re, im; } qcplx;

static qcplx qc_mul(qcplx a, qcplx b)
{
  qcplx r;
  r.re = q_sat((int64_t)oracle_q328_mul(a.re, b.re) - (int64_t)oracle_q328_mul(a.im, b.im));
  r.im = q_sat((int64_t)oracle_q328_mul(a.re, b.im) + (int64_t)oracle_q328_mul(a.im, b.re));
  return r;
}

static qcplx qc_add(qcplx a, qcplx b)
{
  qcplx r;
  r.re = q_sat((int64_t)a.re + b.re);
  r.im = q_sat((int64_t)a.im + b.im);
  return r;
}

/*
 * The gate-by-gate state vector of oracle_statevector in Q3.28: each gate's
 * FP64 matrix rounded once to Q3.28, every output amplitude the saturating
 * sum of the rounded products of its matrix row with the input amplitudes.
 *   psi_out: 2^n complex Q3.28 values, interleaved int32 (re, im).
 * Returns 0, or -1 on a bad gate.
 */
int oracle_statevector_q328(int n, int ngates, const int *kinds, const int *qubits, const double *angles,
                            const double *mats, int32_t *psi_out)
{
  if (n < 1 || n > 34) return -1;
  qcplx *psi = (qcplx *)psi_out;
  const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < dim; ++i) { psi[i].re = 0; psi[i].im = 0; }
  psi[0].re = oracle_q328_from_double(1.0);
  for (int g = 0; g < ngates; ++g) {
    cplx u[16];
    qcplx uq[16];
    if (gate_mat(kinds[g], angles + 3 * g, mats, g, u) != 0) return -1;
    for (int i = 0; i < 16; ++i) {
      uq[i].re = oracle_q328_from_double(u[i].re);
      uq[i].im = oracle_q328_from_double(u[i].im);
    }
    const int two = oracle_is_two_qubit(kinds[g]);
    const int qa = qubits[2 * g], qb = qubits[2 * g + 1];
    if (qa < 0 || qa >= n || (two && (qb < 0 || qb >= n || qb == qa))) return -1;
    const int d = two ? 4 : 2;
    const int pa = n - 1 - qa, pb = two ? n - 1 - qb : 0;
    const int64_t groups = dim >> (two ? 2 : 1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < groups; ++j) {
      /* the basis index with zero bits inserted at the gate's positions (lower one first) */
      int64_t base = j;
      int lo = two ? (pa < pb ? pa : pb) : pa, hi = two ? (pa < pb ? pb : pa) : -1;
      base = ((base >> lo) << (lo + 1)) | (base & (((int64_t)1 << lo) - 1));
      if (two) base = ((base >> hi) << (hi + 1)) | (base & (((int64_t)1 << hi) - 1));
      int64_t idx[4];
      for (int v = 0; v < d; ++v)
        idx[v] = two ? base | ((int64_t)(v >> 1) << pa) | ((int64_t)(v & 1) << pb) : base | ((int64_t)v << pa);
      qcplx in[4];
      for (int v = 0; v < d; ++v) in[v] = psi[idx[v]];
      for (int r = 0; r < d; ++r) {
        qcplx acc = {0, 0};
        for (int c = 0; c < d; ++c) acc = qc_add(acc, qc_mul(uq[d * r + c], in[c]));
        psi[idx[r]] = acc;
      }
    }
  }
  return 0;
}

/* number of OpenMP threads a parallel region uses here */
int oracle_num_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
