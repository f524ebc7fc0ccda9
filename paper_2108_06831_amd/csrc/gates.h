// Gate matrices and gate-recipe evaluation, FP64, callable on host and device.
//
// A tensor of the network that stands for gates (a single gate, or a run of
// gates pre-contracted into one two-qubit block, Sec. 3) is described by a
// recipe: the list of elementary gates in circuit order.  The device
// materialises every recipe at contraction time from the current angles
// (FP64 trigonometry, rounded once to complex64); the host uses the same
// functions to report FP64 tensor values for checks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tn.h"

namespace tnq {

struct c128 {
  double re, im;
};

__host__ __device__ inline c128 cm(double r, double i) { return c128{r, i}; }
__host__ __device__ inline c128 cmul(c128 a, c128 b) { return cm(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
__host__ __device__ inline c128 cadd(c128 a, c128 b) { return cm(a.re + b.re, a.im + b.im); }
__host__ __device__ inline c128 cconj(c128 a) { return cm(a.re, -a.im); }
__host__ __device__ inline c128 cis(double t) { return cm(cos(t), sin(t)); }

__host__ __device__ inline bool gate_is_two_qubit(int kind) {
  return kind == TN_GATE_CZ || kind == TN_GATE_CNOT || kind == TN_GATE_SWAP || kind == TN_GATE_CPHASE ||
         kind == TN_GATE_ZZPHASE || kind == TN_GATE_MATRIX2;
}

__host__ __device__ inline bool gate_is_diagonal(int kind) {
  return kind == TN_GATE_Z || kind == TN_GATE_S || kind == TN_GATE_T || kind == TN_GATE_RZ || kind == TN_GATE_CZ ||
         kind == TN_GATE_CPHASE || kind == TN_GATE_ZZPHASE;
}

__host__ __device__ inline int gate_n_angles(int kind) {
  switch (kind) {
    case TN_GATE_RX: case TN_GATE_RY: case TN_GATE_RZ: case TN_GATE_MIXER: case TN_GATE_CPHASE:
    case TN_GATE_ZZPHASE: return 1;
    case TN_GATE_U3: return 3;
    default: return 0;
  }
}

// Row-major matrix of a named gate (2x2 in m[0..3] or 4x4 in m[0..15]).
// Returns false for an unknown kind.  Explicit matrices are handled by the caller.
__host__ __device__ inline bool gate_matrix(int kind, const double* a, c128* m) {
  for (int i = 0; i < 16; ++i) m[i] = cm(0, 0);
  const double h = 0.70710678118654752440;
  switch (kind) {
    case TN_GATE_H: m[0] = cm(h, 0); m[1] = cm(h, 0); m[2] = cm(h, 0); m[3] = cm(-h, 0); return true;
    case TN_GATE_X: m[1] = cm(1, 0); m[2] = cm(1, 0); return true;
    case TN_GATE_Y: m[1] = cm(0, -1); m[2] = cm(0, 1); return true;
    case TN_GATE_Z: m[0] = cm(1, 0); m[3] = cm(-1, 0); return true;
    case TN_GATE_S: m[0] = cm(1, 0); m[3] = cm(0, 1); return true;
    case TN_GATE_T: m[0] = cm(1, 0); m[3] = cm(h, h); return true;
    case TN_GATE_SX: case TN_GATE_SY: case TN_GATE_SW: {
      // ((1+i) I + (1-i) P) / 2 with P = X, Y or (X+Y)/sqrt2
      c128 off01 = kind == TN_GATE_SX ? cm(1, 0) : kind == TN_GATE_SY ? cm(0, -1) : cm(h, -h);
      c128 off10 = kind == TN_GATE_SX ? cm(1, 0) : kind == TN_GATE_SY ? cm(0, 1) : cm(h, h);
      const c128 d = cm(0.5, 0.5), o = cm(0.5, -0.5);
      m[0] = d; m[3] = d; m[1] = cmul(o, off01); m[2] = cmul(o, off10);
      return true;
    }
    case TN_GATE_RX: { double c = cos(0.5 * a[0]), s = sin(0.5 * a[0]);
      m[0] = cm(c, 0); m[3] = cm(c, 0); m[1] = cm(0, -s); m[2] = cm(0, -s); return true; }
    case TN_GATE_RY: { double c = cos(0.5 * a[0]), s = sin(0.5 * a[0]);
      m[0] = cm(c, 0); m[3] = cm(c, 0); m[1] = cm(-s, 0); m[2] = cm(s, 0); return true; }
    case TN_GATE_RZ: m[0] = cis(-0.5 * a[0]); m[3] = cis(0.5 * a[0]); return true;
    case TN_GATE_U3: { double c = cos(0.5 * a[0]), s = sin(0.5 * a[0]);
      c128 el = cis(a[2]), ef = cis(a[1]), efl = cis(a[1] + a[2]);
      m[0] = cm(c, 0); m[1] = cm(-s * el.re, -s * el.im); m[2] = cm(s * ef.re, s * ef.im);
      m[3] = cm(c * efl.re, c * efl.im); return true; }
    case TN_GATE_MIXER: { double c = cos(a[0]), s = sin(a[0]);
      m[0] = cm(c, 0); m[3] = cm(c, 0); m[1] = cm(0, -s); m[2] = cm(0, -s); return true; }
    case TN_GATE_CZ: m[0] = m[5] = m[10] = cm(1, 0); m[15] = cm(-1, 0); return true;
    case TN_GATE_CNOT: m[0] = m[5] = cm(1, 0); m[11] = m[14] = cm(1, 0); return true;
    case TN_GATE_SWAP: m[0] = m[15] = cm(1, 0); m[6] = m[9] = cm(1, 0); return true;
    case TN_GATE_CPHASE: m[0] = m[5] = m[10] = cm(1, 0); m[15] = cis(a[0]); return true;
    case TN_GATE_ZZPHASE: m[0] = m[15] = cm(1, 0); m[5] = m[10] = cis(-a[0]); return true;
    default: return false;
  }
}

// One elementary gate inside a recipe.
struct RecipeOp {
  int32_t kind;      // tn_gate_kind
  int32_t pos;       // 1-qubit gate in a 2-qubit block: 0 = block's first (more significant) qubit, 1 = second.
                     // 2-qubit gate: 0 = same qubit order as the block, 1 = reversed.
  int32_t param[3];  // -1 = fixed angle
  int32_t mat;       // index of an explicit matrix (32 doubles) for MATRIX kinds, else -1
  double angle[3];
};

// A gate tensor: ops[op_begin, op_end) applied in order to a block of nq qubits.
// Diagonal recipes store only the diagonal (tensor over the wires' hyper-indices).
struct Recipe {
  int32_t nq;
  int32_t diag;
  int32_t op_begin, op_end;
  int32_t split_side;  // -1: the whole block; else the half of a split block on block qubit 0 or 1
  int32_t split_on;    // block qubit (0 or 1) in whose value the block's two-qubit gate is block-diagonal
  int64_t offset;      // element offset of the tensor in the per-batch input buffer
};

// Every array below is indexed by compile-time constants only (loops over
// fixed extents, unrolled; run-time choices made by selects), so that on the
// device the matrices stay in registers instead of per-thread scratch memory.

// The elementary matrix of one recipe op (16 entries, 2x2 or 4x4 row-major).
__host__ __device__ inline void op_matrix(const RecipeOp& op, const double* mats, const double* params, c128* u) {
  double ang[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) ang[j] = op.param[j] >= 0 ? params[op.param[j]] : op.angle[j];
  if (op.kind == TN_GATE_MATRIX1 || op.kind == TN_GATE_MATRIX2) {
    const int n = op.kind == TN_GATE_MATRIX2 ? 16 : 4;
    const double* m = mats + 32 * op.mat;
#pragma unroll
    for (int i = 0; i < 16; ++i) u[i] = i < n ? cm(m[2 * i], m[2 * i + 1]) : cm(0, 0);
  } else {
    gate_matrix(op.kind, ang, u);
  }
}

// M <- G M for the 4x4 block matrix M, G = a one-qubit u on block qubit POS
// (0: the first, more significant qubit).
template <int POS>
__host__ __device__ inline void left_apply1_at(const c128* u, c128* M) {
  c128 T[16];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int xa = x >> 1, xb = x & 1;
    const int r = POS ? xb : xa;                                    // row of u
    const int y0 = POS ? 4 * (2 * xa) : 4 * xb, y1 = POS ? 4 * (2 * xa + 1) : 4 * (2 + xb);  // rows of M
#pragma unroll
    for (int j = 0; j < 4; ++j) T[4 * x + j] = cadd(cmul(u[2 * r], M[y0 + j]), cmul(u[2 * r + 1], M[y1 + j]));
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) M[i] = T[i];
}

__host__ __device__ inline void left_apply1(const c128* u, int pos, c128* M) {
  if (pos) left_apply1_at<1>(u, M); else left_apply1_at<0>(u, M);
}

// a two-qubit u in the block's qubit order (POS 0) or reversed (POS 1)
template <int POS>
__host__ __device__ inline void block_two_qubit_at(const c128* u, c128* G) {
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int xs = POS ? ((x & 1) << 1) | (x >> 1) : x, ys = POS ? ((y & 1) << 1) | (y >> 1) : y;
      G[4 * x + y] = u[4 * xs + ys];
    }
}

__host__ __device__ inline void block_two_qubit(const c128* u, int pos, c128* G) {
  if (pos) block_two_qubit_at<1>(u, G); else block_two_qubit_at<0>(u, G);
}

// d x d matrix (d = 2^nq = D) of a recipe, FP64; get_u(o, u) gives op o's
// elementary matrix.
template <int D, class GetU>
__host__ __device__ inline void recipe_matrix_dg(const Recipe& r, const RecipeOp* ops, GetU get_u, c128* M) {
#pragma unroll
  for (int i = 0; i < D * D; ++i) M[i] = cm((i / D) == (i % D) ? 1.0 : 0.0, 0.0);
  for (int o = r.op_begin; o < r.op_end; ++o) {
    const RecipeOp& op = ops[o];
    c128 u[16];
    get_u(o, u);
    if (D == 2) {
      c128 T[4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) T[2 * i + j] = cadd(cmul(u[2 * i], M[j]), cmul(u[2 * i + 1], M[2 + j]));
#pragma unroll
      for (int i = 0; i < 4; ++i) M[i] = T[i];
    } else if (gate_is_two_qubit(op.kind)) {
      c128 G[16], T[16];
      block_two_qubit(u, op.pos, G);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          c128 acc = cm(0, 0);
#pragma unroll
          for (int k = 0; k < 4; ++k) acc = cadd(acc, cmul(G[4 * i + k], M[4 * k + j]));
          T[4 * i + j] = acc;
        }
#pragma unroll
      for (int i = 0; i < 16; ++i) M[i] = T[i];
    } else {
      left_apply1(u, op.pos, M);
    }
  }
}

template <int D>
__host__ __device__ inline void recipe_matrix_d(const Recipe& r, const RecipeOp* ops, const double* mats,
                                                const double* params, c128* M) {
  recipe_matrix_dg<D>(r, ops, [&](int o, c128* u) { op_matrix(ops[o], mats, params, u); }, M);
}

// d x d matrix (d = 2^nq) of a recipe into M[0 .. d*d), FP64.
__host__ __device__ inline void recipe_matrix(const Recipe& r, const RecipeOp* ops, const double* mats,
                                              const double* params, c128* M) {
  if (r.nq == 2) {
    recipe_matrix_d<4>(r, ops, mats, params, M);
  } else {
    recipe_matrix_d<2>(r, ops, mats, params, M);
  }
}

// A two-qubit block whose two-qubit gate is block-diagonal in the value of one
// of its qubits (CZ, CPHASE, ZZPHASE, CNOT on its control, ...) has the exact
// operator-Schmidt form  sum_k X_k (x) Y_k : with `on` the bond qubit, the
// half on qubit `on` is post . |k><k| . pre and the other half is
// post . G_k . pre with G_k the 2x2 block of the gate at bond value k (pre/post:
// the block's one-qubit gates on that side before/after the two-qubit gate).
// Writes the half on block qubit `side` as the tensor [k][o][i] (8 entries);
// get_u(o, u) gives op o's elementary matrix.
template <class GetU>
__host__ __device__ inline void recipe_split_half_g(const Recipe& r, const RecipeOp* ops, GetU get_u, c128* out) {
  const int side = r.split_side, on = r.split_on;
  // cur: product of this side's one-qubit gates since the two-qubit gate (or
  // the start); it becomes `pre` when the two-qubit gate arrives
  c128 cur[4], pre[4], post[4], U[16];
#pragma unroll
  for (int i = 0; i < 4; ++i) cur[i] = pre[i] = cm((i == 0 || i == 3) ? 1.0 : 0.0, 0.0);
#pragma unroll
  for (int i = 0; i < 16; ++i) U[i] = cm((i / 4) == (i % 4) ? 1.0 : 0.0, 0.0);
  bool after = false;
  for (int o = r.op_begin; o < r.op_end; ++o) {
    const RecipeOp& op = ops[o];
    c128 u[16];
    get_u(o, u);
    if (gate_is_two_qubit(op.kind)) {
      block_two_qubit(u, op.pos, U);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        pre[i] = cur[i];
        cur[i] = cm((i == 0 || i == 3) ? 1.0 : 0.0, 0.0);
      }
      after = true;
      continue;
    }
    if (op.pos != side) continue;
    c128 T[4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) T[2 * i + j] = cadd(cmul(u[2 * i], cur[j]), cmul(u[2 * i + 1], cur[2 + j]));
#pragma unroll
    for (int i = 0; i < 4; ++i) cur[i] = T[i];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const c128 id = cm((i == 0 || i == 3) ? 1.0 : 0.0, 0.0);
    post[i] = after ? cur[i] : id;
    pre[i] = after ? pre[i] : cur[i];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    c128 G[4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const c128 own = cm((x == k && y == k) ? 1.0 : 0.0, 0.0);
        const c128 g0 = U[4 * (2 * k + x) + (2 * k + y)], g1 = U[4 * (2 * x + k) + (2 * y + k)];
        G[2 * x + y] = side == on ? own : (on == 0 ? g0 : g1);
      }
    c128 T[4], V[4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) T[2 * i + j] = cadd(cmul(G[2 * i], pre[j]), cmul(G[2 * i + 1], pre[2 + j]));
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) V[2 * i + j] = cadd(cmul(post[2 * i], T[j]), cmul(post[2 * i + 1], T[2 + j]));
#pragma unroll
    for (int i = 0; i < 4; ++i) out[4 * k + i] = V[i];
  }
}

__host__ __device__ inline void recipe_split_half(const Recipe& r, const RecipeOp* ops, const double* mats,
                                                  const double* params, c128* out) {
  recipe_split_half_g(r, ops, [&](int o, c128* u) { op_matrix(ops[o], mats, params, u); }, out);
}

}  // namespace tnq
