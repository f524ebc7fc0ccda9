// gfx950 kernels of the contraction path.
//
//  * k_materialize / k_projectors: gate tensors from angles (FP64, rounded once
//    to complex64), |0> vectors and one-hot bitstring projectors.
//  * k_skinny: a pairwise contraction whose smaller operand is gate-sized.  It
//    streams the large operand once from HBM (HBM-bound) through strided
//    addresses, so no permute is needed before it.
//  * k_permute: bit-permutation transpose staged through LDS so that both the
//    reads and the writes are coalesced.
//  * k_gemm: complex matrix product on the FP32 matrix cores (4M form through
//    a real embedding, below), batched over the batch modes.
//  * k_expect_* / k_adjoint_*: FP64-accumulated reductions for expectations
//    and the adjoint gradient.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "kernels.h"

namespace tnq {

namespace {

constexpr int kThreads = 256;

__device__ inline float2 f2(float x, float y) { return make_float2(x, y); }

// round-to-nearest-even to bfloat16, returned as float
__device__ inline float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// a*b (real) in the requested precision: FP32, or the three-term bf16 split
template <int PREC>
__device__ inline float rmul(float a, float b) {
  if constexpr (PREC == TN_PREC_C64) {
    return a * b;
  } else {
    const float ah = bf16_round(a), al = bf16_round(a - ah);
    const float bh = bf16_round(b), bl = bf16_round(b - bh);
    return fmaf(ah, bh, fmaf(ah, bl, al * bh));
  }
}

// acc + a b.  In FP32 as two fused multiply-adds per component (a separate
// product, difference and sum would take three instructions each).
template <int PREC>
__device__ inline float2 cmac(float2 acc, float2 a, float2 b) {
  if constexpr (PREC == TN_PREC_C64) {
    acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
    acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
  } else {
    acc.x += rmul<PREC>(a.x, b.x) - rmul<PREC>(a.y, b.y);
    acc.y += rmul<PREC>(a.x, b.y) + rmul<PREC>(a.y, b.x);
  }
  return acc;
}

// a b (no accumulator): one product and one fused multiply-add per component
template <int PREC>
__device__ inline float2 cmul(float2 a, float2 b) {
  if constexpr (PREC == TN_PREC_C64)
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
  else
    return make_float2(rmul<PREC>(a.x, b.x) - rmul<PREC>(a.y, b.y), rmul<PREC>(a.x, b.y) + rmul<PREC>(a.y, b.x));
}

__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  __syncthreads();
  return t;
}

}  // namespace

// ---------------------------------------------------------------------------
// Materialisation of the network's input tensors
// ---------------------------------------------------------------------------
// One block per tensor: the elementary matrices of the tensor's ops (the FP64
// trigonometry) are evaluated in parallel, one op per thread, into LDS; one
// thread then multiplies them in order, with the block matrices in registers
// (every array below is indexed by constants).  Rounded once to complex64.
constexpr int kRecipeThreads = 64;

// The nearest Q3.28 value (raw int32 = value * 2^28), ties to even, saturated.
__device__ inline int32_t q328_from_double(double x) {
  const double r = rint(x * 268435456.0);
  return r >= 2147483647.0 ? 2147483647 : r <= -2147483648.0 ? (int32_t)0x80000000 : (int32_t)r;
}

// One FP64 complex value stored rounded once: to complex64 (Q = false) or to
// a Q3.28 (re, im) pair in the same 8 bytes (Q = true).
template <bool Q>
__device__ inline void store_c(float2* o, int i, const c128& v) {
  if constexpr (Q)
    reinterpret_cast<int2*>(o)[i] = make_int2(q328_from_double(v.re), q328_from_double(v.im));
  else
    o[i] = f2((float)v.re, (float)v.im);
}

template <bool Q, class GetU>
__device__ void write_recipe(const Recipe& r, const RecipeOp* ops, GetU get_u, float2* o) {
  if (r.split_side >= 0) {
    c128 H[8];
    recipe_split_half_g(r, ops, get_u, H);
#pragma unroll
    for (int i = 0; i < 8; ++i) store_c<Q>(o, i, H[i]);
  } else if (r.nq == 2) {
    c128 M[16];
    recipe_matrix_dg<4>(r, ops, get_u, M);
    if (r.diag) {
#pragma unroll
      for (int i = 0; i < 4; ++i) store_c<Q>(o, i, M[5 * i]);
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) store_c<Q>(o, i, M[i]);
    }
  } else {
    c128 M[4];
    recipe_matrix_dg<2>(r, ops, get_u, M);
    if (r.diag) {
      store_c<Q>(o, 0, M[0]);
      store_c<Q>(o, 1, M[3]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) store_c<Q>(o, i, M[i]);
    }
  }
}

template <bool Q>
__global__ __launch_bounds__(kRecipeThreads) void k_materialize(const DevTensor* ts, int nt, const Recipe* rs,
                                                                const RecipeOp* ops, const double* mats,
                                                                const double* params, int64_t pstride, float2* in,
                                                                int64_t in_bs) {
  __shared__ c128 U[kRecipeThreads][16];
  const int t = blockIdx.x;
  const int z = blockIdx.y;
  if (t >= nt) return;
  const DevTensor d = ts[t];
  float2* o = in + (int64_t)z * in_bs + d.offset;
  if (d.kind == TK_KET0) {
    if (threadIdx.x == 0) {
      store_c<Q>(o, 0, c128{1.0, 0.0});
      store_c<Q>(o, 1, c128{0.0, 0.0});
    }
  } else if (d.kind == TK_GATE) {
    const Recipe r = rs[d.recipe];
    const double* p = params ? params + (int64_t)z * pstride : nullptr;
    const int n = r.op_end - r.op_begin;
    if (n <= kRecipeThreads) {
      if ((int)threadIdx.x < n) {
        c128 u[16];
        op_matrix(ops[r.op_begin + threadIdx.x], mats, p, u);
#pragma unroll
        for (int i = 0; i < 16; ++i) U[threadIdx.x][i] = u[i];
      }
      __syncthreads();
      if (threadIdx.x == 0)
        write_recipe<Q>(r, ops, [&](int op, c128* u) {
#pragma unroll
          for (int i = 0; i < 16; ++i) u[i] = U[op - r.op_begin][i];
        }, o);
    } else if (threadIdx.x == 0) {
      write_recipe<Q>(r, ops, [&](int op, c128* u) { op_matrix(ops[op], mats, p, u); }, o);
    }
  }
}

// one_bits: the 32-bit pattern of the value 1 (1.0f, or 2^28 in Q3.28)
__global__ void k_projectors(const uint64_t* bits, int64_t count, int n, int blog2, int64_t first, float2* in,
                             int64_t in_bs, uint32_t one_bits) {
  const int64_t per = (int64_t)1 << blog2;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (i >= per * n) return;
  const int q = (int)(i / per);
  const int64_t s = i % per;
  const int bit = s < count ? (int)((bits[s] >> (n - 1 - q)) & 1) : 0;
  uint2* o = reinterpret_cast<uint2*>(in + (int64_t)z * in_bs + first + (int64_t)q * per * 2 + 2 * s);
  o[0] = make_uint2(bit == 0 ? one_bits : 0u, 0u);
  o[1] = make_uint2(bit == 1 ? one_bits : 0u, 0u);
}

hipError_t launch_materialize(hipStream_t s, const DevTensor* ts, int nt, const Recipe* recipes, const RecipeOp* ops,
                              const double* mats, const double* params, int64_t params_stride, int batch,
                              float2* in, int64_t in_bs, bool q328) {
  if (nt == 0) return hipSuccess;
  if (q328)
    hipLaunchKernelGGL(k_materialize<true>, dim3(nt, batch), dim3(kRecipeThreads), 0, s, ts, nt, recipes, ops, mats,
                       params, params_stride, in, in_bs);
  else
    hipLaunchKernelGGL(k_materialize<false>, dim3(nt, batch), dim3(kRecipeThreads), 0, s, ts, nt, recipes, ops, mats,
                       params, params_stride, in, in_bs);
  return hipGetLastError();
}

hipError_t launch_projectors(hipStream_t s, const uint64_t* bits, int64_t count, int n_qubits, int blog2,
                             int64_t first_offset, int batch, float2* in, int64_t in_bs, bool q328) {
  const int64_t total = ((int64_t)1 << blog2) * n_qubits;
  dim3 grid((unsigned)((total + kThreads - 1) / kThreads), batch);
  const uint32_t one = q328 ? (1u << 28) : 0x3f800000u;
  hipLaunchKernelGGL(k_projectors, grid, dim3(kThreads), 0, s, bits, count, n_qubits, blog2, first_offset, in, in_bs,
                     one);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Q3.28 fixed point: one step of a path as a per-output product over raw int32
// (re, im) pairs (value = raw / 2^28).  Every real product is the exact 64-bit
// product shifted back by 28 bits, rounded to nearest with ties to even and
// saturated; every sum saturates at the int32 range.
// ---------------------------------------------------------------------------
__device__ inline int32_t q_sat(int64_t v) {
  return v > 2147483647ll ? 2147483647 : v < -2147483648ll ? (int32_t)0x80000000 : (int32_t)v;
}
__device__ inline int64_t q_mul(int32_t a, int32_t b) {
  const int64_t p = (int64_t)a * (int64_t)b;
  int64_t q = p >> 28;
  const int64_t rem = p & (((int64_t)1 << 28) - 1);
  q += (rem > ((int64_t)1 << 27)) | ((rem == ((int64_t)1 << 27)) & (q & 1));
  return q_sat(q);
}

constexpr int kQChunks = (kQMaxOutBits + 7) / 8;  // 8-bit chunks of a result index
constexpr int kQKTable = 1024;                    // summed indices resolved through an LDS table

struct QStepArgs {
  const int2* a;
  const int2* b;
  int2* c;
  int64_t a_bs, b_bs, c_bs;
  QStep st;
};

__global__ __launch_bounds__(kThreads) void k_q328_step(QStepArgs g) {
  __shared__ int64_t ta[kQChunks][256], tb[kQChunks][256];
  __shared__ int64_t ka[kQKTable], kb[kQKTable];
  const QStep& q = g.st;
  const int nc = (q.n_out + 7) / 8;
  const int nkl = q.n_k < 10 ? q.n_k : 10;  // low summed bits through the table
  for (int i = threadIdx.x; i < nc * 256; i += kThreads) {
    const int c = i >> 8, v = i & 255;
    int64_t da = 0, db = 0;
    for (int j = 0; j < 8; ++j) {
      const int bit = 8 * c + j;
      if (bit >= q.n_out || !((v >> j) & 1)) continue;
      if (q.a_o[bit] >= 0) da |= (int64_t)1 << q.a_o[bit];
      if (q.b_o[bit] >= 0) db |= (int64_t)1 << q.b_o[bit];
    }
    ta[c][v] = da;
    tb[c][v] = db;
  }
  for (int k = threadIdx.x; k < (1 << nkl); k += kThreads) {
    int64_t da = 0, db = 0;
    for (int j = 0; j < nkl; ++j)
      if ((k >> j) & 1) {
        da |= (int64_t)1 << q.a_k[j];
        db |= (int64_t)1 << q.b_k[j];
      }
    ka[k] = da;
    kb[k] = db;
  }
  __syncthreads();
  const int z = blockIdx.y;
  const int2* A = g.a + (int64_t)z * g.a_bs;
  const int2* B = g.b + (int64_t)z * g.b_bs;
  int2* C = g.c + (int64_t)z * g.c_bs;
  const int64_t n_out = (int64_t)1 << q.n_out;
  const int64_t n_hi = (int64_t)1 << (q.n_k - nkl);
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < n_out; o += (int64_t)gridDim.x * kThreads) {
    int64_t a0 = 0, b0 = 0;
    for (int c = 0; c < nc; ++c) {
      const int v = (int)((o >> (8 * c)) & 255);
      a0 |= ta[c][v];
      b0 |= tb[c][v];
    }
    int32_t re = 0, im = 0;
    for (int64_t h = 0; h < n_hi; ++h) {
      int64_t ah = a0, bh = b0;
      for (int j = nkl; j < q.n_k; ++j)
        if ((h >> (j - nkl)) & 1) {
          ah |= (int64_t)1 << q.a_k[j];
          bh |= (int64_t)1 << q.b_k[j];
        }
      for (int k = 0; k < (1 << nkl); ++k) {
        const int2 x = A[ah | ka[k]], y = B[bh | kb[k]];
        const int32_t pr = q_sat(q_mul(x.x, y.x) - q_mul(x.y, y.y));
        const int32_t pi = q_sat(q_mul(x.x, y.y) + q_mul(x.y, y.x));
        re = q_sat((int64_t)re + pr);
        im = q_sat((int64_t)im + pi);
      }
    }
    C[o] = make_int2(re, im);
  }
}

hipError_t launch_q328_step(hipStream_t s, const QStep& q, const void* a, int64_t a_bs, const void* b, int64_t b_bs,
                            void* c, int64_t c_bs, int batch) {
  if (q.n_out < 0 || q.n_out > kQMaxOutBits || q.n_k < 0 || q.n_k > kQMaxKBits) return hipErrorInvalidValue;
  QStepArgs g;
  g.a = (const int2*)a; g.b = (const int2*)b; g.c = (int2*)c;
  g.a_bs = a_bs; g.b_bs = b_bs; g.c_bs = c_bs;
  g.st = q;
  int64_t blocks = (((int64_t)1 << q.n_out) + kThreads - 1) / kThreads;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_q328_step, dim3((unsigned)blocks, batch), dim3(kThreads), 0, s, g);
  return hipGetLastError();
}

// out[z][o] (complex64) = the Q3.28 value at F[z][deposit(o)], where bit j of o
// sits at bit pos[j] of F's address
__global__ __launch_bounds__(kThreads) void k_q328_finish(const int2* F, int64_t f_bs, float2* out, int64_t out_bs,
                                                          int64_t count, QStep map) {
  __shared__ int64_t ta[kQChunks][256];
  const int nc = (map.n_out + 7) / 8;
  for (int i = threadIdx.x; i < nc * 256; i += kThreads) {
    const int c = i >> 8, v = i & 255;
    int64_t d = 0;
    for (int j = 0; j < 8; ++j) {
      const int bit = 8 * c + j;
      if (bit < map.n_out && ((v >> j) & 1)) d |= (int64_t)1 << map.a_o[bit];
    }
    ta[c][v] = d;
  }
  __syncthreads();
  const int z = blockIdx.y;
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < count; o += (int64_t)gridDim.x * kThreads) {
    int64_t a = 0;
    for (int c = 0; c < nc; ++c) a |= ta[c][(o >> (8 * c)) & 255];
    const int2 v = F[(int64_t)z * f_bs + a];
    out[(int64_t)z * out_bs + o] = f2((float)((double)v.x * (1.0 / 268435456.0)), (float)((double)v.y * (1.0 / 268435456.0)));
  }
}

hipError_t launch_q328_finish(hipStream_t s, const void* f, int64_t f_bs, float2* out, int64_t out_bs, int64_t count,
                              const QStep& map, int batch) {
  if (map.n_out < 0 || map.n_out > kQMaxOutBits) return hipErrorInvalidValue;
  int64_t blocks = (count + kThreads - 1) / kThreads;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_q328_finish, dim3((unsigned)std::max<int64_t>(blocks, 1), batch), dim3(kThreads), 0, s,
                     (const int2*)f, f_bs, out, out_bs, count, map);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small-operand contraction
// ---------------------------------------------------------------------------
struct SkinnyArgs {
  const float2* g;
  const float2* t;
  float2* c;
  int64_t g_bs, t_bs, c_bs;
  int64_t n_outer;
  int32_t nb, c_mode, g_elems, pad;
  int32_t k_pos[kSkinnyMaxK];
  int32_t b_pos[kSkinnyMaxG];
  int64_t kofs[1 << kSkinnyMaxK];
  int64_t mofs[1 << kSkinnyMaxM];
  int32_t gidx[1 << kSkinnyMaxG];
};

template <int NK, int NM, int PREC>
__global__ __launch_bounds__(kThreads) void k_skinny(SkinnyArgs a) {
  __shared__ float2 gs[1 << kSkinnyMaxG];
  const int z = blockIdx.y;
  const float2* G = a.g + (int64_t)z * a.g_bs;
  const float2* Tp = a.t + (int64_t)z * a.t_bs;
  float2* Cp = a.c + (int64_t)z * a.c_bs;
  for (int i = threadIdx.x; i < a.g_elems; i += kThreads) gs[i] = G[a.gidx[i]];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < a.n_outer; o += stride) {
    int64_t tb = o;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const int p = a.k_pos[j];
      tb = ((tb >> p) << (p + 1)) | (tb & (((int64_t)1 << p) - 1));
    }
    int b = 0;
    for (int j = 0; j < a.nb; ++j) b |= (int)((o >> a.b_pos[j]) & 1) << j;
    float2 x[1 << NK];
#pragma unroll
    for (int k = 0; k < (1 << NK); ++k) x[k] = Tp[tb | a.kofs[k]];
    const int64_t cb = a.c_mode ? o : tb;
    const float2* gb = gs + (b << (NM + NK));
#pragma unroll
    for (int m = 0; m < (1 << NM); ++m) {
      float2 acc = f2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < (1 << NK); ++k) acc = cmac<PREC>(acc, gb[(m << NK) + k], x[k]);
      Cp[cb | a.mofs[m]] = acc;
    }
  }
}

// A run of outer products (see OuterChain): block (h, z) writes the 2^t_bits
// elements of C whose vector bits are h, T times the block's factor
// g_1[h_1] .. g_k[h_k].  The factor is formed in FP32 whatever the precision
// of the products (each step has a single term: there is nothing to sum).
struct OuterArgs {
  const float2* t;
  float2* c;
  const float2* in;
  const float2* ws;
  int64_t t_bs, c_bs, in_bs, ws_bs;
  int32_t t_bits, k;
  int64_t vsrc[kOuterMax][2];
};

__global__ __launch_bounds__(kThreads) void k_outer_chain(OuterArgs a) {
  const int z = blockIdx.y;
  const int64_t h = blockIdx.x;
  float2 f = f2(1.f, 0.f);
  for (int i = 0; i < a.k; ++i) {
    const int64_t v = a.vsrc[i][(h >> i) & 1];
    const float2* b = ((v >> 56) & 0x3f) == BUF_IN ? a.in + (int64_t)z * a.in_bs : a.ws + (int64_t)z * a.ws_bs;
    f = cmul<TN_PREC_C64>(f, b[v & (((int64_t)1 << 56) - 1)]);
  }
  // two elements per access (t_bits >= 8)
  const float4* T = reinterpret_cast<const float4*>(a.t + (int64_t)z * a.t_bs);
  float4* C = reinterpret_cast<float4*>(a.c + (int64_t)z * a.c_bs + (h << a.t_bits));
  const int64_t n = (int64_t)1 << (a.t_bits - 1);
  for (int64_t o = threadIdx.x; o < n; o += blockDim.x) {
    const float4 x = T[o];
    const float2 y0 = cmul<TN_PREC_C64>(f, f2(x.x, x.y)), y1 = cmul<TN_PREC_C64>(f, f2(x.z, x.w));
    C[o] = make_float4(y0.x, y0.y, y1.x, y1.y);
  }
}

hipError_t launch_outer_chain(hipStream_t s, const OuterChain& oc, const float2* t, int64_t t_bs, float2* c,
                              int64_t c_bs, const float2* in, int64_t in_bs, const float2* ws, int64_t ws_bs,
                              int batch) {
  if (oc.k < 1 || oc.k > kOuterMax || oc.k > 24 || oc.t_bits < 8 || oc.t_bits > 40) return hipErrorInvalidValue;
  if ((reinterpret_cast<uintptr_t>(t) | reinterpret_cast<uintptr_t>(c)) & 15) return hipErrorInvalidValue;
  if (((t_bs | c_bs) & 1) != 0) return hipErrorInvalidValue;  // float4 accesses in every batch item
  OuterArgs a;
  a.t = t; a.c = c; a.in = in; a.ws = ws;
  a.t_bs = t_bs; a.c_bs = c_bs; a.in_bs = in_bs; a.ws_bs = ws_bs;
  a.t_bits = oc.t_bits;
  a.k = oc.k;
  for (int i = 0; i < kOuterMax; ++i)
    for (int m = 0; m < 2; ++m) a.vsrc[i][m] = i < oc.k ? oc.vsrc[i][m] : 0;
  hipLaunchKernelGGL(k_outer_chain, dim3(1u << oc.k, batch), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <int NK, int NM>
static void* skinny_fn(int prec) {
  return prec == TN_PREC_BF16X3 ? (void*)k_skinny<NK, NM, TN_PREC_BF16X3> : (void*)k_skinny<NK, NM, TN_PREC_C64>;
}

template <int NK>
static void* skinny_fn_m(int nm, int prec) {
  switch (nm) {
    case 0: return skinny_fn<NK, 0>(prec);
    case 1: return skinny_fn<NK, 1>(prec);
    case 2: return skinny_fn<NK, 2>(prec);
    case 3: return skinny_fn<NK, 3>(prec);
    default: return skinny_fn<NK, 4>(prec);
  }
}

hipError_t launch_skinny(hipStream_t s, const SkinnyDesc& d, const float2* g, int64_t g_bs, const float2* t,
                         int64_t t_bs, float2* c, int64_t c_bs, int batch, int precision) {
  SkinnyArgs a;
  a.g = g; a.t = t; a.c = c;
  a.g_bs = g_bs; a.t_bs = t_bs; a.c_bs = c_bs;
  a.n_outer = (int64_t)1 << (d.t_bits - d.nk);
  a.nb = d.nb;
  a.c_mode = d.c_mode;
  a.g_elems = 1 << (d.nb + d.nm + d.nk);
  a.pad = 0;
  for (int j = 0; j < kSkinnyMaxK; ++j) a.k_pos[j] = d.k_pos[j];
  for (int j = 0; j < kSkinnyMaxG; ++j) a.b_pos[j] = d.b_pos[j];
  for (int j = 0; j < (1 << kSkinnyMaxK); ++j) a.kofs[j] = d.kofs[j];
  for (int j = 0; j < (1 << kSkinnyMaxM); ++j) a.mofs[j] = d.mofs[j];
  for (int j = 0; j < (1 << kSkinnyMaxG); ++j) a.gidx[j] = d.gidx[j];
  void* fn;
  switch (d.nk) {
    case 0: fn = skinny_fn_m<0>(d.nm, precision); break;
    case 1: fn = skinny_fn_m<1>(d.nm, precision); break;
    case 2: fn = skinny_fn_m<2>(d.nm, precision); break;
    case 3: fn = skinny_fn_m<3>(d.nm, precision); break;
    default: fn = skinny_fn_m<4>(d.nm, precision); break;
  }
  int64_t blocks = (a.n_outer + kThreads - 1) / kThreads;
  if (blocks > 16384) blocks = 16384;
  void* args[] = {&a};
  return hipLaunchKernel(fn, dim3((unsigned)blocks, batch), dim3(kThreads), args, 0, s);
}

// ---------------------------------------------------------------------------
// Interpreter of small steps (one launch for all the tiny contractions that
// only depend on inputs): each workgroup walks one independent work list.
// A step is computed into registers, then written after a barrier, so a step
// may overwrite one of its own operands.
// ---------------------------------------------------------------------------

// byte j (0..11) of three packed words, sign-extended
__device__ inline int packed_byte(uint32_t w0, uint32_t w1, uint32_t w2, int j) {
  const uint32_t x = j < 4 ? w0 : j < 8 ? w1 : w2;
  return (int)(int8_t)(x >> (8 * (j & 3)));
}

constexpr int kStageInFlight = 8;  // operand loads each interpreter thread issues before it waits

template <int PREC>
__global__ __launch_bounds__(kSmallThreads) void k_small_steps(const SmallStep* steps, const int32_t* list_off,
                                                          const int32_t* level_off, const uint32_t* items,
                                                          float2* in, int64_t in_bs, float2* ws, int64_t ws_bs) {
  __shared__ __attribute__((aligned(16))) SmallStep desc[kSmallDescCache];
  __shared__ __attribute__((aligned(16))) float2 stage[kSmallStage];
  const int w = blockIdx.x, z = blockIdx.y;
  float2* IN = in + (int64_t)z * in_bs;
  float2* WS = ws + (int64_t)z * ws_bs;
  int win0 = -1, win1 = -1;  // steps whose descriptors are in LDS
  for (int lv = list_off[w]; lv < list_off[w + 1]; ++lv) {
    const int l0 = level_off[lv], l1 = level_off[lv + 1];
    for (int cb = l0; cb < l1; cb += kSmallDescCache) {
      const int ce = min(l1, cb + kSmallDescCache), ns = ce - cb;
      if (cb < win0 || ce > win1) {
        // load the descriptors of as many whole following levels as fit (at
        // least this chunk): one global round trip for several levels
        int end = ce;
        if (cb == l0 && l1 - l0 <= kSmallDescCache) {
          int nl = lv + 1;
          while (nl < list_off[w + 1] && level_off[nl + 1] - cb <= kSmallDescCache) ++nl;
          end = level_off[nl];
        }
        const int words = (end - cb) * (int)(sizeof(SmallStep) / 16);
        const uint4* src = reinterpret_cast<const uint4*>(steps + cb);
        uint4* dst = reinterpret_cast<uint4*>(desc);
        __syncthreads();  // the previous window is no longer read
        for (int i = threadIdx.x; i < words; i += kSmallThreads) dst[i] = src[i];
        win0 = cb;
        win1 = end;
        __syncthreads();
      }
      const SmallStep* desc_c = desc + (cb - win0);  // this chunk's descriptors
      // rounds (planned on the host): steps of the level whose operands fit in LDS together
      for (int r0 = 0; r0 < ns;) {
        const int r1 = desc_c[r0].round_end;
        const SmallStep& last = desc_c[r1 - 1];
        const int stage_end = last.stage_b + (1 << last.b_bits);
        // this thread's work items, fetched while the operands are staged
        const int it0 = desc_c[r0].item0, nit = desc_c[r0].n_items;
        const uint32_t my0 = (int)threadIdx.x < nit ? items[it0 + threadIdx.x] : 0u;
        const uint32_t my1 = (int)threadIdx.x + kSmallThreads < nit ? items[it0 + threadIdx.x + kSmallThreads] : 0u;
        // stage the operands: one flat loop over the round's operand elements,
        // every thread keeping kStageInFlight independent loads in flight
        for (int e0 = threadIdx.x; e0 < stage_end; e0 += kStageInFlight * kSmallThreads) {
          float2 v[kStageInFlight];
#pragma unroll
          for (int u = 0; u < kStageInFlight; ++u) {
            const int e = e0 + u * kSmallThreads;
            if (e >= stage_end) break;
            int lo = r0, hi = r1 - 1;  // the step owning staged element e
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (desc_c[mid].stage_a <= e) lo = mid; else hi = mid - 1;
            }
            const SmallStep& st = desc_c[lo];
            const bool is_a = e < st.stage_b;
            const float2* src = is_a ? (st.a_buf == BUF_IN ? IN : WS) + st.a_off + (e - st.stage_a)
                                     : (st.b_buf == BUF_IN ? IN : WS) + st.b_off + (e - st.stage_b);
            v[u] = *src;
          }
#pragma unroll
          for (int u = 0; u < kStageInFlight; ++u) {
            const int e = e0 + u * kSmallThreads;
            if (e >= stage_end) break;
            stage[e] = v[u];
          }
        }
        __syncthreads();
        // each item: the outputs j + t 2^qb of one step; the operand addresses
        // of the first come from the step's index maps (packed in registers),
        // the next ones by flipping the address bits of the output bits that change
        for (int q = 0; q < 2; ++q) {
          if ((int)threadIdx.x + q * kSmallThreads >= nit) break;
          const uint32_t wd = q == 0 ? my0 : my1;
          const SmallStep& st = desc_c[wd & 255u];
          const int o0 = (int)((wd >> 8) & 4095u), qb = (int)(wd >> 20), nt_ = 1 << (st.c_bits - qb);
          const uint32_t* ap = reinterpret_cast<const uint32_t*>(st.apos);
          const uint32_t* bp = reinterpret_cast<const uint32_t*>(st.bpos);
          const uint32_t* ka = reinterpret_cast<const uint32_t*>(st.ka);
          const uint32_t* kb = reinterpret_cast<const uint32_t*>(st.kb);
          const uint32_t ap0 = ap[0], ap1 = ap[1], ap2 = ap[2], bp0 = bp[0], bp1 = bp[1], bp2 = bp[2];
          const uint32_t ka0 = ka[0], ka1 = ka[1], ka2 = ka[2], kb0 = kb[0], kb1 = kb[1], kb2 = kb[2];
          const int nk = 1 << st.k_bits;
          const float2* As = stage + st.stage_a;
          const float2* Bs = stage + st.stage_b;
          float2* C = (st.c_buf == BUF_IN ? IN : WS) + st.c_off;
          int ab = 0, bb = 0;
          for (uint32_t m = (uint32_t)o0; m; m &= m - 1) {
            const int p = __builtin_ctz(m);
            const int pa = packed_byte(ap0, ap1, ap2, p), pb = packed_byte(bp0, bp1, bp2, p);
            if (pa >= 0) ab |= 1 << pa;
            if (pb >= 0) bb |= 1 << pb;
          }
          for (int t = 0; t < nt_; ++t) {
            const int o = o0 | (t << qb);
            if (t != 0)
              for (uint32_t f = (uint32_t)((t ^ (t - 1)) << qb); f; f &= f - 1) {
                const int p = __builtin_ctz(f);
                const int pa = packed_byte(ap0, ap1, ap2, p), pb = packed_byte(bp0, bp1, bp2, p);
                if (pa >= 0) ab ^= 1 << pa;
                if (pb >= 0) bb ^= 1 << pb;
              }
            // summed index in Gray-code order: one address bit flips per term
            int a = ab, b = bb;
            float2 acc = cmul<PREC>(As[a], Bs[b]);
            for (int k = 1; k < nk; ++k) {
              const int j = __builtin_ctz(k);
              a ^= 1 << packed_byte(ka0, ka1, ka2, j);
              b ^= 1 << packed_byte(kb0, kb1, kb2, j);
              acc = cmac<PREC>(acc, As[a], Bs[b]);
            }
            C[o] = acc;
          }
        }
        __syncthreads();
        r0 = r1;
      }
    }
  }
}

hipError_t launch_small_steps(hipStream_t s, const SmallStep* steps, const int32_t* list_off,
                              const int32_t* level_off, const uint32_t* items, int n_lists, float2* in,
                              int64_t in_bs, float2* ws, int64_t ws_bs, int batch, int precision) {
  if (n_lists == 0) return hipSuccess;
  if (precision == TN_PREC_BF16X3)
    hipLaunchKernelGGL(k_small_steps<TN_PREC_BF16X3>, dim3(n_lists, batch), dim3(kSmallThreads), 0, s, steps, list_off,
                       level_off, items, in, in_bs, ws, ws_bs);
  else
    hipLaunchKernelGGL(k_small_steps<TN_PREC_C64>, dim3(n_lists, batch), dim3(kSmallThreads), 0, s, steps, list_off,
                       level_off, items, in, in_bs, ws, ws_bs);
  return hipGetLastError();
}

// deposit(x, pos, nbits): bit j of x (j < nbits) placed at address position
// pos[j]; the address maps of the permute and matrix-product kernels.
// The positions are read four at a time as 32-bit words (each map starts at
// a multiple of 4 bytes of the argument block): word loads of the argument
// block are scalar loads, while a byte-wise read becomes one vector memory
// load per bit that the loop waits for.
static_assert(kGemmMaxBits % 4 == 0, "position maps of whole 32-bit words");
__device__ inline int64_t deposit(int64_t x, const int8_t* pos, int nbits) {
  const int32_t* w = reinterpret_cast<const int32_t*>(pos);
  int64_t r = 0;
  for (int j = 0; j < nbits; j += 4) {
    const int32_t p4 = w[j >> 2];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (j + q < nbits) r |= ((x >> (j + q)) & 1) << ((p4 >> (8 * q)) & 63);
  }
  return r;
}

// ---------------------------------------------------------------------------
// Fused streaming pass: a chunk of 2^l elements (address bits lpos, the five
// lowest always among them so that loads and stores move 256-byte runs) is
// staged in LDS and every gate of the pass is applied to it before it is
// written back: one HBM read and one write for the whole pass.  Gates run in
// segments: each thread holds the 16 elements that differ in the segment's
// four register bits, applies the segment's gates in registers, and the chunk
// goes through LDS only between segments.
// ---------------------------------------------------------------------------
// (lpos and rest start at multiples of 4 bytes: deposit() reads them as 32-bit words)
struct SweepPassArgs {
  const float2* in;
  float2* out;
  int64_t in_bs, out_bs;
  const float2* vals;  // the chain's gathered gate values
  int64_t vals_bs;
  const SweepGateDesc* gates;
  const SweepSegment* segs;
  int32_t n_segs, l, n_rest, pad;
  int32_t ctab_off;          // the pass's power tables in vals
  int32_t lds_off, lds_n;    // the range of vals staged in LDS: the pass's gate values and power
                             // tables when they fit (gates_in_lds), else the power tables only
  int32_t gates_in_lds, pad2;
  int8_t lpos[kSweepMaxLocal];
  int8_t rest[64];
};
static_assert(offsetof(SweepPassArgs, lpos) % 4 == 0 && offsetof(SweepPassArgs, rest) % 4 == 0 &&
                  kSweepMaxLocal % 4 == 0, "position maps aligned to 32-bit words");

__device__ inline int64_t ins0(int64_t x, int p) { return ((x >> p) << (p + 1)) | (x & (((int64_t)1 << p) - 1)); }
__device__ inline int lds_phys(int i) { return i + (i >> 5); }

// Streaming (non-temporal) loads and stores.  The matrix products store their
// results this way: a large product writes far more result than it reads
// operands, and ordinary stores would evict the operand tiles that later
// tiles of the same XCD still read from its L2.  The fused passes move each
// chunk through once.
typedef float float2_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_stream(float2* p, float re, float im) {
  float2_nt v;
  v.x = re;
  v.y = im;
  __builtin_nontemporal_store(v, reinterpret_cast<float2_nt*>(p));
}
__device__ __forceinline__ float2 load_stream(const float2* p) {
  const float2_nt v = __builtin_nontemporal_load(reinterpret_cast<const float2_nt*>(p));
  return f2(v.x, v.y);
}

// Moving a chunk of 2^l = 16 nt elements between HBM and LDS: thread tid
// takes elements tid + k nt, k = 0..15 (consecutive threads on consecutive
// addresses).  The loads are issued eight at a time before their LDS writes,
// so a thread waits for HBM twice per chunk instead of once per element,
// without holding all sixteen in registers (which would lower the occupancy
// of the pass kernels); the empty asm keeps the compiler from merging the two
// halves.
__device__ __forceinline__ void chunk_to_lds(float2* buf, const float2* src, int64_t base, const int64_t* dep_hi,
                                             int tid, int nt) {
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    float2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = tid + (8 * h + k) * nt;
      v[k] = load_stream(&src[base | (i & 31) | dep_hi[i >> 5]]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) buf[lds_phys(tid + (8 * h + k) * nt)] = v[k];
    asm volatile("" ::: "memory");
  }
}
// The same for two tensors at once (eight elements of each in flight).
__device__ __forceinline__ void chunk2_to_lds(float2* buf0, float2* buf1, const float2* src0, const float2* src1,
                                              int64_t base, const int64_t* dep_hi, int tid, int nt) {
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    float2 v[8], w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = tid + (8 * h + k) * nt;
      const int64_t x = base | (i & 31) | dep_hi[i >> 5];
      v[k] = load_stream(&src0[x]);
      w[k] = load_stream(&src1[x]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      buf0[lds_phys(tid + (8 * h + k) * nt)] = v[k];
      buf1[lds_phys(tid + (8 * h + k) * nt)] = w[k];
    }
    asm volatile("" ::: "memory");
  }
}
__device__ __forceinline__ void chunk_from_lds(float2* dst, const float2* buf, int64_t base, const int64_t* dep_hi,
                                               int tid, int nt) {
  // the addresses are computed again here rather than kept in registers since the load
  asm volatile("" ::: "memory");
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    float2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = buf[lds_phys(tid + (8 * h + k) * nt)];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = tid + (8 * h + k) * nt;
      store_stream(&dst[base | (i & 31) | dep_hi[i >> 5]], v[k].x, v[k].y);
    }
    asm volatile("" ::: "memory");
  }
}

// Shapes of a one-qubit matrix that take half the multiplies (known from the
// gate kinds, see GateForm): every entry real (RY, H, X, ...), or a real
// diagonal and an imaginary off-diagonal (RX, Y, the QAOA mixer exp(-i b X)).
enum { kDenseGeneric = 0, kDenseReal = 1, kDenseRxLike = 2 };

// The register-position variants of a helper below are the same code apart
// from which elements they touch, and in reduced precision they are long
// enough that the compiler merges their common tails, selecting the elements
// through pointers, which puts all of them in scratch memory.  A distinct
// (empty) marker at the end of each variant keeps the tails apart.
template <int PREC, int ID>
__device__ __forceinline__ void variant_end() {
  if constexpr (PREC != TN_PREC_C64) asm volatile("; variant %0" ::"n"(ID));
}

template <int PREC, int U, int FORM>
__device__ __forceinline__ void reg_apply1(float2 (&x)[16], const float2* g) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << U)) continue;
    const int r1 = r | (1 << U);
    const float2 a = x[r], b = x[r1];
    if (PREC == TN_PREC_C64 && FORM == kDenseReal) {
      x[r] = f2(fmaf(g[0].x, a.x, g[1].x * b.x), fmaf(g[0].x, a.y, g[1].x * b.y));
      x[r1] = f2(fmaf(g[2].x, a.x, g[3].x * b.x), fmaf(g[2].x, a.y, g[3].x * b.y));
    } else if (PREC == TN_PREC_C64 && FORM == kDenseRxLike) {
      // g1 = i g1.y, g2 = i g2.y: i t (u + i v) = -t v + i t u
      x[r] = f2(fmaf(g[0].x, a.x, -g[1].y * b.y), fmaf(g[0].x, a.y, g[1].y * b.x));
      x[r1] = f2(fmaf(g[3].x, b.x, -g[2].y * a.y), fmaf(g[3].x, b.y, g[2].y * a.x));
    } else {
      x[r] = cmac<PREC>(cmul<PREC>(g[0], a), g[1], b);
      x[r1] = cmac<PREC>(cmul<PREC>(g[2], a), g[3], b);
    }
  }
  variant_end<PREC, U * 3 + FORM>();
}

// A dense one-qubit gate on register bit rb, its values in the given form, on
// one state (NS = 1) or on x and y (NS = 2).  Bit and form are compile-time
// constants in every case: a form tested inside the unrolled element loop
// would be turned into per-element selects between the variants.
template <int PREC, int NS>
__device__ __forceinline__ void apply_dense1(float2 (&x)[16], float2 (&y)[16], const float2* g, int rb, int form) {
#define TNQ_DENSE1(U, F)                   \
  reg_apply1<PREC, U, F>(x, g);            \
  if (NS == 2) reg_apply1<PREC, U, F>(y, g); \
  break;
  // (the reduced-precision products take one form for all: identical cases would be merged
  // into code that indexes the elements through pointers, which keeps them out of registers)
  switch (rb * 3 + (PREC == TN_PREC_C64 ? form : kDenseGeneric)) {
    case 0: TNQ_DENSE1(0, 0)
    case 1: TNQ_DENSE1(0, 1)
    case 2: TNQ_DENSE1(0, 2)
    case 3: TNQ_DENSE1(1, 0)
    case 4: TNQ_DENSE1(1, 1)
    case 5: TNQ_DENSE1(1, 2)
    case 6: TNQ_DENSE1(2, 0)
    case 7: TNQ_DENSE1(2, 1)
    case 8: TNQ_DENSE1(2, 2)
    case 9: TNQ_DENSE1(3, 0)
    case 10: TNQ_DENSE1(3, 1)
    default: TNQ_DENSE1(3, 2)
  }
#undef TNQ_DENSE1
}

// A run of two to four dense one-qubit gates of one form on the register bits
// of mask M, in increasing bit order (the k-th gate's values at gp[k]), on x
// (NS = 1) or on x and y (NS = 2): straight-line code, where gate-by-gate
// dispatch would end every gate with a copy of the elements back into the
// registers the loop carries them in.
template <int PREC, int NS, int M, int F>
__device__ __forceinline__ void run_apply(float2 (&x)[16], float2 (&y)[16], const float2* const (&gp)[4]) {
  int k = 0;
  if constexpr ((M & 1) != 0) {
    reg_apply1<PREC, 0, F>(x, gp[k]);
    if (NS == 2) reg_apply1<PREC, 0, F>(y, gp[k]);
    ++k;
  }
  if constexpr ((M & 2) != 0) {
    reg_apply1<PREC, 1, F>(x, gp[k]);
    if (NS == 2) reg_apply1<PREC, 1, F>(y, gp[k]);
    ++k;
  }
  if constexpr ((M & 4) != 0) {
    reg_apply1<PREC, 2, F>(x, gp[k]);
    if (NS == 2) reg_apply1<PREC, 2, F>(y, gp[k]);
    ++k;
  }
  if constexpr ((M & 8) != 0) {
    reg_apply1<PREC, 3, F>(x, gp[k]);
    if (NS == 2) reg_apply1<PREC, 3, F>(y, gp[k]);
  }
  variant_end<PREC, 200 + M * 8 + NS * 4 + F>();
}

template <int PREC, int NS>
__device__ __forceinline__ void apply_dense1_run(float2 (&x)[16], float2 (&y)[16], const float2* const (&g)[4],
                                                 int mask, int form) {
#define TNQ_RUN(M)                                                   \
  case M * 3 + kDenseGeneric: run_apply<PREC, NS, M, kDenseGeneric>(x, y, g); break; \
  case M * 3 + kDenseReal: run_apply<PREC, NS, M, kDenseReal>(x, y, g); break;       \
  case M * 3 + kDenseRxLike: run_apply<PREC, NS, M, kDenseRxLike>(x, y, g); break;
  switch (mask * 3 + (PREC == TN_PREC_C64 ? form : kDenseGeneric)) {
    TNQ_RUN(3) TNQ_RUN(5) TNQ_RUN(6) TNQ_RUN(7) TNQ_RUN(9) TNQ_RUN(10) TNQ_RUN(11) TNQ_RUN(12) TNQ_RUN(13)
    TNQ_RUN(14)
    default: run_apply<PREC, NS, 15, kDenseGeneric>(x, y, g); break;  // mask 15, generic form
    case 15 * 3 + kDenseReal: run_apply<PREC, NS, 15, kDenseReal>(x, y, g); break;
    case 15 * 3 + kDenseRxLike: run_apply<PREC, NS, 15, kDenseRxLike>(x, y, g); break;
  }
#undef TNQ_RUN
}

template <int PREC, int U0, int U1>
__device__ __forceinline__ void reg_apply2(float2 (&x)[16], const float2* g) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & ((1 << U0) | (1 << U1))) continue;
    const int id[4] = {r, r | (1 << U0), r | (1 << U1), r | (1 << U0) | (1 << U1)};
    float2 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = x[id[k]];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      float2 acc = f2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc = cmac<PREC>(acc, g[4 * m + k], v[k]);
      x[id[m]] = acc;
    }
  }
  variant_end<PREC, 16 + U0 * 4 + U1>();
}

// Diagonal factor on the 16 register elements, with the bits of the factor's
// index resolved at compile time: e_{bit U of r} ...
template <int PREC, int U>
__device__ __forceinline__ void diag_reg1(float2 (&x)[16], float2 e0, float2 e1) {
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = cmul<PREC>((r >> U) & 1 ? e1 : e0, x[r]);
  variant_end<PREC, 32 + U>();
}
// ... or d_{bit U0 of r + 2 bit U1 of r}
template <int PREC, int U0, int U1>
__device__ __forceinline__ void diag_reg2(float2 (&x)[16], float2 d0, float2 d1, float2 d2, float2 d3) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int b = ((r >> U0) & 1) | (((r >> U1) & 1) << 1);
    x[r] = cmul<PREC>(b == 0 ? d0 : b == 1 ? d1 : b == 2 ? d2 : d3, x[r]);
  }
  variant_end<PREC, 48 + U0 * 4 + U1>();
}

// x[r] *= d_b, b = bit0 + 2 bit1 of the diagonal's index.  Bit j is register
// bit k_j of r (k_j in 0..3), or, for k_j < 0, the constant bit j of c.  All
// selections are per gate and thread, none per element.
template <int PREC>
__device__ __forceinline__ void apply_diag(float2 (&x)[16], int n, int k0, int k1, int c, float2 d0, float2 d1, float2 d2,
                                  float2 d3) {
  if (n == 2 && k0 >= 0 && k1 >= 0) {
    switch (k0 * 4 + k1) {
      case 1: diag_reg2<PREC, 0, 1>(x, d0, d1, d2, d3); break;
      case 2: diag_reg2<PREC, 0, 2>(x, d0, d1, d2, d3); break;
      case 3: diag_reg2<PREC, 0, 3>(x, d0, d1, d2, d3); break;
      case 4: diag_reg2<PREC, 1, 0>(x, d0, d1, d2, d3); break;
      case 6: diag_reg2<PREC, 1, 2>(x, d0, d1, d2, d3); break;
      case 7: diag_reg2<PREC, 1, 3>(x, d0, d1, d2, d3); break;
      case 8: diag_reg2<PREC, 2, 0>(x, d0, d1, d2, d3); break;
      case 9: diag_reg2<PREC, 2, 1>(x, d0, d1, d2, d3); break;
      case 11: diag_reg2<PREC, 2, 3>(x, d0, d1, d2, d3); break;
      case 12: diag_reg2<PREC, 3, 0>(x, d0, d1, d2, d3); break;
      case 13: diag_reg2<PREC, 3, 1>(x, d0, d1, d2, d3); break;
      default: diag_reg2<PREC, 3, 2>(x, d0, d1, d2, d3); break;
    }
    return;
  }
  int k = -1;
  float2 e0, e1;
  if (n == 2 && k0 >= 0) {  // bit 1 constant
    k = k0;
    e0 = (c & 2) ? d2 : d0;
    e1 = (c & 2) ? d3 : d1;
  } else if (n == 2 && k1 >= 0) {  // bit 0 constant
    k = k1;
    e0 = (c & 1) ? d1 : d0;
    e1 = (c & 1) ? d3 : d2;
  } else if (n == 1 && k0 >= 0) {
    k = k0;
    e0 = d0;
    e1 = d1;
  }
  if (k < 0) {  // constant over the thread's elements
    const float2 f = c == 0 ? d0 : c == 1 ? d1 : c == 2 ? d2 : d3;
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = cmul<PREC>(f, x[r]);
    return;
  }
  switch (k) {
    case 0: diag_reg1<PREC, 0>(x, e0, e1); break;
    case 1: diag_reg1<PREC, 1>(x, e0, e1); break;
    case 2: diag_reg1<PREC, 2>(x, e0, e1); break;
    default: diag_reg1<PREC, 3>(x, e0, e1); break;
  }
}

// Unit-modulus diagonals with the entry of index 0 factored out: the caller
// multiplies d0 into the thread's deferred phase, and only the elements whose
// index is not 0 are multiplied, by d_b conj(d0); an entry whose ratio is
// exactly 1 (the ZZ phase diag(1, e, e, 1) has d3 = d0) is skipped.
// (NS = 2: the same factors on a second state y)
template <int PREC, int NS, int U0, int U1>
__device__ __forceinline__ void diag_reg2_rel(float2 (&x)[16], float2 (&y)[16], float2 q1, float2 q2, float2 q3,
                                              int skip) {
  const bool s1 = (skip >> 1) & 1, s2 = (skip >> 2) & 1, s3 = (skip >> 3) & 1;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int b = ((r >> U0) & 1) | (((r >> U1) & 1) << 1);  // compile-time per r
    if (b == 0 || (b == 1 && s1) || (b == 2 && s2) || (b == 3 && s3)) continue;
    const float2 q = b == 1 ? q1 : b == 2 ? q2 : q3;
    x[r] = cmul<PREC>(q, x[r]);
    if (NS == 2) y[r] = cmul<PREC>(q, y[r]);
  }
  variant_end<PREC, 64 + NS * 16 + U0 * 4 + U1>();
}
template <int PREC, int NS, int U>
__device__ __forceinline__ void diag_reg1_rel(float2 (&x)[16], float2 (&y)[16], float2 q1) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if ((r >> U) & 1) {
      x[r] = cmul<PREC>(q1, x[r]);
      if (NS == 2) y[r] = cmul<PREC>(q1, y[r]);
    }
  variant_end<PREC, 112 + NS * 4 + U>();
}
__device__ inline bool is_one(float2 v) { return v.x == 1.f && v.y == 0.f; }

// x[r] *= d_b (unit-modulus entries) as ph *= d_{b0} and x[r] *= d_b conj(d_{b0}),
// b0 the index value of r = 0 (bits as in apply_diag: register bits k_j, else
// bit j of c).  Returns with nothing done to x when no bit is a register bit.
template <int PREC, int NS>
__device__ __forceinline__ void apply_diag_unit(float2 (&x)[16], float2 (&y)[16], float2& ph, int n, int k0, int k1,
                                                int c, float2 d0, float2 d1, float2 d2, float2 d3) {
  auto rel = [](float2 d, float2 base) { return cmul<TN_PREC_C64>(d, f2(base.x, -base.y)); };
  auto mulph = [&](float2 f) { ph = cmul<TN_PREC_C64>(ph, f); };
  if (n == 2 && k0 >= 0 && k1 >= 0) {
    mulph(d0);
    const float2 q1 = rel(d1, d0), q2 = rel(d2, d0), q3 = rel(d3, d0);
    const int skip = (is_one(q1) << 1) | (is_one(q2) << 2) | (is_one(q3) << 3);
    switch (k0 * 4 + k1) {
      case 1: diag_reg2_rel<PREC, NS, 0, 1>(x, y, q1, q2, q3, skip); break;
      case 2: diag_reg2_rel<PREC, NS, 0, 2>(x, y, q1, q2, q3, skip); break;
      case 3: diag_reg2_rel<PREC, NS, 0, 3>(x, y, q1, q2, q3, skip); break;
      case 4: diag_reg2_rel<PREC, NS, 1, 0>(x, y, q1, q2, q3, skip); break;
      case 6: diag_reg2_rel<PREC, NS, 1, 2>(x, y, q1, q2, q3, skip); break;
      case 7: diag_reg2_rel<PREC, NS, 1, 3>(x, y, q1, q2, q3, skip); break;
      case 8: diag_reg2_rel<PREC, NS, 2, 0>(x, y, q1, q2, q3, skip); break;
      case 9: diag_reg2_rel<PREC, NS, 2, 1>(x, y, q1, q2, q3, skip); break;
      case 11: diag_reg2_rel<PREC, NS, 2, 3>(x, y, q1, q2, q3, skip); break;
      case 12: diag_reg2_rel<PREC, NS, 3, 0>(x, y, q1, q2, q3, skip); break;
      case 13: diag_reg2_rel<PREC, NS, 3, 1>(x, y, q1, q2, q3, skip); break;
      default: diag_reg2_rel<PREC, NS, 3, 2>(x, y, q1, q2, q3, skip); break;
    }
    return;
  }
  int k = -1;
  float2 e0, e1;
  if (n == 2 && k0 >= 0) {  // bit 1 constant
    k = k0;
    e0 = (c & 2) ? d2 : d0;
    e1 = (c & 2) ? d3 : d1;
  } else if (n == 2 && k1 >= 0) {  // bit 0 constant
    k = k1;
    e0 = (c & 1) ? d1 : d0;
    e1 = (c & 1) ? d3 : d2;
  } else if (n == 1 && k0 >= 0) {
    k = k0;
    e0 = d0;
    e1 = d1;
  }
  if (k < 0) return;
  mulph(e0);
  const float2 q1 = rel(e1, e0);
  switch (k) {
    case 0: diag_reg1_rel<PREC, NS, 0>(x, y, q1); break;
    case 1: diag_reg1_rel<PREC, NS, 1>(x, y, q1); break;
    case 2: diag_reg1_rel<PREC, NS, 2>(x, y, q1); break;
    default: diag_reg1_rel<PREC, NS, 3>(x, y, q1); break;
  }
}

// A run of one-bit unit diagonal gates on the register bits of mask M, in
// increasing bit order, each already split as in apply_diag_unit (its first
// entry joined the deferred phase; q[k]: the k-th gate's second entry relative
// to its first): straight-line code, without the gate loop's copy per gate.
template <int PREC, int NS, int M>
__device__ __forceinline__ void diag_run_m(float2 (&x)[16], float2 (&y)[16], const float2 (&q)[4]) {
  int k = 0;
  if constexpr ((M & 1) != 0) diag_reg1_rel<PREC, NS, 0>(x, y, q[k++]);
  if constexpr ((M & 2) != 0) diag_reg1_rel<PREC, NS, 1>(x, y, q[k++]);
  if constexpr ((M & 4) != 0) diag_reg1_rel<PREC, NS, 2>(x, y, q[k++]);
  if constexpr ((M & 8) != 0) diag_reg1_rel<PREC, NS, 3>(x, y, q[k]);
  variant_end<PREC, 500 + NS * 16 + M>();
}

template <int PREC, int NS>
__device__ __forceinline__ void diag_run(float2 (&x)[16], float2 (&y)[16], const float2 (&q)[4], int mask) {
  switch (mask) {
    case 3: diag_run_m<PREC, NS, 3>(x, y, q); break;
    case 5: diag_run_m<PREC, NS, 5>(x, y, q); break;
    case 6: diag_run_m<PREC, NS, 6>(x, y, q); break;
    case 7: diag_run_m<PREC, NS, 7>(x, y, q); break;
    case 9: diag_run_m<PREC, NS, 9>(x, y, q); break;
    case 10: diag_run_m<PREC, NS, 10>(x, y, q); break;
    case 11: diag_run_m<PREC, NS, 11>(x, y, q); break;
    case 12: diag_run_m<PREC, NS, 12>(x, y, q); break;
    case 13: diag_run_m<PREC, NS, 13>(x, y, q); break;
    case 14: diag_run_m<PREC, NS, 14>(x, y, q); break;
    default: diag_run_m<PREC, NS, 15>(x, y, q); break;
  }
}

// The thread's elements that a diagonal with entries +-1 negates, as a 16-bit
// mask over the register combinations r: entry b (bit 0 from register bit k0
// or constant bit 0 of c, bit 1 likewise from k1 or c) is -1 where bit b of
// `signs` is set, as in apply_signs.
__device__ __forceinline__ int sign_pattern(int n, int k0, int k1, int c, int signs) {
  auto ones = [](int k) { return k == 0 ? 0xAAAA : k == 1 ? 0xCCCC : k == 2 ? 0xF0F0 : 0xFF00; };
  const int A = k0 >= 0 ? ones(k0) : ((c & 1) ? 0xFFFF : 0);
  const int B = n == 2 ? (k1 >= 0 ? ones(k1) : ((c & 2) ? 0xFFFF : 0)) : 0;
  int m = 0;
  if (signs & 1) m |= ~A & ~B;
  if (signs & 2) m |= A & ~B;
  if (signs & 4) m |= ~A & B;
  if (signs & 8) m |= A & B;
  return m & 0xFFFF;
}

// x[r] = -x[r] where bit r of m is set (sign-bit flips, no multiplies)
__device__ __forceinline__ void flip_signs(float2 (&x)[16], int m) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const unsigned s = (unsigned)((m >> r) & 1) << 31;
    x[r] = f2(__uint_as_float(__float_as_uint(x[r].x) ^ s), __uint_as_float(__float_as_uint(x[r].y) ^ s));
  }
}

// Sign mask of a diagonal whose used entries are all +1 or -1 (CZ, Z), or -1.
__device__ __forceinline__ int sign_mask(int n, float2 d0, float2 d1, float2 d2, float2 d3) {
  auto pm1 = [](float2 d) { return d.y == 0.f && fabsf(d.x) == 1.f; };
  const bool two = n == 2;
  if (!pm1(d0) || !pm1(d1) || (two && (!pm1(d2) || !pm1(d3)))) return -1;
  return (d0.x < 0.f) | ((d1.x < 0.f) << 1) | (two ? ((d2.x < 0.f) << 2) | ((d3.x < 0.f) << 3) : 0);
}

// x[r] = -x[r] where the diagonal's entry b is -1 (bit b of mask), b resolved as in apply_diag
template <int U>
__device__ __forceinline__ void signs_reg1(float2 (&x)[16], int m01) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if ((m01 >> ((r >> U) & 1)) & 1) x[r] = f2(-x[r].x, -x[r].y);
}
template <int U0, int U1>
__device__ __forceinline__ void signs_reg2(float2 (&x)[16], int mask) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int b = ((r >> U0) & 1) | (((r >> U1) & 1) << 1);
    if ((mask >> b) & 1) x[r] = f2(-x[r].x, -x[r].y);
  }
}
__device__ __forceinline__ void apply_signs(float2 (&x)[16], int n, int k0, int k1, int c, int mask) {
  if (n == 2 && k0 >= 0 && k1 >= 0) {
    switch (k0 * 4 + k1) {
      case 1: signs_reg2<0, 1>(x, mask); break;
      case 2: signs_reg2<0, 2>(x, mask); break;
      case 3: signs_reg2<0, 3>(x, mask); break;
      case 4: signs_reg2<1, 0>(x, mask); break;
      case 6: signs_reg2<1, 2>(x, mask); break;
      case 7: signs_reg2<1, 3>(x, mask); break;
      case 8: signs_reg2<2, 0>(x, mask); break;
      case 9: signs_reg2<2, 1>(x, mask); break;
      case 11: signs_reg2<2, 3>(x, mask); break;
      case 12: signs_reg2<3, 0>(x, mask); break;
      case 13: signs_reg2<3, 1>(x, mask); break;
      default: signs_reg2<3, 2>(x, mask); break;
    }
    return;
  }
  int k = -1, m01 = 0;  // signs of the register bit's two values
  if (n == 2 && k0 >= 0) {
    k = k0;
    m01 = (c & 2) ? (mask >> 2) & 3 : mask & 3;
  } else if (n == 2 && k1 >= 0) {
    k = k1;
    m01 = (c & 1) ? ((mask >> 1) & 1) | (((mask >> 3) & 1) << 1) : (mask & 1) | (((mask >> 2) & 1) << 1);
  } else if (n == 1 && k0 >= 0) {
    k = k0;
    m01 = mask & 3;
  }
  if (k < 0) {
    if ((mask >> c) & 1)
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = f2(-x[r].x, -x[r].y);
    return;
  }
  switch (k) {
    case 0: signs_reg1<0>(x, m01); break;
    case 1: signs_reg1<1>(x, m01); break;
    case 2: signs_reg1<2>(x, m01); break;
    default: signs_reg1<3>(x, m01); break;
  }
}


// A count group: x[r] *= w^cut(r), cut(r) the number of the group's E member
// edges whose two bits differ at the thread's element r.  An edge between
// two bits outside the registers adds a per-thread constant; an edge from
// register bit j to a constant bit b adds 1 where bit j of r differs from b;
// an edge between register bits j and k (the same for every thread) adds 1
// where they differ.  The powers come from the pass's LDS table tab.
__device__ __forceinline__ int count_pair(int j, int k) {  // 0..5 for the unordered pairs of 0..3
  const int lo = j < k ? j : k, hi = j < k ? k : j;
  return lo == 0 ? hi - 1 : lo == 1 ? hi + 1 : 5;
}
template <int PREC>
__device__ __forceinline__ void apply_count_group(float2 (&x)[16], const SweepGateDesc* __restrict__ m, int E, int ob,
                                                  int64_t base, const float2* tab) {
  int K = 0;                  // constant edges that differ
  uint32_t to0 = 0, to1 = 0;  // per register bit j (8-bit fields): edges to a constant 0 / 1
  uint64_t pr = 0;            // per register-bit pair (8-bit fields): edges between two register bits
  for (int e = 0; e < E; ++e) {
    const int k0 = m[e].kreg[0], k1 = m[e].kreg[1];
    auto cbit = [&](int j) {
      const int cs = m[e].csrc[j];
      return cs >= 64 ? (int)((base >> (cs - 64)) & 1) : ((ob >> cs) & 1);
    };
    if (k0 < 0 && k1 < 0) {
      K += cbit(0) ^ cbit(1);
    } else if (k0 >= 0 && k1 >= 0) {
      pr += (uint64_t)1 << (8 * count_pair(k0, k1));
    } else {
      const int j = k0 >= 0 ? k0 : k1;
      if (cbit(k0 >= 0 ? 1 : 0)) to1 += 1u << (8 * j);
      else to0 += 1u << (8 * j);
    }
  }
  // partial sums over register bits {0, 1} and {2, 3}: where bit j is set the edges to a
  // constant 0 differ, where it is clear those to a constant 1
  int s01[4], s23[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    s01[b] = K + (int)(((b & 1 ? to0 : to1) >> 0) & 255) + (int)(((b & 2 ? to0 : to1) >> 8) & 255);
    s23[b] = (int)(((b & 1 ? to0 : to1) >> 16) & 255) + (int)(((b & 2 ? to0 : to1) >> 24) & 255);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    int pc = 0;  // register-register edges that differ at r (the same for every thread)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = j + 1; k < 4; ++k)
        if (((r >> j) ^ (r >> k)) & 1) pc += (int)((pr >> (8 * count_pair(j, k))) & 255);
    x[r] = cmul<PREC>(tab[s01[r & 3] + s23[r >> 2] + pc], x[r]);
  }
}

// The descriptor and value tables come as separate __restrict__ arguments: the
// compiler may then read them with scalar loads (nothing the kernel writes can
// alias them) instead of vector memory loads on every gate.  VL: the gate
// values are read from their LDS copy (a compile-time choice: a pointer that
// may point to LDS or to global memory would be read with flat loads, whose
// latency every gate would wait on).
template <int PREC, bool VL>
__global__ __launch_bounds__(kThreads) void k_sweep_pass(SweepPassArgs a, const SweepGateDesc* __restrict__ gates,
                                                          const SweepSegment* __restrict__ segs,
                                                          const float2* __restrict__ vals) {
  __shared__ float2 buf[(1 << kSweepMaxLocal) + (1 << (kSweepMaxLocal - 5))];
  __shared__ int64_t dep_hi[1 << (kSweepMaxLocal - 5)];
  __shared__ float2 vtab[kPassValMax];  // see SweepPassArgs::lds_off
  const int z = blockIdx.y;
  const int64_t c = blockIdx.x;
  const int L = 1 << a.l;
  const int nt = blockDim.x, tid = threadIdx.x;
  const int64_t base = deposit(c, a.rest, a.n_rest);
  // address bits of local index bits 5.. (the five lowest local bits are address bits 0..4)
  for (int h = tid; h < (L >> 5); h += nt) dep_hi[h] = deposit((int64_t)h << 5, a.lpos, a.l);
  __syncthreads();
  const float2* in = a.in + (int64_t)z * a.in_bs;
  float2* out = a.out + (int64_t)z * a.out_bs;
  const float2* V0 = vals + (int64_t)z * a.vals_bs;
  for (int t = tid; t < a.lds_n; t += nt) vtab[t] = V0[a.lds_off + t];
  const float2* ctab = vtab + (a.ctab_off - a.lds_off);
  chunk_to_lds(buf, in, base, dep_hi, tid, nt);
  __syncthreads();
  for (int sg = 0; sg < a.n_segs; ++sg) {
    const SweepSegment& seg = segs[sg];
    // the thread's local bits outside the registers, and its slots (see SweepSegment)
    int ob = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) ob |= ((tid >> t) & 1) << seg.tpos[t];
    const int pob = ob + (ob >> 5);
    float2 x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = buf[pob + seg.physoff[r]];
    // diagonal factors that are the same for all of a thread's elements (every
    // bit of the gate outside the register set) commute with every gate of the
    // segment: they are multiplied into one per-thread factor, applied once
    float2 ph = f2(1.f, 0.f);
    bool ph_used = false;  // the same for the whole block: set where a gate's descriptor sends it to ph
    const int g_end = seg.first_gate + seg.n_gates;
    int gi = seg.first_gate;
    // the segment's leading diagonal gates with no bit in the registers (the
    // planner puts them first): only the per-thread factor changes, so this
    // loop carries no register elements (the main loop below copies them back
    // into place on every gate)
    for (; gi < g_end; ++gi) {
      const SweepGateDesc& gd = gates[gi];
      if (!gd.diag || gd.form == kFormCount || gd.form == kFormCountMember || gd.kreg[0] >= 0 ||
          (gd.n == 2 && gd.kreg[1] >= 0))
        break;
      const float2* V = VL ? vtab + (gd.voff - a.lds_off) : V0 + gd.voff;
      int cb = 0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (j >= gd.n) continue;
        const int cs = gd.csrc[j];
        cb |= (cs >= 64 ? (int)((base >> (cs - 64)) & 1) : ((ob >> cs) & 1)) << j;
      }
      const bool two = gd.n == 2;
      const float2 d0 = V[0], d1 = V[1], d2 = two ? V[2] : d0, d3 = two ? V[3] : d0;
      const float2 f = cb == 0 ? d0 : cb == 1 ? d1 : cb == 2 ? d2 : d3;
      ph_used = true;
      if (gd.form == kFormSigns) {
        if (f.x < 0.f) ph = f2(-ph.x, -ph.y);
      } else {
        ph = cmul<TN_PREC_C64>(ph, f);
      }
    }
    for (; gi < g_end; ++gi) {
      const SweepGateDesc& gd = gates[gi];
      const float2* V = VL ? vtab + (gd.voff - a.lds_off) : V0 + gd.voff;
      if (gd.form == kFormCount) {
        apply_count_group<PREC>(x, gates + gi + 1, gd.n, ob, base, ctab + gd.voff);
        gi += gd.n;
        continue;
      }
      if (gd.diag && gd.run_mask && gd.form == kFormSigns) {  // run_mask gates with entries +-1
        int m = 0;
        for (int j = 0; j < gd.run_mask; ++j) {
          const SweepGateDesc& gj = gates[gi + j];
          const float2* Vj = VL ? vtab + (gj.voff - a.lds_off) : V0 + gj.voff;
          const bool two = gj.n == 2;
          const int sm = (Vj[0].x < 0.f) | ((Vj[1].x < 0.f) << 1) | (two ? ((Vj[2].x < 0.f) << 2) | ((Vj[3].x < 0.f) << 3) : 0);
          int cb = 0;
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            if (t >= gj.n || gj.kreg[t] >= 0) continue;
            const int cs = gj.csrc[t];
            cb |= (cs >= 64 ? (int)((base >> (cs - 64)) & 1) : ((ob >> cs) & 1)) << t;
          }
          m ^= sign_pattern(gj.n, gj.kreg[0], two ? gj.kreg[1] : -1, cb, sm);
        }
        flip_signs(x, m);
        gi += gd.run_mask - 1;
        continue;
      }
      if (gd.diag && gd.run_mask) {  // one-bit unit diagonals on the mask's register bits, in bit order
        const int cnt = __builtin_popcount(gd.run_mask);
        float2 q[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int vo = j < cnt ? gates[gi + j].voff : gd.voff;
          const float2* Vj = VL ? vtab + (vo - a.lds_off) : V0 + vo;
          const float2 e0 = Vj[0], e1 = Vj[1];
          if (j < cnt) ph = cmul<TN_PREC_C64>(ph, e0);
          q[j] = cmul<TN_PREC_C64>(e1, f2(e0.x, -e0.y));
        }
        ph_used = true;
        diag_run<PREC, 1>(x, x, q, gd.run_mask);
        gi += cnt - 1;
        continue;
      }
      if (gd.diag) {
        const bool two = gd.n == 2;
        const float2 d0 = V[0], d1 = V[1];
        const float2 d2 = two ? V[2] : f2(1.f, 0.f), d3 = two ? V[3] : f2(1.f, 0.f);
        const int k0 = gd.kreg[0], k1 = two ? gd.kreg[1] : -1;
        int cb = 0;  // the index bits that are constant over the thread's elements
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (j >= gd.n || gd.kreg[j] >= 0) continue;
          const int cs = gd.csrc[j];
          cb |= (cs >= 64 ? (int)((base >> (cs - 64)) & 1) : ((ob >> cs) & 1)) << j;
        }
        if (gd.form == kFormSigns) {  // entries +-1: sign flips, no multiplies
          const int sm = (d0.x < 0.f) | ((d1.x < 0.f) << 1) | ((d2.x < 0.f) << 2) | ((d3.x < 0.f) << 3);
          if (k0 < 0 && k1 < 0) {
            ph_used = true;
            if ((sm >> cb) & 1) ph = f2(-ph.x, -ph.y);
          } else {
            apply_signs(x, gd.n, k0, k1, cb, sm);
          }
        } else if (k0 < 0 && k1 < 0) {
          const float2 f = cb == 0 ? d0 : cb == 1 ? d1 : cb == 2 ? d2 : d3;
          ph = cmul<TN_PREC_C64>(ph, f);
          ph_used = true;
        } else if (gd.form == kFormUnit) {
          apply_diag_unit<PREC, 1>(x, x, ph, gd.n, k0, k1, cb, d0, d1, d2, d3);
          ph_used = true;
        } else {
          apply_diag<PREC>(x, gd.n, k0, k1, cb, d0, d1, d2, d3);
        }
      } else if (gd.n == 1) {
        const int form = gd.form == kFormReal ? kDenseReal : gd.form == kFormRxLike ? kDenseRxLike : kDenseGeneric;
        if (gd.run_mask) {  // this gate and the next ones: one per bit of the mask, one form
          const int cnt = __builtin_popcount(gd.run_mask);
          const float2* gp[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int vo = j < cnt ? gates[gi + j].voff : gd.voff;
            gp[j] = VL ? vtab + (vo - a.lds_off) : V0 + vo;
          }
          apply_dense1_run<PREC, 1>(x, x, gp, gd.run_mask, form);
          gi += cnt - 1;
          continue;
        }
        const float2 g[4] = {V[0], V[1], V[2], V[3]};
        apply_dense1<PREC, 1>(x, x, g, gd.rb[0], form);
      } else {
        float2 g[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) g[e] = V[e];
        switch (gd.rb[0] * 4 + gd.rb[1]) {
          case 1: reg_apply2<PREC, 0, 1>(x, g); break;
          case 2: reg_apply2<PREC, 0, 2>(x, g); break;
          case 3: reg_apply2<PREC, 0, 3>(x, g); break;
          case 6: reg_apply2<PREC, 1, 2>(x, g); break;
          case 7: reg_apply2<PREC, 1, 3>(x, g); break;
          default: reg_apply2<PREC, 2, 3>(x, g); break;
        }
      }
    }
    if (ph_used) {
#pragma unroll
      for (int r = 0; r < 16; ++r) buf[pob + seg.physoff[r]] = cmul<TN_PREC_C64>(ph, x[r]);
    } else {  // no gate of the segment touched the factor (it is 1)
#pragma unroll
      for (int r = 0; r < 16; ++r) buf[pob + seg.physoff[r]] = x[r];
    }
    __syncthreads();
  }
  chunk_from_lds(out, buf, base, dep_hi, tid, nt);
}

// The gate values of a chain's passes in one table (see SweepChain).
__global__ void k_gather_vals(const int64_t* src, int n, const float2* IN, int64_t in_bs, const float2* WS,
                              int64_t ws_bs, float2* out, int64_t out_bs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (i >= n) return;
  const int64_t v = src[i];
  const int64_t off = v & (((int64_t)1 << kValExpShift) - 1);
  const float2* b = ((v >> 56) & 0x3f) == BUF_IN ? IN + (int64_t)z * in_bs : WS + (int64_t)z * ws_bs;
  float2 r = b[off];
  if (v & kValPow) {  // w^e by repeated multiplication in FP64, rounded once
    const int e = (int)((v >> kValExpShift) & 0xff);
    double pr = 1.0, pi = 0.0;
    for (int k = 0; k < e; ++k) {
      const double t = pr * r.x - pi * r.y;
      pi = pr * r.y + pi * r.x;
      pr = t;
    }
    r = f2((float)pr, (float)pi);
  }
  out[(int64_t)z * out_bs + i] = r;
}

hipError_t launch_gather_vals(hipStream_t s, const int64_t* src, int n, const float2* IN, int64_t in_bs,
                              const float2* WS, int64_t ws_bs, float2* out, int64_t out_bs, int batch) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((n + kThreads - 1) / kThreads), batch), dim3(kThreads), 0, s,
                     src, n, IN, in_bs, WS, ws_bs, out, out_bs);
  return hipGetLastError();
}

hipError_t launch_sweep_pass(hipStream_t s, const SweepPass& ps, int bits, const SweepGateDesc* gates_dev,
                             const SweepSegment* segs_dev, const float2* in, int64_t in_bs, float2* out,
                             int64_t out_bs, const float2* vals, int64_t vals_bs, int batch, int precision) {
  SweepPassArgs a;
  a.in = in; a.out = out; a.in_bs = in_bs; a.out_bs = out_bs;
  a.vals = vals; a.vals_bs = vals_bs;
  a.gates = gates_dev;
  a.segs = segs_dev + ps.first_seg;
  a.n_segs = ps.n_segs;
  a.l = ps.l;
  a.pad = 0;
  a.ctab_off = ps.ctab_off;
  const int n_all = ps.ctab_off + ps.ctab_n - ps.val_off;  // the pass's values and tables
  a.gates_in_lds = n_all <= kPassValMax ? 1 : 0;
  a.lds_off = a.gates_in_lds ? ps.val_off : ps.ctab_off;
  a.lds_n = a.gates_in_lds ? n_all : ps.ctab_n;
  a.pad2 = 0;
  if (ps.l < kSweepMinLocal || ps.l > kSweepMaxLocal) return hipErrorInvalidValue;
  if (ps.ctab_n < 0 || ps.ctab_n > kCountTabMax || n_all < 0 || (a.lds_n > 0 && !vals)) return hipErrorInvalidValue;
  static_assert(kCountTabMax <= kPassValMax, "the power tables alone always fit");
  std::vector<char> local(bits, 0);
  for (int j = 0; j < ps.l; ++j) {
    a.lpos[j] = ps.lpos[j];
    if (ps.lpos[j] < 0 || ps.lpos[j] >= bits || (j < 5 && ps.lpos[j] != j)) return hipErrorInvalidValue;
    local[ps.lpos[j]] = 1;
  }
  int nr = 0;
  for (int p = 0; p < bits; ++p)
    if (!local[p]) a.rest[nr++] = (int8_t)p;
  a.n_rest = nr;
  const int64_t chunks = (int64_t)1 << nr;
  if (chunks > ((int64_t)1 << 24)) return hipErrorInvalidValue;
  const int threads = 1 << (ps.l - 4);
  const dim3 grid((unsigned)chunks, batch);
  if (precision == TN_PREC_BF16X3) {
    if (a.gates_in_lds)
      hipLaunchKernelGGL((k_sweep_pass<TN_PREC_BF16X3, true>), grid, dim3(threads), 0, s, a, a.gates, a.segs, a.vals);
    else
      hipLaunchKernelGGL((k_sweep_pass<TN_PREC_BF16X3, false>), grid, dim3(threads), 0, s, a, a.gates, a.segs, a.vals);
  } else {
    if (a.gates_in_lds)
      hipLaunchKernelGGL((k_sweep_pass<TN_PREC_C64, true>), grid, dim3(threads), 0, s, a, a.gates, a.segs, a.vals);
    else
      hipLaunchKernelGGL((k_sweep_pass<TN_PREC_C64, false>), grid, dim3(threads), 0, s, a, a.gates, a.segs, a.vals);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Index slicing: the input tensors of one slice gathered from the full ones,
// and the slices' results summed.
// ---------------------------------------------------------------------------
__global__ void k_slice_gather(const SliceTensor* ts, int nt, const float2* full, int64_t full_bs, float2* sl,
                               int64_t sl_bs, int64_t slice) {
  const int t = blockIdx.x, z = blockIdx.y;
  if (t >= nt) return;
  const SliceTensor st = ts[t];
  int64_t cut = 0;  // the fixed bits of this slice, at their places in the full tensor
  for (int k = 0; k < st.n_cut; ++k) cut |= ((slice >> st.cut_src[k]) & 1) << st.cut_pos[k];
  const float2* src = full + (int64_t)z * full_bs + st.src_off;
  float2* dst = sl + (int64_t)z * sl_bs + st.dst_off;
  const int64_t n = (int64_t)1 << st.n_keep;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    int64_t a = cut;
    for (int j = 0; j < st.n_keep; ++j) a |= ((i >> j) & 1) << st.keep_pos[j];
    dst[i] = src[a];
  }
}

hipError_t launch_slice_gather(hipStream_t s, const SliceTensor* ts, int nt, const float2* full, int64_t full_bs,
                               float2* sl, int64_t sl_bs, int64_t slice, int batch) {
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_gather, dim3(nt, batch), dim3(64), 0, s, ts, nt, full, full_bs, sl, sl_bs, slice);
  return hipGetLastError();
}

// acc = src (first) or acc += src
__global__ void k_accumulate(const float2* src, int64_t src_bs, float2* acc, int64_t acc_bs, int64_t n, int first) {
  const int z = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const float2 v = src[(int64_t)z * src_bs + i];
    float2& a = acc[(int64_t)z * acc_bs + i];
    a = first ? v : f2(a.x + v.x, a.y + v.y);
  }
}

hipError_t launch_accumulate(hipStream_t s, const float2* src, int64_t src_bs, float2* acc, int64_t acc_bs, int64_t n,
                             int first, int batch) {
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_accumulate, dim3((unsigned)std::max<int64_t>(blocks, 1), batch), dim3(kThreads), 0, s, src,
                     src_bs, acc, acc_bs, n, first);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bit-permutation transpose through LDS
// ---------------------------------------------------------------------------
constexpr int kMaxTileBits = 10;

// (every map starts at a multiple of 4 bytes: deposit() reads them as 32-bit words)
struct PermArgs {
  const float2* in;
  float2* out;
  int64_t in_bs, out_bs;
  int64_t n_blocks;
  int32_t tile_bits, rest_bits;
  int8_t rest_in[64];
  int8_t rest_out[64];
  int8_t tin[kMaxTileBits + 2];   // input position of tile-index bit j (load order)
  int8_t tsrc[kMaxTileBits + 2];  // store order: bit j of the store index = load-index bit tsrc[j]
  int8_t tout[kMaxTileBits + 2];  // output position of store-index bit j
};
static_assert(offsetof(PermArgs, rest_in) % 4 == 0 && offsetof(PermArgs, tin) % 4 == 0 &&
                  offsetof(PermArgs, tsrc) % 4 == 0 && offsetof(PermArgs, tout) % 4 == 0,
              "position maps aligned to 32-bit words");

__global__ __launch_bounds__(kThreads) void k_permute(PermArgs a) {
  __shared__ float2 buf[(1 << kMaxTileBits) + (1 << (kMaxTileBits - 5))];
  const int z = blockIdx.y;
  const float2* in = a.in + (int64_t)z * a.in_bs;
  float2* out = a.out + (int64_t)z * a.out_bs;
  const int tile = 1 << a.tile_bits;
  constexpr int kPer = (1 << kMaxTileBits) / kThreads;
  int64_t in_off[kPer], out_off[kPer];
  int lds_src[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int l = threadIdx.x + e * kThreads;
    in_off[e] = deposit(l, a.tin, a.tile_bits);
    out_off[e] = deposit(l, a.tout, a.tile_bits);
    const int src = (int)deposit(l, a.tsrc, a.tile_bits);
    lds_src[e] = src + (src >> 5);
  }
  for (int64_t blk = blockIdx.x; blk < a.n_blocks; blk += gridDim.x) {
    const int64_t ib = deposit(blk, a.rest_in, a.rest_bits), ob = deposit(blk, a.rest_out, a.rest_bits);
    for (int e = 0; e < kPer; ++e) {
      const int l = threadIdx.x + e * kThreads;
      if (l < tile) buf[l + (l >> 5)] = in[ib | in_off[e]];
    }
    __syncthreads();
    for (int e = 0; e < kPer; ++e) {
      const int l = threadIdx.x + e * kThreads;
      if (l < tile) out[ob | out_off[e]] = buf[lds_src[e]];
    }
    __syncthreads();
  }
}

hipError_t launch_permute(hipStream_t s, const PermuteDesc& d, const float2* in, int64_t in_bs, float2* out,
                          int64_t out_bs, int batch) {
  const int R = d.bits;
  // tile: the low input bits plus the input bits that land on the low output bits,
  // grown while it fits in kMaxTileBits
  std::vector<int> best;
  for (int a = 1; a <= R; ++a) {
    std::vector<char> in_tile(R, 0);
    for (int p = 0; p < a; ++p) in_tile[p] = 1;
    for (int p = 0; p < R; ++p)
      if (d.dst[p] < a) in_tile[p] = 1;
    std::vector<int> t;
    for (int p = 0; p < R; ++p)
      if (in_tile[p]) t.push_back(p);
    if ((int)t.size() > kMaxTileBits) break;
    best = t;
  }
  PermArgs a;
  a.in = in; a.out = out; a.in_bs = in_bs; a.out_bs = out_bs;
  a.tile_bits = (int)best.size();
  for (int j = 0; j < a.tile_bits; ++j) a.tin[j] = (int8_t)best[j];
  // store order: tile bits by ascending output position
  std::vector<int> order(a.tile_bits);
  for (int j = 0; j < a.tile_bits; ++j) order[j] = j;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return d.dst[best[x]] < d.dst[best[y]]; });
  for (int j = 0; j < a.tile_bits; ++j) {
    a.tsrc[j] = (int8_t)order[j];
    a.tout[j] = (int8_t)d.dst[best[order[j]]];
  }
  int nr = 0;
  for (int p = 0; p < R; ++p) {
    if (std::find(best.begin(), best.end(), p) != best.end()) continue;
    a.rest_in[nr] = (int8_t)p;
    a.rest_out[nr] = (int8_t)d.dst[p];
    ++nr;
  }
  a.rest_bits = nr;
  a.n_blocks = (int64_t)1 << nr;
  int64_t blocks = a.n_blocks;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)blocks, batch), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Complex GEMM on the FP32 matrix cores
//
// With complex64 stored as interleaved (re, im), A (M x K complex) is read as
// the real M x 2K matrix A_r, and B (K x N complex) is expanded on the fly
// into the real 2K x 2N matrix B' whose 2x2 block (k, n) is
// [[Re b, Im b], [-Im b, Re b]].  Then A_r B' is the interleaved real view of
// A B (4M form: 4 real multiply-adds per complex one).  One
// v_mfma_f32_32x32x2f32 consumes exactly one complex k: lanes 0-31 carry
// Re A / the first row of the block of B', lanes 32-63 Im A / the second row,
// and produces a 32 x 16 complex tile.
// ---------------------------------------------------------------------------
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kBK = kGemmBK;          // complex k per staged K tile
constexpr int kB3Row = 2 * kBK + 8;   // bf16 per LDS row of a split-precision K tile (16-byte pad)

// Operands and result are read and written through bit-deposit maps: the
// address of logical index x of an operand is the OR of x's bits moved to
// their positions in that operand's layout.  A tile's base address is the
// deposit of its (multiple-of-tile) origin; the offsets inside a tile come
// from small LDS tables, so no separate permute pass is needed.
struct GemmArgs {
  const float2* A;
  const float2* B;
  float2* C;
  int64_t a_bs, b_bs, c_bs;
  int64_t batch, M, N, K;
  int64_t tiles_m, tiles_n;
  int64_t band_n;   // tile columns per band of the tile order (divides tiles_n)
  int64_t c_elems;  // elements of C per parameter vector (split-K partial stride)
  int32_t nbb, nbm, nbn, nbk, split, xcd;
  int8_t a_b[kGemmMaxBits], a_m[kGemmMaxBits], a_k[kGemmMaxBits];
  int8_t b_b[kGemmMaxBits], b_k[kGemmMaxBits], b_n[kGemmMaxBits];
  int8_t c_b[kGemmMaxBits], c_m[kGemmMaxBits], c_n[kGemmMaxBits];
};

// Tile order of the matrix-product kernels.  The GPU hands consecutive
// workgroup ids to its eight XCDs in turn, and each XCD has its own L2.  With
// xcd set (the grid is a multiple of 8), workgroup h takes logical id
// (h mod 8) * (grid / 8) + h / 8, so each XCD runs one contiguous range of
// logical ids, in order.  Logical ids walk the tile grid in bands of band_n
// tile columns, n fastest inside a band: an XCD's range then covers a block of
// rows of one band, whose B column tiles stay in its L2 while the rows pass
// and whose A row tiles are used band_n times in a row.
struct TileCoord {
  int64_t tm, tn, rest;  // rest: the split, batch and parameter-vector index
};

__device__ inline TileCoord tile_coord(const GemmArgs& g) {
  int64_t bid = blockIdx.x;
  if (g.xcd) {
    const int64_t per = (int64_t)gridDim.x >> 3;
    bid = (bid & 7) * per + (bid >> 3);
  }
  const int64_t tmn = g.tiles_m * g.tiles_n;
  const int64_t r = bid % tmn, band_tiles = g.tiles_m * g.band_n;
  const int64_t band = r / band_tiles, q = r - band * band_tiles;
  return {q / g.band_n, band * g.band_n + q % g.band_n, bid / tmn};
}

// BF16x3 split precision: x_hi = bf16(x), x_lo = bf16(x - x_hi), both round
// to nearest even; the product keeps a_hi b_hi + a_hi b_lo + a_lo b_hi.
__device__ inline void split_bf16(float2 v, uint32_t* hi, uint32_t* lo) {
  const __bf16 h0 = (__bf16)v.x, h1 = (__bf16)v.y;
  const __bf16 l0 = (__bf16)(v.x - (float)h0), l1 = (__bf16)(v.y - (float)h1);
  const bf16x2 H = {h0, h1}, L = {l0, l1};
  *hi = __builtin_bit_cast(uint32_t, H);
  *lo = __builtin_bit_cast(uint32_t, L);
}

// (re, im) bf16 pairs of B -> the B' column entries of real column parity d:
// (re, -im) for even real columns, (im, re) for odd ones
__device__ inline bf16x8 b_embed(uint4 w, int d) {
  uint4 r;
  r.x = d ? ((w.x >> 16) | (w.x << 16)) : (w.x ^ 0x80000000u);
  r.y = d ? ((w.y >> 16) | (w.y << 16)) : (w.y ^ 0x80000000u);
  r.z = d ? ((w.z >> 16) | (w.z << 16)) : (w.z ^ 0x80000000u);
  r.w = d ? ((w.w >> 16) | (w.w << 16)) : (w.w ^ 0x80000000u);
  return __builtin_bit_cast(bf16x8, r);
}

// Complex GEMM on the matrix cores.
//
// With complex64 stored as interleaved (re, im), A (M x K complex) is read as
// the real M x 2K matrix A_r, and B (K x N complex) is expanded on the fly
// into the real 2K x 2N matrix B' whose 2x2 block (k, n) is
// [[Re b, Im b], [-Im b, Re b]].  Then A_r B' is the interleaved real view of
// A B (4M form: 4 real multiply-adds per complex one).
//
// Four waves in a 2 x 2 arrangement; each wave owns TM x TN result tiles of
// 32 x 16 complex, so a block computes (64 TM) x (32 TN).  Form F = 0: FP32,
// one v_mfma_f32_32x32x2f32 per complex k (lanes 0-31 carry Re A / the first
// row of B's 2x2 block, lanes 32-63 Im A / the second row).  Form F = 1:
// BF16x3 on the bf16 matrix cores, v_mfma_f32_32x32x16_bf16 covering 8
// complex k: lane l holds the eight consecutive k' = 8*(l/32) .. +7 of row
// (A) or column (B) l%32, i.e. four complex values of one A row as stored,
// or four complex values of one B column turned into B' entries (b_embed).
// Operands are split into hi/lo once, while a tile is staged into LDS.
template <int AK, int BNF, int TM, int TN, int F>
__global__ __launch_bounds__(kThreads) void k_gemm(GemmArgs g) {
  constexpr int BM = 64 * TM, BN = 32 * TN;
  constexpr int kPA = (BM * kBK) / kThreads, kPB = (BN * kBK) / kThreads;
  constexpr int kF32Bytes = 2 * kBK * (BM + 1) * 4 + kBK * (BN + 1) * 8;
  constexpr int kB3Bytes = 2 * BM * kB3Row * 2 + 2 * BN * kB3Row * 2;
  constexpr int kSmem = F == 0 ? kF32Bytes : kB3Bytes;
  __shared__ __attribute__((aligned(16))) char smem[kSmem];
  __shared__ int64_t TAm[BM], TCm[BM], TBn[BN], TCn[BN], TAk[kBK], TBk[kBK];
  constexpr int kKt = 64;  // K tiles whose origin deposits are tabulated (the rest computed on the fly)
  __shared__ int64_t TAt[kKt], TBt[kKt];
  float (*As_re)[BM + 1] = reinterpret_cast<float (*)[BM + 1]>(smem);
  float (*As_im)[BM + 1] = reinterpret_cast<float (*)[BM + 1]>(smem + kBK * (BM + 1) * 4);
  float2 (*Bs)[BN + 1] = reinterpret_cast<float2 (*)[BN + 1]>(smem + 2 * kBK * (BM + 1) * 4);
  __bf16 (*Ah)[kB3Row] = reinterpret_cast<__bf16 (*)[kB3Row]>(smem);
  __bf16 (*Al)[kB3Row] = reinterpret_cast<__bf16 (*)[kB3Row]>(smem + BM * kB3Row * 2);
  __bf16 (*Bh)[kB3Row] = reinterpret_cast<__bf16 (*)[kB3Row]>(smem + 2 * BM * kB3Row * 2);
  __bf16 (*Bl)[kB3Row] = reinterpret_cast<__bf16 (*)[kB3Row]>(smem + 2 * BM * kB3Row * 2 + BN * kB3Row * 2);

  const TileCoord tc = tile_coord(g);
  const int64_t tn = tc.tn, tm = tc.tm;
  int64_t bid = tc.rest;
  const int64_t ks = bid % g.split;
  bid /= g.split;
  const int64_t gb = bid % g.batch;
  const int64_t z = bid / g.batch;
  const float2* A = g.A + z * g.a_bs;
  const float2* B = g.B + z * g.b_bs;
  float2* C = g.C + z * g.c_bs + ks * g.c_elems;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t kchunk = g.K / g.split;
  const int64_t kbeg = ks * kchunk, kend = kbeg + kchunk;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int64_t base_a = deposit(gb, g.a_b, g.nbb) | deposit(m0, g.a_m, g.nbm);
  const int64_t base_b = deposit(gb, g.b_b, g.nbb) | deposit(n0, g.b_n, g.nbn);
  const int64_t base_c = deposit(gb, g.c_b, g.nbb) | deposit(m0, g.c_m, g.nbm) | deposit(n0, g.c_n, g.nbn);
  constexpr int kLogBM = 6 + (TM == 2), kLogBN = 5 + (TN == 2);
  if (tid < BM) {
    const int nb = min(g.nbm, kLogBM);
    TAm[tid] = deposit(tid, g.a_m, nb);
    TCm[tid] = deposit(tid, g.c_m, nb);
  }
  if (tid < BN) {
    const int nb = min(g.nbn, kLogBN);
    TBn[tid] = deposit(tid, g.b_n, nb);
    TCn[tid] = deposit(tid, g.c_n, nb);
  }
  if (tid < kBK) {
    const int nb = min(g.nbk, 4);
    TAk[tid] = deposit(tid, g.a_k, nb);
    TBk[tid] = deposit(tid, g.b_k, nb);
  }
  if (tid < kKt && kbeg + (int64_t)tid * kBK < kend) {
    TAt[tid] = deposit(kbeg + (int64_t)tid * kBK, g.a_k, g.nbk);
    TBt[tid] = deposit(kbeg + (int64_t)tid * kBK, g.b_k, g.nbk);
  }
  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
  __syncthreads();

  // tile element e of this thread: (row or column, k) inside the tile
  auto a_elem = [&](int e, int& mm, int& kk) {
    const int idx = tid + e * kThreads;
    if (AK) { mm = idx / kBK; kk = idx % kBK; } else { mm = idx % BM; kk = idx / BM; }
  };
  auto b_elem = [&](int e, int& nn, int& kk) {
    const int idx = tid + e * kThreads;
    if (BNF) { nn = idx % BN; kk = idx / BN; } else { nn = idx / kBK; kk = idx % kBK; }
  };
  // software pipeline: the next K tile is fetched into registers while the
  // current one is multiplied out of LDS
  // per-thread element addresses without the K tile's origin, fixed for the block
  const float2* pa[kPA];
  const float2* pb[kPB];
  bool va[kPA], vb[kPB];
  int ka_e[kPA], kb_e[kPB];
#pragma unroll
  for (int e = 0; e < kPA; ++e) {
    int mm, kk;
    a_elem(e, mm, kk);
    pa[e] = A + (base_a | TAm[mm] | TAk[kk]);
    va[e] = m0 + mm < g.M;
    ka_e[e] = kk;
  }
#pragma unroll
  for (int e = 0; e < kPB; ++e) {
    int nn, kk;
    b_elem(e, nn, kk);
    pb[e] = B + (base_b | TBn[nn] | TBk[kk]);
    vb[e] = n0 + nn < g.N;
    kb_e[e] = kk;
  }
  const bool interior = m0 + BM <= g.M && n0 + BN <= g.N;
  float2 ra[kPA], rb[kPB];
  auto fetch = [&](int64_t k0) {
    const int64_t t = (k0 - kbeg) / kBK;
    const int64_t ka = t < kKt ? TAt[t] : deposit(k0, g.a_k, g.nbk);
    const int64_t kb = t < kKt ? TBt[t] : deposit(k0, g.b_k, g.nbk);
    const int64_t rem = kend - k0;
    const int kleft = rem < kBK ? (int)rem : kBK;  // valid k of this tile
    if (interior && kleft == kBK) {  // whole tile inside the operands: no guards
#pragma unroll
      for (int e = 0; e < kPA; ++e) ra[e] = pa[e][ka];
#pragma unroll
      for (int e = 0; e < kPB; ++e) rb[e] = pb[e][kb];
    } else {
#pragma unroll
      for (int e = 0; e < kPA; ++e) ra[e] = (va[e] && ka_e[e] < kleft) ? pa[e][ka] : f2(0.f, 0.f);
#pragma unroll
      for (int e = 0; e < kPB; ++e) rb[e] = (vb[e] && kb_e[e] < kleft) ? pb[e][kb] : f2(0.f, 0.f);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int e = 0; e < kPA; ++e) {
      int mm, kk;
      a_elem(e, mm, kk);
      if constexpr (F == 0) {
        As_re[kk][mm] = ra[e].x;
        As_im[kk][mm] = ra[e].y;
      } else {
        uint32_t h, l;
        split_bf16(ra[e], &h, &l);
        *reinterpret_cast<uint32_t*>(&Ah[mm][2 * kk]) = h;
        *reinterpret_cast<uint32_t*>(&Al[mm][2 * kk]) = l;
      }
    }
#pragma unroll
    for (int e = 0; e < kPB; ++e) {
      int nn, kk;
      b_elem(e, nn, kk);
      if constexpr (F == 0) {
        Bs[kk][nn] = rb[e];
      } else {
        uint32_t h, l;
        split_bf16(rb[e], &h, &l);
        *reinterpret_cast<uint32_t*>(&Bh[nn][2 * kk]) = h;
        *reinterpret_cast<uint32_t*>(&Bl[nn][2 * kk]) = l;
      }
    }
  };
  fetch(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
    stage();
    __syncthreads();
    if (k0 + kBK < kend) fetch(k0 + kBK);
    if constexpr (F == 0) {
#pragma unroll 4
      for (int kk = 0; kk < kBK; ++kk) {
        float av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const int row = wm * 32 * TM + i * 32 + (lane & 31);
          av[i] = lane < 32 ? As_re[kk][row] : As_im[kk][row];
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const float2 bb = Bs[kk][wn * 16 * TN + j * 16 + ((lane & 31) >> 1)];
          const bool odd = lane & 1;
          bv[j] = lane < 32 ? (odd ? bb.y : bb.x) : (odd ? bb.x : -bb.y);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    } else {
      const int half = lane >> 5, d = lane & 1;
#pragma unroll
      for (int kq = 0; kq < kBK / 8; ++kq) {
        const int col = kq * 16 + half * 8;  // first bf16 of this lane's eight
        bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const int row = wm * 32 * TM + i * 32 + (lane & 31);
          ah[i] = *reinterpret_cast<const bf16x8*>(&Ah[row][col]);
          al[i] = *reinterpret_cast<const bf16x8*>(&Al[row][col]);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int nn = wn * 16 * TN + j * 16 + ((lane & 31) >> 1);
          bh[j] = b_embed(*reinterpret_cast<const uint4*>(&Bh[nn][col]), d);
          bl[j] = b_embed(*reinterpret_cast<const uint4*>(&Bl[nn][col]), d);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* Cf = reinterpret_cast<float*>(C);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = wm * 32 * TM + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int jj = lane & 31;
        const int cl = wn * 16 * TN + j * 16 + (jj >> 1);
        if (m0 + rl < g.M && n0 + cl < g.N)
          __builtin_nontemporal_store(acc[i][j][v], &Cf[(base_c | TCm[rl] | TCn[cl]) * 2 + (jj & 1)]);
      }
}

// 3M form on the FP32 matrix cores: with A = Ar + i Ai and B = Br + i Bi,
//   Re C = Ar Br - Ai Bi,   Im C = (Ar + Ai)(Br + Bi) - Ar Br - Ai Bi,
// three real products instead of the four of the real embedding.  Operands
// are staged as interleaved complex and split into real and imaginary parts
// as a lane reads them; one v_mfma_f32_32x32x2f32 takes
// two complex k (lanes 0-31 the first, 32-63 the second) and a 32 x 32
// complex tile keeps three accumulators (P1 = Ar Br, P2 = Ai Bi,
// P3 = (Ar + Ai)(Br + Bi)).  Four waves in a 2 x 2 arrangement, each owning
// TM tiles of 32 x 32 complex: the block computes (64 TM) x 64.
template <int AK, int BNF, int TM, int BK, int NW, int BP>
__global__ __launch_bounds__(kThreads, TM == 1 && !BP ? 4 : 2) void k_gemm3m(GemmArgs g) {
  // BP = 1 (batch-packed): four batch items of at most 32 x 32 per block, wave
  // w computing item w; operand "rows" are (item, m) for A and (item, n) for
  // B.  BP = 2 (column-packed): M <= 32 and four 32-column slices of N per
  // block, wave w computing slice w; A's rows repeat per slice, B's rows are
  // n - n0.
  static_assert(!BP || TM == 1, "packed blocks hold one 32 x 32 tile per wave");
  constexpr int BM = BP ? 128 : 64 * TM, BN = BP ? 128 : 64;
  constexpr int kPA = (BM * BK) / kThreads, kPB = (BN * BK) / kThreads;
  constexpr int kLogBK = BK == 32 ? 5 : 4;
  // operands staged as interleaved complex with k contiguous per row of A and
  // per column of B, rows kRow = 2 BK + 4 words apart: a lane reads four
  // consecutive complex k of its row as two 16-byte loads, and 16 consecutive
  // rows start on distinct multiples of 4 banks (36 r mod 64)
  static_assert(BK % 8 == 0, "whole 16-byte operand reads");
  constexpr int kRow = 2 * BK + 4;
  __shared__ __attribute__((aligned(16))) float As[BM * kRow], Bs[BN * kRow];
  __shared__ int64_t TAm[BM], TCm[BM], TBn[BN], TCn[BN], TAk[BK], TBk[BK];
  constexpr int kKt = 64;  // K tiles whose origin deposits are tabulated (the rest computed on the fly)
  __shared__ int64_t TAt[kKt], TBt[kKt];
  const TileCoord tc = tile_coord(g);
  const int64_t tn = tc.tn, tm = tc.tm;
  int64_t bid = tc.rest;
  const int64_t ks = bid % g.split;
  bid /= g.split;
  const int64_t n_bgroups = BP == 1 ? g.batch / 4 : g.batch;
  const int64_t gb = (bid % n_bgroups) * (BP == 1 ? 4 : 1);
  const int64_t z = bid / n_bgroups;
  const float2* A = g.A + z * g.a_bs;
  const float2* B = g.B + z * g.b_bs;
  float2* C = g.C + z * g.c_bs + ks * g.c_elems;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t kchunk = g.K / g.split;
  const int64_t kbeg = ks * kchunk, kend = kbeg + kchunk;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int64_t base_a = deposit(gb, g.a_b, g.nbb) | deposit(m0, g.a_m, g.nbm);
  const int64_t base_b = deposit(gb, g.b_b, g.nbb) | deposit(n0, g.b_n, g.nbn);
  const int64_t base_c = deposit(gb, g.c_b, g.nbb) | deposit(m0, g.c_m, g.nbm) | deposit(n0, g.c_n, g.nbn);
  constexpr int kLogBM = 6 + (TM == 2);
  if constexpr (BP == 1) {
    if (tid < 128) {  // row tid: item tid >> 5 (the two lowest batch bits), m or n tid & 31
      const int it = tid >> 5, r = tid & 31, nbi = min(g.nbb, 2);
      TAm[tid] = deposit(r, g.a_m, min(g.nbm, 5)) | deposit(it, g.a_b, nbi);
      TCm[tid] = deposit(r, g.c_m, min(g.nbm, 5)) | deposit(it, g.c_b, nbi);
      TBn[tid] = deposit(r, g.b_n, min(g.nbn, 5)) | deposit(it, g.b_b, nbi);
      TCn[tid] = deposit(r, g.c_n, min(g.nbn, 5));
    }
  } else if constexpr (BP == 2) {
    if (tid < 128) {  // row tid of A: slice tid >> 5, m tid & 31; row tid of B: n - n0 = tid
      const int r = tid & 31;
      TAm[tid] = deposit(r, g.a_m, min(g.nbm, 5));
      TCm[tid] = deposit(r, g.c_m, min(g.nbm, 5)) | deposit(tid & ~31, g.c_n, min(g.nbn, 7));
      TBn[tid] = deposit(tid, g.b_n, min(g.nbn, 7));
      TCn[tid] = deposit(r, g.c_n, min(g.nbn, 5));
    }
  } else {
    if (tid < BM) {
      const int nb = min(g.nbm, kLogBM);
      TAm[tid] = deposit(tid, g.a_m, nb);
      TCm[tid] = deposit(tid, g.c_m, nb);
    }
    if (tid < BN) {
      const int nb = min(g.nbn, 6);
      TBn[tid] = deposit(tid, g.b_n, nb);
      TCn[tid] = deposit(tid, g.c_n, nb);
    }
  }
  if (tid < BK) {
    const int nb = min(g.nbk, kLogBK);
    TAk[tid] = deposit(tid, g.a_k, nb);
    TBk[tid] = deposit(tid, g.b_k, nb);
  }
  if (tid < kKt && kbeg + (int64_t)tid * BK < kend) {
    TAt[tid] = deposit(kbeg + (int64_t)tid * BK, g.a_k, g.nbk);
    TBt[tid] = deposit(kbeg + (int64_t)tid * BK, g.b_k, g.nbk);
  }
  floatx16 p1[TM], p2[TM], p3[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) p1[i][v] = p2[i][v] = p3[i][v] = 0.f;
  __syncthreads();

  // Staging order (16-wide K tiles, four waves), element e of a thread at row
  // rt + row_e(e), complex k kt + k_e(e) of its operand tile:
  //  - k fastest in the operand: a quarter-wave loads 16 consecutive k of one
  //    row (a 128-byte run) and writes them as 8-byte words; the two rows of
  //    a half-wave are 8 apart (36 * 8 = 32 mod 64 banks), so its 64 words
  //    fall on distinct banks;
  //  - m or n fastest: a wave loads 64 consecutive rows at one k per load and
  //    each thread writes its four consecutive k of a row as two 16-byte
  //    words (16 consecutive rows per LDS cycle, distinct banks).
  static_assert(BK == 16 && kThreads == 256 && (BN == 64 || BN == 128), "staging order assumes 16-wide K tiles");
  auto slot_t = [&](bool k_fast, int& r, int& kk) {
    if (k_fast) {
      r = w + 4 * ((lane >> 5) & 1) + 8 * ((lane >> 4) & 1);
      kk = lane & 15;
    } else {
      r = lane;
      kk = 4 * w;
    }
  };
  auto row_e = [](bool k_fast, int e) { return k_fast ? 16 * e : 64 * (e >> 2); };
  auto k_e = [](bool k_fast, int e) { return k_fast ? 0 : (e & 3); };
  constexpr bool kfa = AK != 0, kfb = BNF == 0;
  int a_rt, a_kt, b_rt, b_kt;
  slot_t(kfa, a_rt, a_kt);
  slot_t(kfb, b_rt, b_kt);
  // element offsets within a K tile, without the tile's origin: 32-bit byte
  // offsets from a block-uniform base when every offset of the tile stays
  // below 2^32 bytes (NW), else full pointers
  const float2* pa[NW ? 1 : kPA];
  const float2* pb[NW ? 1 : kPB];
  uint32_t oa[NW ? kPA : 1], ob[NW ? kPB : 1];
#pragma unroll
  for (int e = 0; e < kPA; ++e) {
    const int64_t off = TAm[a_rt + row_e(kfa, e)] | TAk[a_kt + k_e(kfa, e)];
    if constexpr (NW) oa[e] = (uint32_t)off * (uint32_t)sizeof(float2);
    else pa[e] = A + (base_a | off);
  }
#pragma unroll
  for (int e = 0; e < kPB; ++e) {
    const int64_t off = TBn[b_rt + row_e(kfb, e)] | TBk[b_kt + k_e(kfb, e)];
    if constexpr (NW) ob[e] = (uint32_t)off * (uint32_t)sizeof(float2);
    else pb[e] = B + (base_b | off);
  }
  const bool interior = BP == 1   ? g.M == 32 && g.N == 32
                        : BP == 2 ? g.M == 32 && n0 + BN <= g.N
                                  : m0 + BM <= g.M && n0 + BN <= g.N;
  // whether tile row r of A (of B) lies inside the operand
  auto a_in = [&](int r) { return BP ? (r & 31) < g.M : m0 + r < g.M; };
  auto b_in = [&](int r) { return BP == 1 ? (r & 31) < g.N : n0 + r < g.N; };
  float2 ra[kPA], rb[kPB];
  auto fetch = [&](int64_t k0) {
    const int64_t t = (k0 - kbeg) / BK;
    int64_t ka = t < kKt ? TAt[t] : deposit(k0, g.a_k, g.nbk);
    int64_t kb = t < kKt ? TBt[t] : deposit(k0, g.b_k, g.nbk);
    // the same value in every lane: keep it in scalar registers
    ka = ((int64_t)__builtin_amdgcn_readfirstlane((int)(ka >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)ka);
    kb = ((int64_t)__builtin_amdgcn_readfirstlane((int)(kb >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)kb);
    const char* a_org = reinterpret_cast<const char*>(A + (base_a | ka));
    const char* b_org = reinterpret_cast<const char*>(B + (base_b | kb));
    auto lda = [&](int e) -> float2 {
      if constexpr (NW) return *reinterpret_cast<const float2*>(a_org + oa[e]);
      else return pa[e][ka];
    };
    auto ldb = [&](int e) -> float2 {
      if constexpr (NW) return *reinterpret_cast<const float2*>(b_org + ob[e]);
      else return pb[e][kb];
    };
    const int64_t rem = kend - k0;
    const int kleft = rem < BK ? (int)rem : BK;  // valid k of this tile
    if (interior && kleft == BK) {  // whole tile inside the operands: no guards
#pragma unroll
      for (int e = 0; e < kPA; ++e) ra[e] = lda(e);
#pragma unroll
      for (int e = 0; e < kPB; ++e) rb[e] = ldb(e);
    } else {
#pragma unroll
      for (int e = 0; e < kPA; ++e)
        ra[e] = (a_in(a_rt + row_e(kfa, e)) && a_kt + k_e(kfa, e) < kleft) ? lda(e) : f2(0.f, 0.f);
#pragma unroll
      for (int e = 0; e < kPB; ++e)
        rb[e] = (b_in(b_rt + row_e(kfb, e)) && b_kt + k_e(kfb, e) < kleft) ? ldb(e) : f2(0.f, 0.f);
    }
  };
  float* const as_t = As + a_rt * kRow + 2 * a_kt;
  float* const bs_t = Bs + b_rt * kRow + 2 * b_kt;
  auto put = [&](float* dst, bool k_fast, const float2* r, int n) {
    if (k_fast) {
#pragma unroll
      for (int e = 0; e < n; ++e) *reinterpret_cast<float2*>(dst + row_e(true, e) * kRow) = r[e];
    } else {
#pragma unroll
      for (int e = 0; e < n; e += 4) {
        float* d = dst + row_e(false, e) * kRow;
        *reinterpret_cast<float4*>(d) = make_float4(r[e].x, r[e].y, r[e + 1].x, r[e + 1].y);
        *reinterpret_cast<float4*>(d + 4) = make_float4(r[e + 2].x, r[e + 2].y, r[e + 3].x, r[e + 3].y);
      }
    }
  };
  auto stage = [&]() {
    put(as_t, kfa, ra, kPA);
    put(bs_t, kfb, rb, kPB);
  };
  const int h = lane >> 5, r32 = lane & 31;
  const int col = BP ? 32 * w + r32 : wn * 32 + r32;
  fetch(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    stage();
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
    // MFMA step s takes k = s on lanes 0-31 and k = BK/2 + s on lanes 32-63
    // (the same order for A and B), so a lane's operands for the whole tile are
    // the BK/2 contiguous k values of its row or column starting at h BK/2
    constexpr int kHalf = BK / 2;
#pragma unroll
    for (int hh = 0; hh < kHalf / 4; ++hh) {  // groups of four steps: four k values per lane and plane
      const int kw = 2 * (kHalf * h + 4 * hh);  // word offset of the lane's four complex k
      const float4 b0 = *reinterpret_cast<const float4*>(&Bs[col * kRow + kw]);
      const float4 b1 = *reinterpret_cast<const float4*>(&Bs[col * kRow + kw + 4]);
      const float br[4] = {b0.x, b0.z, b1.x, b1.z}, bi[4] = {b0.y, b0.w, b1.y, b1.w};
      float ar[TM][4], ai[TM][4];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int row = BP ? 32 * w + r32 : wm * 32 * TM + i * 32 + r32;
        const float4 a0 = *reinterpret_cast<const float4*>(&As[row * kRow + kw]);
        const float4 a1 = *reinterpret_cast<const float4*>(&As[row * kRow + kw + 4]);
        ar[i][0] = a0.x; ar[i][1] = a0.z; ar[i][2] = a1.x; ar[i][3] = a1.z;
        ai[i][0] = a0.y; ai[i][1] = a0.w; ai[i][2] = a1.y; ai[i][3] = a1.w;
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const float bs = br[st] + bi[st];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          p1[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i][st], br[st], p1[i], 0, 0, 0);
          p2[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[i][st], bi[st], p2[i], 0, 0, 0);
          p3[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i][st] + ai[i][st], bs, p3[i], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int rl = (BP ? 32 * w : wm * 32 * TM + i * 32) + 8 * (v >> 2) + 4 * h + (v & 3);
      const int cl = BP ? r32 : wn * 32 + r32;
      if (a_in(rl) && (BP == 1 ? cl < g.N : BP == 2 ? n0 + 32 * w + cl < g.N : n0 + cl < g.N)) {
        const float a = p1[i][v], b = p2[i][v];
        store_stream(&C[base_c | TCm[rl] | TCn[cl]], a - b, p3[i][v] - a - b);
      }
    }
}

// Products too narrow for the matrix-core tiles (M < 64 or N < 32, e.g. a
// 4096-way batch of 2x2 outer products): one thread per output element, the
// same deposit-map addressing, K loop on the vector ALUs.
template <int PREC>
__global__ __launch_bounds__(kThreads) void k_contract_elem(GemmArgs g) {
  __shared__ int64_t TKa[kElemMaxK], TKb[kElemMaxK];
  const int z = blockIdx.y;
  const float2* A = g.A + (int64_t)z * g.a_bs;
  const float2* B = g.B + (int64_t)z * g.b_bs;
  float2* C = g.C + (int64_t)z * g.c_bs;
  const int K = (int)g.K;
  for (int k = threadIdx.x; k < K; k += kThreads) {
    TKa[k] = deposit(k, g.a_k, g.nbk);
    TKb[k] = deposit(k, g.b_k, g.nbk);
  }
  __syncthreads();
  const int64_t total = g.batch * g.M * g.N;
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < total; o += (int64_t)gridDim.x * kThreads) {
    const int64_t n = o & (g.N - 1);
    const int64_t m = (o >> g.nbn) & (g.M - 1);
    const int64_t b = o >> (g.nbn + g.nbm);
    const int64_t db_a = deposit(b, g.a_b, g.nbb), db_b = deposit(b, g.b_b, g.nbb);
    const int64_t ab = db_a | deposit(m, g.a_m, g.nbm);
    const int64_t bb = db_b | deposit(n, g.b_n, g.nbn);
    float2 acc = f2(0.f, 0.f);
    int k = 0;
    // eight operand pairs in flight at a time (the loads do not wait on the sum)
    for (; k + 8 <= K; k += 8) {
      float2 av[8], bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        av[u] = A[ab | TKa[k + u]];
        bv[u] = B[bb | TKb[k + u]];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cmac<PREC>(acc, av[u], bv[u]);
    }
    for (; k < K; ++k) acc = cmac<PREC>(acc, A[ab | TKa[k]], B[bb | TKb[k]]);
    C[deposit(b, g.c_b, g.nbb) | deposit(m, g.c_m, g.nbm) | deposit(n, g.c_n, g.nbn)] = acc;
  }
}

constexpr int kElemChunks = (kElemGroupOutBits + 5) / 6;

// A grouped member with long sums: thread t takes result o = t >> lane_bits
// and the terms k = s, s + L, s + 2L, ... (s = t mod L, L = 2^lane_bits); the
// L lanes of a result are adjacent lanes of one wave, leave the loop together
// (2^(out_bits + lane_bits) is a multiple of L) and combine their partial sums
// with cross-lane adds.
template <int PREC>
__device__ void elem_sum_lanes(const ElemMember& e, const int64_t* TO, const int64_t* TKa, const int64_t* TKb,
                               const float2* A, const float2* B, float2* C, int blk, int nblk) {
  const int lb = e.lane_bits, L = 1 << lb, s = threadIdx.x & (L - 1);
  const int KL = (1 << e.k_bits) >> lb;  // terms per lane, at least 4
  const int n_thr = 1 << (e.out_bits + lb);
  for (int t = blk * kThreads + threadIdx.x; t < n_thr; t += nblk * kThreads) {
    const int o = t >> lb;
    int64_t ab = 0, bb = 0, cc = 0;
#pragma unroll
    for (int ch = 0; ch < kElemChunks; ++ch) {
      const int i = ch * 64 + ((o >> (6 * ch)) & 63);
      ab |= TO[i];
      bb |= TO[kElemChunks * 64 + i];
      cc |= TO[2 * kElemChunks * 64 + i];
    }
    float2 acc = f2(0.f, 0.f);
    for (int j = 0; j < KL; j += 4) {  // four operand pairs in flight at a time
      float2 av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = s + ((j + u) << lb);
        av[u] = A[ab | TKa[k]];
        bv[u] = B[bb | TKb[k]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = cmac<PREC>(acc, av[u], bv[u]);
    }
    for (int off = L >> 1; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    if (s == 0) C[cc] = acc;
  }
}

// Grouped form of the per-output products: every member's address maps are
// turned into LDS tables (four 6-bit chunks of the result index, one table of
// summed offsets per operand), so an output costs twelve table reads before
// its sum.
static_assert(offsetof(ElemMember, bo) == offsetof(ElemMember, ao) + kElemGroupOutBits &&
                  offsetof(ElemMember, co) == offsetof(ElemMember, bo) + kElemGroupOutBits &&
                  offsetof(ElemMember, ak) == offsetof(ElemMember, co) + kElemGroupOutBits &&
                  offsetof(ElemMember, bk) == offsetof(ElemMember, ak) + kElemKBits,
              "the position maps of a member are consecutive bytes");

template <int PREC>
__global__ __launch_bounds__(kThreads) void k_elem_group(ElemGroupArgs g) {
  __shared__ int64_t TO[3 * kElemChunks * 64];  // [operand A, B, C][chunk][chunk value]
  __shared__ int64_t TKa[kElemMaxK], TKb[kElemMaxK];
  const int bx = blockIdx.x, z = blockIdx.y;
  int mi = 0;
  for (int i = 1; i < g.n; ++i)
    if (bx >= g.m[i].block0) mi = i;
  const ElemMember& e = g.m[mi];
  const int nblk = (mi + 1 < g.n ? g.m[mi + 1].block0 : g.total_blocks) - e.block0;
  const int ob = e.out_bits, kb = e.k_bits;
  // the member's position maps (ao, bo, co, ak, bk: consecutive bytes) staged in LDS with one
  // load per thread: read from the argument block at a run-time member index, each byte
  // would be a vector memory load that the table loops below wait for
  constexpr int kPosBytes = 3 * kElemGroupOutBits + 2 * kElemKBits;
  __shared__ int8_t PM[kPosBytes];
  for (int t = threadIdx.x; t < kPosBytes; t += kThreads) PM[t] = e.ao[t];
  __syncthreads();
  const int8_t* pak = PM + 3 * kElemGroupOutBits;
  const int8_t* pbk = pak + kElemKBits;
  for (int t = threadIdx.x; t < 3 * kElemChunks * 64; t += kThreads) {
    const int map = t / (kElemChunks * 64), ch = (t >> 6) % kElemChunks, x = t & 63;
    const int8_t* pos = PM + map * kElemGroupOutBits;
    int64_t r = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int bit = ch * 6 + j;
      if (bit < ob && ((x >> j) & 1)) {
        const int p = pos[bit];
        if (p >= 0) r |= (int64_t)1 << p;
      }
    }
    TO[t] = r;
  }
  const int K = 1 << kb;
  for (int k = threadIdx.x; k < K; k += kThreads) {
    int64_t ra = 0, rb = 0;
#pragma unroll
    for (int j = 0; j < kElemKBits; ++j)
      if (j < kb && ((k >> j) & 1)) {
        ra |= (int64_t)1 << pak[j];
        rb |= (int64_t)1 << pbk[j];
      }
    TKa[k] = ra;
    TKb[k] = rb;
  }
  __syncthreads();
  const float2* A = e.A + (int64_t)z * e.a_bs;
  const float2* B = e.B + (int64_t)z * e.b_bs;
  float2* C = e.C + (int64_t)z * e.c_bs;
  if (e.lane_bits > 0) {
    elem_sum_lanes<PREC>(e, TO, TKa, TKb, A, B, C, bx - e.block0, nblk);
    return;
  }
  const int n_out = 1 << ob;
  for (int o = (bx - e.block0) * kThreads + threadIdx.x; o < n_out; o += nblk * kThreads) {
    int64_t ab = 0, bb = 0, cc = 0;
#pragma unroll
    for (int ch = 0; ch < kElemChunks; ++ch) {
      const int i = ch * 64 + ((o >> (6 * ch)) & 63);
      ab |= TO[i];
      bb |= TO[kElemChunks * 64 + i];
      cc |= TO[2 * kElemChunks * 64 + i];
    }
    float2 acc = f2(0.f, 0.f);
    int k = 0;
    for (; k + 8 <= K; k += 8) {
      float2 av[8], bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        av[u] = A[ab | TKa[k + u]];
        bv[u] = B[bb | TKb[k + u]];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cmac<PREC>(acc, av[u], bv[u]);
    }
    for (; k < K; ++k) acc = cmac<PREC>(acc, A[ab | TKa[k]], B[bb | TKb[k]]);
    C[cc] = acc;
  }
}

ElemMember elem_member(const GemmDesc& d, const float2* a, int64_t a_bs, const float2* b, int64_t b_bs, float2* c,
                       int64_t c_bs) {
  ElemMember m;
  m.A = a;
  m.B = b;
  m.C = c;
  m.a_bs = a_bs;
  m.b_bs = b_bs;
  m.c_bs = c_bs;
  m.block0 = 0;  // laid out by the launcher
  m.out_bits = d.nbb + d.nbm + d.nbn;
  m.k_bits = d.nbk;
  m.lane_bits = 0;  // laid out by the launcher
  // result index bits: n lowest, then m, then batch
  for (int j = 0; j < kElemGroupOutBits; ++j) {
    m.ao[j] = m.bo[j] = m.co[j] = -1;
    if (j < d.nbn) {
      m.bo[j] = d.b_n[j];
      m.co[j] = d.c_n[j];
    } else if (j < d.nbn + d.nbm) {
      m.ao[j] = d.a_m[j - d.nbn];
      m.co[j] = d.c_m[j - d.nbn];
    } else if (j < m.out_bits) {
      m.ao[j] = d.a_b[j - d.nbn - d.nbm];
      m.bo[j] = d.b_b[j - d.nbn - d.nbm];
      m.co[j] = d.c_b[j - d.nbn - d.nbm];
    }
  }
  for (int j = 0; j < kElemKBits; ++j) {
    m.ak[j] = j < d.nbk ? d.a_k[j] : 0;
    m.bk[j] = j < d.nbk ? d.b_k[j] : 0;
  }
  return m;
}

hipError_t launch_elem_group(hipStream_t s, const ElemGroupArgs& a, int batch, int precision) {
  if (a.n < 1 || a.n > kElemGroupMax || batch < 1) return hipErrorInvalidValue;
  ElemGroupArgs g = a;
  int32_t blocks = 0;
  for (int i = 0; i < g.n; ++i) {
    ElemMember& m = g.m[i];
    if (m.out_bits < 0 || m.out_bits > kElemGroupOutBits || m.k_bits < 0 || m.k_bits > kElemKBits)
      return hipErrorInvalidValue;
    // one thread per result, or for sums of 128 terms and more 2^lane_bits
    // lanes per result, about eight terms each (at most 32 lanes, and at most
    // 2^20 threads for the member)
    int lb = m.k_bits >= 7 ? std::min(m.k_bits - 3, 5) : 0;
    while (lb > 0 && m.out_bits + lb > 20) --lb;
    m.lane_bits = lb;
    m.block0 = blocks;
    blocks += (int32_t)((((int64_t)1 << (m.out_bits + lb)) + kThreads - 1) / kThreads);
  }
  g.total_blocks = blocks;
  const void* fn = precision == TN_PREC_BF16X3 ? (const void*)k_elem_group<TN_PREC_BF16X3>
                                               : (const void*)k_elem_group<TN_PREC_C64>;
  void* args[] = {&g};
  return hipLaunchKernel(fn, dim3((unsigned)blocks, batch), dim3(kThreads), args, 0, s);
}

// C[i] = sum over s of partial[s][i] (split-K), contiguous per parameter vector
__global__ void k_sum_partials(const float2* part, int64_t part_bs, int split, int64_t n, float2* C, int64_t c_bs) {
  const int z = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    float2 acc = f2(0.f, 0.f);
    for (int s = 0; s < split; ++s) {
      const float2 v = part[(int64_t)z * part_bs + (int64_t)s * n + i];
      acc.x += v.x;
      acc.y += v.y;
    }
    C[(int64_t)z * c_bs + i] = acc;
  }
}

template <int TM, int TN, int F>
static void* gemm_fn(int ak, int bnf) {
  if (ak && bnf) return (void*)k_gemm<1, 1, TM, TN, F>;
  if (ak) return (void*)k_gemm<1, 0, TM, TN, F>;
  if (bnf) return (void*)k_gemm<0, 1, TM, TN, F>;
  return (void*)k_gemm<0, 0, TM, TN, F>;
}

template <int TM, int BK, int NW, int BP = 0>
static void* gemm3m_fn_nw(int ak, int bnf) {
  if (ak && bnf) return (void*)k_gemm3m<1, 1, TM, BK, NW, BP>;
  if (ak) return (void*)k_gemm3m<1, 0, TM, BK, NW, BP>;
  if (bnf) return (void*)k_gemm3m<0, 1, TM, BK, NW, BP>;
  return (void*)k_gemm3m<0, 0, TM, BK, NW, BP>;
}

template <int TM, int BK>
static void* gemm3m_fn(int ak, int bnf, bool narrow) {
  return narrow ? gemm3m_fn_nw<TM, BK, 1>(ak, bnf) : gemm3m_fn_nw<TM, BK, 0>(ak, bnf);
}

template <int F>
static void* gemm_fn_tile(int tile, int ak, int bnf, bool narrow) {
  switch (tile) {
    case 0: return gemm_fn<2, 2, F>(ak, bnf);
    case 1: return gemm_fn<2, 1, F>(ak, bnf);
    case 2: return gemm_fn<1, 2, F>(ak, bnf);
    case 3: return gemm_fn<1, 1, F>(ak, bnf);
    case 5: return gemm3m_fn<2, 16>(ak, bnf, narrow);
    case 7: return narrow ? gemm3m_fn_nw<1, 16, 1, 1>(ak, bnf) : nullptr;
    case 8: return narrow ? gemm3m_fn_nw<1, 16, 1, 2>(ak, bnf) : nullptr;
    default: return gemm3m_fn<1, 16>(ak, bnf, narrow);
  }
}

// Whether every element offset inside one operand tile (its tile-local m or n
// bits, k bits and, batch-packed, batch bits, without the tile's origin) is
// below 2^32 bytes.
static bool tile_offsets_narrow(const int8_t* pos_mn, int n_mn, const int8_t* pos_k, int n_k,
                                const int8_t* pos_b = nullptr, int n_b = 0) {
  int top = -1;
  for (int j = 0; j < n_mn; ++j) top = pos_mn[j] > top ? pos_mn[j] : top;
  for (int j = 0; j < n_k; ++j) top = pos_k[j] > top ? pos_k[j] : top;
  for (int j = 0; j < n_b; ++j) top = pos_b[j] > top ? pos_b[j] : top;
  return top + 1 + 3 <= 32;  // 8-byte elements
}

static bool tile_narrow(const GemmDesc& d, int tile) {
  const int lbk = std::min(d.nbk, 4);
  if (tile == kGemmBatchPacked)
    return tile_offsets_narrow(d.a_m, std::min(d.nbm, 5), d.a_k, lbk, d.a_b, std::min(d.nbb, 2)) &&
           tile_offsets_narrow(d.b_n, std::min(d.nbn, 5), d.b_k, lbk, d.b_b, std::min(d.nbb, 2));
  if (tile == kGemmColumnPacked)
    return tile_offsets_narrow(d.a_m, std::min(d.nbm, 5), d.a_k, lbk) &&
           tile_offsets_narrow(d.b_n, std::min(d.nbn, 7), d.b_k, lbk);
  const int lbm = kGemmTileM[tile] == 128 ? 7 : 6, lbn = kGemmTileN[tile] == 64 ? 6 : 5;
  return tile_offsets_narrow(d.a_m, std::min(d.nbm, lbm), d.a_k, lbk) &&
         tile_offsets_narrow(d.b_n, std::min(d.nbn, lbn), d.b_k, lbk);
}

bool gemm_tile_supported(const GemmDesc& d, int tile) {
  if (tile < 0 || tile >= kGemmTiles) return false;
  if (tile == kGemmBatchPacked)  // four whole batch items of at most 32 x 32 per block
    return d.M <= 32 && d.N <= 32 && d.nbb >= 2 && tile_narrow(d, tile);
  if (tile == kGemmColumnPacked)  // M <= 32, four 32-column slices per block
    return d.M <= 32 && d.N >= 64 && tile_narrow(d, tile);
  return true;
}

hipError_t launch_gemm(hipStream_t s, const GemmDesc& d, int tile, int split, const float2* a, int64_t a_bs,
                       const float2* b, int64_t b_bs, float2* c, int64_t c_bs, float2* tmp, int64_t tmp_bs, int batch,
                       int precision) {
  if (!gemm_tile_supported(d, tile)) return hipErrorInvalidValue;
  if (tile > kGemmVector && precision != TN_PREC_C64) return hipErrorInvalidValue;  // 3M: FP32 only
  GemmArgs g;
  g.A = a; g.B = b;
  g.batch = d.batch; g.M = d.M; g.N = d.N; g.K = d.K;
  g.split = split > 1 ? split : 1;
  g.c_elems = d.batch * d.M * d.N;
  g.a_bs = a_bs; g.b_bs = b_bs;
  g.nbb = d.nbb; g.nbm = d.nbm; g.nbn = d.nbn; g.nbk = d.nbk; g.xcd = 0;
  g.band_n = 1;
  for (int j = 0; j < kGemmMaxBits; ++j) {
    g.a_b[j] = d.a_b[j]; g.a_m[j] = d.a_m[j]; g.a_k[j] = d.a_k[j];
    g.b_b[j] = d.b_b[j]; g.b_k[j] = d.b_k[j]; g.b_n[j] = d.b_n[j];
    g.c_b[j] = d.c_b[j]; g.c_m[j] = d.c_m[j]; g.c_n[j] = d.c_n[j];
  }
  if (tile == kGemmVector) {
    if (d.K > kElemMaxK) return hipErrorInvalidValue;
    if (d.nbb + d.nbm + d.nbn <= kElemGroupOutBits && d.nbk <= kElemKBits) {  // the table-driven kernel
      ElemGroupArgs ga;
      ga.n = 1;
      ga.total_blocks = 0;
      ga.m[0] = elem_member(d, a, a_bs, b, b_bs, c, c_bs);
      return launch_elem_group(s, ga, batch, precision);
    }
    g.C = c;
    g.c_bs = c_bs;
    g.split = 1;
    g.tiles_m = g.tiles_n = 1;
    int64_t eb = (g.c_elems + kThreads - 1) / kThreads;
    if (eb > 65535) eb = 65535;
    if (precision == TN_PREC_BF16X3)
      hipLaunchKernelGGL(k_contract_elem<TN_PREC_BF16X3>, dim3((unsigned)eb, batch), dim3(kThreads), 0, s, g);
    else
      hipLaunchKernelGGL(k_contract_elem<TN_PREC_C64>, dim3((unsigned)eb, batch), dim3(kThreads), 0, s, g);
    return hipGetLastError();
  }
  if (g.split > 1) {
    if (d.K % g.split != 0 || g.split > d.max_split || !tmp) return hipErrorInvalidValue;
    g.C = tmp;
    g.c_bs = tmp_bs;
  } else {
    g.C = c;
    g.c_bs = c_bs;
  }
  g.tiles_m = (d.M + kGemmTileM[tile] - 1) / kGemmTileM[tile];
  g.tiles_n = (d.N + kGemmTileN[tile] - 1) / kGemmTileN[tile];
  const int64_t batch_blocks = tile == kGemmBatchPacked ? d.batch / 4 : d.batch;
  const int64_t blocks = g.tiles_m * g.tiles_n * g.split * batch_blocks * batch;
  if (blocks > ((int64_t)1 << 24)) return hipErrorInvalidValue;  // grid of < 2^32 work-items
  // bands of a quarter of the tile columns on large grids (two XCDs per band), whole rows otherwise
  g.band_n = g.tiles_n >= 16 && g.tiles_n % 4 == 0 && g.tiles_m >= 16 ? g.tiles_n / 4 : g.tiles_n;
  g.xcd = blocks % 8 == 0 ? 1 : 0;
  const bool narrow = tile_narrow(d, tile);
  void* fn = precision == TN_PREC_BF16X3 ? gemm_fn_tile<1>(tile, d.a_kfast, d.b_nfast, narrow)
                                         : gemm_fn_tile<0>(tile, d.a_kfast, d.b_nfast, narrow);
  void* args[] = {&g};
  hipError_t e = hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(kThreads), args, 0, s);
  if (e != hipSuccess || g.split == 1) return e;
  int64_t rb = (g.c_elems + kThreads - 1) / kThreads;
  if (rb > 16384) rb = 16384;
  hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)rb, batch), dim3(kThreads), 0, s, tmp, tmp_bs, g.split, g.c_elems,
                     c, c_bs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions (FP64 accumulation)
// ---------------------------------------------------------------------------
__device__ inline double zdiag(uint64_t x, const ZTerms& t) {
  double d = 0;
  for (int i = 0; i < t.n; ++i) d += (__popcll(x & t.mask[i]) & 1) ? -t.coeff[i] : t.coeff[i];
  return d;
}

__global__ __launch_bounds__(kThreads) void k_expect_partial(const float2* psi, int64_t bs, int64_t n, ZTerms t,
                                                             double* partial) {
  __shared__ double red[kThreads / 64];
  const int z = blockIdx.y;
  const float2* p = psi + (int64_t)z * bs;
  double acc = 0;
  for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
    const float2 v = p[x];
    const double pr = (double)v.x * v.x + (double)v.y * v.y;
    acc += pr * zdiag((uint64_t)x, t);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)z * kExpectBlocks + blockIdx.x] = s;
}

// one block per parameter vector; fixed summation order (deterministic)
__global__ __launch_bounds__(kThreads) void k_reduce_rows(const double* partial, int nb, double* out,
                                                          int64_t out_stride) {
  __shared__ double red[kThreads / 64];
  const int z = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < nb; i += kThreads) s += partial[(int64_t)z * kExpectBlocks + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[(int64_t)z * out_stride] = s;
}

// D at the 16 addresses base + 256 j (j = 0..15, base with bits 8..11 clear):
// each term's sign over the bits other than 8..11 is taken once per thread,
// the sums per pattern mu of bits 8..11 go into w[mu], and a 16-point
// Walsh-Hadamard transform gives D(base + 256 j) = sum_mu w[mu] (-1)^popc(j & mu).
__device__ inline void zdiag16(uint64_t base, const ZTerms& t, double (&w)[16]) {
#pragma unroll
  for (int mu = 0; mu < 16; ++mu) {
    double acc = 0;
    for (int i = t.mu_start[mu]; i < t.mu_start[mu + 1]; ++i)
      acc += (__popcll(base & t.mask[i]) & 1) ? -t.coeff[i] : t.coeff[i];
    w[mu] = acc;
  }
#pragma unroll
  for (int h = 1; h < 16; h <<= 1)
#pragma unroll
    for (int a = 0; a < 16; a += 2 * h)
#pragma unroll
      for (int b = a; b < a + h; ++b) {
        const double u = w[b], v = w[b + h];
        w[b] = u + v;
        w[b + h] = u - v;
      }
}

// blocks of 4096 consecutive elements: thread t takes base + t + 256 j
__global__ __launch_bounds__(kThreads) void k_expect_partial16(const float2* psi, int64_t bs, int64_t n, ZTerms t,
                                                               double* partial) {
  __shared__ double red[kThreads / 64];
  const int z = blockIdx.y;
  const float2* p = psi + (int64_t)z * bs;
  double acc = 0;
  for (int64_t c = blockIdx.x; c < (n >> 12); c += gridDim.x) {
    const int64_t base = (c << 12) | threadIdx.x;
    double w[16];
    zdiag16((uint64_t)base, t, w);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const float2 v = p[base + 256 * j];
      acc += ((double)v.x * v.x + (double)v.y * v.y) * w[j];
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)z * kExpectBlocks + blockIdx.x] = s;
}

hipError_t launch_expectation(hipStream_t s, const float2* psi, int64_t psi_bs, int64_t n_elems, const ZTerms& terms,
                              int batch, double* partial, double* out, int64_t out_stride) {
  int64_t blocks;
  if (n_elems >= 4096) {
    blocks = std::min<int64_t>(n_elems >> 12, kExpectBlocks);
    hipLaunchKernelGGL(k_expect_partial16, dim3((unsigned)blocks, batch), dim3(kThreads), 0, s, psi, psi_bs, n_elems,
                       terms, partial);
  } else {
    blocks = std::min<int64_t>((n_elems + kThreads - 1) / kThreads, kExpectBlocks);
    hipLaunchKernelGGL(k_expect_partial, dim3((unsigned)blocks, batch), dim3(kThreads), 0, s, psi, psi_bs, n_elems,
                       terms, partial);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_rows, dim3(batch), dim3(kThreads), 0, s, partial, (int)blocks, out, out_stride);
  return hipGetLastError();
}

__global__ void k_copy(const float2* in, int64_t in_bs, float2* out, int64_t out_bs, int64_t n) {
  const int z = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    out[(int64_t)z * out_bs + i] = in[(int64_t)z * in_bs + i];
}

hipError_t launch_copy(hipStream_t s, const float2* in, int64_t in_bs, float2* out, int64_t out_bs, int64_t n,
                       int batch) {
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks, batch), dim3(kThreads), 0, s, in, in_bs, out, out_bs, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint sweep
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_apply_diag_obs(const float2* psi, int64_t psi_bs, float2* lam,
                                                             int64_t lam_bs, int64_t n, ZTerms t) {
  const int z = blockIdx.y;
  for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
    const float2 v = psi[(int64_t)z * psi_bs + x];
    const double d = zdiag((uint64_t)x, t);
    lam[(int64_t)z * lam_bs + x] = f2((float)(d * v.x), (float)(d * v.y));
  }
}

__global__ __launch_bounds__(kThreads) void k_apply_diag_obs16(const float2* psi, int64_t psi_bs, float2* lam,
                                                               int64_t lam_bs, int64_t n, ZTerms t) {
  const int z = blockIdx.y;
  for (int64_t c = blockIdx.x; c < (n >> 12); c += gridDim.x) {
    const int64_t base = (c << 12) | threadIdx.x;
    double w[16];
    zdiag16((uint64_t)base, t, w);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const float2 v = psi[(int64_t)z * psi_bs + base + 256 * j];
      lam[(int64_t)z * lam_bs + base + 256 * j] = f2((float)(w[j] * v.x), (float)(w[j] * v.y));
    }
  }
}

hipError_t launch_apply_diag_obs(hipStream_t s, const float2* psi, int64_t psi_bs, float2* lam, int64_t lam_bs,
                                 int64_t n_elems, const ZTerms& terms, int batch) {
  if (n_elems >= 4096) {
    const int64_t blocks = std::min<int64_t>(n_elems >> 12, 16384);
    hipLaunchKernelGGL(k_apply_diag_obs16, dim3((unsigned)blocks, batch), dim3(kThreads), 0, s, psi, psi_bs, lam,
                       lam_bs, n_elems, terms);
    return hipGetLastError();
  }
  int64_t blocks = (n_elems + kThreads - 1) / kThreads;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_apply_diag_obs, dim3((unsigned)blocks, batch), dim3(kThreads), 0, s, psi, psi_bs, lam, lam_bs,
                     n_elems, terms);
  return hipGetLastError();
}

// Im(conj(l) * p)
__device__ inline double im_cl_p(float2 l, float2 p) { return (double)l.x * p.y - (double)l.y * p.x; }
// Re(conj(l) * p)
__device__ inline double re_cl_p(float2 l, float2 p) { return (double)l.x * p.x + (double)l.y * p.y; }

template <int NQ, int PREC>
__global__ __launch_bounds__(kThreads) void k_adjoint_step(SweepArgs a, const float2* U, int64_t u_bs, float2* psi,
                                                           int64_t psi_bs, float2* lam, int64_t lam_bs,
                                                           int64_t n_groups, double* partials, int64_t pstride) {
  __shared__ double red[kThreads / 64];
  constexpr int D = 1 << NQ;
  const int z = blockIdx.y;
  float2* P = psi + (int64_t)z * psi_bs;
  float2* L = lam + (int64_t)z * lam_bs;
  float2 u[D * D];
  for (int i = 0; i < D * D; ++i) u[i] = U[(int64_t)z * u_bs + i];
  int lo = a.pos[0], hi = a.pos[0];
  if (NQ == 2) { lo = min(a.pos[0], a.pos[1]); hi = max(a.pos[0], a.pos[1]); }
  double g = 0;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n_groups; j += (int64_t)gridDim.x * kThreads) {
    int64_t base = ((j >> lo) << (lo + 1)) | (j & (((int64_t)1 << lo) - 1));
    if (NQ == 2) base = ((base >> hi) << (hi + 1)) | (base & (((int64_t)1 << hi) - 1));
    int64_t idx[D];
    if (NQ == 1) {
      idx[0] = base;
      idx[1] = base | ((int64_t)1 << a.pos[0]);
    } else {
      for (int v = 0; v < 4; ++v)
        idx[v] = base | ((int64_t)(v >> 1) << a.pos[0]) | ((int64_t)(v & 1) << a.pos[1]);
    }
    float2 p[D], l[D];
    for (int v = 0; v < D; ++v) { p[v] = P[idx[v]]; l[v] = L[idx[v]]; }
    switch (a.gen) {
      case GEN_X_HALF: g += im_cl_p(l[0], p[1]) + im_cl_p(l[1], p[0]); break;
      case GEN_X: g += 2.0 * (im_cl_p(l[0], p[1]) + im_cl_p(l[1], p[0])); break;
      case GEN_Y_HALF:  // Y p = (-i p1, i p0);  Im(conj(l) (-i p)) = -Re(conj(l) p)
        g += -re_cl_p(l[0], p[1]) + re_cl_p(l[1], p[0]); break;
      case GEN_Z_HALF: g += im_cl_p(l[0], p[0]) - im_cl_p(l[1], p[1]); break;
      case GEN_ZZ_PHASE: if (NQ == 2) g += 2.0 * (im_cl_p(l[1], p[1]) + im_cl_p(l[2], p[2])); break;
      case GEN_CPHASE: if (NQ == 2) g += -2.0 * im_cl_p(l[3], p[3]); break;
      default: break;
    }
    // psi <- U^dagger psi, lam <- U^dagger lam (products in the requested precision)
    for (int r = 0; r < D; ++r) {
      float2 ap = f2(0.f, 0.f), al = f2(0.f, 0.f);
      for (int c = 0; c < D; ++c) {
        const float2 uc = f2(u[c * D + r].x, -u[c * D + r].y);  // conj(U[c][r])
        ap = cmac<PREC>(ap, uc, p[c]);
        al = cmac<PREC>(al, uc, l[c]);
      }
      P[idx[r]] = ap;
      L[idx[r]] = al;
    }
  }
  if (a.slot >= 0) {
    const double s = block_sum(g, red);
    if (threadIdx.x == 0) partials[(int64_t)z * pstride + (int64_t)a.slot * kReduceBlocks + blockIdx.x] = s;
  }
}

hipError_t launch_adjoint_step(hipStream_t s, const SweepArgs& a, const float2* u, int64_t u_bs, float2* psi,
                               int64_t psi_bs, float2* lam, int64_t lam_bs, int64_t n_elems, int batch,
                               double* partials, int64_t partial_stride, int precision) {
  const int64_t groups = n_elems >> a.nq;
  // a fixed grid so that every partial slot is written
  const int blocks = kReduceBlocks;
  const bool bf = precision == TN_PREC_BF16X3;
  void* fn = a.nq == 2 ? (bf ? (void*)k_adjoint_step<2, TN_PREC_BF16X3> : (void*)k_adjoint_step<2, TN_PREC_C64>)
                       : (bf ? (void*)k_adjoint_step<1, TN_PREC_BF16X3> : (void*)k_adjoint_step<1, TN_PREC_C64>);
  SweepArgs aa = a;
  void* args[] = {&aa, (void*)&u, (void*)&u_bs, (void*)&psi, (void*)&psi_bs, (void*)&lam, (void*)&lam_bs,
                  (void*)&groups, (void*)&partials, (void*)&partial_stride};
  return hipLaunchKernel(fn, dim3(blocks, batch), dim3(kThreads), args, 0, s);
}

// Fused adjoint pass (see AdjGateDesc).  Two chunks (psi and lambda) in LDS;
// per segment each thread holds 16 elements of each in registers.
struct AdjPassArgs {
  float2* psi;
  float2* lam;
  int64_t psi_bs, lam_bs;
  const float2* U;
  int64_t u_bs;
  const AdjGateDesc* gates;
  const SweepSegment* segs;
  double* partials;
  int64_t pstride;
  int64_t n_chunks;
  int32_t n_segs, l, n_rest, n_red;
  int32_t first_gate, n_gates;
  int8_t lpos[kSweepMaxLocal];
  int8_t rest[64];
};
static_assert(offsetof(AdjPassArgs, lpos) % 4 == 0 && offsetof(AdjPassArgs, rest) % 4 == 0,
              "position maps aligned to 32-bit words");

__device__ inline float im_conj_mul(float2 l, float2 q) { return l.x * q.y - l.y * q.x; }
__device__ inline float2 cmulf(float2 a, float2 b) { return f2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// sum over the register pairs along bit U of Im(conj(l_m) (G p)_m)
template <int U>
__device__ __forceinline__ float reg_grad1(const float2 (&p)[16], const float2 (&l)[16], const float2* G) {
  float g = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << U)) continue;
    const int r1 = r | (1 << U);
    const float2 q0 = f2(G[0].x * p[r].x - G[0].y * p[r].y + G[1].x * p[r1].x - G[1].y * p[r1].y,
                         G[0].x * p[r].y + G[0].y * p[r].x + G[1].x * p[r1].y + G[1].y * p[r1].x);
    const float2 q1 = f2(G[2].x * p[r].x - G[2].y * p[r].y + G[3].x * p[r1].x - G[3].y * p[r1].y,
                         G[2].x * p[r].y + G[2].y * p[r].x + G[3].x * p[r1].y + G[3].y * p[r1].x);
    g += im_conj_mul(l[r], q0) + im_conj_mul(l[r1], q1);
  }
  return g;
}

// Sum over the 16 register elements of q_b Im(conj(l) p), b resolved as in
// apply_diag (the diagonal generators Z, 1 - ZZ and |11><11| are real)
template <int U>
__device__ __forceinline__ float dgrad_reg1(const float2 (&p)[16], const float2 (&l)[16], float e0, float e1) {
  float g = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) g += ((r >> U) & 1 ? e1 : e0) * im_conj_mul(l[r], p[r]);
  return g;
}
template <int U0, int U1>
__device__ __forceinline__ float dgrad_reg2(const float2 (&p)[16], const float2 (&l)[16], float q0, float q1, float q2,
                                   float q3) {
  float g = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int b = ((r >> U0) & 1) | (((r >> U1) & 1) << 1);
    g += (b == 0 ? q0 : b == 1 ? q1 : b == 2 ? q2 : q3) * im_conj_mul(l[r], p[r]);
  }
  return g;
}
__device__ __forceinline__ float diag_grad(const float2 (&p)[16], const float2 (&l)[16], int n, int k0, int k1, int c,
                                  float q0, float q1, float q2, float q3) {
  if (n == 2 && k0 >= 0 && k1 >= 0) {
    switch (k0 * 4 + k1) {
      case 1: return dgrad_reg2<0, 1>(p, l, q0, q1, q2, q3);
      case 2: return dgrad_reg2<0, 2>(p, l, q0, q1, q2, q3);
      case 3: return dgrad_reg2<0, 3>(p, l, q0, q1, q2, q3);
      case 4: return dgrad_reg2<1, 0>(p, l, q0, q1, q2, q3);
      case 6: return dgrad_reg2<1, 2>(p, l, q0, q1, q2, q3);
      case 7: return dgrad_reg2<1, 3>(p, l, q0, q1, q2, q3);
      case 8: return dgrad_reg2<2, 0>(p, l, q0, q1, q2, q3);
      case 9: return dgrad_reg2<2, 1>(p, l, q0, q1, q2, q3);
      case 11: return dgrad_reg2<2, 3>(p, l, q0, q1, q2, q3);
      case 12: return dgrad_reg2<3, 0>(p, l, q0, q1, q2, q3);
      case 13: return dgrad_reg2<3, 1>(p, l, q0, q1, q2, q3);
      default: return dgrad_reg2<3, 2>(p, l, q0, q1, q2, q3);
    }
  }
  int k = -1;
  float e0 = 0.f, e1 = 0.f;
  if (n == 2 && k0 >= 0) {
    k = k0;
    e0 = (c & 2) ? q2 : q0;
    e1 = (c & 2) ? q3 : q1;
  } else if (n == 2 && k1 >= 0) {
    k = k1;
    e0 = (c & 1) ? q1 : q0;
    e1 = (c & 1) ? q3 : q2;
  } else if (n == 1 && k0 >= 0) {
    k = k0;
    e0 = q0;
    e1 = q1;
  }
  if (k < 0) {
    const float f = c == 0 ? q0 : c == 1 ? q1 : c == 2 ? q2 : q3;
    float g = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) g += im_conj_mul(l[r], p[r]);
    return f * g;
  }
  switch (k) {
    case 0: return dgrad_reg1<0>(p, l, e0, e1);
    case 1: return dgrad_reg1<1>(p, l, e0, e1);
    case 2: return dgrad_reg1<2>(p, l, e0, e1);
    default: return dgrad_reg1<3>(p, l, e0, e1);
  }
}

// dense generators: c X (gradient c [Im(conj(l0) p1) + Im(conj(l1) p0)]) and Y
template <int U>
__device__ __forceinline__ float reg_grad_x(const float2 (&p)[16], const float2 (&l)[16], float c) {
  float g = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << U)) continue;
    const int r1 = r | (1 << U);
    g += im_conj_mul(l[r], p[r1]) + im_conj_mul(l[r1], p[r]);
  }
  return c * g;
}
template <int U>
__device__ __forceinline__ float reg_grad_y(const float2 (&p)[16], const float2 (&l)[16]) {
  float g = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << U)) continue;
    const int r1 = r | (1 << U);
    // Y p = (-i p1, i p0): Im(conj(l0)(-i p1)) + Im(conj(l1)(i p0)) = -Re(conj(l0) p1) + Re(conj(l1) p0)
    g += (l[r1].x * p[r].x + l[r1].y * p[r].y) - (l[r].x * p[r1].x + l[r].y * p[r1].y);
  }
  return g;
}

// Sum over the 64 lanes of a wave, the result in lane 63: DPP moves within
// quads, half rows and rows, then the row broadcasts of lane 15 and lane 31
// (six dependent VALU operations; a shuffle network would wait on LDS at each
// of its six steps).
__device__ __forceinline__ float wave_sum_to_63(float v) {
  auto dpp = [](float x, int ctrl, int row_mask) -> float {
    switch (ctrl) {  // the control word must be a compile-time constant
      case 0xb1: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xb1, 0xf, 0xf, false));
      case 0x4e: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4e, 0xf, 0xf, false));
      case 0x141: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xf, 0xf, false));
      case 0x140: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xf, 0xf, false));
      case 0x142: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xa, 0xf, false));
      default: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xc, 0xf, false));
    }
  };
  v += dpp(v, 0xb1, 0xf);   // quad_perm [1, 0, 3, 2]
  v += dpp(v, 0x4e, 0xf);   // quad_perm [2, 3, 0, 1]
  v += dpp(v, 0x141, 0xf);  // row_half_mirror
  v += dpp(v, 0x140, 0xf);  // row_mirror: every lane of a row holds the row's sum
  v += dpp(v, 0x142, 0xa);  // row_bcast:15 into rows 1 and 3
  v += dpp(v, 0x143, 0xc);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
  return v;
}

// One gate of a run of dense one-qubit gates in the reverse sweep (see
// run_apply): its gradient term from the states as they stand, then
// U^dagger on register bit R of both states, R and U's form F fixed.
template <int PREC, int R, int F, class AddGrad>
__device__ __forceinline__ void adj_run_slot(float2 (&xp)[16], float2 (&xl)[16], const AdjGateDesc& gd,
                                             const float2* Up, AddGrad& add_grad) {
  if (gd.red >= 0) {
    const float2* G = reinterpret_cast<const float2*>(gd.gen);
    const float g = gd.form == ADJ_GEN_X ? reg_grad_x<R>(xp, xl, G[2].x)
                    : gd.form == ADJ_GEN_Y ? reg_grad_y<R>(xp, xl)
                                           : reg_grad1<R>(xp, xl, G);
    add_grad(gd.red, g);
  }
  // U^dagger[m][k] = conj(U[k][m])
  const float2 ud[4] = {f2(Up[0].x, -Up[0].y), f2(Up[2].x, -Up[2].y), f2(Up[1].x, -Up[1].y), f2(Up[3].x, -Up[3].y)};
  reg_apply1<PREC, R, F>(xp, ud);
  reg_apply1<PREC, R, F>(xl, ud);
}

// The run of mask M: its k-th gate (descriptor gd[k], U entries Up[k]) on the k-th bit of M.
template <int PREC, int M, int F, class AddGrad>
__device__ __forceinline__ void adj_run(float2 (&xp)[16], float2 (&xl)[16], const AdjGateDesc* gd,
                                        const float2 (*Up)[4], AddGrad& add_grad) {
  int k = 0;
  if constexpr ((M & 1) != 0) { adj_run_slot<PREC, 0, F>(xp, xl, gd[k], Up[k], add_grad); ++k; }
  if constexpr ((M & 2) != 0) { adj_run_slot<PREC, 1, F>(xp, xl, gd[k], Up[k], add_grad); ++k; }
  if constexpr ((M & 4) != 0) { adj_run_slot<PREC, 2, F>(xp, xl, gd[k], Up[k], add_grad); ++k; }
  if constexpr ((M & 8) != 0) adj_run_slot<PREC, 3, F>(xp, xl, gd[k], Up[k], add_grad);
  variant_end<PREC, 400 + M * 4 + F>();
}

template <int PREC, class AddGrad>
__device__ __forceinline__ void adj_apply_run(float2 (&xp)[16], float2 (&xl)[16], const AdjGateDesc* gd,
                                              const float2 (*Up)[4], AddGrad& add_grad, int mask, int form) {
#define TNQ_ADJ_RUN(M)                                                                              \
  case M * 3 + kDenseGeneric: adj_run<PREC, M, kDenseGeneric>(xp, xl, gd, Up, add_grad); break; \
  case M * 3 + kDenseReal: adj_run<PREC, M, kDenseReal>(xp, xl, gd, Up, add_grad); break;       \
  case M * 3 + kDenseRxLike: adj_run<PREC, M, kDenseRxLike>(xp, xl, gd, Up, add_grad); break;
  switch (mask * 3 + (PREC == TN_PREC_C64 ? form : kDenseGeneric)) {
    TNQ_ADJ_RUN(3) TNQ_ADJ_RUN(5) TNQ_ADJ_RUN(6) TNQ_ADJ_RUN(7) TNQ_ADJ_RUN(9) TNQ_ADJ_RUN(10) TNQ_ADJ_RUN(11)
    TNQ_ADJ_RUN(12) TNQ_ADJ_RUN(13) TNQ_ADJ_RUN(14)
    default: adj_run<PREC, 15, kDenseGeneric>(xp, xl, gd, Up, add_grad); break;  // mask 15, generic form
    case 15 * 3 + kDenseReal: adj_run<PREC, 15, kDenseReal>(xp, xl, gd, Up, add_grad); break;
    case 15 * 3 + kDenseRxLike: adj_run<PREC, 15, kDenseRxLike>(xp, xl, gd, Up, add_grad); break;
  }
#undef TNQ_ADJ_RUN
}

template <int PREC>
__global__ __launch_bounds__(kThreads) void k_adjoint_pass(AdjPassArgs a, const AdjGateDesc* __restrict__ gates,
                                                            const SweepSegment* __restrict__ segs,
                                                            const float2* __restrict__ Uall) {
  constexpr int kBuf = (1 << kSweepMaxLocal) + (1 << (kSweepMaxLocal - 5));
  __shared__ float2 bp[kBuf], bl[kBuf];
  __shared__ int64_t dep_hi[1 << (kSweepMaxLocal - 5)];
  __shared__ double red[kAdjMaxRed][kThreads / 64];
  __shared__ float2 upre[kAdjPreGates][4];  // the entries of U the pass's first gates use (see below)
  const int z = blockIdx.y;
  const int L = 1 << a.l;
  const int nt = blockDim.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  if (blockIdx.x >= a.n_chunks) {  // no chunk for this block: its partial of every gradient term is zero
    for (int gi = a.first_gate + tid; gi < a.first_gate + a.n_gates; gi += nt) {
      const AdjGateDesc& gd = gates[gi];
      if (gd.red >= 0 && gd.slot >= 0)
        a.partials[(int64_t)z * a.pstride + (int64_t)gd.slot * kReduceBlocks + blockIdx.x] = 0.0;
    }
    return;
  }
  const float2* Uz = Uall + (int64_t)z * a.u_bs;
  // U of the pass's gates (at most kAdjPreGates) staged in LDS, one load per thread, all in flight
  // together: diagonal U[0], U[3] (one bit) or U[0], U[5], U[10], U[15] (two bits); one-qubit dense
  // U[0..3]; two-qubit dense gates read U from memory
  for (int i = tid; i < a.n_gates * 4; i += nt) {
    const int g = i >> 2, e = i & 3;
    const AdjGateDesc& gd = gates[a.first_gate + g];
    const int idx = gd.diag ? (gd.n == 2 ? 5 * e : (e == 1 ? 3 : 0)) : e;
    upre[g][e] = Uz[(int64_t)gd.gate * 16 + idx];
  }
  for (int h = tid; h < (L >> 5); h += nt) dep_hi[h] = deposit((int64_t)h << 5, a.lpos, a.l);
  __syncthreads();
  float2* P = a.psi + (int64_t)z * a.psi_bs;
  float2* Lm = a.lam + (int64_t)z * a.lam_bs;
  // gradient sums of this wave in registers: lane j holds slot j (accA) and slot 64 + j (accB)
  double accA = 0.0, accB = 0.0;
  auto add_grad = [&](int slot, float v) {
    v = wave_sum_to_63(v);
    const double sv = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
    const double add = lane == (slot & 63) ? sv : 0.0;  // selects only: no run-time choice of a register
    accA += slot < 64 ? add : 0.0;
    accB += slot < 64 ? 0.0 : add;
  };
  for (int64_t c = blockIdx.x; c < a.n_chunks; c += gridDim.x) {
    const int64_t base = deposit(c, a.rest, a.n_rest);
    chunk2_to_lds(bp, bl, P, Lm, base, dep_hi, tid, nt);
    __syncthreads();
    for (int sg = 0; sg < a.n_segs; ++sg) {
      const SweepSegment& seg = segs[sg];
      int ob = 0;
#pragma unroll
      for (int t = 0; t < 8; ++t) ob |= ((tid >> t) & 1) << seg.tpos[t];
      const int pob = ob + (ob >> 5);
      float2 xp[16], xl[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        xp[r] = bp[pob + seg.physoff[r]];
        xl[r] = bl[pob + seg.physoff[r]];
      }
      // unit-modulus diagonal factors that are the same for all of a thread's
      // elements go into one per-thread factor, applied to both states at the
      // segment's end; they commute with the segment's gates and leave every
      // gradient term Im<lambda|G|psi> unchanged (|factor|^2 = 1)
      float2 ph = f2(1.f, 0.f);
      bool ph_used = false;  // the same for the whole block (set by gates' descriptors)
      // Im(conj(lambda) psi) at each element is unchanged by unit-modulus diagonal gates, so
      // along a run of diagonal gates its sums are formed once: over the thread's elements
      // (tT) and over those whose register bit j is 1 (tS[j]); a one-bit diagonal generator's
      // term is then q0 (tT - s1) + q1 s1, s1 the sum where the gate's bit is 1
      bool have_t = false;
      float tT = 0.f, tS0 = 0.f, tS1 = 0.f, tS2 = 0.f, tS3 = 0.f;
      const int g_end = seg.first_gate + seg.n_gates;
      int gi = seg.first_gate;
      // the segment's leading diagonal gates with no bit in the registers (the planner puts
      // them first; they commute with the rest of the segment): their gradient terms need only
      // tT, and they change only ph, so this loop carries no register elements
      for (; gi < g_end; ++gi) {
        const AdjGateDesc& gd = gates[gi];
        if (!gd.diag || gd.kreg[0] >= 0 || (gd.n == 2 && gd.kreg[1] >= 0)) break;
        int c = 0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (j >= gd.n) continue;
          const int cs = gd.csrc[j];
          c |= (cs >= 64 ? (int)((base >> (cs - 64)) & 1) : ((ob >> cs) & 1)) << j;
        }
        ph_used = true;
        if (gd.form & ADJ_DIAG_SIGNS) {
          if (((gd.form >> 8) >> c) & 1) ph = f2(-ph.x, -ph.y);
          continue;
        }
        const float2* Up = upre[gi - a.first_gate];
        if (gd.red >= 0) {
          if (!have_t) {
            tT = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) tT += im_conj_mul(xl[r], xp[r]);
            have_t = true;
          }
          const float* G = gd.gen;  // diagonal generator entries, re/im interleaved
          const float q = c == 0 ? G[0] : c == 1 ? G[2] : c == 2 ? G[4] : G[6];
          add_grad(gd.red, q * tT);
        }
        const bool two = gd.n == 2;
        const float2 u0 = Up[0], u1 = Up[1], u2 = two ? Up[2] : u0, u3 = two ? Up[3] : u0;
        const float2 u = c == 0 ? u0 : c == 1 ? u1 : c == 2 ? u2 : u3;  // U^dagger: conj(U[b][b])
        ph = cmul<TN_PREC_C64>(ph, f2(u.x, -u.y));
      }
      have_t = false;  // the main loop's sums also split tT by register bit
      for (; gi < g_end; ++gi) {
        const AdjGateDesc& gd = gates[gi];
        const float2* U = Uz + (int64_t)gd.gate * 16;
        const float2* G = reinterpret_cast<const float2*>(gd.gen);
        const float2* Up = upre[gi - a.first_gate];
        if (!gd.diag) have_t = false;
        if (gd.diag && gd.run_mask && (gd.form & ADJ_DIAG_SIGNS)) {  // run_mask gates with entries +-1
          // (U^dagger = U; no gradient terms; sign flips of both states leave Im(conj(l) p) as it was)
          int m = 0;
          for (int j = 0; j < gd.run_mask; ++j) {
            const AdjGateDesc& gj = gates[gi + j];
            const bool two = gj.n == 2;
            int cj = 0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              if (t >= gj.n || gj.kreg[t] >= 0) continue;
              const int cs = gj.csrc[t];
              cj |= (cs >= 64 ? (int)((base >> (cs - 64)) & 1) : ((ob >> cs) & 1)) << t;
            }
            m ^= sign_pattern(gj.n, gj.kreg[0], two ? gj.kreg[1] : -1, cj, gj.form >> 8);
          }
          flip_signs(xp, m);
          flip_signs(xl, m);
          gi += gd.run_mask - 1;
          continue;
        }
        if (gd.diag && gd.run_mask) {  // one-bit unit diagonals on the mask's register bits, in bit order
          const int cnt = __builtin_popcount(gd.run_mask);
          // their gradient terms: a unit diagonal applied to both states leaves Im(conj(l) p)
          // unchanged, so the whole run shares one set of sums
          bool any_red = false;
#pragma unroll
          for (int j = 0; j < 4; ++j) any_red |= j < cnt && gates[gi + j].red >= 0;
          if (any_red && !have_t) {
            tT = tS0 = tS1 = tS2 = tS3 = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float t = im_conj_mul(xl[r], xp[r]);
              tT += t;
              if (r & 1) tS0 += t;
              if (r & 2) tS1 += t;
              if (r & 4) tS2 += t;
              if (r & 8) tS3 += t;
            }
            have_t = true;
          }
          float2 q[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            q[j] = f2(1.f, 0.f);
            if (j >= cnt) continue;
            const AdjGateDesc& gj = gates[gi + j];  // the run's gates are in register-bit order
            if (gj.red >= 0) {
              const float2* Gj = reinterpret_cast<const float2*>(gj.gen);
              const int b = gj.kreg[0];
              const float s1 = b == 0 ? tS0 : b == 1 ? tS1 : b == 2 ? tS2 : tS3;
              add_grad(gj.red, Gj[0].x * (tT - s1) + Gj[1].x * s1);
            }
            // U^dagger: conj of the entries; the first joins the deferred phase
            const float2* Uj = upre[gi + j - a.first_gate];
            const float2 e0 = f2(Uj[0].x, -Uj[0].y), e1 = f2(Uj[1].x, -Uj[1].y);
            ph = cmul<TN_PREC_C64>(ph, e0);
            q[j] = cmul<TN_PREC_C64>(e1, f2(e0.x, -e0.y));
          }
          ph_used = true;
          diag_run<PREC, 2>(xp, xl, q, gd.run_mask);
          gi += cnt - 1;
          continue;
        }
        if (gd.diag) {
          const int k[2] = {gd.kreg[0], gd.n == 2 ? gd.kreg[1] : -1};
          int c = 0;  // the index bits that are constant over the thread's elements
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            if (j >= gd.n || gd.kreg[j] >= 0) continue;
            const int cs = gd.csrc[j];
            c |= (cs >= 64 ? (int)((base >> (cs - 64)) & 1) : ((ob >> cs) & 1)) << j;
          }
          const bool two = gd.n == 2;
          const bool uniform = k[0] < 0 && k[1] < 0;  // the same entry for every element of the thread
          if (gd.form & ADJ_DIAG_SIGNS) {  // Z, CZ: U^dagger = U, entries +-1
            if (uniform) {
              ph_used = true;
              if (((gd.form >> 8) >> c) & 1) ph = f2(-ph.x, -ph.y);
              continue;
            }
            apply_signs(xp, gd.n, k[0], k[1], c, gd.form >> 8);
            apply_signs(xl, gd.n, k[0], k[1], c, gd.form >> 8);
            continue;
          }
          // U^dagger diagonal: conj(U[b][b])
          const float2 u0 = Up[0], u1 = Up[1], u2 = two ? Up[2] : f2(1.f, 0.f), u3 = two ? Up[3] : f2(1.f, 0.f);
          if (gd.red >= 0) {
            float v;
            if (!two) {
              if (!have_t) {
                tT = tS0 = tS1 = tS2 = tS3 = 0.f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                  const float t = im_conj_mul(xl[r], xp[r]);
                  tT += t;
                  if (r & 1) tS0 += t;
                  if (r & 2) tS1 += t;
                  if (r & 4) tS2 += t;
                  if (r & 8) tS3 += t;
                }
                have_t = true;
              }
              const float s1 = k[0] >= 0 ? (k[0] == 0 ? tS0 : k[0] == 1 ? tS1 : k[0] == 2 ? tS2 : tS3) : (c ? tT : 0.f);
              v = G[0].x * (tT - s1) + G[1].x * s1;
            } else {
              v = diag_grad(xp, xl, gd.n, k[0], k[1], c, G[0].x, G[1].x, G[2].x, G[3].x);
            }
            add_grad(gd.red, v);
          }
          const float2 d0 = f2(u0.x, -u0.y), d1 = f2(u1.x, -u1.y), d2 = f2(u2.x, -u2.y), d3 = f2(u3.x, -u3.y);
          ph_used = true;
          if (uniform) {
            const float2 f = c == 0 ? d0 : c == 1 ? d1 : c == 2 ? d2 : d3;
            ph = cmul<TN_PREC_C64>(ph, f);
            continue;
          }
          // unitary gates: the entries have unit modulus, so the first one joins the deferred phase
          apply_diag_unit<PREC, 2>(xp, xl, ph, gd.n, k[0], k[1], c, d0, d1, d2, d3);
        } else if (gd.n == 1) {
          if (gd.run_mask) {  // this gate and the next ones: one per bit of the mask, one form of U
            const int f = gd.uform == kFormReal ? kDenseReal : gd.uform == kFormRxLike ? kDenseRxLike : kDenseGeneric;
            adj_apply_run<PREC>(xp, xl, gates + gi, upre + (gi - a.first_gate), add_grad, gd.run_mask, f);
            gi += __builtin_popcount(gd.run_mask) - 1;
            continue;
          }
          if (gd.red >= 0) {
            float g;
            if (gd.form == ADJ_GEN_X) {
              const float cx = G[2].x;
              switch (gd.rb[0]) {
                case 0: g = reg_grad_x<0>(xp, xl, cx); break;
                case 1: g = reg_grad_x<1>(xp, xl, cx); break;
                case 2: g = reg_grad_x<2>(xp, xl, cx); break;
                default: g = reg_grad_x<3>(xp, xl, cx); break;
              }
            } else if (gd.form == ADJ_GEN_Y) {
              switch (gd.rb[0]) {
                case 0: g = reg_grad_y<0>(xp, xl); break;
                case 1: g = reg_grad_y<1>(xp, xl); break;
                case 2: g = reg_grad_y<2>(xp, xl); break;
                default: g = reg_grad_y<3>(xp, xl); break;
              }
            } else {
              switch (gd.rb[0]) {
                case 0: g = reg_grad1<0>(xp, xl, G); break;
                case 1: g = reg_grad1<1>(xp, xl, G); break;
                case 2: g = reg_grad1<2>(xp, xl, G); break;
                default: g = reg_grad1<3>(xp, xl, G); break;
              }
            }
            add_grad(gd.red, g);
          }
          // U^dagger[m][k] = conj(U[k][m])
          const float2 w0 = Up[0], w1 = Up[1], w2 = Up[2], w3 = Up[3];
          float2 ud[4];
          ud[0] = f2(w0.x, -w0.y);
          ud[1] = f2(w2.x, -w2.y);
          ud[2] = f2(w1.x, -w1.y);
          ud[3] = f2(w3.x, -w3.y);
          const int form = gd.uform == kFormReal ? kDenseReal : gd.uform == kFormRxLike ? kDenseRxLike : kDenseGeneric;
          apply_dense1<PREC, 2>(xp, xl, ud, gd.rb[0], form);
        } else {
          // dense two-qubit gates carry no gradient term (the planner checks)
          float2 ud[16];
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < 4; ++k) ud[4 * m + k] = f2(U[4 * k + m].x, -U[4 * k + m].y);
          switch (gd.rb[0] * 4 + gd.rb[1]) {
            case 1: reg_apply2<PREC, 0, 1>(xp, ud); reg_apply2<PREC, 0, 1>(xl, ud); break;
            case 4: reg_apply2<PREC, 1, 0>(xp, ud); reg_apply2<PREC, 1, 0>(xl, ud); break;
            case 2: reg_apply2<PREC, 0, 2>(xp, ud); reg_apply2<PREC, 0, 2>(xl, ud); break;
            case 8: reg_apply2<PREC, 2, 0>(xp, ud); reg_apply2<PREC, 2, 0>(xl, ud); break;
            case 3: reg_apply2<PREC, 0, 3>(xp, ud); reg_apply2<PREC, 0, 3>(xl, ud); break;
            case 12: reg_apply2<PREC, 3, 0>(xp, ud); reg_apply2<PREC, 3, 0>(xl, ud); break;
            case 6: reg_apply2<PREC, 1, 2>(xp, ud); reg_apply2<PREC, 1, 2>(xl, ud); break;
            case 9: reg_apply2<PREC, 2, 1>(xp, ud); reg_apply2<PREC, 2, 1>(xl, ud); break;
            case 7: reg_apply2<PREC, 1, 3>(xp, ud); reg_apply2<PREC, 1, 3>(xl, ud); break;
            case 13: reg_apply2<PREC, 3, 1>(xp, ud); reg_apply2<PREC, 3, 1>(xl, ud); break;
            case 11: reg_apply2<PREC, 2, 3>(xp, ud); reg_apply2<PREC, 2, 3>(xl, ud); break;
            default: reg_apply2<PREC, 3, 2>(xp, ud); reg_apply2<PREC, 3, 2>(xl, ud); break;
          }
        }
      }
      if (ph_used) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          bp[pob + seg.physoff[r]] = cmul<TN_PREC_C64>(ph, xp[r]);
          bl[pob + seg.physoff[r]] = cmul<TN_PREC_C64>(ph, xl[r]);
        }
      } else {  // no gate of the segment touched the factor (it is 1)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          bp[pob + seg.physoff[r]] = xp[r];
          bl[pob + seg.physoff[r]] = xl[r];
        }
      }
      __syncthreads();
    }
    chunk_from_lds(P, bp, base, dep_hi, tid, nt);
    chunk_from_lds(Lm, bl, base, dep_hi, tid, nt);
    __syncthreads();
  }
  red[lane][wv] = accA;
  red[64 + lane][wv] = accB;
  __syncthreads();
  // every (slot, block) entry of the pass's gates is written
  for (int gi = a.first_gate + tid; gi < a.first_gate + a.n_gates; gi += nt) {
    const AdjGateDesc& gd = gates[gi];
    if (gd.red < 0 || gd.slot < 0) continue;
    double v = 0;
    for (int w = 0; w < nw; ++w) v += red[gd.red][w];
    a.partials[(int64_t)z * a.pstride + (int64_t)gd.slot * kReduceBlocks + blockIdx.x] = v;
  }
}

hipError_t launch_adjoint_pass(hipStream_t s, const SweepPass& ps, int bits, const AdjGateDesc* gates_dev,
                               const SweepSegment* segs_dev, const float2* u, int64_t u_bs, float2* psi,
                               int64_t psi_bs, float2* lam, int64_t lam_bs, int batch, double* partials,
                               int64_t partial_stride, int precision) {
  AdjPassArgs a;
  a.psi = psi; a.lam = lam; a.psi_bs = psi_bs; a.lam_bs = lam_bs;
  a.U = u; a.u_bs = u_bs;
  a.gates = gates_dev;
  a.segs = segs_dev + ps.first_seg;
  a.partials = partials;
  a.pstride = partial_stride;
  a.n_segs = ps.n_segs;
  a.l = ps.l;
  a.n_red = ps.n_red;
  a.first_gate = ps.first_gate;
  a.n_gates = ps.n_gates;
  // 64 threads at least (whole waves for the gradient reductions), 256 at most
  if (ps.l < 10 || ps.l > kSweepMaxLocal || ps.n_red < 0 || ps.n_red > kAdjMaxRed || ps.n_gates < 0 ||
      ps.n_gates > kAdjPreGates)
    return hipErrorInvalidValue;
  std::vector<char> local(bits, 0);
  for (int j = 0; j < ps.l; ++j) {
    a.lpos[j] = ps.lpos[j];
    if (ps.lpos[j] < 0 || ps.lpos[j] >= bits || (j < 5 && ps.lpos[j] != j)) return hipErrorInvalidValue;
    local[ps.lpos[j]] = 1;
  }
  int nr = 0;
  for (int p = 0; p < bits; ++p)
    if (!local[p]) a.rest[nr++] = (int8_t)p;
  a.n_rest = nr;
  a.n_chunks = (int64_t)1 << nr;
  const int threads = 1 << (ps.l - 4);
  if (precision == TN_PREC_BF16X3)
    hipLaunchKernelGGL(k_adjoint_pass<TN_PREC_BF16X3>, dim3(kReduceBlocks, batch), dim3(threads), 0, s, a, a.gates,
                       a.segs, a.U);
  else
    hipLaunchKernelGGL(k_adjoint_pass<TN_PREC_C64>, dim3(kReduceBlocks, batch), dim3(threads), 0, s, a, a.gates, a.segs,
                       a.U);
  return hipGetLastError();
}

__global__ void k_slot_sums(double* partials, int64_t pstride, int n_slots, int batch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_slots * batch) return;
  const int z = (int)(i / n_slots), sl = (int)(i % n_slots);
  double* p = partials + (int64_t)z * pstride + (int64_t)sl * kReduceBlocks;
  double s = 0;
  for (int b = 0; b < kReduceBlocks; ++b) s += p[b];
  p[0] = s;
}

__global__ void k_param_sums(const double* partials, int64_t pstride, int n_slots, const int32_t* slot_param,
                             int n_params, const double* grad_out, int batch, double* grad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_params * batch) return;
  const int z = (int)(i / n_params), pp = (int)(i % n_params);
  double s = 0;
  for (int sl = 0; sl < n_slots; ++sl)
    if (slot_param[sl] == pp) s += partials[(int64_t)z * pstride + (int64_t)sl * kReduceBlocks];
  const double scale = grad_out ? grad_out[z] : 1.0;
  grad[(int64_t)z * n_params + pp] = scale * s;
}

hipError_t launch_gradient_reduce(hipStream_t s, const double* partials, int64_t partial_stride, int n_slots,
                                  const int32_t* slot_param, int n_params, const double* grad_out, int batch,
                                  double* grad) {
  if (n_slots > 0) {
    const int64_t n1 = (int64_t)n_slots * batch;
    hipLaunchKernelGGL(k_slot_sums, dim3((unsigned)((n1 + 127) / 128)), dim3(128), 0, s, (double*)partials,
                       partial_stride, n_slots, batch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t n2 = (int64_t)n_params * batch;
  if (n2 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_param_sums, dim3((unsigned)((n2 + 127) / 128)), dim3(128), 0, s, partials, partial_stride,
                     n_slots, slot_param, n_params, grad_out, batch, grad);
  return hipGetLastError();
}

__global__ __launch_bounds__(kRecipeThreads) void k_sweep_matrices(const Recipe* rs, int n, const RecipeOp* ops,
                                                                    const double* mats,
                                 const double* params, int64_t pstride, float2* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (i >= n) return;
  const double* p = params ? params + (int64_t)z * pstride : nullptr;
  float2* o = out + ((int64_t)z * n + i) * 16;
  if (rs[i].nq == 2) {
    c128 M[16];
    recipe_matrix_d<4>(rs[i], ops, mats, p, M);
#pragma unroll
    for (int k = 0; k < 16; ++k) o[k] = f2((float)M[k].re, (float)M[k].im);
  } else {
    c128 M[4];
    recipe_matrix_d<2>(rs[i], ops, mats, p, M);
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = f2((float)M[k].re, (float)M[k].im);
  }
}

hipError_t launch_sweep_matrices(hipStream_t s, const Recipe* recipes, int n, const RecipeOp* ops, const double* mats,
                                 const double* params, int64_t params_stride, int batch, float2* out) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sweep_matrices, dim3((n + kRecipeThreads - 1) / kRecipeThreads, batch), dim3(kRecipeThreads),
                     0, s, recipes, n, ops, mats, params, params_stride, out);
  return hipGetLastError();
}

}  // namespace tnq
