// Launchers for the gfx950 kernels.  Every launcher enqueues on `stream` and
// returns hipSuccess or the launch error.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace tnq {

struct DevTensor {
  int32_t kind, recipe, qubit, pad;
  int64_t offset, size;
};

// Gate materialisation: every KET0 and GATE tensor of the network, for each
// of `batch` parameter vectors (params: [batch][params_stride] or NULL).
// q328: store Q3.28 (re, im) int32 pairs instead of complex64 (same 8 bytes per element).
hipError_t launch_materialize(hipStream_t s, const DevTensor* ts, int nt, const Recipe* recipes, const RecipeOp* ops,
                              const double* mats, const double* params, int64_t params_stride, int batch,
                              float2* in, int64_t in_bs, bool q328 = false);
// One-hot projectors P_q[s][w] = [w == bit_q(b_s)] for the last n tensors.
hipError_t launch_projectors(hipStream_t s, const uint64_t* bits, int64_t count, int n_qubits, int blog2,
                             int64_t first_offset, int batch, float2* in, int64_t in_bs, bool q328 = false);

// Q3.28 fixed point: one step (see QStep) over raw int32 pairs; and the final
// tensor F to complex64, out[o] = F[deposit(o)] with bit j of o at F bit map.a_o[j]
// (map.n_out bits; `count` outputs per batch item).
hipError_t launch_q328_step(hipStream_t s, const QStep& q, const void* a, int64_t a_bs, const void* b, int64_t b_bs,
                            void* c, int64_t c_bs, int batch);
hipError_t launch_q328_finish(hipStream_t s, const void* f, int64_t f_bs, float2* out, int64_t out_bs, int64_t count,
                              const QStep& map, int batch);

// Small-operand contraction streaming over the large operand (see SkinnyDesc).
hipError_t launch_skinny(hipStream_t s, const SkinnyDesc& d, const float2* g, int64_t g_bs, const float2* t,
                         int64_t t_bs, float2* c, int64_t c_bs, int batch, int precision);

// A run of outer products with one-qubit vectors in one launch (see OuterChain);
// the vectors' values are read from `in` or `ws` by their sources.
hipError_t launch_outer_chain(hipStream_t s, const OuterChain& oc, const float2* t, int64_t t_bs, float2* c,
                              int64_t c_bs, const float2* in, int64_t in_bs, const float2* ws, int64_t ws_bs,
                              int batch);

// Bit permutation of a 2^bits array: input bit p -> output bit dst[p].
hipError_t launch_permute(hipStream_t s, const PermuteDesc& d, const float2* in, int64_t in_bs, float2* out,
                          int64_t out_bs, int batch);

// C[b] = A[b] B[b] on complex64, FP32 accumulation: FP32 matrix cores, or the
// BF16x3 split on the bf16 matrix cores (precision TN_PREC_BF16X3).  `tile`
// (< kGemmVector: MFMA tile shape; kGemmVector: one output per thread on the
// vector ALUs) and `split` (K ranges, partials in `tmp` = [split][C], summed
// into C) choose the launch shape.
// Whether launch shape `tile` can run product d (the batch-packed tile needs
// M, N <= 32, a batch of at least 4 and tile offsets below 2^32 bytes).
bool gemm_tile_supported(const GemmDesc& d, int tile);
hipError_t launch_gemm(hipStream_t s, const GemmDesc& d, int tile, int split, const float2* a, int64_t a_bs,
                       const float2* b, int64_t b_bs, float2* c, int64_t c_bs, float2* tmp, int64_t tmp_bs, int batch,
                       int precision);

// Several independent per-output products in one launch.  Member i owns
// blocks [block0_i, block0_{i+1}); result element o (per batch item) has bit j
// at position co[j] of C and reads A at ao[j] and B at bo[j] (-1: absent),
// summed bit j at A position ak[j] and B position bk[j].
struct ElemMember {
  const float2* A;
  const float2* B;
  float2* C;
  int64_t a_bs, b_bs, c_bs;  // strides between parameter vectors
  int32_t block0;
  int32_t out_bits;  // 2^out_bits result elements per batch item
  int32_t k_bits;    // 2^k_bits summed terms
  int32_t lane_bits;  // 2^lane_bits adjacent lanes share one result's sum (set by the launcher)
  int8_t ao[kElemGroupOutBits], bo[kElemGroupOutBits], co[kElemGroupOutBits];
  int8_t ak[kElemKBits], bk[kElemKBits];
};
struct ElemGroupArgs {
  int32_t n, total_blocks;
  ElemMember m[kElemGroupMax];
};
hipError_t launch_elem_group(hipStream_t s, const ElemGroupArgs& a, int batch, int precision);
// The member for product d (orientation as given) with operands a, b and result c.
ElemMember elem_member(const GemmDesc& d, const float2* a, int64_t a_bs, const float2* b, int64_t b_bs, float2* c,
                       int64_t c_bs);

// Expectation of a diagonal Z-string observable: out[z] = sum_x |psi_z[x]|^2 D(x),
// FP64 accumulation (block partials + a fixed-order second pass).
constexpr int kMaxTerms = 128;
struct ZTerms {
  int32_t n;
  uint64_t mask[kMaxTerms];  // address-bit masks, sorted by their bits 8..11
  double coeff[kMaxTerms];
  int32_t mu_start[17];      // terms whose bits 8..11 equal mu: [mu_start[mu], mu_start[mu + 1])
};
constexpr int kReduceBlocks = 512;   // blocks of the adjoint step (one partial per block and gate)
constexpr int kExpectBlocks = 4096;  // blocks of the expectation reduction
hipError_t launch_expectation(hipStream_t s, const float2* psi, int64_t psi_bs, int64_t n_elems, const ZTerms& terms,
                              int batch, double* partial, double* out, int64_t out_stride);

// Interpreter of small steps: work list w (levels list_off[w] .. list_off[w+1]-1,
// level i = steps level_off[i] .. level_off[i+1]-1, each depending only on
// inputs or on earlier levels of the same list) runs in workgroup (w, batch item);
// items: the rounds' work items (SmallStep::item0).
hipError_t launch_small_steps(hipStream_t s, const SmallStep* steps, const int32_t* list_off,
                              const int32_t* level_off, const uint32_t* items, int n_lists, float2* in,
                              int64_t in_bs, float2* ws, int64_t ws_bs, int batch, int precision);

// One fused streaming pass over a 2^bits tensor (see SweepPass); vals: the
// chain's gate values gathered by launch_gather_vals.
hipError_t launch_sweep_pass(hipStream_t s, const SweepPass& ps, int bits, const SweepGateDesc* gates_dev,
                             const SweepSegment* segs_dev, const float2* in, int64_t in_bs, float2* out,
                             int64_t out_bs, const float2* vals, int64_t vals_bs, int batch, int precision);
// out[z][i] = value i of a chain's table: src[i] = element offset | (BUF_IN or BUF_WS) << 56.
hipError_t launch_gather_vals(hipStream_t s, const int64_t* src, int n, const float2* IN, int64_t in_bs,
                              const float2* WS, int64_t ws_bs, float2* out, int64_t out_bs, int batch);

// Index slicing: the sliced input tensors of slice `slice` from the full ones
// (see SliceTensor), and acc = src (first != 0) or acc += src over n elements.
hipError_t launch_slice_gather(hipStream_t s, const SliceTensor* ts, int nt, const float2* full, int64_t full_bs,
                               float2* sl, int64_t sl_bs, int64_t slice, int batch);
hipError_t launch_accumulate(hipStream_t s, const float2* src, int64_t src_bs, float2* acc, int64_t acc_bs, int64_t n,
                             int first, int batch);

// Contiguous copy of `n` complex64 per batch item.
hipError_t launch_copy(hipStream_t s, const float2* in, int64_t in_bs, float2* out, int64_t out_bs, int64_t n,
                       int batch);

// ---- adjoint sweep
struct SweepArgs {
  int32_t nq;
  int32_t pos[2];      // address-bit positions of the gate's qubits (q[0], q[1])
  int32_t gen;         // GenKind of the gate (GEN_NONE: no gradient term)
  int32_t slot;        // column of the gradient-partials table for this gate (or -1)
};
// lambda_z[x] = D(x) psi_z[x]
hipError_t launch_apply_diag_obs(hipStream_t s, const float2* psi, int64_t psi_bs, float2* lam, int64_t lam_bs,
                                 int64_t n_elems, const ZTerms& terms, int batch);
// one reverse step: g = 2 Im<lam|G|psi> (partials), then psi <- U^dagger psi, lam <- U^dagger lam, the
// products of the un-applied gates in `precision` (the gradient terms in FP32, summed in FP64).
// U: complex64 [batch][u_bs] matrix (2x2 or 4x4, row-major).
hipError_t launch_adjoint_step(hipStream_t s, const SweepArgs& a, const float2* u, int64_t u_bs, float2* psi,
                               int64_t psi_bs, float2* lam, int64_t lam_bs, int64_t n_elems, int batch,
                               double* partials, int64_t partial_stride, int precision);
// One fused pass of the reverse sweep over psi and lambda (2^bits elements
// each, per parameter vector): for every gate of the pass, in order, its
// gradient term (if any) into partials[z][slot][block], then both states
// undone by U^dagger.  U: [batch][u_bs] matrices, 16 complex64 per gate.
// Grid: kReduceBlocks blocks per parameter vector, each taking chunks in turn.
hipError_t launch_adjoint_pass(hipStream_t s, const SweepPass& ps, int bits, const AdjGateDesc* gates_dev,
                               const SweepSegment* segs_dev, const float2* u, int64_t u_bs, float2* psi,
                               int64_t psi_bs, float2* lam, int64_t lam_bs, int batch, double* partials,
                               int64_t partial_stride, int precision);
// grad[z][p] = scale_z * sum over slots with param p and blocks of partials
hipError_t launch_gradient_reduce(hipStream_t s, const double* partials, int64_t partial_stride, int n_slots,
                                  const int32_t* slot_param, int n_params, const double* grad_out, int batch,
                                  double* grad);
// sweep gate matrices: recipe r of the sweep -> [batch][n_sweep][16] complex64
hipError_t launch_sweep_matrices(hipStream_t s, const Recipe* recipes, int n, const RecipeOp* ops, const double* mats,
                                 const double* params, int64_t params_stride, int batch, float2* out);

}  // namespace tnq
