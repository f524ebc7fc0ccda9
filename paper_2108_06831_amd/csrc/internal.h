// Internal data structures shared by the host-side network builder, planner,
// program compiler and the device runtime.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "gates.h"
#include "tn.h"

namespace tnq {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
tn_status set_error(tn_status s, const std::string& msg);
void clear_error();

// ---------------------------------------------------------------------------
// Network
// ---------------------------------------------------------------------------
enum TensorKind { TK_GATE = 0, TK_KET0 = 1, TK_PROJ = 2 };

struct TensorDef {
  std::vector<int32_t> modes;  // C order
  int32_t kind;                // TensorKind
  int32_t recipe;              // TK_GATE: index into recipes
  int32_t qubit;               // TK_KET0 / TK_PROJ
  int64_t size;                // elements
  int64_t offset;              // element offset in the per-batch input buffer
};

// One gate of the original (unfused) circuit, as the adjoint sweep needs it:
// U3 gates that read parameters are expanded into RZ RY RZ (up to a global
// phase, which no expectation sees).
struct SweepGate {
  int32_t nq;
  int32_t q[2];
  int32_t recipe;     // a one-op recipe giving the gate's matrix
  int32_t gen;        // generator kind for parametric gates (GEN_*), GEN_NONE otherwise
  int32_t param;      // parameter index, or -1
};

enum GenKind { GEN_NONE = 0, GEN_X_HALF, GEN_Y_HALF, GEN_Z_HALF, GEN_X, GEN_ZZ_PHASE, GEN_CPHASE };

}  // namespace tnq

struct tn_network {
  int32_t n_qubits = 0;
  int32_t n_params = 0;
  int32_t output_kind = TN_OUT_STATEVECTOR;
  int32_t flags = 0;
  int64_t n_bitstrings = 0;
  int32_t batch_log2 = 0;      // log2 of the padded bitstring batch (AMPLITUDES)
  int32_t batch_mode = -1;     // the hyper batch mode (AMPLITUDES)
  std::vector<int32_t> mode_log2;  // per mode: log2(extent)
  std::vector<tnq::TensorDef> tensors;
  std::vector<int32_t> output_modes;
  std::vector<int32_t> wire_final;  // per qubit: mode of its output leg
  std::vector<tnq::Recipe> recipes;
  std::vector<tnq::RecipeOp> ops;
  std::vector<double> matrices;      // 32 doubles per explicit matrix
  int64_t input_elems = 0;           // per batch item
  // adjoint sweep description (unfused gates, circuit order)
  std::vector<tnq::SweepGate> sweep;
  std::vector<tnq::Recipe> sweep_recipes;
  std::vector<tnq::RecipeOp> sweep_ops;
  bool has_matrix_param = false;
  // device-side copies (owned, created lazily)
  void* dev = nullptr;
};

namespace tnq {

// ---------------------------------------------------------------------------
// Compiled program
// ---------------------------------------------------------------------------
enum BufId { BUF_IN = 0, BUF_WS = 1, BUF_OUT = 2, BUF_AUX = 3 };

struct BufRef {
  int32_t buf = BUF_WS;
  int64_t off = 0;           // elements (complex64) from the buffer's base
  int64_t batch_stride = 0;  // elements between consecutive parameter vectors
};

constexpr int kSkinnyMaxK = 4;  // at most 2^4 summed elements per output
constexpr int kSkinnyMaxM = 4;  // at most 2^4 outputs per thread
constexpr int kSkinnyMaxG = 8;  // small operand of at most 2^8 elements

struct SkinnyDesc {
  BufRef g, t, c;
  int32_t t_bits;         // address bits of T
  int32_t nk, nm, nb;     // summed bits, output bits of G, batch bits shared by G and T
  int32_t k_pos[kSkinnyMaxK];       // ascending positions of the summed bits in T
  int32_t b_pos[kSkinnyMaxG];       // position, in the outer index, of G's batch bit j
  int32_t c_mode;                   // 0: C keeps T's layout with M bits at the K positions; 1: C = [M | outer]
  int64_t kofs[1 << kSkinnyMaxK];   // offset in T of summed index k
  int64_t mofs[1 << kSkinnyMaxM];   // offset in C of output index m
  int32_t gidx[1 << kSkinnyMaxG];   // G element of (b, m, k), b slowest
};

struct PermuteDesc {
  BufRef in, out;
  int32_t bits;                 // total address bits
  int32_t dst[64];              // input bit p goes to output bit dst[p]
};

struct GemmDesc {
  BufRef a, b, c;
  int64_t batch, M, N, K;
  int32_t a_kfast;  // A stored [batch][M][K] (1) or [batch][K][M] (0)
  int32_t b_nfast;  // B stored [batch][K][N] (1) or [batch][N][K] (0)
};

// A small step executed inside the interpreter kernel: every operand and the
// result fit in a few KB.  C's address bit p comes from A's bit apos[p] and/or
// B's bit bpos[p] (-1: absent); summed bit j sits at A bit ka[j] and B bit kb[j].
constexpr int kSmallMaxBits = 12;
constexpr int kSmallMaxMacLog2 = 20;
struct SmallStep {
  int32_t a_buf, b_buf, c_buf;
  int32_t c_bits, k_bits, pad;
  int64_t a_off, b_off, c_off;
  int8_t apos[kSmallMaxBits], bpos[kSmallMaxBits];
  int8_t ka[kSmallMaxBits], kb[kSmallMaxBits];
};

enum StepKind { SK_SKINNY = 0, SK_GEMM = 1, SK_SMALL = 2 };

struct StepProgram {
  int32_t kind;
  SmallStep sm;
  std::vector<PermuteDesc> pre;  // operand permutes before the product
  SkinnyDesc sk;
  GemmDesc gm;
  double flops = 0, bytes = 0;
  int64_t gemm_bmnk[4] = {0, 0, 0, 0};
};

}  // namespace tnq

struct tn_path {
  std::vector<int32_t> pairs;            // 2 per step
  std::vector<std::vector<int32_t>> step_modes;  // logical modes of each result (memory order)
  std::vector<tnq::StepProgram> steps;
  // layout of the final tensor: bit labels (mode*64 + bit), most significant first
  std::vector<int32_t> final_bits;
  tnq::BufRef final_ref;
  int64_t final_elems = 0;
  int64_t ws_elems = 0;  // per batch item (complex64 elements)
  int32_t n_inputs = 0;
  // leading steps run by the interpreter kernel: independent sub-trees, one work list each
  int32_t n_small = 0;
  std::vector<tnq::SmallStep> small_steps;   // grouped by work list
  std::vector<int32_t> small_lists;          // offsets into small_steps, size n_lists + 1
  int64_t small_region = 0;                  // workspace elements reserved for their results
  tn_path_stats stats{};
  void* dev = nullptr;   // device-side cache
};

namespace tnq {
// planner.cpp
tn_status plan_order(const tn_network* net, const tn_plan_opts& opts, std::vector<int32_t>& pairs,
                     double* max_log2_out, double alpha = 1.0, double temp = 0.0, uint64_t seed = 0);
uint64_t splitmix(uint64_t& s);
double modeled_seconds(const tn_path* path);
// program.cpp
tn_status compile_program(const tn_network* net, tn_path* path);
// moves every step that is small and depends only on inputs or such steps to the front
std::vector<int32_t> reorder_small_first(const tn_network* net, const std::vector<int32_t>& pairs, int* n_small,
                                         int64_t* small_region);
// network.cpp
void network_values_host(const tn_network* net, const double* params, const uint64_t* bits, double* out);
// runtime
void device_release_network(tn_network* net);
void device_release_path(tn_path* path);
}  // namespace tnq
