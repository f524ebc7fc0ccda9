// Internal data structures shared by the host-side network builder, planner,
// program compiler and the device runtime.
#pragma once
#include <stdint.h>

#include <memory>
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
  int32_t diag;       // the gate's matrix is diagonal
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
enum BufId { BUF_IN = 0, BUF_WS = 1, BUF_OUT = 2, BUF_AUX = 3, BUF_LDS0 = 4, BUF_LDS1 = 5 };

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
  int32_t bt_pos[kSkinnyMaxG];      // position in T of G's batch bit j
  int32_t g_unit;                   // G is a diagonal gate whose entries all have modulus one
  int32_t g_form;                   // shape of G's values that fewer multiplies serve (kForm*), from the gate kinds
};

// Shapes of a gate tensor's values, known from its gate kinds: a dense
// one-qubit matrix that is real (H, X, RY, ...) or has a real diagonal and an
// imaginary off-diagonal (RX, Y, the QAOA mixer); a diagonal whose entries are
// all +1 or -1 (Z, CZ), or all of modulus one (RZ, S, T, CPHASE, ZZPHASE).
enum GateForm { kFormGeneric = 0, kFormReal = 1, kFormRxLike = 2, kFormUnit = 3, kFormSigns = 4,
                // a group of ZZ phase gates with one angle (in a pass: a header, then its members):
                // the product of their diagonals is w^cut(x), w the phase of one differing edge and
                // cut(x) the number of member edges whose two bits differ
                kFormCount = 5, kFormCountMember = 6 };
constexpr int kCountMaxEdges = 64;   // members of one group
constexpr int kCountTabMax = 512;    // entries of a pass's power tables (w^0 .. w^E per group), staged in LDS
constexpr int kPassValMax = 640;     // a pass's gate values and power tables staged in LDS together (when they fit)
// a gathered gate value (SweepChain::vals): offset | buffer << 56, or with kValPow the
// value at offset raised to the power in bits 48..55
constexpr int64_t kValPow = (int64_t)1 << 62;
constexpr int kValExpShift = 48;

// Fused streaming of a chain of gate-sized steps on one large tensor: the
// chain is split into passes; a pass keeps a chunk of 2^l elements (the bits
// `lpos`, ascending, always including the lowest bits) in LDS and applies all
// its gates there, so each pass reads and writes the tensor once.
constexpr int kSweepMaxLocal = 12;
constexpr int kSweepMinLocal = 8;
struct SweepGateDesc {
  int32_t diag;          // 0: dense gate on n local bits (G[m][k]); 1: diagonal factor G[b] on n bits
  int32_t n;             // 1 or 2
  int32_t lidx[2];       // local bit index of bit j of the gate's index; a diagonal gate's bit outside
                         // the chunk is -(address position + 1)
  int32_t rb[2];         // dense gates: index in the segment's register bits of bit j
  int32_t unit;          // diagonal with unit-modulus entries
  int32_t g_buf;
  int32_t form;          // GateForm of the values
  int32_t voff;          // the gate's values in the chain's value table: dense (m, k) row-major, diagonal by b
  int64_t g_off;
  int32_t gidx[16];      // element of G for (m, k) (dense, m*2^n + k) or b (diagonal)
  // diagonal gates, resolved for the gate's segment: bit j of the index is register bit kreg[j]
  // (>= 0), else the thread's local bit csrc[j] (0..l-1) or the chunk base's address bit csrc[j] - 64
  int32_t kreg[2], csrc[2];
  // on the first of two to four consecutive gates on distinct register bits, in increasing bit
  // order, the mask of those bits (0: no run); the kernels apply the run as straight-line code.
  // The gates of a run are all dense one-qubit gates of one form, or all one-bit diagonal gates
  // with unit-modulus entries.  On the first of a run of diagonal gates with entries +-1 (CZ, Z)
  // and a bit in the registers, it holds instead the number of the run's gates (2 to 16)
  int32_t run_mask = 0;
};
// Inside a pass, gates run in segments: a segment names four local bits
// (`rbits`, indices into lpos) that each thread holds in registers (16
// elements per thread); its dense gates act only on those bits, its diagonal
// gates on any bits.  Between segments the chunk goes through LDS once.
// (Every field of the descriptors the pass kernels read per gate and segment
// is 32 bits wide: the kernels then fetch them with scalar loads, whereas
// narrower fields are read with vector memory loads whose latency every gate
// would wait for.)
struct SweepSegment {
  int32_t rbits[4];
  int32_t first_gate, n_gates;
  // thread index bit t -> local bit tpos[t] (the local bits outside the registers, ascending);
  // physoff[r]: LDS slot offset (padded) of the register combination r
  int32_t tpos[8];
  int32_t physoff[16];
};
struct SweepPass {
  int32_t l;
  int8_t lpos[kSweepMaxLocal];
  int32_t first_gate, n_gates;
  int32_t first_seg, n_segs;
  int32_t n_red;  // adjoint passes: gradient accumulators of the pass
  int32_t ctab_off = 0, ctab_n = 0;  // the pass's power tables in the chain's value table
  int32_t val_off = 0;               // the pass's first gate value (its values run up to ctab_off + ctab_n)
};

// Reverse sweep of the adjoint gradient in fused passes: psi and lambda
// chunks of 2^l elements stay in LDS while every gate of the pass is undone
// on both, each parametric gate first adding its chunk's share of
// Im<lambda|G|psi> to an accumulator of its own (`red`).
constexpr int kAdjMaxRed = 128;     // two per lane of a wave (the kernel's register accumulators)
constexpr int kAdjPreGates = 128;   // gates of an adjoint pass at most (the kernel stages their U entries in LDS)
struct AdjGateDesc {
  int32_t diag, n;
  int32_t lidx[2];  // as in SweepGateDesc
  int32_t rb[2];
  int32_t gate;     // index in the network's gate sweep (matrix U of the gate)
  int32_t red;      // accumulator of the pass, or -1 (no gradient term)
  int32_t slot;     // gradient-partials column, or -1
  int32_t form;     // ADJ_*: shape of the generator (dense gates) / of U (diagonal gates)
  float gen[8];     // generator G: dense 2x2 row-major, or diagonal entries (complex, re/im interleaved)
  int32_t uform;    // dense one-qubit gates: GateForm of U (kFormReal, kFormRxLike or kFormGeneric)
  int32_t kreg[2], csrc[2];  // diagonal gates, resolved for the gate's segment as in SweepGateDesc
  int32_t run_mask = 0;      // as in SweepGateDesc (the run's gates share uform)
};
// dense one-qubit generators c X or Y, real diagonal generators, diagonal
// gates whose entries are all +1 or -1 (applied as sign flips; bit b of
// `form >> 8` set: entry b is -1)
enum AdjForm { ADJ_GENERIC = 0, ADJ_GEN_X = 1, ADJ_GEN_Y = 2, ADJ_DIAG_SIGNS = 4 };
struct SweepChain {
  BufRef in, out;
  int32_t bits;
  int32_t first_pass, n_passes;
  int32_t n_steps;
  // the chain's gate values, gathered into one table before its passes (sources in the path's
  // sweep_val_src, first_val .. first_val + n_vals; the table at `vals` in the workspace)
  int32_t first_val, n_vals;
  BufRef vals;
};

struct PermuteDesc {
  BufRef in, out;
  int32_t bits;                 // total address bits
  int32_t dst[64];              // input bit p goes to output bit dst[p]
};

// Batched complex product over arbitrary bit layouts: bit j of the batch, m,
// n or k index sits at address position x_y[j] of operand x (no permute
// kernel; the product reads and writes through per-tile deposit tables).
constexpr int kGemmMaxBits = 40;
struct GemmDesc {
  BufRef a, b, c;
  int64_t batch, M, N, K;
  int32_t nbb, nbm, nbn, nbk;  // bit counts of the batch, m, n, k indices
  int32_t swapped;  // A and B are the step's second and first operands (C = B^T A^T)
  int32_t a_kfast;  // A tile loads walk k fastest (A's lowest m/k address bit is a k bit)
  int32_t b_nfast;  // B tile loads walk n fastest
  int8_t a_b[kGemmMaxBits], a_m[kGemmMaxBits], a_k[kGemmMaxBits];
  int8_t b_b[kGemmMaxBits], b_k[kGemmMaxBits], b_n[kGemmMaxBits];
  int8_t c_b[kGemmMaxBits], c_m[kGemmMaxBits], c_n[kGemmMaxBits];
  // launch shape per precision (index TN_PREC_*): tile[p] != kGemmVector is an
  // MFMA tile of kGemmTileM x kGemmTileN complex, kGemmVector the per-output
  // vector kernel; split[p] > 1 cuts K into ranges whose partial products land
  // in `tmp` and are summed.  `tmp` holds max_split copies of C.
  int32_t tile[2], split[2];
  int32_t max_split;
  BufRef tmp;
};
// tiles 0-3: real-embedding (4M) MFMA tiles; 4: vector kernel; 5-6: 3M MFMA
// tiles (FP32 only); 7: 3M, batch-packed (four batch items of at most 32 x 32
// per block, one per wave; batch of at least 4, FP32 only); 8: 3M,
// column-packed (M <= 32, four 32-column slices of N per block, one per wave;
// FP32 only)
constexpr int kGemmVector = 4;
constexpr int kGemmBatchPacked = 7;
constexpr int kGemmColumnPacked = 8;
constexpr int kGemmTiles = 9;
constexpr int kGemmTileM[kGemmTiles] = {128, 128, 64, 64, 1, 128, 64, 32, 32};
constexpr int kGemmTileN[kGemmTiles] = {64, 32, 64, 32, 1, 64, 64, 32, 128};
constexpr int kGemmMaxSplit = 8;
constexpr int kGemmBK = 16;      // complex k per staged K tile of the MFMA kernels
constexpr int kElemMaxK = 1024;  // longest K of the per-output kernel
// The table-driven per-output kernel (k_elem_group): up to kElemGroupMax
// independent products in one launch, each with a result of at most
// 2^kElemGroupOutBits elements per batch item and at most 2^kElemKBits summed
// terms.  The planner places products with results of at most 2^kElemSmallBits
// elements side by side so that they can share a launch.
constexpr int kElemGroupMax = 16;
constexpr int kElemGroupOutBits = 24;
constexpr int kElemSmallBits = 16;
constexpr int kElemKBits = 10;
// small gate-sized products (result of at most 2^kElemSkinnyBits elements)
// become per-output products, which can share a launch
constexpr int kElemSkinnyBits = 15;
// A product (bit counts of its result, of A's and B's own indices and of the
// summed index) that the default launch shape runs on the per-output kernel
// and that may share a launch with its neighbours.
inline bool elem_group_shape(int out_bits, int m_bits, int n_bits, int k_bits) {
  return out_bits <= kElemSmallBits && k_bits <= kElemKBits && (m_bits < 6 || n_bits < 5 || k_bits <= 5);
}
// default launch shape of a product (before any measurement)
void gemm_default_launch(const GemmDesc& g, int* tile, int* split);

// A small step executed inside the interpreter kernel: every operand and the
// result fit in a few KB.  C's address bit p comes from A's bit apos[p] and/or
// B's bit bpos[p] (-1: absent); summed bit j sits at A bit ka[j] and B bit kb[j].
constexpr int kSmallMaxBits = 12;
constexpr int kSmallMaxMacLog2 = 20;
constexpr int kSmallDescCache = 128;  // step descriptors staged in LDS at a time
constexpr int kSmallStage = 12288;    // operand elements staged in LDS per round (96 KB)
struct SmallStep {
  int32_t a_buf, b_buf, c_buf;  // BUF_IN / BUF_WS
  int32_t c_bits, k_bits;
  int16_t a_bits, b_bits;       // operand sizes (log2 elements)
  int64_t a_off, b_off, c_off;
  int8_t apos[kSmallMaxBits], bpos[kSmallMaxBits];
  int8_t ka[kSmallMaxBits], kb[kSmallMaxBits];
  // planned on the host: a level is run in rounds of steps whose operands fit
  // the LDS stage together; offsets of this step's operands in the stage and
  // of its first output among the round's outputs, and (on a round's first
  // step) the index, within the level's chunk, one past the round's last step
  int32_t stage_a, stage_b, out0, round_end;
  // on a round's first step: the round's work items (kSmallItem*), one per
  // thread, small_items[item0 .. item0 + n_items)
  int32_t item0, n_items, pad2[2];
};
// A work item of the interpreter: the outputs j + t 2^q (t = 0 .. 2^(c - q) - 1)
// of one step of the round with 2^c outputs, packed as step (index in the
// level's chunk, 8 bits) | j << 8 (12 bits) | q << 20 (4 bits).  The 2^q items
// of a step take interleaved outputs, so that neighbouring threads touch
// neighbouring elements.
constexpr int kSmallThreads = 1024;  // threads of an interpreter workgroup (one work list each)
constexpr int kSmallMaxItems = 2 * kSmallThreads;  // per round: at most two per thread
static_assert(sizeof(SmallStep) % 16 == 0, "SmallStep is copied in 16-byte words");

enum StepKind { SK_SKINNY = 0, SK_GEMM = 1, SK_SMALL = 2 };

// A run of outer products of a tensor with one-qubit vectors: skinny steps with
// no summed, batch or shared bits and one output bit, each on the previous
// step's result.  Each step puts its vector's bit above the bits it was given,
// so the run's result is C[m_k .. m_1 | o] = T[o] g_1[m_1] .. g_k[m_k]: one
// launch writes it, where the steps would write every intermediate.
constexpr int kOuterMax = 24;
struct OuterChain {
  BufRef t, c;
  int32_t t_bits, k;              // T has 2^t_bits elements; k vectors
  int64_t vsrc[kOuterMax][2];     // g_i[m]: element offset | buffer << 56
  double flops = 0, bytes = 0;    // per batch item, for kernel timing
};

struct StepProgram {
  int32_t kind;
  int32_t chain = -1;  // >= 0: first step of fused chain `chain`; -2: inside a chain (skipped)
  int32_t outer = -1;  // >= 0: first step of outer-product run `outer` (run in one launch); -2: inside one
  SmallStep sm;
  std::vector<PermuteDesc> pre;  // operand permutes before the product
  SkinnyDesc sk;
  GemmDesc gm[2];       // matrix product as C = A B (0) and as C = B^T A^T (1)
  int32_t orient[2];    // per precision: which of the two runs
  // steps grp_from..this one are pairwise independent and touch disjoint
  // workspace ranges where one of them writes (they may run in one launch)
  int32_t grp_from = -1;
  // a gate-sized step whose gate is one ZZ phase exp(-i t (1 - Z Z) / 2): the angle's
  // parameter index (-1: fixed angle zz_angle); -2 otherwise
  int32_t zz_param = -2;
  double zz_angle = 0;
  double flops = 0, bytes = 0;
  int64_t gemm_bmnk[4] = {0, 0, 0, 0};
};

// a product step the grouped per-output kernel can run at `precision`
inline bool elem_groupable(const StepProgram& P, int precision) {
  if (P.kind != SK_GEMM || P.chain != -1 || !P.pre.empty()) return false;
  const GemmDesc& g = P.gm[P.orient[precision]];
  return g.tile[precision] == kGemmVector && g.nbb + g.nbm + g.nbn <= kElemGroupOutBits && g.nbk <= kElemKBits;
}

// Q3.28 fixed-point mode (TN_PREC_Q3_28): every step of the path is one launch
// of a per-output product over int32 (re, im) pairs, each real product rounded
// to Q3.28 (ties to even) and every sum saturating.  Operand and result
// layouts: input tensors as the network stores them, each intermediate C-ordered
// over its modes.  Result bit j (C address bit j) sits at A bit a_o[j] and/or B
// bit b_o[j] (-1: absent); summed bit j at A bit a_k[j] and B bit b_k[j].
constexpr int kQMaxOutBits = 40;
constexpr int kQMaxKBits = 20;
struct QStep {
  int32_t a_buf, b_buf;          // BUF_IN / BUF_WS (the result is always in the workspace)
  int64_t a_off, b_off, c_off;   // complex elements from the buffer's base
  int32_t n_out, n_k;
  int8_t a_o[kQMaxOutBits], b_o[kQMaxOutBits];
  int8_t a_k[kQMaxKBits], b_k[kQMaxKBits];
};

// Index slicing: input tensor t of the sliced network (its sliced modes take
// no address bits) is gathered from the full tensor: sliced address bit j is
// full address bit keep_pos[j]; full address bit cut_pos[k] is bit cut_src[k]
// of the slice index.
constexpr int kSliceMaxKeep = 40;
constexpr int kSliceMaxCut = 16;
struct SliceTensor {
  int64_t src_off, dst_off;  // elements, in the full and in the sliced input buffer
  int32_t n_keep, n_cut;
  int8_t keep_pos[kSliceMaxKeep];
  int8_t cut_pos[kSliceMaxCut], cut_src[kSliceMaxCut];
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
  std::vector<tnq::SmallStep> small_steps;   // grouped by work list, and by level inside a list
  std::vector<int32_t> small_lists;          // list w owns levels small_lists[w] .. small_lists[w+1]-1
  std::vector<int32_t> small_levels;         // level i owns steps small_levels[i] .. small_levels[i+1]-1
  std::vector<uint32_t> small_items;         // work items of every round (see SmallStep::item0)
  int64_t small_region = 0;                  // workspace elements reserved for their results
  // runs of outer products written in one launch
  std::vector<tnq::OuterChain> outers;
  // fused streaming chains
  std::vector<tnq::SweepChain> chains;
  std::vector<tnq::SweepPass> passes;
  std::vector<tnq::SweepSegment> segments;
  std::vector<tnq::SweepGateDesc> sweep_gates;
  std::vector<int64_t> sweep_val_src;        // gate values of the chains: element offset | (buffer << 56)
  // adjoint gradient passes over the final tensor (built on first use; adj_state 1: built, -1: not possible)
  int32_t adj_state = 0;
  // the layout (labels, C order) the passes run in: the final tensor's, or the qubit order when
  // that needs fewer passes (adj_perm = 1: the state is permuted into it first)
  std::vector<int32_t> adj_bits;
  int32_t adj_perm = 0;
  std::vector<tnq::SweepPass> adj_passes;
  std::vector<tnq::SweepSegment> adj_segments;
  std::vector<tnq::AdjGateDesc> adj_gates;
  // index slicing: the program runs on `sliced_net` (the network with the modes slice_modes fixed);
  // 2^slice_bits slices, slice index bits in the order of slice_modes, each mode's bits low to high
  int32_t slice_bits = 0;
  std::shared_ptr<tn_network> sliced_net;
  std::vector<int32_t> slice_modes;
  std::vector<tnq::SliceTensor> slice_tensors;
  // Q3.28 fixed-point program (q_state 1: built; -1: a step exceeds the kernel's bit limits)
  int32_t q_state = 0;
  std::vector<tnq::QStep> q_steps;
  int64_t q_ws_elems = 0;            // per batch item
  tnq::BufRef q_final;               // the final tensor, C-ordered over q_final_modes
  std::vector<int32_t> q_final_modes;
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
tn_status compile_program(const tn_network* net, tn_path* path, const std::vector<int32_t>* final_layout = nullptr);
std::vector<int32_t> output_layout(const tn_network* net);
// fused passes of the adjoint sweep over the path's final tensor (sets path->adj_state)
void build_adjoint_plan(const tn_network* net, tn_path* path, const std::vector<int32_t>& slot_of_gate);
// moves every step that is small and depends only on inputs or such steps to the
// front; of the rest, likely per-output products that are ready together are
// placed next to each other
std::vector<int32_t> reorder_small_first(const tn_network* net, const std::vector<int32_t>& pairs, int* n_small,
                                         int64_t* small_region);
// fixedpoint.cpp: the Q3.28 program of a path (sets q_state)
void build_q328_program(const tn_network* net, tn_path* path);
// slicing.cpp: bond modes to fix so that `pairs` keeps every intermediate within 2^cap_log2 (TN_ELIMIT if
// more than max_bits address bits would be needed); the network with those modes fixed; and the gather
// tables from the full input tensors to the sliced ones
tn_status choose_slices(const tn_network* net, const std::vector<int32_t>& pairs, int cap_log2, int max_bits,
                        std::vector<int32_t>* slice_modes);
std::shared_ptr<tn_network> sliced_network(const tn_network* net, const std::vector<int32_t>& slice_modes);
tn_status slice_gather_tables(const tn_network* net, const tn_network* sliced, const std::vector<int32_t>& slice_modes,
                              std::vector<SliceTensor>* out);
// network.cpp
void network_values_host(const tn_network* net, const double* params, const uint64_t* bits, double* out);
// runtime
void device_release_network(tn_network* net);
void device_release_path(tn_path* path);
}  // namespace tnq
