/*
 * tn.h -- C ABI of the tensor-network quantum-circuit contraction library
 * (gfx950 / MI355X).
 *
 * The method (Sec. 2.2.3 of "Tensor Networks for Simulating Quantum Circuits
 * on FPGAs"): write a circuit as a network of low-order tensors (qubit state
 * vectors and gate tensors, Sec. 2.2.2, eq. (2.3)), choose a contraction
 * order (Sec. 2.2.3; the order is a free hyperparameter because contraction is
 * associative), and contract the network pair by pair, each pairwise step
 * being a sum over shared indices (Sec. 2.2.1, eq. (2.2)) executed as a mode
 * permutation followed by a (batched) complex matrix product (Sec. 3, where
 * order-(p,q) tensors are turned into block-diagonal matrices -- a batched
 * matrix product -- before being multiplied).  Closing the network with the
 * tensor of a final basis state gives that state's amplitude (Sec. 2.2.3).
 *
 * Conventions
 *  - Qubit 0 is the most significant bit of a basis-state index (Sec. 2.1:
 *    the first Kronecker factor is the most significant).  A bitstring b
 *    holds qubit q in bit (n-1-q).
 *  - A gate acts as psi' = U psi (upper index = row = output, Sec. 2.2.1).  A
 *    two-qubit gate on (a, b) is U[2 o_a + o_b][2 i_a + i_b]; its tensor has
 *    modes (o_a, o_b, i_a, i_b) in C order.
 *  - Complex data are complex64: interleaved (re, im) float32, 8 bytes per
 *    element, the layout of torch.complex64.  Tensors are C-ordered over
 *    their mode lists.  Every mode extent is a power of two.
 *  - Contraction is bilinear: no operand is conjugated (Sec. 2.2.1).
 *
 * Memory and streams
 *  - tn_network / tn_path handles are owned by the library (host memory and
 *    small device buffers for gate recipes, allocated on first use on the
 *    device that is current at that time).
 *  - Every other device buffer (workspace, parameters, bitstrings, outputs)
 *    is owned by the caller.  Device work is enqueued asynchronously on the
 *    caller's stream (a hipStream_t passed as void*; NULL = the null
 *    stream); the caller synchronises.
 *  - Calls that share a handle must not run concurrently from several host
 *    threads.
 *
 * Errors: every entry point returns a tn_status; tn_last_error() gives a
 * thread-local message for the last non-OK status.  On error nothing is
 * launched, except for TN_EDEVICE (a HIP runtime error), after which the
 * contents of output buffers are undefined.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TN_OK = 0,
  TN_EINVAL = 1,       /* bad argument: qubit index, mode mismatch, null pointer ... */
  TN_ENOMEM = 2,       /* caller's workspace smaller than required, or a host allocation failed */
  TN_ELIMIT = 3,       /* the plan's largest intermediate exceeds the requested cap */
  TN_EDEVICE = 4,      /* a HIP runtime error */
  TN_EUNSUPPORTED = 5  /* a valid request the library does not handle (e.g. a non power-of-two extent) */
} tn_status;

/* Arithmetic of the pairwise products.  C64: complex64 operands, FP32
 * multiply-accumulate.  BF16X3: each FP32 component is split as hi + lo in
 * bfloat16 and a*b is formed as hi*hi + hi*lo + lo*hi with FP32 accumulation
 * (split-precision emulation; storage stays complex64).  Q3_28: the paper's
 * FPGA arithmetic (Sec. 3: 32-bit fixed point, 28 bits behind the binary
 * point), read as two's-complement Q3.28: every tensor a pair of int32
 * (value = raw / 2^28), gate entries rounded once from FP64, every real
 * product rounded to nearest with ties to even, every sum saturating; each step
 * of the path one per-output product on the vector ALUs (an error-study mode,
 * tn_contract_path and tn_amplitudes only; the output is converted to
 * complex64; TN_EUNSUPPORTED elsewhere, or for a step wider than 2^40 results
 * or 2^20 summed terms). */
typedef enum { TN_PREC_C64 = 0, TN_PREC_BF16X3 = 1, TN_PREC_Q3_28 = 2 } tn_precision;

/* What closes the network (Sec. 2.2.3). */
typedef enum {
  TN_OUT_STATEVECTOR = 0, /* open output legs: the full 2^n state, qubit order */
  TN_OUT_AMPLITUDES = 1   /* one projector <b_s| per qubit sharing a batch index s */
} tn_output_kind;

/* Gate kinds (matrix definitions in the implementation's gate header):
 *   H, X, Y, Z, S = diag(1,i), T = diag(1,e^{i pi/4}),
 *   SX/SY/SW: principal square roots ((1+i)I + (1-i)P)/2 of X, Y, W=(X+Y)/sqrt2,
 *   RX/RY/RZ(t) = exp(-i t P/2),
 *   U3(t,f,l) = [[cos t/2, -e^{il} sin t/2], [e^{if} sin t/2, e^{i(f+l)} cos t/2]],
 *   MIXER(b) = exp(-i b X)  (QAOA mixer),
 *   CZ, CNOT (control = first qubit), SWAP,
 *   CPHASE(l) = diag(1,1,1,e^{il}),
 *   ZZPHASE(g) = exp(-i g (1 - Z Z)/2) = diag(1,e^{-ig},e^{-ig},1)  (QAOA phase separator),
 *   MATRIX1 / MATRIX2: explicit 2x2 / 4x4 matrices. */
typedef enum {
  TN_GATE_H = 1, TN_GATE_X, TN_GATE_Y, TN_GATE_Z, TN_GATE_S, TN_GATE_T,
  TN_GATE_SX, TN_GATE_SY, TN_GATE_SW,
  TN_GATE_RX, TN_GATE_RY, TN_GATE_RZ, TN_GATE_U3, TN_GATE_MIXER,
  TN_GATE_CZ, TN_GATE_CNOT, TN_GATE_SWAP, TN_GATE_CPHASE, TN_GATE_ZZPHASE,
  TN_GATE_MATRIX1, TN_GATE_MATRIX2
} tn_gate_kind;

typedef struct {
  int32_t kind;          /* tn_gate_kind */
  int32_t q[2];          /* q[0] (and q[1] for two-qubit gates), 0 <= q < n_qubits */
  double angle[3];       /* fixed angles (RX/RY/RZ/MIXER/CPHASE/ZZPHASE: angle[0]; U3: all three) */
  int32_t param[3];      /* -1: use angle[i]; >= 0: angle i is params[param[i]] at contraction time */
  const double* matrix;  /* MATRIX1/MATRIX2: host, row-major complex128 (re,im) pairs; copied. Else NULL */
} tn_gate;

/* Diagonal observable D = sum_t coeff[t] prod_{q in mask t} Z_q (host arrays,
 * z_mask bit n-1-q selects qubit q; mask 0 is the identity).  MaxCut's
 * C = sum_(u,v) (1 - Z_u Z_v)/2 is one such sum. */
typedef struct {
  int32_t n_terms;
  const uint64_t* z_mask;
  const double* coeff;
} tn_observable;

typedef enum {
  TN_PATH_GREEDY = 0,     /* size-minimising greedy (default) */
  TN_PATH_SEQUENTIAL = 1, /* input tensors in network order (gate-by-gate state vector) */
  TN_PATH_RANDOM = 2,     /* a seeded random connected order (for testing order independence) */
  TN_PATH_SEARCH = 3      /* strategy selection (Sec. 3): the greedy order, the sequential order and `trials`
                             randomised greedy orders (objective |C| - alpha(|A|+|B|) with Gumbel noise, alpha
                             and the noise scale drawn per trial), each compiled and scored by a model of its
                             run time on the GPU; the fastest order within the intermediate cap is kept */
} tn_path_kind;

typedef struct {
  int32_t kind;                  /* tn_path_kind */
  int32_t max_log2_intermediate; /* TN_ELIMIT if an intermediate exceeds 2^this elements; <= 0: 40 */
  uint64_t seed;                 /* TN_PATH_RANDOM and TN_PATH_SEARCH */
  int32_t trials;                /* TN_PATH_SEARCH: randomised trials; <= 0: 64 */
  int32_t max_slice_bits;        /* index slicing: when no order of `kind` keeps every intermediate within
                                    the cap, fix the values of bond indices of at most this many address bits
                                    in total (2^bits slices, contracted one after another and summed);
                                    0: never slice (TN_ELIMIT instead) */
} tn_plan_opts;

typedef struct {
  double flops;                  /* sum over steps of 8 * batch * M * N * K (complex multiply-add = 8 flops) */
  double bytes;                  /* sum over steps of 8 (|A| + |B| + |C|) plus 16 |T| per executed permute */
  double max_intermediate_elems; /* largest intermediate, elements */
  double large_step_flops;       /* flops of the steps with >= 1e9 flops and >= 40 flop/byte */
  double plan_seconds;           /* host time spent planning */
  double modeled_seconds;        /* the planner's model of the program's GPU run time */
  int32_t n_steps;
  int32_t n_permutes;            /* explicit permute launches in the compiled program */
  int32_t n_gemm_steps;          /* steps executed by the MFMA matrix-product kernel */
  int32_t n_skinny_steps;        /* steps executed by the small-operand streaming kernel */
  int32_t n_small_steps;         /* leading small steps run together by one interpreter launch */
  int32_t n_small_lists;         /* independent work lists of that launch (one workgroup each) */
  int32_t n_sweep_steps;         /* gate-sized steps on one large tensor executed by fused streaming passes */
  int32_t n_sweep_passes;        /* those passes (each reads and writes the tensor once) */
  int32_t n_product_launches;    /* launches of the steps outside the interpreter and the fused passes, with
                                    the default launch shapes in complex64: independent per-output products
                                    that follow each other share a launch */
  int32_t n_slice_bits;          /* address bits of the sliced bond indices: 2^n_slice_bits slices (0: none);
                                    flops, bytes and max_intermediate_elems are per slice */
  int32_t n_sweep_gate_runs;     /* runs of two to four gates on distinct register bits of a segment (dense
                                    one-qubit gates of one form, or one-bit unit diagonals) that the fused
                                    passes apply as straight-line code (their gates are among n_sweep_steps) */
} tn_path_stats;

typedef struct tn_network tn_network;
typedef struct tn_path tn_path;

/* Flags for tn_build_network. */
#define TN_FUSE_2Q 1 /* pre-contract each run of one-qubit gates into the adjacent two-qubit gate (Sec. 3) */
#define TN_FUSE_SPLIT 2 /* with TN_FUSE_2Q: keep a fused block whose two-qubit gate is block-diagonal in one
                           qubit's value (CZ, CNOT, CPHASE, ZZPHASE, ...) in its exact operator-Schmidt form,
                           two 3-leg tensors joined by a bond of extent 2, so that orders can cut through it */

/*
 * Circuit -> tensor network (Sec. 2.2.2-2.2.3; the "pre-contract the first
 * tensors" step of Sec. 3 is TN_FUSE_2Q).  One |0> vector per qubit, one
 * tensor per gate (diagonal gates become tensors on the wire's hyper-index,
 * dense gates tensors with separate input and output modes), and the
 * output: open legs, or for TN_OUT_AMPLITUDES one projector per qubit on a
 * batch index of extent n_bitstrings rounded up to a power of two.
 *   n_qubits 1..62; gates: host array of n_gates; n_params: length of the
 *   parameter vector that param[] indexes.
 * Returns TN_EINVAL for a bad qubit index, equal qubits in a two-qubit gate, a
 * parameter index out of range or an unknown kind.  *net_out owned by the
 * caller, release with tn_network_destroy.  Host only: no device call.
 */
tn_status tn_build_network(int32_t n_qubits, const tn_gate* gates, int32_t n_gates, int32_t n_params,
                           int32_t output_kind, int64_t n_bitstrings, int32_t flags, tn_network** net_out);
void tn_network_destroy(tn_network* net);

/* Introspection (host only).  Tensors are numbered 0..n_tensors-1 in network
 * order; modes 0..n_modes-1.  Arrays are caller-allocated with room for
 * TN_MAX_RANK entries. */
#define TN_MAX_RANK 64
tn_status tn_network_info(const tn_network* net, int32_t* n_tensors, int32_t* n_modes, int32_t* n_qubits,
                          int32_t* n_output_modes);
tn_status tn_network_tensor(const tn_network* net, int32_t t, int32_t* rank, int32_t* modes, int64_t* extents);
tn_status tn_network_output(const tn_network* net, int32_t* modes, int64_t* extents);
/* FP64 host values of every input tensor for one parameter vector (params:
 * host, n_params doubles or NULL) and bitstrings (host, AMPLITUDES only):
 * complex128 pairs, tensors concatenated in network order.  Used to check the
 * network itself; the device path materialises tensors on the GPU. */
tn_status tn_network_values(const tn_network* net, const double* params, const uint64_t* bitstrings,
                            double* out, int64_t out_len_doubles);

/*
 * Index slicing (opts.max_slice_bits > 0; Sec. 2.2.3: the order is a free
 * hyperparameter, and Sec. 3 names the size of the intermediates as the
 * binding constraint).  When no order fits the cap, bond indices (modes that
 * are not outputs) are chosen greedily -- each time the index whose removal
 * most reduces the largest intermediate of an uncapped greedy order -- until
 * the order fits; the sliced network (those indices fixed) is planned again
 * under the cap.  A sum over a bond index is the sum of the contractions with
 * that index fixed to each value, so the 2^bits slices are contracted one
 * after another and their results summed.  tn_contract_path, tn_amplitudes
 * and tn_expectation run sliced paths; tn_backward, tn_autotune, the Q3.28
 * mode and tn_contract_path_noalloc return TN_EUNSUPPORTED for them.
 *
 * Contraction order (Sec. 2.2.3 and Sec. 3: greedy search over pairwise
 * contractions).  Greedy: among pairs of live tensors that share a mode,
 * contract the pair minimising |C| - |A| - |B| (elements); ties by smaller |C|,
 * then fewer flops, then smaller (min id, max id).  A mode is summed only when
 * no other live tensor and no output holds it (hyper-indices stay).  If no
 * pair shares a mode, the two smallest tensors are joined by an outer
 * product.  Also compiles the executable program (mode layouts, permutes,
 * kernel choice, workspace offsets).  Host only.
 *   stats_out may be NULL.  *path_out released with tn_path_destroy.
 */
tn_status tn_plan_path(const tn_network* net, const tn_plan_opts* opts, tn_path** path_out,
                       tn_path_stats* stats_out);
void tn_path_destroy(tn_path* path);
/* SSA pairs: step s contracts ids pairs[2s], pairs[2s+1] into id n_tensors+s. */
tn_status tn_path_pairs(const tn_path* path, int32_t* n_steps, int32_t* pairs, int32_t capacity);
/* Sliced bond modes of the path (index slicing; none for an unsliced path):
 * *n_modes of them, written to modes[0..capacity).  Slice number sigma fixes
 * the sliced modes' indices to sigma's bits, the modes in this order and each
 * mode's bits from least significant up.  The pairs and step modes above are
 * those of the sliced network, whose tensors lack these modes. */
tn_status tn_path_slices(const tn_path* path, int32_t* n_modes, int32_t* modes, int32_t capacity);
/* Modes of the tensor produced by step s (C order, as laid out in memory),
 * and the step's GEMM view. kind: 0 = streaming small-operand kernel,
 * 1 = MFMA matrix product, 2 = interpreter of small steps. */
tn_status tn_path_step(const tn_path* path, int32_t s, int32_t* rank, int32_t* modes, int64_t* gemm_bmnk,
                       int32_t* kind);

/* Device workspace needed by tn_contract_path / tn_amplitudes /
 * tn_expectation / tn_backward for `batch` parameter vectors (bytes). */
size_t tn_workspace_bytes(const tn_network* net, const tn_path* path, int32_t batch);

/*
 * Contract the network along the path on the GPU (TN_OUT_STATEVECTOR): the
 * open-legged network of Sec. 2.2.2 (eq. (2.3): the state is the network of
 * the |0> vectors and the gate tensors with the output legs left open),
 * contracted pair by pair along the order (Sec. 2.2.3), each pairwise step a
 * sum over shared indices (eq. (2.2)) run as a matrix product (Sec. 3, Sec. 5).
 *   params_dev: device, [batch][n_params] float64 (NULL if n_params == 0);
 *   workspace_dev: device, >= tn_workspace_bytes(net, path, batch) bytes;
 *   out_dev: device, [batch][2^n] complex64 in qubit order (qubit 0 = MSB).
 * Gate tensors are materialised on the device from their angles in FP64 and
 * rounded once to complex64.  TN_ENOMEM if the workspace is too small.
 */
tn_status tn_contract_path(void* stream, int32_t precision, tn_network* net, tn_path* path,
                           const double* params_dev, int32_t batch, void* workspace_dev, size_t workspace_bytes,
                           void* out_dev);

/*
 * tn_contract_path without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same contraction and kernels as
 * tn_contract_path, with the workspace in a static device array of
 * TN_NOALLOC_SCRATCH_BYTES per GPU (held by each GPU the library runs on until
 * the process ends) instead of a caller's buffer.  The caller still passes the
 * parameters and the output.
 *   Preconditions: tn_contract_path has run once with this network and path
 *   on the current device (it creates their device tables; TN_EINVAL
 *   otherwise).  TN_ENOMEM if tn_workspace_bytes(net, path, batch) exceeds
 *   TN_NOALLOC_SCRATCH_BYTES.  Kernel timing (tn_profile_*) is not recorded.
 *   Calls no hipMalloc/hipFree.  Every call on one GPU shares that GPU's array
 *   and leaves its contents behind (nothing in it needs to start at zero):
 *   calls that overlap on one GPU (concurrent streams or threads) race.
 */
#define TN_NOALLOC_SCRATCH_BYTES (64u << 20)
tn_status tn_contract_path_noalloc(void* stream, int32_t precision, tn_network* net, tn_path* path,
                                   const double* params_dev, int32_t batch, void* out_dev);

/*
 * Amplitudes <b_s|U|0> for a batch of bitstrings (TN_OUT_AMPLITUDES network,
 * Sec. 2.2.3: close the network with the final basis states).
 *   bitstrings_dev: device uint64[count], count <= the network's n_bitstrings;
 *   qubit q is bit n-1-q and bits n..63 are ignored (b and b + k 2^n give the
 *   same amplitude); the batch slots count..padded-1 are contracted with the
 *   all-zeros bitstring and not returned;
 *   out_dev: device complex64[count].
 */
tn_status tn_amplitudes(void* stream, int32_t precision, tn_network* net, tn_path* path, const double* params_dev,
                        const uint64_t* bitstrings_dev, int64_t count, void* workspace_dev, size_t workspace_bytes,
                        void* out_dev);

/*
 * Expectations <psi|D|psi> of diagonal observables for several circuits
 * (TN_OUT_STATEVECTOR networks) and parameter batches in one call; the sum
 * over basis states accumulates in FP64.  Each state is the contraction of
 * the open-legged network of Sec. 2.2.2 (eq. (2.3)) along its order (Sec.
 * 2.2.3); the bra is the complex conjugate of the ket (only bras conjugate,
 * Sec. 2.2.1), and a diagonal D only weights |psi_x|^2 per basis state.
 *   nets/paths/obs: host arrays of n_circuits;
 *   params_dev: host array of n_circuits device pointers, each [batch][n_params_c] float64 (or NULL);
 *   workspace_dev: device, >= tn_expectation_workspace_bytes(...) (up to twelve circuits run
 *     at once, each in its own slot of the workspace);
 *   out_dev: device float64[n_circuits][batch].
 * The circuits are independent: the library spreads them over the caller's
 * stream and up to eleven streams of its own, which wait for the caller's
 * stream at the start and which the caller's stream waits for at the end, so
 * the work is ordered on `stream` as one call (and a capture of `stream`
 * records all of it).  With kernel timing on (tn_profile_enable) every circuit
 * runs on `stream`.
 */
size_t tn_expectation_workspace_bytes(tn_network* const* nets, tn_path* const* paths, int32_t n_circuits,
                                      int32_t batch);
tn_status tn_expectation(void* stream, int32_t precision, tn_network* const* nets, tn_path* const* paths,
                         int32_t n_circuits, const double* const* params_dev, int32_t batch,
                         const tn_observable* obs, void* workspace_dev, size_t workspace_bytes, double* out_dev);

/*
 * Value and gradient of E(theta) = <psi(theta)|D|psi(theta)> for `batch`
 * parameter vectors by the adjoint method: contract the network forward to
 * psi, set lambda = D psi, then sweep the gates in reverse, un-applying each
 * gate U_j from psi and lambda and accumulating dE/dtheta = Im<lambda|G|psi>
 * for each parametric gate exp(-i theta G) in FP64 (summed over every gate
 * that reads the parameter).  The states are the contractions of Sec. 2.2.2
 * (eq. (2.3)); the derivative itself is not in the paper.  `precision`
 * selects the products of both the forward contraction and the un-applied
 * gates of the reverse sweep; the gradient terms are formed in FP32 and
 * summed in FP64 in either mode.
 *   grad_out_dev: device float64[batch] (dL/dE, NULL = ones);
 *   value_dev: device float64[batch]; grad_dev: device float64[batch][n_params].
 * Workspace: tn_backward_workspace_bytes.  TN_EUNSUPPORTED for a parametric
 * gate whose generator the library does not know (MATRIX gates are fixed).
 */
size_t tn_backward_workspace_bytes(const tn_network* net, const tn_path* path, int32_t batch);
tn_status tn_backward(void* stream, int32_t precision, tn_network* net, tn_path* path, const double* params_dev,
                      int32_t batch, const tn_observable* obs, const double* grad_out_dev, void* workspace_dev,
                      size_t workspace_bytes, double* value_dev, double* grad_dev);

/*
 * One pairwise contraction C = sum over contracted modes of A * B (Sec. 2.2.1,
 * eq. (2.2)).  A mode present in A and B and in C is a batch (hyper) mode; in
 * A and B but not in C it is summed; in one operand only it must be in C.
 *   a, b, c: device complex64, C-ordered over modes_*; ext_*: extents
 *   (powers of two; a mode shared by operands has equal extents).
 *   workspace_dev: device, >= tn_contract_pair_workspace_bytes(...) (may be
 *   NULL when that is 0); used for operand permutations.
 * TN_EINVAL on a mode mismatch; TN_EUNSUPPORTED for a non power-of-two extent.
 */
size_t tn_contract_pair_workspace_bytes(int32_t rank_a, const int32_t* modes_a, const int64_t* ext_a,
                                        int32_t rank_b, const int32_t* modes_b, const int64_t* ext_b,
                                        int32_t rank_c, const int32_t* modes_c);
tn_status tn_contract_pair(void* stream, int32_t precision, const void* a, int32_t rank_a, const int32_t* modes_a,
                           const int64_t* ext_a, const void* b, int32_t rank_b, const int32_t* modes_b,
                           const int64_t* ext_b, void* c, int32_t rank_c, const int32_t* modes_c,
                           void* workspace_dev, size_t workspace_bytes);

/*
 * HIP graphs.  tn_graph_begin starts capturing `stream` (not the null stream);
 * every entry point called on that stream by this thread until tn_graph_end
 * is recorded instead of run, and tn_graph_end instantiates the recording.
 * tn_graph_launch replays all of it as one graph launch, with the device
 * pointers given at capture time (update params, inputs and bitstrings in
 * place between launches).  Device-side tables of a network and a path are
 * created on their first use and cannot be created during a capture: run the
 * calls once before capturing them (TN_EDEVICE otherwise).  Kernel timing
 * must be off while capturing.  The library's kernels clear no memory with
 * memset nodes, so replays are self-contained.
 */
typedef struct tn_graph tn_graph;
tn_status tn_graph_begin(void* stream);
tn_status tn_graph_end(void* stream, tn_graph** graph_out);
tn_status tn_graph_launch(const tn_graph* graph, void* stream);
void tn_graph_destroy(tn_graph* graph);

/*
 * Autotuner for the launch shapes of the matrix-product steps.
 * Runs the path's steps once on `stream` (gate tensors from params_dev, for
 * `batch` parameter vectors; amplitude projectors are left zero), then for
 * every matrix-product step times each candidate launch shape -- an MFMA tile
 * of 128x64, 128x32, 64x64 or 64x32 complex (4M form) or, for TN_PREC_C64,
 * 128x64 or 64x64 in the 3M form, K cut into 1, 2, 4 or 8 ranges
 * where the step's result is small, the one-output-per-thread vector kernel
 * where K <= 1024, each for C = A B and for C = B^T A^T -- over `reps` launches (hipEvents on `stream`) and
 * keeps the fastest in the path for `precision`.  Synchronises the stream.
 * Later contractions along the path give the same results up to rounding
 * order (a K split sums partial products in another order).
 *   workspace_dev: >= tn_workspace_bytes(net, path, batch) bytes (contents
 *   overwritten);  report (may be NULL): number of product steps, steps whose
 *   shape changed, and the sum of their measured times before and after.
 */
typedef struct {
  int32_t n_products, n_changed;
  double seconds_before, seconds_after;
} tn_tune_report;
tn_status tn_autotune(void* stream, int32_t precision, tn_network* net, tn_path* path, const double* params_dev,
                      int32_t batch, void* workspace_dev, size_t workspace_bytes, int32_t reps,
                      tn_tune_report* report);
/* Launch shape of matrix-product step `step` for `precision`: read (set == 0)
 * into *tile / *split / *transposed, or replace it (set != 0) with the values
 * given, e.g. to restore shapes tuned earlier.  tile: 0..3 = MFMA tiles
 * 128x64, 128x32, 64x64, 64x32 complex in the real-embedding (4M) form;
 * 4 = vector kernel (K <= 1024 only, split 1); 5, 6 = MFMA tiles 128x64,
 * 64x64 in the three-product (3M) form (TN_PREC_C64 only); 7 = 3M,
 * batch-packed: four batch items of at most 32 x 32 per workgroup, one per
 * wave (TN_PREC_C64, M and N <= 32, a batch of at least 4 only); 8 = 3M,
 * column-packed: M <= 32 and four 32-column slices of N per workgroup, one
 * per wave (TN_PREC_C64, N >= 64 only).
 * split: 1, 2, 4 or 8, dividing K, at most the step's reserved
 * maximum.  transposed: 0 computes C = A B, 1 computes C = B^T A^T (operands
 * trade places; same result layout).  TN_EINVAL for a step that is not a
 * matrix product or an invalid shape. */
tn_status tn_path_gemm_config(tn_path* path, int32_t step, int32_t precision, int32_t* tile, int32_t* split,
                              int32_t* transposed, int32_t set);

/*
 * Kernel timing for measurement.  While enabled, the kernel launches of the
 * entry points above are bracketed by hipEvents recorded on the launch's own
 * stream, and tagged with the launch's algorithmic work: bytes that must
 * cross HBM (operands read once, result written once) and flops (8 per
 * complex multiply-add).  Within the steps of a contraction, consecutive
 * timed launches of one kind share one event pair (an event recorded between
 * two kernels idles the GPU for a few microseconds); every other launch gets a
 * pair of its own, and so does a TN_KERNEL_GEMM_LARGE product while that kind
 * is selected (it is then counted under TN_KERNEL_GEMM too if that is
 * selected).  tn_profile_read synchronises on the recorded events and returns
 * one record per kernel kind (at most `capacity`, returns the number
 * written).  Not thread-safe.
 */
typedef enum {
  TN_KERNEL_MATERIALIZE = 0, TN_KERNEL_SKINNY = 1, TN_KERNEL_PERMUTE = 2, TN_KERNEL_GEMM = 3,
  TN_KERNEL_REDUCE = 4, TN_KERNEL_COPY = 5, TN_KERNEL_ADJOINT = 6, TN_KERNEL_INTERP = 7, TN_KERNEL_SWEEP = 8,
  TN_KERNEL_GEMM_LARGE = 9, /* the subset of TN_KERNEL_GEMM launches with >= 1e9 flops and >= 40 flops per
                                algorithmic byte, counted again under this kind (same events) */
  TN_KERNEL_KINDS = 10
} tn_kernel_kind;
typedef struct {
  int32_t kind;       /* tn_kernel_kind */
  int64_t launches;
  double seconds;     /* sum of event-measured durations (of single launches or runs of launches) */
  double bytes;       /* sum of algorithmic bytes */
  double flops;       /* sum of algorithmic flops */
} tn_kernel_profile;
tn_status tn_profile_enable(int32_t on);
/* Kernel kinds timed while timing is enabled: bit k for tn_kernel_kind k
 * (default: all).  Every event pair costs a few microseconds of queue time,
 * so a measurement of one kind's launches should select that kind alone. */
tn_status tn_profile_select(uint32_t kind_mask);
int32_t tn_profile_read(tn_kernel_profile* out, int32_t capacity);
void tn_profile_reset(void);

/* Thread-local description of the last non-OK status ("" if none). */
const char* tn_last_error(void);
/* Library version string. */
const char* tn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TN_H */
