// Device runtime: uploads network tables, lays out the caller's workspace,
// executes compiled programs and implements the device entry points of tn.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace tnq {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

tn_status set_error(tn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
void clear_error() { g_err.clear(); }

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return set_error(TN_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));      \
  } while (0)

// ---------------------------------------------------------------------------
// kernel timing (tn_profile_*)
// ---------------------------------------------------------------------------
struct ProfRec {
  int kind;
  hipEvent_t a, b;
  double bytes, flops;
  int launches;  // timed launches between a and b
  bool owner;    // the record that returns a and b to the pool (a launch may be counted under two kinds)
};
static bool g_prof = false;
static uint32_t g_prof_mask = ~0u;  // kernel kinds timed while enabled
static std::vector<ProfRec> g_recs;
static std::vector<hipEvent_t> g_pool;

static hipEvent_t pool_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  // timing-only events: no system-scope fence (no cache writeback and
  // invalidation around the timed kernels)
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Every event recorded between two kernels leaves the GPU idle for a few
// microseconds.  Inside a contraction, consecutive timed launches of one kind
// therefore share one event pair (a run, closed by the next launch of another
// kind or by the end of the steps); a large product keeps a pair of its own.
static bool g_coalesce = false;
static bool g_run_open = false;
static ProfRec g_run;
static hipEvent_t const kRunMember = reinterpret_cast<hipEvent_t>(&g_run);  // prof_start's token for a run member

static bool large_product(double bytes, double flops) { return flops >= 1e9 && flops >= 40.0 * bytes; }

static void prof_close_run(hipStream_t s) {
  if (!g_run_open) return;
  g_run_open = false;
  hipEvent_t b = pool_event();
  if (!b) {
    g_pool.push_back(g_run.a);
    return;
  }
  (void)hipEventRecord(b, s);
  g_run.b = b;
  g_recs.push_back(g_run);
}

static bool prof_selected(int kind) { return g_prof && ((g_prof_mask >> kind) & 1u); }

// large: a large product, timed alone (a pair of its own, even inside a run)
// when TN_KERNEL_GEMM_LARGE is selected
static hipEvent_t prof_start(hipStream_t s, int kind, bool large = false) {
  const bool own_pair = large && prof_selected(TN_KERNEL_GEMM_LARGE);
  const bool timed = prof_selected(kind) || own_pair;
  if (g_run_open && (!timed || own_pair || g_run.kind != kind)) prof_close_run(s);
  if (!timed) return nullptr;
  if (g_coalesce && !own_pair) {
    if (!g_run_open) {
      hipEvent_t e = pool_event();
      if (!e) return nullptr;
      (void)hipEventRecord(e, s);
      g_run = ProfRec{kind, e, nullptr, 0.0, 0.0, 0, true};
      g_run_open = true;
    }
    return kRunMember;
  }
  hipEvent_t e = pool_event();
  if (e) (void)hipEventRecord(e, s);
  return e;
}

static void prof_stop(hipStream_t s, hipEvent_t a, int kind, double bytes, double flops) {
  if (!a) return;
  if (a == kRunMember) {
    g_run.bytes += bytes;
    g_run.flops += flops;
    g_run.launches += 1;
    return;
  }
  hipEvent_t b = pool_event();
  if (!b) return;
  (void)hipEventRecord(b, s);
  const bool large = kind == TN_KERNEL_GEMM && large_product(bytes, flops) && prof_selected(TN_KERNEL_GEMM_LARGE);
  if (prof_selected(kind)) {
    g_recs.push_back(ProfRec{kind, a, b, bytes, flops, 1, true});
    // products that are large by flops and intensity are also tallied on their own
    if (large) g_recs.push_back(ProfRec{TN_KERNEL_GEMM_LARGE, a, b, bytes, flops, 1, false});
  } else if (large) {
    g_recs.push_back(ProfRec{TN_KERNEL_GEMM_LARGE, a, b, bytes, flops, 1, true});
  }
}

// ---------------------------------------------------------------------------
// device copies of a network's tables
// ---------------------------------------------------------------------------
struct DevNet {
  int device = -1;
  DevTensor* tensors = nullptr;
  Recipe* recipes = nullptr;
  RecipeOp* ops = nullptr;
  double* mats = nullptr;
  Recipe* sweep_recipes = nullptr;
  RecipeOp* sweep_ops = nullptr;
  int32_t* slot_param = nullptr;
  std::vector<int32_t> slot_of_gate;  // per sweep gate: gradient slot or -1
  int n_slots = 0;
};

// set between tn_graph_begin and tn_graph_end on this thread: device-side
// tables must exist before a capture starts (their upload is not a graph node)
static thread_local bool g_capturing = false;

template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return hipSuccess;
  if (g_capturing) return hipErrorStreamCaptureUnsupported;
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

static tn_status ensure_device(tn_network* net, DevNet** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DevNet* d = (DevNet*)net->dev;
  if (d && d->device == dev) { *out = d; return TN_OK; }
  if (d) { device_release_network(net); }
  d = new DevNet();
  d->device = dev;
  net->dev = d;
  std::vector<DevTensor> ts;
  for (const TensorDef& t : net->tensors) {
    DevTensor x;
    x.kind = t.kind; x.recipe = t.recipe; x.qubit = t.qubit; x.pad = 0;
    x.offset = t.offset; x.size = t.size;
    ts.push_back(x);
  }
  HIP_TRY(upload(&d->tensors, ts));
  HIP_TRY(upload(&d->recipes, net->recipes));
  HIP_TRY(upload(&d->ops, net->ops));
  HIP_TRY(upload(&d->mats, net->matrices));
  HIP_TRY(upload(&d->sweep_recipes, net->sweep_recipes));
  HIP_TRY(upload(&d->sweep_ops, net->sweep_ops));
  std::vector<int32_t> sp;
  d->slot_of_gate.assign(net->sweep.size(), -1);
  for (size_t i = 0; i < net->sweep.size(); ++i)
    if (net->sweep[i].gen != GEN_NONE) {
      d->slot_of_gate[i] = (int32_t)sp.size();
      sp.push_back(net->sweep[i].param);
    }
  d->n_slots = (int)sp.size();
  HIP_TRY(upload(&d->slot_param, sp));
  *out = d;
  return TN_OK;
}

void device_release_network(tn_network* net) {
  DevNet* d = (DevNet*)net->dev;
  if (!d) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(d->device);
  (void)hipFree(d->tensors); (void)hipFree(d->recipes); (void)hipFree(d->ops); (void)hipFree(d->mats);
  (void)hipFree(d->sweep_recipes); (void)hipFree(d->sweep_ops); (void)hipFree(d->slot_param);
  (void)hipSetDevice(cur);
  delete d;
  net->dev = nullptr;
}

struct DevPath {
  int device = -1;
  SmallStep* steps = nullptr;
  int32_t* lists = nullptr;
  int32_t* levels = nullptr;
  uint32_t* items = nullptr;
  SweepGateDesc* sweep_gates = nullptr;
  SweepSegment* segments = nullptr;
  int64_t* sweep_val_src = nullptr;
  SliceTensor* slice_tensors = nullptr;
  AdjGateDesc* adj_gates = nullptr;     // uploaded on the first backward call
  SweepSegment* adj_segments = nullptr;
};

static tn_status ensure_path_device(tn_path* path, DevPath** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DevPath* d = (DevPath*)path->dev;
  if (d && d->device == dev) { *out = d; return TN_OK; }
  if (d) device_release_path(path);
  d = new DevPath();
  d->device = dev;
  path->dev = d;
  HIP_TRY(upload(&d->steps, path->small_steps));
  HIP_TRY(upload(&d->lists, path->small_lists));
  HIP_TRY(upload(&d->levels, path->small_levels));
  HIP_TRY(upload(&d->items, path->small_items));
  HIP_TRY(upload(&d->sweep_gates, path->sweep_gates));
  HIP_TRY(upload(&d->segments, path->segments));
  HIP_TRY(upload(&d->sweep_val_src, path->sweep_val_src));
  HIP_TRY(upload(&d->slice_tensors, path->slice_tensors));
  *out = d;
  return TN_OK;
}

void device_release_path(tn_path* path) {
  DevPath* d = (DevPath*)path->dev;
  if (!d) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(d->device);
  (void)hipFree(d->steps);
  (void)hipFree(d->lists);
  (void)hipFree(d->levels);
  (void)hipFree(d->items);
  (void)hipFree(d->sweep_gates);
  (void)hipFree(d->segments);
  (void)hipFree(d->sweep_val_src);
  (void)hipFree(d->slice_tensors);
  (void)hipFree(d->adj_gates);
  (void)hipFree(d->adj_segments);
  (void)hipSetDevice(cur);
  delete d;
  path->dev = nullptr;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
  size_t in_off, arena_off, aux_off, total;
};

static WsLayout layout_ws(const tn_network* net, const tn_path* path, int batch, size_t aux_bytes) {
  WsLayout L;
  L.in_off = 0;
  L.arena_off = align256(L.in_off + sizeof(float2) * (size_t)net->input_elems * batch);
  L.aux_off = align256(L.arena_off + sizeof(float2) * (size_t)path->ws_elems * batch);
  L.total = align256(L.aux_off + aux_bytes);
  return L;
}

static size_t expect_aux(int batch) { return sizeof(double) * (size_t)kExpectBlocks * batch; }

// ---------------------------------------------------------------------------
// program execution
// ---------------------------------------------------------------------------
struct Bases {
  float2* in = nullptr;
  int64_t in_bs = 0;
  float2* ws = nullptr;
  int64_t ws_bs = 0;
  float2* out = nullptr;
  int64_t out_bs = 0;
  // when set, the last step (a matrix product) writes here instead of its workspace buffer
  float2* final_out = nullptr;
  int64_t final_out_bs = 0;
  // contract_pair: inputs are two separate user buffers
  const float2* pair_a = nullptr;
  const float2* pair_b = nullptr;
  int64_t pair_a_elems = 0;
};

static float2* resolve(const Bases& b, const BufRef& r, int64_t* bs) {
  switch (r.buf) {
    case BUF_IN:
      if (b.pair_a) {
        *bs = 0;
        return r.off < b.pair_a_elems ? (float2*)b.pair_a + r.off : (float2*)b.pair_b + (r.off - b.pair_a_elems);
      }
      *bs = b.in_bs;
      return b.in + r.off;
    case BUF_WS: *bs = b.ws_bs; return b.ws + r.off;
    case BUF_OUT: *bs = b.out_bs; return b.out + r.off;
    default: *bs = 0; return nullptr;
  }
}

// End (exclusive) of the run of products starting at step si that share one
// launch of the grouped per-output kernel (si + 1: si runs alone).
static size_t group_end(const tn_path* path, size_t si, int precision) {
  size_t e = si + 1;
  if (!elem_groupable(path->steps[si], precision)) return e;
  while (e < path->steps.size() && e - si < (size_t)kElemGroupMax && elem_groupable(path->steps[e], precision) &&
         path->steps[e].grp_from <= (int)si)
    ++e;
  return e;
}

static tn_status run_steps_body(hipStream_t s, tn_path* path, const Bases& B, int batch, int precision) {
  DevPath* dp = nullptr;
  if (path->n_small > 0 || !path->chains.empty()) {
    tn_status st = ensure_path_device(path, &dp);
    if (st != TN_OK) return st;
  }
  if (path->n_small > 0) {
    int64_t ibs, wbs;
    BufRef ri, rw;
    ri.buf = BUF_IN;
    rw.buf = BUF_WS;
    float2* ip = resolve(B, ri, &ibs);
    float2* wp = resolve(B, rw, &wbs);
    if (B.pair_a) return set_error(TN_EINVAL, "internal: interpreter steps in a single pairwise contraction");
    hipEvent_t ev = prof_start(s, TN_KERNEL_INTERP);
    HIP_TRY(launch_small_steps(s, dp->steps, dp->lists, dp->levels, dp->items, (int)path->small_lists.size() - 1, ip,
                               ibs, wp, wbs, batch, precision));
    double fl = 0, by = 0;
    for (int i = 0; i < path->n_small; ++i) { fl += path->steps[i].flops; by += path->steps[i].bytes; }
    prof_stop(s, ev, TN_KERNEL_INTERP, by * batch, fl * batch);
  }
  for (size_t si = path->n_small; si < path->steps.size(); ++si) {
    const StepProgram& P = path->steps[si];
    if (P.chain == -2) continue;
    if (P.chain >= 0) {
      const SweepChain& ch = path->chains[P.chain];
      int64_t ibs, obs, IN_bs, WS_bs;
      float2* ip = resolve(B, ch.in, &ibs);
      float2* op = resolve(B, ch.out, &obs);
      BufRef ri, rw;
      ri.buf = BUF_IN;
      rw.buf = BUF_WS;
      float2* INp = resolve(B, ri, &IN_bs);
      float2* WSp = resolve(B, rw, &WS_bs);
      int64_t vbs = 0;
      float2* vals = ch.n_vals > 0 ? resolve(B, ch.vals, &vbs) : nullptr;
      if (ch.n_vals > 0)
        HIP_TRY(launch_gather_vals(s, dp->sweep_val_src + ch.first_val, ch.n_vals, INp, IN_bs, WSp, WS_bs, vals, vbs,
                                   batch));
      for (int k = 0; k < ch.n_passes; ++k) {
        const SweepPass& ps = path->passes[ch.first_pass + k];
        hipEvent_t ev = prof_start(s, TN_KERNEL_SWEEP);
        HIP_TRY(launch_sweep_pass(s, ps, ch.bits, dp->sweep_gates, dp->segments, k == 0 ? ip : op,
                                  k == 0 ? ibs : obs, op, obs, vals, vbs, batch, precision));
        double fl = 0;
        for (int g = 0; g < ps.n_gates; ++g) {
          const SweepGateDesc& gd = path->sweep_gates[ps.first_gate + g];
          if (gd.form == kFormCount) continue;  // its member gates are counted
          fl += gd.diag ? 8.0 : 8.0 * (1 << gd.n);
        }
        prof_stop(s, ev, TN_KERNEL_SWEEP, 16.0 * std::ldexp(1.0, ch.bits) * batch,
                  fl * std::ldexp(1.0, ch.bits) * batch);
      }
      continue;
    }
    if (P.outer >= 0 && !B.pair_a) {
      // a run of outer products in one launch (its steps run one by one when T or C is not
      // 16-byte aligned in every batch item)
      const OuterChain& oc = path->outers[P.outer];
      int64_t tbs, cbs, IN_bs, WS_bs;
      const float2* t = resolve(B, oc.t, &tbs);
      float2* c = resolve(B, oc.c, &cbs);
      BufRef ri, rw;
      ri.buf = BUF_IN;
      rw.buf = BUF_WS;
      const float2* INp = resolve(B, ri, &IN_bs);
      const float2* WSp = resolve(B, rw, &WS_bs);
      const bool aligned = t && c && ((reinterpret_cast<uintptr_t>(t) | reinterpret_cast<uintptr_t>(c)) & 15) == 0 &&
                           (batch == 1 || ((tbs | cbs) & 1) == 0);
      if (aligned) {
        hipEvent_t ev = prof_start(s, TN_KERNEL_SKINNY);
        HIP_TRY(launch_outer_chain(s, oc, t, batch == 1 ? 0 : tbs, c, batch == 1 ? 0 : cbs, INp, IN_bs, WSp, WS_bs,
                                   batch));
        prof_stop(s, ev, TN_KERNEL_SKINNY, oc.bytes * batch, oc.flops * batch);
        si += oc.k - 1;
        continue;
      }
    }
    for (const PermuteDesc& pd : P.pre) {
      int64_t ibs, obs;
      float2* ip = resolve(B, pd.in, &ibs);
      float2* op = resolve(B, pd.out, &obs);
      hipEvent_t ev = prof_start(s, TN_KERNEL_PERMUTE);
      HIP_TRY(launch_permute(s, pd, ip, ibs, op, obs, batch));
      prof_stop(s, ev, TN_KERNEL_PERMUTE, 16.0 * (double)((int64_t)1 << pd.bits) * batch, 0.0);
    }
    if (P.kind == SK_SKINNY) {
      int64_t gbs, tbs, cbs;
      float2* g = resolve(B, P.sk.g, &gbs);
      float2* t = resolve(B, P.sk.t, &tbs);
      float2* c = resolve(B, P.sk.c, &cbs);
      const SkinnyDesc& d = P.sk;
      const double te = (double)((int64_t)1 << d.t_bits);
      const double ce = d.c_mode ? (double)((int64_t)1 << (d.t_bits - d.nk + d.nm)) : te;
      const double ge = (double)((int64_t)1 << (d.nb + d.nm + d.nk));
      hipEvent_t ev = prof_start(s, TN_KERNEL_SKINNY);
      HIP_TRY(launch_skinny(s, P.sk, g, gbs, t, tbs, c, cbs, batch, precision));
      prof_stop(s, ev, TN_KERNEL_SKINNY, 8.0 * batch * (ge + te + ce), P.flops * batch);
    } else {
      {
        const size_t e = group_end(path, si, precision);
        if (e - si >= 2) {
          ElemGroupArgs ga;
          ga.n = (int32_t)(e - si);
          double bytes = 0, flops = 0;
          for (size_t t = si; t < e; ++t) {
            const StepProgram& Q = path->steps[t];
            const GemmDesc& d = Q.gm[Q.orient[precision]];
            int64_t abs_, bbs, cbs;
            const float2* ma = resolve(B, d.a, &abs_);
            const float2* mb = resolve(B, d.b, &bbs);
            float2* mc = resolve(B, d.c, &cbs);
            if (t + 1 == path->steps.size() && B.final_out) {
              mc = B.final_out;
              cbs = B.final_out_bs;
            }
            ga.m[t - si] = elem_member(d, ma, abs_, mb, bbs, mc, cbs);
            bytes += 8.0 * batch * (double)d.batch * (double)(d.M * d.K + d.K * d.N + d.M * d.N);
            flops += Q.flops * batch;
          }
          ga.total_blocks = 0;
          hipEvent_t ev = prof_start(s, TN_KERNEL_GEMM);
          HIP_TRY(launch_elem_group(s, ga, batch, precision));
          prof_stop(s, ev, TN_KERNEL_GEMM, bytes, flops);
          si = e - 1;
          continue;
        }
      }
      int64_t abs_, bbs, cbs;
      const GemmDesc& g = P.gm[P.orient[precision]];
      float2* a = resolve(B, g.a, &abs_);
      float2* b = resolve(B, g.b, &bbs);
      float2* c = resolve(B, g.c, &cbs);
      const double bytes = 8.0 * batch * (double)g.batch * (double)(g.M * g.K + g.K * g.N + g.M * g.N);
      int64_t tbs = 0;
      float2* tmp = g.max_split > 1 ? resolve(B, g.tmp, &tbs) : nullptr;
      if (si + 1 == path->steps.size() && B.final_out) {
        c = B.final_out;  // the last product writes the caller's output directly
        cbs = B.final_out_bs;
      }
      hipEvent_t ev = prof_start(s, TN_KERNEL_GEMM, large_product(bytes, P.flops * batch));
      HIP_TRY(launch_gemm(s, g, g.tile[precision], g.split[precision], a, abs_, b, bbs, c, cbs, tmp, tbs, batch,
                          precision));
      prof_stop(s, ev, TN_KERNEL_GEMM, bytes, P.flops * batch);
    }
  }
  return TN_OK;
}

static tn_status run_steps(hipStream_t s, tn_path* path, const Bases& B, int batch, int precision) {
  g_coalesce = true;
  const tn_status st = run_steps_body(s, path, B, batch, precision);
  prof_close_run(s);
  g_coalesce = false;
  return st;
}

static tn_status materialize(hipStream_t s, tn_network* net, DevNet* d, const double* params, int batch,
                             const uint64_t* bits, int64_t count, float2* in) {
  hipEvent_t ev = prof_start(s, TN_KERNEL_MATERIALIZE);
  HIP_TRY(launch_materialize(s, d->tensors, (int)net->tensors.size(), d->recipes, d->ops, d->mats, params,
                             net->n_params, batch, in, net->input_elems));
  if (net->output_kind == TN_OUT_AMPLITUDES) {
    const int64_t first = net->tensors[net->tensors.size() - net->n_qubits].offset;
    HIP_TRY(launch_projectors(s, bits, count, net->n_qubits, net->batch_log2, first, batch, in, net->input_elems));
  }
  prof_stop(s, ev, TN_KERNEL_MATERIALIZE, 8.0 * (double)net->input_elems * batch, 0.0);
  return TN_OK;
}

static int32_t lab(int mode, int j) { return mode * 64 + j; }

static int pos_in(const std::vector<int32_t>& bits, int32_t l) {
  for (size_t i = 0; i < bits.size(); ++i)
    if (bits[i] == l) return (int)(bits.size() - 1 - i);
  return -1;
}

// move the final tensor (layout `from`) into `dst` with layout `to`
// the final tensor f (stride fbs per batch item, layout path->final_bits) into dst
static tn_status finish_to(hipStream_t s, const float2* f, int64_t fbs, const tn_path* path,
                           const std::vector<int32_t>& to, float2* dst, int64_t dst_bs, int64_t n_copy, int batch,
                           float2* scratch) {
  const std::vector<int32_t>& from = path->final_bits;
  if (from == to) {
    hipEvent_t ev = prof_start(s, TN_KERNEL_COPY);
    HIP_TRY(launch_copy(s, f, fbs, dst, dst_bs, n_copy, batch));
    prof_stop(s, ev, TN_KERNEL_COPY, 16.0 * (double)n_copy * batch, 0.0);
    return TN_OK;
  }
  PermuteDesc pd;
  pd.bits = (int32_t)from.size();
  for (size_t i = 0; i < from.size(); ++i) pd.dst[from.size() - 1 - i] = pos_in(to, from[i]);
  if (n_copy == path->final_elems) {
    hipEvent_t ev = prof_start(s, TN_KERNEL_PERMUTE);
    HIP_TRY(launch_permute(s, pd, f, fbs, dst, dst_bs, batch));
    prof_stop(s, ev, TN_KERNEL_PERMUTE, 16.0 * (double)n_copy * batch, 0.0);
  } else {
    HIP_TRY(launch_permute(s, pd, f, fbs, scratch, path->final_elems, batch));
    HIP_TRY(launch_copy(s, scratch, path->final_elems, dst, dst_bs, n_copy, batch));
  }
  return TN_OK;
}

static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

// map qubit masks to address-bit masks of the final tensor
// The observable's Z strings as address masks of a state in layout `bits` (labels, C order).
static tn_status make_terms(const tn_network* net, const std::vector<int32_t>& bits, const tn_observable* obs,
                            ZTerms* t) {
  if (!obs || obs->n_terms < 0 || (obs->n_terms > 0 && (!obs->z_mask || !obs->coeff)))
    return set_error(TN_EINVAL, "bad observable");
  if (obs->n_terms > kMaxTerms)
    return set_error(TN_EUNSUPPORTED, "observable has more than " + std::to_string(kMaxTerms) + " terms");
  const int n = net->n_qubits;
  t->n = obs->n_terms;
  for (int i = 0; i < obs->n_terms; ++i) {
    uint64_t m = 0;
    const uint64_t qm = obs->z_mask[i];
    if (n < 64 && (qm >> n) != 0) return set_error(TN_EINVAL, "observable mask names a qubit >= n_qubits");
    for (int q = 0; q < n; ++q)
      if ((qm >> (n - 1 - q)) & 1) {
        const int p = pos_in(bits, lab(net->wire_final[q], 0));
        if (p < 0) return set_error(TN_EINVAL, "qubit leg missing from the final tensor");
        m |= (uint64_t)1 << p;
      }
    t->mask[i] = m;
    t->coeff[i] = obs->coeff[i];
  }
  // group the terms by their address bits 8..11 (the reduction kernels sum
  // each group once per thread and spread it over 16 elements)
  std::vector<int> order(t->n);
  for (int i = 0; i < t->n; ++i) order[i] = i;
  auto mu = [&](int i) { return (int)((t->mask[i] >> 8) & 15); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mu(a) < mu(b); });
  uint64_t mk[kMaxTerms];
  double cf[kMaxTerms];
  for (int i = 0; i < t->n; ++i) {
    mk[i] = t->mask[order[i]];
    cf[i] = t->coeff[order[i]];
  }
  for (int i = 0; i < t->n; ++i) {
    t->mask[i] = mk[i];
    t->coeff[i] = cf[i];
  }
  for (int m = 0, i = 0; m <= 16; ++m) {
    while (i < t->n && mu(i) < m) ++i;
    t->mu_start[m] = i;
  }
  return TN_OK;
}

}  // namespace tnq

using namespace tnq;

extern "C" const char* tn_last_error(void) { return g_err.c_str(); }

extern "C" tn_status tn_profile_enable(int32_t on) {
  clear_error();
  g_prof = on != 0;
  return TN_OK;
}

extern "C" tn_status tn_profile_select(uint32_t kind_mask) {
  clear_error();
  g_prof_mask = kind_mask;
  return TN_OK;
}

extern "C" void tn_profile_reset(void) {
  for (ProfRec& r : g_recs) {
    (void)hipEventSynchronize(r.b);
    if (r.owner) {
      g_pool.push_back(r.a);
      g_pool.push_back(r.b);
    }
  }
  g_recs.clear();
}

extern "C" int32_t tn_profile_read(tn_kernel_profile* out, int32_t capacity) {
  tn_kernel_profile acc[TN_KERNEL_KINDS];
  for (int k = 0; k < TN_KERNEL_KINDS; ++k) acc[k] = tn_kernel_profile{k, 0, 0.0, 0.0, 0.0};
  for (ProfRec& r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      acc[r.kind].launches += r.launches;
      acc[r.kind].seconds += 1e-3 * ms;
      acc[r.kind].bytes += r.bytes;
      acc[r.kind].flops += r.flops;
    }
    if (r.owner) {
      g_pool.push_back(r.a);
      g_pool.push_back(r.b);
    }
  }
  g_recs.clear();
  int n = 0;
  for (int k = 0; k < TN_KERNEL_KINDS && n < capacity; ++k)
    if (acc[k].launches) out[n++] = acc[k];
  return n;
}
extern "C" const char* tn_version(void) { return "tnq 0.1 (gfx950)"; }

// Workspace of a sliced path: [full input tensors x batch][sum of the slices x batch]
// [the sliced program's workspace: its inputs, arena and aux, as layout_ws on the sliced network]
struct SliceLayout {
  size_t full_off, acc_off, prog_off, total;
  WsLayout prog;  // relative to prog_off
};

static SliceLayout layout_sliced(const tn_network* net, const tn_path* path, int batch, size_t aux_bytes) {
  SliceLayout L;
  L.full_off = 0;
  L.acc_off = align256(sizeof(float2) * (size_t)net->input_elems * batch);
  L.prog_off = align256(L.acc_off + sizeof(float2) * (size_t)path->final_elems * batch);
  L.prog = layout_ws(path->sliced_net.get(), path, batch, aux_bytes);
  L.total = align256(L.prog_off + L.prog.total);
  return L;
}

// Contract every slice and sum them into the accumulator (final layout, final_elems per batch item).
static tn_status run_slices(hipStream_t s, tn_network* net, tn_path* path, DevNet* d, const double* params,
                            int batch, const uint64_t* bits, int64_t count, char* w, const SliceLayout& L,
                            int precision) {
  DevPath* dp;
  tn_status st = ensure_path_device(path, &dp);
  if (st != TN_OK) return st;
  const tn_network* sn = path->sliced_net.get();
  float2* full = (float2*)(w + L.full_off);
  float2* acc = (float2*)(w + L.acc_off);
  char* pw = w + L.prog_off;
  Bases B;
  B.in = (float2*)(pw + L.prog.in_off);
  B.in_bs = sn->input_elems;
  B.ws = (float2*)(pw + L.prog.arena_off);
  B.ws_bs = path->ws_elems;
  if ((st = materialize(s, net, d, params, batch, bits, count, full)) != TN_OK) return st;
  const int64_t n_slices = (int64_t)1 << path->slice_bits;
  for (int64_t sl = 0; sl < n_slices; ++sl) {
    HIP_TRY(launch_slice_gather(s, dp->slice_tensors, (int)path->slice_tensors.size(), full, net->input_elems, B.in,
                                B.in_bs, sl, batch));
    if ((st = run_steps(s, path, B, batch, precision)) != TN_OK) return st;
    int64_t fbs;
    const float2* f = resolve(B, path->final_ref, &fbs);
    HIP_TRY(launch_accumulate(s, f, fbs, acc, path->final_elems, path->final_elems, sl == 0, batch));
  }
  return TN_OK;
}

static tn_status refuse_sliced(const tn_path* path, const char* what) {
  if (path && path->slice_bits > 0)
    return set_error(TN_EUNSUPPORTED, std::string(what) + " does not run sliced paths");
  return TN_OK;
}

// workspace of the Q3.28 program: [input tensors x batch][arena x batch]
static WsLayout layout_q328(const tn_network* net, const tn_path* path, int batch) {
  WsLayout L;
  L.in_off = 0;
  L.arena_off = align256(sizeof(float2) * (size_t)net->input_elems * batch);
  L.aux_off = align256(L.arena_off + sizeof(float2) * (size_t)path->q_ws_elems * batch);
  L.total = L.aux_off;
  return L;
}

extern "C" size_t tn_workspace_bytes(const tn_network* net, const tn_path* path, int32_t batch) {
  if (!net || !path || batch < 1) return 0;
  const size_t final_tmp = sizeof(float2) * (size_t)path->final_elems * batch;
  if (path->slice_bits > 0) return layout_sliced(net, path, batch, std::max(expect_aux(batch), final_tmp)).total;
  size_t n = layout_ws(net, path, batch, std::max(expect_aux(batch), final_tmp)).total;
  if (path->q_state == 1) n = std::max(n, layout_q328(net, path, batch).total);
  return n;
}

static tn_status check_common(const tn_network* net, const tn_path* path, const double* params, int32_t batch,
                              int32_t precision, bool q328_ok = false) {
  if (!net || !path) return set_error(TN_EINVAL, "NULL network or path");
  if (path->n_inputs != (int32_t)net->tensors.size()) return set_error(TN_EINVAL, "path was planned for another network");
  if (batch < 1 || batch > 65535) return set_error(TN_EINVAL, "batch must be in 1..65535");
  if (net->n_params > 0 && !params) return set_error(TN_EINVAL, "params_dev required (n_params > 0)");
  if (precision == TN_PREC_Q3_28) {
    if (!q328_ok) return set_error(TN_EUNSUPPORTED, "TN_PREC_Q3_28 is offered by tn_contract_path and tn_amplitudes");
    if (path->slice_bits > 0) return set_error(TN_EUNSUPPORTED, "TN_PREC_Q3_28 does not run sliced paths");
    if (path->q_state != 1)
      return set_error(TN_EUNSUPPORTED, "a step of this path exceeds the fixed-point kernel's index limits");
    return TN_OK;
  }
  if (precision != TN_PREC_C64 && precision != TN_PREC_BF16X3) return set_error(TN_EINVAL, "unknown precision");
  return TN_OK;
}

// The Q3.28 program (Sec. 3's fixed-point arithmetic): materialise the inputs
// as Q3.28 pairs (bits: the amplitude network's bitstrings, `count` of them),
// run every step of the path as one fixed-point product, then convert the
// final tensor to complex64 in the order `to` (bit labels, most significant
// first): `count` outputs per batch item, `out_bs` apart.
static tn_status run_q328(hipStream_t s, tn_network* net, tn_path* path, DevNet* d, const double* params, int batch,
                          const uint64_t* bits, int64_t count, char* w, const std::vector<int32_t>& to,
                          float2* out, int64_t out_bs) {
  const WsLayout L = layout_q328(net, path, batch);
  float2* in = (float2*)(w + L.in_off);
  char* arena = w + L.arena_off;
  const int64_t in_bs = net->input_elems, ws_bs = path->q_ws_elems;
  HIP_TRY(launch_materialize(s, d->tensors, (int)net->tensors.size(), d->recipes, d->ops, d->mats, params,
                             net->n_params, batch, in, in_bs, true));
  if (net->output_kind == TN_OUT_AMPLITUDES) {
    const int64_t first = net->tensors[net->tensors.size() - net->n_qubits].offset;
    HIP_TRY(launch_projectors(s, bits, count, net->n_qubits, net->batch_log2, first, batch, in, in_bs, true));
  }
  auto base = [&](int32_t buf, int64_t off, int64_t* bs) -> const void* {
    *bs = buf == BUF_IN ? in_bs : ws_bs;
    return buf == BUF_IN ? (const void*)(in + off) : (const void*)((float2*)arena + off);
  };
  for (const QStep& q : path->q_steps) {
    int64_t abs_, bbs;
    const void* a = base(q.a_buf, q.a_off, &abs_);
    const void* b = base(q.b_buf, q.b_off, &bbs);
    HIP_TRY(launch_q328_step(s, q, a, abs_, b, bbs, (float2*)arena + q.c_off, ws_bs, batch));
  }
  // result index bit j (from the least significant) -> bit of the final tensor
  QStep map{};
  map.n_out = (int32_t)to.size();
  if (map.n_out > kQMaxOutBits) return set_error(TN_EUNSUPPORTED, "output too wide for the fixed-point kernel");
  for (int j = 0; j < map.n_out; ++j) {
    const int32_t lab = to[to.size() - 1 - j];
    const int m = lab / 64, bit = lab % 64;
    int below = 0, pos = -1;
    for (size_t i = path->q_final_modes.size(); i-- > 0;) {
      if (path->q_final_modes[i] == m) { pos = below + bit; break; }
      below += net->mode_log2[path->q_final_modes[i]];
    }
    if (pos < 0) return set_error(TN_EINVAL, "internal: output leg missing from the final tensor");
    map.a_o[j] = (int8_t)pos;
  }
  int64_t fbs;
  const void* f = base(path->q_final.buf, path->q_final.off, &fbs);
  HIP_TRY(launch_q328_finish(s, f, fbs, out, out_bs, count, map, batch));
  return TN_OK;
}

// The statevector contraction into a workspace `w` of tn_workspace_bytes,
// with the network's device tables `d` already in place.
static tn_status contract_path_in(hipStream_t s, int32_t precision, tn_network* net, tn_path* path, DevNet* d,
                                  const double* params_dev, int32_t batch, char* w, void* out_dev) {
  tn_status st;
  const size_t final_tmp = sizeof(float2) * (size_t)path->final_elems * batch;
  WsLayout L = layout_ws(net, path, batch, std::max(expect_aux(batch), final_tmp));
  Bases B;
  B.in = (float2*)(w + L.in_off);
  B.in_bs = net->input_elems;
  B.ws = (float2*)(w + L.arena_off);
  B.ws_bs = path->ws_elems;
  B.out = (float2*)out_dev;
  B.out_bs = (int64_t)1 << net->n_qubits;
  std::vector<int32_t> to;
  for (int q = 0; q < net->n_qubits; ++q) to.push_back(lab(net->wire_final[q], 0));
  const bool direct = !path->steps.empty() && path->steps.back().kind == SK_GEMM && path->steps.back().chain == -1 &&
                      path->final_bits == to;
  if (direct) {
    B.final_out = B.out;
    B.final_out_bs = B.out_bs;
  }
  if ((st = materialize(s, net, d, params_dev, batch, nullptr, 0, B.in)) != TN_OK) return st;
  if ((st = run_steps(s, path, B, batch, precision)) != TN_OK) return st;
  if (direct) return TN_OK;
  int64_t fbs;
  const float2* f = resolve(B, path->final_ref, &fbs);
  return finish_to(s, f, fbs, path, to, B.out, B.out_bs, B.out_bs, batch, (float2*)(w + L.aux_off));
}

extern "C" tn_status tn_contract_path(void* stream, int32_t precision, tn_network* net, tn_path* path,
                                      const double* params_dev, int32_t batch, void* workspace_dev,
                                      size_t workspace_bytes, void* out_dev) {
  clear_error();
  tn_status st = check_common(net, path, params_dev, batch, precision, true);
  if (st != TN_OK) return st;
  if (net->output_kind != TN_OUT_STATEVECTOR) return set_error(TN_EINVAL, "network does not output a statevector");
  if (!out_dev || !workspace_dev) return set_error(TN_EINVAL, "NULL device buffer");
  const size_t need = tn_workspace_bytes(net, path, batch);
  if (workspace_bytes < need)
    return set_error(TN_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  DevNet* d;
  if ((st = ensure_device(net, &d)) != TN_OK) return st;
  if (precision == TN_PREC_Q3_28) {
    std::vector<int32_t> to;
    for (int q = 0; q < net->n_qubits; ++q) to.push_back(lab(net->wire_final[q], 0));
    const int64_t n_out = (int64_t)1 << net->n_qubits;
    return run_q328((hipStream_t)stream, net, path, d, params_dev, batch, nullptr, n_out, (char*)workspace_dev, to,
                    (float2*)out_dev, n_out);
  }
  if (path->slice_bits > 0) {
    hipStream_t s = (hipStream_t)stream;
    const size_t final_tmp = sizeof(float2) * (size_t)path->final_elems * batch;
    const SliceLayout L = layout_sliced(net, path, batch, std::max(expect_aux(batch), final_tmp));
    char* w = (char*)workspace_dev;
    if ((st = run_slices(s, net, path, d, params_dev, batch, nullptr, 0, w, L, precision)) != TN_OK) return st;
    std::vector<int32_t> to;
    for (int q = 0; q < net->n_qubits; ++q) to.push_back(lab(net->wire_final[q], 0));
    const int64_t n_out = (int64_t)1 << net->n_qubits;
    return finish_to(s, (float2*)(w + L.acc_off), path->final_elems, path, to, (float2*)out_dev, n_out, n_out, batch,
                     (float2*)(w + L.prog_off + L.prog.aux_off));
  }
  return contract_path_in((hipStream_t)stream, precision, net, path, d, params_dev, batch, (char*)workspace_dev,
                          out_dev);
}

// ---------------------------------------------------------------------------
// tn_contract_path_noalloc: the same contraction with its workspace in a
// file-scope device array instead of a caller's buffer, for callers that
// cannot allocate.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol): the device address of each
// device's copy is looked up once with hipGetSymbolAddress and kept.  The
// array has external linkage (in this library's namespace): with internal
// linkage it would be a local symbol of the code object, which the runtime's
// symbol lookup cannot see.
// ---------------------------------------------------------------------------
namespace tnq {
__device__ __align__(256) char scratch[TN_NOALLOC_SCRATCH_BYTES];
}

constexpr int kMaxDevices = 64;
static char* g_scratch_ptr[kMaxDevices];  // per device, set on the first call on that device
static std::mutex g_scratch_mu;

static tn_status scratch_for_device(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(TN_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(tnq::scratch));
    if (e != hipSuccess || !p)
      return set_error(TN_EDEVICE, std::string("hipGetSymbolAddress(tnq::scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return TN_OK;
}

extern "C" tn_status tn_contract_path_noalloc(void* stream, int32_t precision, tn_network* net, tn_path* path,
                                              const double* params_dev, int32_t batch, void* out_dev) {
  clear_error();
  tn_status st = check_common(net, path, params_dev, batch, precision);
  if (st != TN_OK) return st;
  if (net->output_kind != TN_OUT_STATEVECTOR) return set_error(TN_EINVAL, "network does not output a statevector");
  if (!out_dev) return set_error(TN_EINVAL, "NULL output buffer");
  if ((st = refuse_sliced(path, "tn_contract_path_noalloc")) != TN_OK) return st;
  const size_t need = tn_workspace_bytes(net, path, batch);
  if (need > (size_t)TN_NOALLOC_SCRATCH_BYTES)
    return set_error(TN_ENOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the static scratch of " +
                                    std::to_string((size_t)TN_NOALLOC_SCRATCH_BYTES) + " bytes");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  // device-side tables are created (allocated) by the other entry points only
  DevNet* d = (DevNet*)net->dev;
  if (!d || d->device != dev)
    return set_error(TN_EINVAL, "the network's device tables are not on this device: run tn_contract_path once "
                                "with this network on this device first");
  const bool needs_path_tables = path->n_small > 0 || !path->chains.empty();
  const DevPath* dp = (const DevPath*)path->dev;
  if (needs_path_tables && (!dp || dp->device != dev))
    return set_error(TN_EINVAL, "the path's device tables are not on this device: run tn_contract_path once "
                                "with this path on this device first");
  char* w = nullptr;
  if ((st = scratch_for_device(dev, &w)) != TN_OK) return st;
  // kernel timing creates events: it is left out of this call
  const bool prof = g_prof;
  g_prof = false;
  st = contract_path_in((hipStream_t)stream, precision, net, path, d, params_dev, batch, w, out_dev);
  g_prof = prof;
  return st;
}

extern "C" tn_status tn_amplitudes(void* stream, int32_t precision, tn_network* net, tn_path* path,
                                   const double* params_dev, const uint64_t* bitstrings_dev, int64_t count,
                                   void* workspace_dev, size_t workspace_bytes, void* out_dev) {
  clear_error();
  tn_status st = check_common(net, path, params_dev, 1, precision, true);
  if (st != TN_OK) return st;
  if (net->output_kind != TN_OUT_AMPLITUDES) return set_error(TN_EINVAL, "network does not output amplitudes");
  if (count < 1 || count > net->n_bitstrings) return set_error(TN_EINVAL, "count must be in 1..n_bitstrings");
  if (!out_dev || !workspace_dev || !bitstrings_dev) return set_error(TN_EINVAL, "NULL device buffer");
  const size_t need = tn_workspace_bytes(net, path, 1);
  if (workspace_bytes < need)
    return set_error(TN_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  hipStream_t s = (hipStream_t)stream;
  DevNet* d;
  if ((st = ensure_device(net, &d)) != TN_OK) return st;
  if (precision == TN_PREC_Q3_28) {
    std::vector<int32_t> to;
    for (int j = net->batch_log2 - 1; j >= 0; --j) to.push_back(lab(net->batch_mode, j));
    return run_q328(s, net, path, d, params_dev, 1, bitstrings_dev, count, (char*)workspace_dev, to,
                    (float2*)out_dev, count);
  }
  if (path->slice_bits > 0) {
    const size_t final_tmp = sizeof(float2) * (size_t)path->final_elems;
    const SliceLayout L = layout_sliced(net, path, 1, std::max(expect_aux(1), final_tmp));
    char* w = (char*)workspace_dev;
    if ((st = run_slices(s, net, path, d, params_dev, 1, bitstrings_dev, count, w, L, precision)) != TN_OK) return st;
    std::vector<int32_t> to;
    for (int j = net->batch_log2 - 1; j >= 0; --j) to.push_back(lab(net->batch_mode, j));
    return finish_to(s, (float2*)(w + L.acc_off), path->final_elems, path, to, (float2*)out_dev, count, count, 1,
                     (float2*)(w + L.prog_off + L.prog.aux_off));
  }
  const size_t final_tmp = sizeof(float2) * (size_t)path->final_elems;
  WsLayout L = layout_ws(net, path, 1, std::max(expect_aux(1), final_tmp));
  char* w = (char*)workspace_dev;
  Bases B;
  B.in = (float2*)(w + L.in_off);
  B.in_bs = net->input_elems;
  B.ws = (float2*)(w + L.arena_off);
  B.ws_bs = path->ws_elems;
  std::vector<int32_t> to;
  for (int j = net->batch_log2 - 1; j >= 0; --j) to.push_back(lab(net->batch_mode, j));
  const bool direct = !path->steps.empty() && path->steps.back().kind == SK_GEMM && path->steps.back().chain == -1 &&
                      path->final_bits == to && count == path->final_elems;
  if (direct) {
    B.final_out = (float2*)out_dev;
    B.final_out_bs = count;
  }
  if ((st = materialize(s, net, d, params_dev, 1, bitstrings_dev, count, B.in)) != TN_OK) return st;
  if ((st = run_steps(s, path, B, 1, precision)) != TN_OK) return st;
  if (direct) return TN_OK;
  int64_t fbs;
  const float2* f = resolve(B, path->final_ref, &fbs);
  return finish_to(s, f, fbs, path, to, (float2*)out_dev, count, count, 1, (float2*)(w + L.aux_off));
}

// Circuits of one tn_expectation call are independent: they run on kExpLanes
// streams at once (the caller's and kExpLanes - 1 of the library's, forked
// from and joined back into the caller's stream with events, so the call stays
// ordered on it and captures into one graph), each lane with its own
// workspace slot.  Small circuits then fill the GPU beside large ones.  (On
// 512 QAOA circuits of 16 to 26 qubits, 4, 8, 12 and 16 lanes measured 411,
// 360, 351 and 353 ms per call, with the runtime's default four hardware
// queues; more hardware queues made it slower.)
constexpr int kExpLanes = 12;

static size_t expect_slot_bytes(tn_network* const* nets, tn_path* const* paths, int32_t n_circuits, int32_t batch) {
  size_t mx = 0;
  for (int i = 0; i < n_circuits; ++i) {
    if (!nets || !paths || !nets[i] || !paths[i]) return 0;
    mx = std::max(mx, paths[i]->slice_bits > 0 ? layout_sliced(nets[i], paths[i], batch, expect_aux(batch)).total
                                               : layout_ws(nets[i], paths[i], batch, expect_aux(batch)).total);
  }
  return align256(mx);
}

static int expect_lanes(int32_t n_circuits) { return std::max(1, std::min((int)n_circuits, kExpLanes)); }

extern "C" size_t tn_expectation_workspace_bytes(tn_network* const* nets, tn_path* const* paths, int32_t n_circuits,
                                                 int32_t batch) {
  if (n_circuits < 1) return 0;
  return expect_slot_bytes(nets, paths, n_circuits, batch) * (size_t)expect_lanes(n_circuits);
}

// the library's side streams and fork/join events, per device (created on first use; default priority)
struct SideLanes {
  hipStream_t stream[kExpLanes - 1] = {};
  hipEvent_t fork = nullptr, join[kExpLanes - 1] = {};
};
static std::mutex g_lanes_mu;
static SideLanes* g_lanes[64];

static tn_status side_lanes(SideLanes** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return set_error(TN_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_lanes_mu);
  if (!g_lanes[dev]) {
    SideLanes* L = new SideLanes();
    for (int k = 0; k < kExpLanes - 1; ++k) {
      HIP_TRY(hipStreamCreateWithFlags(&L->stream[k], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&L->join[k], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&L->fork, hipEventDisableTiming));
    g_lanes[dev] = L;
  }
  *out = g_lanes[dev];
  return TN_OK;
}

extern "C" tn_status tn_expectation(void* stream, int32_t precision, tn_network* const* nets, tn_path* const* paths,
                                    int32_t n_circuits, const double* const* params_dev, int32_t batch,
                                    const tn_observable* obs, void* workspace_dev, size_t workspace_bytes,
                                    double* out_dev) {
  clear_error();
  if (n_circuits < 1 || !nets || !paths || !obs || !out_dev || !workspace_dev)
    return set_error(TN_EINVAL, "NULL argument or no circuits");
  const size_t need = tn_expectation_workspace_bytes(nets, paths, n_circuits, batch);
  if (need == 0) return set_error(TN_EINVAL, "NULL network or path");
  if (workspace_bytes < need) return set_error(TN_ENOMEM, "workspace too small: need " + std::to_string(need));
  const size_t slot = expect_slot_bytes(nets, paths, n_circuits, batch);
  // every check and host-side table before the first launch, so that an error leaves no lane forked
  std::vector<ZTerms> all_terms(n_circuits);
  std::vector<DevNet*> devs(n_circuits);
  for (int c = 0; c < n_circuits; ++c) {
    const double* prm = params_dev ? params_dev[c] : nullptr;
    tn_status st = check_common(nets[c], paths[c], prm, batch, precision);
    if (st != TN_OK) return set_error(st, "circuit " + std::to_string(c) + ": " + g_err);
    if (nets[c]->output_kind != TN_OUT_STATEVECTOR)
      return set_error(TN_EINVAL, "expectation needs a statevector network");
    if ((st = make_terms(nets[c], paths[c]->final_bits, &obs[c], &all_terms[c])) != TN_OK) return st;
    if ((st = ensure_device(nets[c], &devs[c])) != TN_OK) return st;
    DevPath* dp;
    if ((st = ensure_path_device(paths[c], &dp)) != TN_OK) return st;
  }
  hipStream_t s0 = (hipStream_t)stream;
  // kernel timing measures per stream: with it on, every circuit runs on the caller's stream
  const int lanes = g_prof ? 1 : expect_lanes(n_circuits);
  SideLanes* SL_ = nullptr;
  if (lanes > 1) {
    tn_status st = side_lanes(&SL_);
    if (st != TN_OK) return st;
    HIP_TRY(hipEventRecord(SL_->fork, s0));
    for (int k = 0; k < lanes - 1; ++k) HIP_TRY(hipStreamWaitEvent(SL_->stream[k], SL_->fork, 0));
  }
  // circuits to lanes by the planner's run-time model, largest first, each to the lane with the
  // least work so far (ties: the lower lane), so that the lanes finish close together
  std::vector<int> lane_of(n_circuits, 0);
  if (lanes > 1) {
    std::vector<int> order(n_circuits);
    std::vector<double> cost(n_circuits);
    for (int c = 0; c < n_circuits; ++c) {
      order[c] = c;
      cost[c] = paths[c]->stats.modeled_seconds * std::ldexp(1.0, paths[c]->slice_bits);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<double> load(lanes, 0.0);
    for (int c : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      lane_of[c] = k;
      load[k] += cost[c];
    }
  }
  tn_status result = TN_OK;
  for (int c = 0; c < n_circuits && result == TN_OK; ++c) {
    tn_network* net = nets[c];
    tn_path* path = paths[c];
    const double* prm = params_dev ? params_dev[c] : nullptr;
    const int lane = lane_of[c];
    hipStream_t s = lane == 0 ? s0 : SL_->stream[lane - 1];
    const ZTerms& terms = all_terms[c];
    DevNet* d = devs[c];
    char* w = (char*)workspace_dev + (size_t)lane * slot;
    tn_status st;
    if (path->slice_bits > 0) {  // the state is the sum of the slices
      const SliceLayout SL = layout_sliced(net, path, batch, expect_aux(batch));
      if ((st = run_slices(s, net, path, d, prm, batch, nullptr, 0, w, SL, precision)) != TN_OK) {
        result = st;
        break;
      }
      hipEvent_t ev = prof_start(s, TN_KERNEL_REDUCE);
      const hipError_t e = launch_expectation(s, (float2*)(w + SL.acc_off), path->final_elems, path->final_elems,
                                              terms, batch, (double*)(w + SL.prog_off + SL.prog.aux_off),
                                              out_dev + (int64_t)c * batch, 1);
      if (e != hipSuccess) {
        result = set_error(TN_EDEVICE, std::string("expectation: ") + hipGetErrorString(e));
        break;
      }
      prof_stop(s, ev, TN_KERNEL_REDUCE, 8.0 * (double)path->final_elems * batch, 0.0);
      continue;
    }
    WsLayout L = layout_ws(net, path, batch, expect_aux(batch));
    Bases B;
    B.in = (float2*)(w + L.in_off);
    B.in_bs = net->input_elems;
    B.ws = (float2*)(w + L.arena_off);
    B.ws_bs = path->ws_elems;
    if ((st = materialize(s, net, d, prm, batch, nullptr, 0, B.in)) != TN_OK ||
        (st = run_steps(s, path, B, batch, precision)) != TN_OK) {
      result = st;
      break;
    }
    int64_t fbs;
    float2* f = resolve(B, path->final_ref, &fbs);
    hipEvent_t ev = prof_start(s, TN_KERNEL_REDUCE);
    const hipError_t e = launch_expectation(s, f, fbs, path->final_elems, terms, batch, (double*)(w + L.aux_off),
                                            out_dev + (int64_t)c * batch, 1);
    if (e != hipSuccess) {
      result = set_error(TN_EDEVICE, std::string("expectation: ") + hipGetErrorString(e));
      break;
    }
    prof_stop(s, ev, TN_KERNEL_REDUCE, 8.0 * (double)path->final_elems * batch, 0.0);
  }
  // join the lanes back into the caller's stream (also after an error, so no lane stays forked)
  for (int k = 0; k < lanes - 1; ++k) {
    const hipError_t e1 = hipEventRecord(SL_->join[k], SL_->stream[k]);
    const hipError_t e2 = hipStreamWaitEvent(s0, SL_->join[k], 0);
    if (result == TN_OK && (e1 != hipSuccess || e2 != hipSuccess))
      result = set_error(TN_EDEVICE, std::string("joining the expectation lanes: ") +
                                         hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  return result;
}

// ---------------------------------------------------------------------------
// adjoint gradient
// ---------------------------------------------------------------------------
struct BackLayout {
  WsLayout base;
  size_t lam_off, mats_off, part_off, total;
};

static BackLayout back_layout(const tn_network* net, const tn_path* path, int batch, int n_slots) {
  BackLayout L;
  L.base = layout_ws(net, path, batch, expect_aux(batch));
  L.lam_off = L.base.total;
  L.mats_off = align256(L.lam_off + sizeof(float2) * (size_t)path->final_elems * batch);
  L.part_off = align256(L.mats_off + sizeof(float2) * 16 * net->sweep.size() * batch);
  L.total = align256(L.part_off + sizeof(double) * (size_t)std::max(n_slots, 1) * kReduceBlocks * batch);
  return L;
}

static int count_slots(const tn_network* net) {
  int n = 0;
  for (const SweepGate& g : net->sweep) n += g.gen != GEN_NONE;
  return n;
}

extern "C" size_t tn_backward_workspace_bytes(const tn_network* net, const tn_path* path, int32_t batch) {
  if (!net || !path || batch < 1) return 0;
  return back_layout(net, path, batch, count_slots(net)).total;
}

extern "C" tn_status tn_backward(void* stream, int32_t precision, tn_network* net, tn_path* path,
                                 const double* params_dev, int32_t batch, const tn_observable* obs,
                                 const double* grad_out_dev, void* workspace_dev, size_t workspace_bytes,
                                 double* value_dev, double* grad_dev) {
  clear_error();
  tn_status st = check_common(net, path, params_dev, batch, precision);
  if (st != TN_OK) return st;
  if ((st = refuse_sliced(path, "tn_backward")) != TN_OK) return st;
  if (net->output_kind != TN_OUT_STATEVECTOR) return set_error(TN_EINVAL, "backward needs a statevector network");
  if (!workspace_dev || !value_dev || (net->n_params > 0 && !grad_dev)) return set_error(TN_EINVAL, "NULL buffer");
  const size_t need = tn_backward_workspace_bytes(net, path, batch);
  if (workspace_bytes < need) return set_error(TN_ENOMEM, "workspace too small: need " + std::to_string(need));
  if (path->adj_state == 0) {
    DevNet* d0;
    if ((st = ensure_device(net, &d0)) != TN_OK) return st;
    build_adjoint_plan(net, path, d0->slot_of_gate);
  }
  // the passes' layout: the final tensor's, or the qubit order (the state is permuted first)
  const bool perm = path->adj_state == 1 && path->adj_perm;
  ZTerms terms;
  if ((st = make_terms(net, perm ? path->adj_bits : path->final_bits, obs, &terms)) != TN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  DevNet* d;
  if ((st = ensure_device(net, &d)) != TN_OK) return st;
  BackLayout L = back_layout(net, path, batch, d->n_slots);
  char* w = (char*)workspace_dev;
  Bases B;
  B.in = (float2*)(w + L.base.in_off);
  B.in_bs = net->input_elems;
  B.ws = (float2*)(w + L.base.arena_off);
  B.ws_bs = path->ws_elems;
  // forward contraction to psi (left in the workspace arena)
  if ((st = materialize(s, net, d, params_dev, batch, nullptr, 0, B.in)) != TN_OK) return st;
  if ((st = run_steps(s, path, B, batch, precision)) != TN_OK) return st;
  int64_t pbs;
  float2* psi = resolve(B, path->final_ref, &pbs);
  if (path->final_ref.buf != BUF_WS) return set_error(TN_EUNSUPPORTED, "backward of a network without contraction steps");
  const int64_t n = path->final_elems;
  double* partial = (double*)(w + L.base.aux_off);
  float2* lam = (float2*)(w + L.lam_off);
  int64_t lbs = n;
  if (perm) {
    // psi into the qubit order, in lambda's buffer; lambda then takes psi's
    PermuteDesc pd;
    pd.bits = (int32_t)path->final_bits.size();
    for (int p = 0; p < pd.bits; ++p) {
      const int32_t label = path->final_bits[pd.bits - 1 - p];
      const int q = pos_in(path->adj_bits, label);
      if (q < 0) return set_error(TN_EINVAL, "internal: adjoint layout misses a leg of the final tensor");
      pd.dst[p] = q;
    }
    hipEvent_t ev = prof_start(s, TN_KERNEL_PERMUTE);
    HIP_TRY(launch_permute(s, pd, psi, pbs, lam, n, batch));
    prof_stop(s, ev, TN_KERNEL_PERMUTE, 16.0 * (double)n * batch, 0.0);
    std::swap(psi, lam);
    std::swap(pbs, lbs);
  }
  HIP_TRY(launch_expectation(s, psi, pbs, n, terms, batch, partial, value_dev, 1));
  HIP_TRY(launch_apply_diag_obs(s, psi, pbs, lam, lbs, n, terms, batch));
  float2* umats = (float2*)(w + L.mats_off);
  HIP_TRY(launch_sweep_matrices(s, d->sweep_recipes, (int)net->sweep.size(), d->sweep_ops, d->mats, params_dev,
                                net->n_params, batch, umats));
  double* parts = (double*)(w + L.part_off);
  const int64_t pstride = (int64_t)std::max(d->n_slots, 1) * kReduceBlocks;
  if (path->adj_state == 1) {
    // fused passes: both states stream through LDS once per pass
    DevPath* dp;
    if ((st = ensure_path_device(path, &dp)) != TN_OK) return st;
    if (!dp->adj_gates) {
      HIP_TRY(upload(&dp->adj_gates, path->adj_gates));
      HIP_TRY(upload(&dp->adj_segments, path->adj_segments));
    }
    const int bits = (int)path->final_bits.size();
    for (const SweepPass& ps : path->adj_passes) {
      double fl = 0;
      for (int i = ps.first_gate; i < ps.first_gate + ps.n_gates; ++i) {
        const AdjGateDesc& gd = path->adj_gates[i];
        // per element and state: 8 for a diagonal factor, 8 * 2^n for a dense gate on n qubits (one
        // complex multiply-add per matrix entry); 8 more per element for a gradient term
        const double per = gd.diag ? 8.0 : 8.0 * (double)(1 << gd.n);
        fl += 2.0 * per * (double)n + (gd.red >= 0 ? 8.0 * (double)n : 0.0);
      }
      hipEvent_t ev = prof_start(s, TN_KERNEL_ADJOINT);
      HIP_TRY(launch_adjoint_pass(s, ps, bits, dp->adj_gates, dp->adj_segments, umats,
                                  (int64_t)net->sweep.size() * 16, psi, pbs, lam, lbs, batch, parts, pstride,
                                  precision));
      prof_stop(s, ev, TN_KERNEL_ADJOINT, 32.0 * (double)n * batch, fl * batch);
    }
  }
  for (int gi = path->adj_state == 1 ? -1 : (int)net->sweep.size() - 1; gi >= 0; --gi) {
    const SweepGate& g = net->sweep[gi];
    SweepArgs a;
    a.nq = g.nq;
    a.pos[0] = pos_in(path->final_bits, lab(net->wire_final[g.q[0]], 0));
    a.pos[1] = g.nq == 2 ? pos_in(path->final_bits, lab(net->wire_final[g.q[1]], 0)) : 0;
    a.gen = g.gen;
    a.slot = d->slot_of_gate[gi];
    if (a.pos[0] < 0 || a.pos[1] < 0 || (1ll << a.pos[0]) >= n || (1ll << a.pos[1]) >= n)
      return set_error(TN_EINVAL, "internal: qubit leg missing from the final tensor");
    hipEvent_t ev = prof_start(s, TN_KERNEL_ADJOINT);
    HIP_TRY(launch_adjoint_step(s, a, umats + (int64_t)gi * 16, (int64_t)net->sweep.size() * 16, psi, pbs, lam, lbs,
                                n, batch, parts, pstride, precision));
    const double per = 8.0 * (double)(1 << g.nq);  // dense U^dagger on both states, as in the fused passes
    prof_stop(s, ev, TN_KERNEL_ADJOINT, 32.0 * (double)n * batch,
              (2.0 * per + (a.slot >= 0 ? 8.0 : 0.0)) * (double)n * batch);
  }
  if (net->n_params > 0)
    HIP_TRY(launch_gradient_reduce(s, parts, pstride, d->n_slots, d->slot_param, net->n_params, grad_out_dev, batch,
                                   grad_dev));
  return TN_OK;
}

// ---------------------------------------------------------------------------
// HIP graphs of whole calls
// ---------------------------------------------------------------------------
struct tn_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
};

extern "C" tn_status tn_graph_begin(void* stream) {
  clear_error();
  if (!stream) return set_error(TN_EINVAL, "capture needs a stream other than the null stream");
  if (g_prof) return set_error(TN_EINVAL, "disable kernel timing (tn_profile_enable(0)) before capturing");
  if (g_capturing) return set_error(TN_EINVAL, "a capture is already open on this thread");
  HIP_TRY(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
  g_capturing = true;
  return TN_OK;
}

extern "C" tn_status tn_graph_end(void* stream, tn_graph** out) {
  clear_error();
  if (!g_capturing) return set_error(TN_EINVAL, "no capture open on this thread");
  g_capturing = false;
  if (!stream || !out) {
    hipGraph_t g = nullptr;
    if (stream && hipStreamEndCapture((hipStream_t)stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    return set_error(TN_EINVAL, "NULL stream or output handle");
  }
  *out = nullptr;
  tn_graph* G = new tn_graph();
  hipError_t e = hipStreamEndCapture((hipStream_t)stream, &G->graph);
  if (e == hipSuccess) e = hipGetDevice(&G->device);
  if (e == hipSuccess) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return set_error(TN_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  *out = G;
  return TN_OK;
}

extern "C" tn_status tn_graph_launch(const tn_graph* g, void* stream) {
  clear_error();
  if (!g || !g->exec) return set_error(TN_EINVAL, "NULL graph");
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return TN_OK;
}

extern "C" void tn_graph_destroy(tn_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

// ---------------------------------------------------------------------------
// launch-shape autotuner
// ---------------------------------------------------------------------------
static bool gemm_shape_ok(const GemmDesc& g, int tile, int split, int precision) {
  if (!gemm_tile_supported(g, tile)) return false;
  if (tile > kGemmVector && precision != TN_PREC_C64) return false;  // 3M tiles: FP32 only
  if (split != 1 && split != 2 && split != 4 && split != 8) return false;
  if (tile == kGemmVector) return split == 1 && g.K <= kElemMaxK;
  return split <= std::max(g.max_split, 1) && g.K % split == 0;
}

extern "C" tn_status tn_path_gemm_config(tn_path* path, int32_t step, int32_t precision, int32_t* tile,
                                         int32_t* split, int32_t* transposed, int32_t set) {
  clear_error();
  if (!path || !tile || !split || !transposed) return set_error(TN_EINVAL, "NULL argument");
  if (precision != TN_PREC_C64 && precision != TN_PREC_BF16X3) return set_error(TN_EINVAL, "unknown precision");
  if (step < 0 || step >= (int32_t)path->steps.size() || path->steps[step].kind != SK_GEMM ||
      path->steps[step].chain != -1)
    return set_error(TN_EINVAL, "step is not a matrix product");
  StepProgram& P = path->steps[step];
  if (!set) {
    const GemmDesc& g = P.gm[P.orient[precision]];
    *tile = g.tile[precision];
    *split = g.split[precision];
    *transposed = P.orient[precision];
    return TN_OK;
  }
  if (*transposed != 0 && *transposed != 1) return set_error(TN_EINVAL, "transposed must be 0 or 1");
  GemmDesc& g = P.gm[*transposed];
  if (!gemm_shape_ok(g, *tile, *split, precision))
    return set_error(TN_EINVAL, "launch shape not valid for this step");
  g.tile[precision] = *tile;
  g.split[precision] = *split;
  P.orient[precision] = *transposed;
  return TN_OK;
}

extern "C" tn_status tn_autotune(void* stream, int32_t precision, tn_network* net, tn_path* path,
                                 const double* params_dev, int32_t batch, void* workspace_dev, size_t workspace_bytes,
                                 int32_t reps, tn_tune_report* report) {
  clear_error();
  tn_status st = check_common(net, path, params_dev, batch, precision);
  if (st != TN_OK) return st;
  if ((st = refuse_sliced(path, "tn_autotune")) != TN_OK) return st;
  if (!workspace_dev) return set_error(TN_EINVAL, "NULL workspace");
  if (reps < 1 || reps > 1000) return set_error(TN_EINVAL, "reps must be in 1..1000");
  const size_t need = tn_workspace_bytes(net, path, batch);
  if (workspace_bytes < need) return set_error(TN_ENOMEM, "workspace too small: need " + std::to_string(need));
  hipStream_t s = (hipStream_t)stream;
  DevNet* d;
  if ((st = ensure_device(net, &d)) != TN_OK) return st;
  WsLayout L = layout_ws(net, path, batch, 0);
  char* w = (char*)workspace_dev;
  Bases B;
  B.in = (float2*)(w + L.in_off);
  B.in_bs = net->input_elems;
  B.ws = (float2*)(w + L.arena_off);
  B.ws_bs = path->ws_elems;
  HIP_TRY(hipMemsetAsync(w, 0, L.aux_off, s));
  HIP_TRY(launch_materialize(s, d->tensors, (int)net->tensors.size(), d->recipes, d->ops, d->mats, params_dev,
                             net->n_params, batch, B.in, net->input_elems));
  if ((st = run_steps(s, path, B, batch, precision)) != TN_OK) return st;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  HIP_TRY(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  tn_tune_report rep{0, 0, 0.0, 0.0};
  tn_status result = TN_OK;
  // products that share a launch keep their shape: alone, another shape would
  // have to save more than the launch it adds
  std::vector<char> grouped(path->steps.size(), 0);
  for (size_t si = path->n_small; si < path->steps.size();) {
    const size_t e = group_end(path, si, precision);
    if (e - si >= 2)
      for (size_t t = si; t < e; ++t) grouped[t] = 1;
    si = e;
  }
  for (size_t si = 0; si < path->steps.size() && result == TN_OK; ++si) {
    StepProgram& P = path->steps[si];
    if (P.kind != SK_GEMM || P.chain != -1) continue;
    auto time_shape = [&](const GemmDesc& g, int tile, int split, double* sec) -> hipError_t {
      int64_t abs_, bbs, cbs, tbs = 0;
      float2* a = resolve(B, g.a, &abs_);
      float2* b = resolve(B, g.b, &bbs);
      float2* c = resolve(B, g.c, &cbs);
      float2* tmp = g.max_split > 1 ? resolve(B, g.tmp, &tbs) : nullptr;
      hipError_t e = launch_gemm(s, g, tile, split, a, abs_, b, bbs, c, cbs, tmp, tbs, batch, precision);
      if (e != hipSuccess) return e;
      if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
      for (int r = 0; r < reps; ++r)
        if ((e = launch_gemm(s, g, tile, split, a, abs_, b, bbs, c, cbs, tmp, tbs, batch, precision)) != hipSuccess)
          return e;
      if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
      float ms = 0;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
      *sec = 1e-3 * ms / reps;
      return hipSuccess;
    };
    const int o0 = P.orient[precision];
    const int t0 = P.gm[o0].tile[precision], s0 = P.gm[o0].split[precision];
    double best = 0;
    hipError_t e = time_shape(P.gm[o0], t0, s0, &best);
    if (e != hipSuccess) { result = set_error(TN_EDEVICE, std::string("autotune: ") + hipGetErrorString(e)); break; }
    rep.n_products++;
    rep.seconds_before += best;
    int bo = o0, bt = t0, bs = s0;
    for (int o = 0; o < 2 && result == TN_OK && !grouped[si]; ++o)
      for (int tile = 0; tile < kGemmTiles && result == TN_OK; ++tile)
        for (int split = 1; split <= kGemmMaxSplit; split *= 2) {
          const GemmDesc& g = P.gm[o];
          if ((o == o0 && tile == t0 && split == s0) || !gemm_shape_ok(g, tile, split, precision)) continue;
          if (tile != kGemmVector && split > 1 && g.K / split < kGemmBK) continue;
          double sec = 0;
          e = time_shape(g, tile, split, &sec);
          if (e != hipSuccess) {
            result = set_error(TN_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
            break;
          }
          if (sec < 0.97 * best) { best = sec; bo = o; bt = tile; bs = split; }
        }
    if (bo != o0 || bt != t0 || bs != s0) rep.n_changed++;
    P.orient[precision] = bo;
    P.gm[bo].tile[precision] = bt;
    P.gm[bo].split[precision] = bs;
    rep.seconds_after += best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (report) *report = rep;
  return result;
}

// ---------------------------------------------------------------------------
// single pairwise contraction
// ---------------------------------------------------------------------------
namespace {

struct PairPlan {
  tn_network net;
  tn_path path;
  std::vector<int32_t> c_bits;
  int64_t a_elems = 0, c_elems = 0;
};

tn_status make_pair_plan(int32_t rank_a, const int32_t* modes_a, const int64_t* ext_a, int32_t rank_b,
                         const int32_t* modes_b, const int64_t* ext_b, int32_t rank_c, const int32_t* modes_c,
                         PairPlan* pp) {
  if (rank_a < 0 || rank_b < 0 || rank_c < 0 || rank_a > TN_MAX_RANK || rank_b > TN_MAX_RANK || rank_c > TN_MAX_RANK)
    return set_error(TN_EINVAL, "bad rank");
  if ((rank_a && (!modes_a || !ext_a)) || (rank_b && (!modes_b || !ext_b)) || (rank_c && !modes_c))
    return set_error(TN_EINVAL, "NULL mode array");
  std::map<int32_t, int> id;
  std::map<int32_t, int64_t> ext;
  auto reg = [&](int32_t m, int64_t e) -> tn_status {
    if (!is_pow2(e)) return set_error(TN_EUNSUPPORTED, "extents must be powers of two");
    auto it = ext.find(m);
    if (it != ext.end() && it->second != e) return set_error(TN_EINVAL, "shared mode with different extents");
    ext[m] = e;
    if (!id.count(m)) id[m] = (int)id.size();
    return TN_OK;
  };
  auto dup = [](int32_t r, const int32_t* ms) {
    for (int i = 0; i < r; ++i)
      for (int j = i + 1; j < r; ++j)
        if (ms[i] == ms[j]) return true;
    return false;
  };
  if (dup(rank_a, modes_a) || dup(rank_b, modes_b) || dup(rank_c, modes_c))
    return set_error(TN_EINVAL, "repeated mode within a tensor");
  tn_status st;
  for (int i = 0; i < rank_a; ++i) if ((st = reg(modes_a[i], ext_a[i])) != TN_OK) return st;
  for (int i = 0; i < rank_b; ++i) if ((st = reg(modes_b[i], ext_b[i])) != TN_OK) return st;
  auto has = [](int32_t r, const int32_t* ms, int32_t m) {
    for (int i = 0; i < r; ++i) if (ms[i] == m) return true;
    return false;
  };
  for (int i = 0; i < rank_c; ++i)
    if (!ext.count(modes_c[i])) return set_error(TN_EINVAL, "output mode absent from both operands");
  for (auto& kv : ext) {
    const bool ia = has(rank_a, modes_a, kv.first), ib = has(rank_b, modes_b, kv.first);
    if ((ia != ib) && !has(rank_c, modes_c, kv.first))
      return set_error(TN_EINVAL, "a mode of one operand only must appear in the output");
  }
  tn_network& net = pp->net;
  net.mode_log2.assign(id.size(), 0);
  for (auto& kv : ext) {
    int l = 0;
    while (((int64_t)1 << l) < kv.second) ++l;
    net.mode_log2[id[kv.first]] = l;
  }
  TensorDef ta, tb;
  for (int i = 0; i < rank_a; ++i) ta.modes.push_back(id[modes_a[i]]);
  for (int i = 0; i < rank_b; ++i) tb.modes.push_back(id[modes_b[i]]);
  ta.kind = tb.kind = TK_GATE;
  ta.recipe = tb.recipe = -1;
  ta.qubit = tb.qubit = 0;
  ta.size = tb.size = 1;
  for (int m : ta.modes) ta.size <<= net.mode_log2[m];
  for (int m : tb.modes) tb.size <<= net.mode_log2[m];
  ta.offset = 0;
  tb.offset = ta.size;
  net.tensors = {ta, tb};
  for (int i = 0; i < rank_c; ++i) net.output_modes.push_back(id[modes_c[i]]);
  net.input_elems = ta.size + tb.size;
  pp->path.pairs = {0, 1};
  pp->a_elems = ta.size;
  pp->c_elems = 1;
  for (int i = 0; i < rank_c; ++i) {
    const int m = id[modes_c[i]];
    for (int j = net.mode_log2[m] - 1; j >= 0; --j) pp->c_bits.push_back(lab(m, j));
    pp->c_elems <<= net.mode_log2[m];
  }
  if ((st = compile_program(&net, &pp->path, &pp->c_bits)) != TN_OK) return st;
  return TN_OK;
}

}  // namespace

extern "C" size_t tn_contract_pair_workspace_bytes(int32_t rank_a, const int32_t* modes_a, const int64_t* ext_a,
                                                   int32_t rank_b, const int32_t* modes_b, const int64_t* ext_b,
                                                   int32_t rank_c, const int32_t* modes_c) {
  PairPlan pp;
  if (make_pair_plan(rank_a, modes_a, ext_a, rank_b, modes_b, ext_b, rank_c, modes_c, &pp) != TN_OK) return 0;
  return align256(sizeof(float2) * (size_t)pp.path.ws_elems);
}

extern "C" tn_status tn_contract_pair(void* stream, int32_t precision, const void* a, int32_t rank_a,
                                      const int32_t* modes_a, const int64_t* ext_a, const void* b, int32_t rank_b,
                                      const int32_t* modes_b, const int64_t* ext_b, void* c, int32_t rank_c,
                                      const int32_t* modes_c, void* workspace_dev, size_t workspace_bytes) {
  clear_error();
  if (precision != TN_PREC_C64 && precision != TN_PREC_BF16X3) return set_error(TN_EINVAL, "unknown precision");
  if (!a || !b || !c) return set_error(TN_EINVAL, "NULL operand");
  PairPlan pp;
  tn_status st = make_pair_plan(rank_a, modes_a, ext_a, rank_b, modes_b, ext_b, rank_c, modes_c, &pp);
  if (st != TN_OK) return st;
  const size_t need = align256(sizeof(float2) * (size_t)pp.path.ws_elems);
  if (workspace_bytes < need || !workspace_dev)
    return set_error(TN_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  hipStream_t s = (hipStream_t)stream;
  Bases B;
  B.pair_a = (const float2*)a;
  B.pair_b = (const float2*)b;
  B.pair_a_elems = pp.a_elems;
  B.ws = (float2*)workspace_dev;
  B.ws_bs = 0;
  const bool direct = pp.path.steps.back().kind == SK_GEMM && pp.path.final_bits == pp.c_bits;
  if (direct) {
    B.final_out = (float2*)c;
    B.final_out_bs = 0;
  }
  if ((st = run_steps(s, &pp.path, B, 1, precision)) != TN_OK) return st;
  if (direct) return TN_OK;
  int64_t fbs;
  const float2* f = resolve(B, pp.path.final_ref, &fbs);
  return finish_to(s, f, fbs, &pp.path, pp.c_bits, (float2*)c, 0, pp.c_elems, 1, nullptr);
}
