// Compile a contraction order into an executable program: memory layouts of
// every intermediate, the kernel for each pairwise step, the operand permutes
// it needs, and workspace offsets.
//
// Every extent is a power of two, so a tensor is a 2^R array whose address
// bits are labelled (mode, bit-of-mode); a mode permutation is a permutation of
// address bits.  A pairwise step (Sec. 2.2.1, eq. (2.2)) classifies modes as
// batch (in A, B and C -- the block-diagonal structure that Sec. 3 builds
// with block_diag), M (A and C), N (B and C) and K (A and B, summed):
//   * small operand (gate-like, <= 2^8 elements, <= 2^4 summed and <= 2^4
//     output combinations): a streaming kernel that reads the large operand
//     in place through strided addresses and writes C with the large
//     operand's layout (no permute);
//   * otherwise: the MFMA complex matrix product on [batch][M][K] x
//     [batch][K][N] -> [batch][M][N], permuting an operand first only when
//     its bits are not already grouped that way.
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <thread>
#include <cmath>
#include <map>
#include <set>
#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"
#include "passes.h"

namespace tnq {

namespace {

inline int32_t label(int mode, int j) { return mode * 64 + j; }
inline int mode_of(int32_t lab) { return lab / 64; }

std::vector<int32_t> bits_of_modes(const tn_network* net, const std::vector<int32_t>& modes) {
  std::vector<int32_t> b;
  for (int m : modes)
    for (int j = net->mode_log2[m] - 1; j >= 0; --j) b.push_back(label(m, j));
  return b;
}

// address position of the label in a layout (MSB-first list)
int pos_of(const std::vector<int32_t>& bits, int32_t lab) {
  for (size_t i = 0; i < bits.size(); ++i)
    if (bits[i] == lab) return (int)(bits.size() - 1 - i);
  return -1;
}

struct Alloc {
  std::map<int64_t, int64_t> free_;  // offset -> size
  int64_t top = 0, peak = 0;
  static int64_t round(int64_t n) { return (n + 31) & ~(int64_t)31; }  // 256-byte granules
  int64_t get(int64_t n) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        int64_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > n) free_[off + n] = sz - n;
        return off;
      }
    }
    int64_t off = top;
    top += n;
    peak = std::max(peak, top);
    return off;
  }
  void put(int64_t off, int64_t n) {
    n = round(n);
    free_[off] = n;
    // coalesce
    auto it = free_.find(off);
    if (it != free_.begin()) {
      auto p = std::prev(it);
      if (p->first + p->second == it->first) { p->second += it->second; free_.erase(it); it = p; }
    }
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
    if (it->first + it->second == top) { top = it->first; free_.erase(it); }
  }
};

struct Loc {
  BufRef ref;
  std::vector<int32_t> bits;
  int64_t elems = 0;
  bool input = false;
  int last_use = -1;
};

enum Cls { C_BATCH = 0, C_M = 1, C_N = 2, C_K = 3 };

PermuteDesc make_permute(const BufRef& in, const std::vector<int32_t>& from, const BufRef& out,
                         const std::vector<int32_t>& to) {
  PermuteDesc p;
  p.in = in;
  p.out = out;
  p.bits = (int32_t)from.size();
  for (int i = 0; i < 64; ++i) p.dst[i] = 0;
  for (size_t i = 0; i < from.size(); ++i) {
    int pin = (int)(from.size() - 1 - i);
    p.dst[pin] = pos_of(to, from[i]);
  }
  return p;
}

// is `bits` = [batch run][X run][Y run] with {X, Y} = {c1, c2}?  returns orientation via fast_cls
bool grouped(const std::vector<int32_t>& bits, const std::map<int32_t, int>& cls, int c1, int c2, int* fast_cls) {
  size_t i = 0;
  while (i < bits.size() && cls.at(bits[i]) == C_BATCH) ++i;
  if (i == bits.size()) { *fast_cls = c2; return true; }
  int first = cls.at(bits[i]);
  if (first != c1 && first != c2) return false;
  while (i < bits.size() && cls.at(bits[i]) == first) ++i;
  if (i == bits.size()) { *fast_cls = first; return true; }
  int second = cls.at(bits[i]);
  if (second == first || (second != c1 && second != c2)) return false;
  while (i < bits.size() && cls.at(bits[i]) == second) ++i;
  if (i != bits.size()) return false;
  *fast_cls = second;
  return true;
}

std::vector<int32_t> filter(const std::vector<int32_t>& bits, const std::map<int32_t, int>& cls, int c) {
  std::vector<int32_t> out;
  for (int32_t b : bits)
    if (cls.at(b) == c) out.push_back(b);
  return out;
}

std::vector<int32_t> cat(std::vector<int32_t> a, const std::vector<int32_t>& b, const std::vector<int32_t>& c) {
  a.insert(a.end(), b.begin(), b.end());
  a.insert(a.end(), c.begin(), c.end());
  return a;
}

}  // namespace

std::vector<int32_t> reorder_small_first(const tn_network* net, const std::vector<int32_t>& pairs, int* n_small,
                                         int64_t* small_region) {
  const int T = (int)net->tensors.size();
  const int S = (int)pairs.size() / 2;
  std::vector<std::vector<int32_t>> modes(T + S);
  std::vector<int> lsz(T + S, 0);
  std::vector<int> holders(net->mode_log2.size(), 0);
  std::vector<char> is_out(net->mode_log2.size(), 0);
  for (int m : net->output_modes) is_out[m] = 1;
  for (int t = 0; t < T; ++t) {
    modes[t] = net->tensors[t].modes;
    for (int m : modes[t]) { holders[m]++; lsz[t] += net->mode_log2[m]; }
  }
  std::vector<char> small(S, 0), early(S, 0), groupable(S, 0);
  for (int s = 0; s < S; ++s) {
    const int a = pairs[2 * s], b = pairs[2 * s + 1];
    auto in = [](const std::vector<int32_t>& v, int m) { return std::find(v.begin(), v.end(), m) != v.end(); };
    std::vector<int32_t> cm;
    int f = 0, kb = 0, mb = 0, nb = 0;
    for (int m : modes[a]) {
      f += net->mode_log2[m];
      const bool sh = in(modes[b], m);
      const bool kept = is_out[m] || holders[m] > (sh ? 2 : 1);
      if (kept) cm.push_back(m);
      if (sh && !kept) kb += net->mode_log2[m];
      if (!sh) mb += net->mode_log2[m];
    }
    for (int m : modes[b])
      if (!in(modes[a], m)) { f += net->mode_log2[m]; nb += net->mode_log2[m]; cm.push_back(m); }
    for (int m : modes[a]) holders[m]--;
    for (int m : modes[b]) holders[m]--;
    for (int m : cm) holders[m]++;
    modes[T + s] = cm;
    for (int m : cm) lsz[T + s] += net->mode_log2[m];
    small[s] = lsz[a] <= kSmallMaxBits && lsz[b] <= kSmallMaxBits && lsz[T + s] <= kSmallMaxBits &&
               f <= kSmallMaxMacLog2 && (f - lsz[T + s]) <= kSmallMaxBits;
    early[s] = small[s] && (a < T || early[a - T]) && (b < T || early[b - T]);
    // a likely per-output product (narrow result side, short sum) with a small result
    groupable[s] = elem_group_shape(lsz[T + s], mb, nb, kb);
  }
  std::vector<int> order;
  for (int s = 0; s < S; ++s)
    if (early[s]) order.push_back(s);
  *n_small = (int)order.size();
  *small_region = 0;
  for (int s : order) *small_region += ((((int64_t)1 << lsz[T + s]) + 31) & ~(int64_t)31);
  // the rest in path order, except that next to a likely per-output product
  // the other such products that are ready at the same time move up, so that
  // one launch can run them together
  std::vector<int> pending(S, 0);  // operands not yet available
  std::vector<int> consumer(T + S, -1);
  for (int s = 0; s < S; ++s)
    for (int k = 0; k < 2; ++k) {
      const int id = pairs[2 * s + k];
      consumer[id] = s;
      if (id >= T && !early[id - T]) pending[s]++;
    }
  std::set<int> ready;
  for (int s = 0; s < S; ++s)
    if (!early[s] && pending[s] == 0) ready.insert(s);
  auto emit = [&](int s) {
    order.push_back(s);
    ready.erase(s);
    const int c = consumer[T + s];
    if (c >= 0 && --pending[c] == 0) ready.insert(c);
  };
  while (!ready.empty()) {
    const int s = *ready.begin();
    if (!groupable[s]) {
      emit(s);
      continue;
    }
    std::vector<int> mates;  // ready now, so independent of s and of each other
    for (int t : ready)
      if (t != s && groupable[t] && (int)mates.size() + 1 < kElemGroupMax) mates.push_back(t);
    emit(s);
    for (int t : mates) emit(t);
  }
  if ((int)order.size() != S) return pairs;  // not a tree over the inputs: keep the path order
  std::vector<int> newid(T + S);
  for (int t = 0; t < T; ++t) newid[t] = t;
  for (int i = 0; i < S; ++i) newid[T + order[i]] = T + i;
  std::vector<int32_t> out(2 * S);
  for (int i = 0; i < S; ++i) {
    out[2 * i] = newid[pairs[2 * order[i]]];
    out[2 * i + 1] = newid[pairs[2 * order[i] + 1]];
  }
  return out;
}

namespace {

// A segment's thread-bit map and the LDS slots of its register combinations
// (slot of local index i: i + i/32; the map from a thread's bits and the
// register bits are disjoint, so a slot is the sum of their two slots).
void fill_segment_tables(SweepSegment& seg, int l) {
  int t = 0;
  for (int j = 0; j < 8; ++j) seg.tpos[j] = 0;
  for (int b = 0; b < l && t < 8; ++b) {
    bool reg = false;
    for (int r = 0; r < 4; ++r) reg |= seg.rbits[r] == b;
    if (!reg) seg.tpos[t++] = (int8_t)b;
  }
  for (int r = 0; r < 16; ++r) {
    int off = 0;
    for (int j = 0; j < 4; ++j)
      if ((r >> j) & 1) off |= 1 << seg.rbits[j];
    seg.physoff[r] = (uint16_t)(off + (off >> 5));
  }
}

// Group chains of consecutive gate-sized steps on one large tensor into fused
// streaming passes (light-cone rule: a gate joins the current pass if its bits
// fit in the pass's local set and no earlier gate left out of the pass touches
// them; gates on disjoint bits commute).

// Runs of dense one-qubit gates for the pass kernels.  A dense one-qubit gate
// on register bit r commutes with every gate that leaves bit r alone, so for
// each such gate the first later gates of the same form on the other three
// register bits, each reached without crossing a gate on its bit, move up
// beside it; when there are two to four of them they are put in register-bit
// order, the first carries the mask of their bits, and the kernels apply them
// as one straight-line run.
inline int run_form(const SweepGateDesc& d) { return d.form; }
inline int run_form(const AdjGateDesc& d) { return d.uform; }  // the gradient's generator may differ
inline bool group_header(const SweepGateDesc& d) { return d.diag && d.form == kFormCount; }
inline bool group_header(const AdjGateDesc&) { return false; }

inline bool unit_diag1(const SweepGateDesc& d) { return d.diag && d.n == 1 && d.kreg[0] >= 0 && d.form == kFormUnit; }
inline bool unit_diag1(const AdjGateDesc& d) {
  return d.diag && d.n == 1 && d.kreg[0] >= 0 && !(d.form & ADJ_DIAG_SIGNS);
}

// Runs of one-bit unit diagonal gates on register bits (RZ and its like), found
// as the dense runs are: a diagonal gate on register bit r commutes with every
// gate but a dense one on bit r, so it moves up past the others beside the
// first such gate; two to four on distinct bits make a run.
template <class Desc>
void mark_diag_runs(Desc* g, int n) {
  const std::vector<Desc> v(g, g + n);
  std::vector<char> used(n, 0);
  int o = 0;
  for (int i = 0; i < n; ++i) {
    if (used[i]) continue;
    const Desc& d = v[i];
    if (unit_diag1(d) && d.run_mask == 0) {
      int pick[4] = {-1, -1, -1, -1};
      const int b0 = d.kreg[0];
      pick[b0] = i;
      int mask = 1 << b0;
      for (int r = 0; r < 4; ++r) {
        if (r == b0) continue;
        for (int j = i + 1; j < n; ++j) {
          if (used[j]) continue;
          const Desc& e = v[j];
          if (unit_diag1(e) && e.kreg[0] == r) {
            pick[r] = j;
            mask |= 1 << r;
            break;
          }
          if (!e.diag && (e.rb[0] == r || (e.n == 2 && e.rb[1] == r))) break;
        }
      }
      if (mask != (1 << b0)) {
        bool first = true;
        for (int r = 0; r < 4; ++r) {
          if (pick[r] < 0) continue;
          g[o] = v[pick[r]];
          g[o].run_mask = first ? mask : 0;
          first = false;
          used[pick[r]] = 1;
          ++o;
        }
        continue;
      }
    }
    g[o] = v[i];
    used[i] = 1;
    ++o;
  }
}

inline int reg_bits(const SweepGateDesc& d) {
  return (d.kreg[0] >= 0 ? 1 << d.kreg[0] : 0) | (d.n == 2 && d.kreg[1] >= 0 ? 1 << d.kreg[1] : 0);
}
inline int reg_bits(const AdjGateDesc& d) {
  return (d.kreg[0] >= 0 ? 1 << d.kreg[0] : 0) | (d.n == 2 && d.kreg[1] >= 0 ? 1 << d.kreg[1] : 0);
}
inline bool sign_diag(const SweepGateDesc& d) { return d.diag && d.form == kFormSigns && reg_bits(d) != 0; }
inline bool sign_diag(const AdjGateDesc& d) {
  return d.diag && (d.form & ADJ_DIAG_SIGNS) && d.red < 0 && reg_bits(d) != 0;
}

// Runs of diagonal gates with entries +-1 and a bit in the registers (CZ, Z):
// such a gate commutes with every gate but a dense one on its register bits,
// so later ones move up beside the first while no dense gate on their bits
// lies in between; two to sixteen make a run, whose sign flips the kernels
// combine into one mask over the thread's elements.
template <class Desc>
void mark_sign_runs(Desc* g, int n) {
  const std::vector<Desc> v(g, g + n);
  std::vector<char> used(n, 0);
  int o = 0;
  for (int i = 0; i < n; ++i) {
    if (used[i]) continue;
    if (sign_diag(v[i]) && v[i].run_mask == 0) {
      std::vector<int> pick{i};
      int blocked = 0;  // register bits of the dense gates passed
      for (int j = i + 1; j < n && pick.size() < 16; ++j) {
        if (used[j]) continue;
        const Desc& e = v[j];
        if (!e.diag) {
          blocked |= 1 << e.rb[0];
          if (e.n == 2) blocked |= 1 << e.rb[1];
          continue;
        }
        if (sign_diag(e) && e.run_mask == 0 && !(reg_bits(e) & blocked)) pick.push_back(j);
      }
      if (pick.size() >= 2) {
        for (size_t k = 0; k < pick.size(); ++k) {
          g[o] = v[pick[k]];
          g[o].run_mask = k == 0 ? (int32_t)pick.size() : 0;
          used[pick[k]] = 1;
          ++o;
        }
        continue;
      }
    }
    g[o] = v[i];
    used[i] = 1;
    ++o;
  }
}

template <class Desc>
void mark_runs(Desc* g, int n) {
  // whether d acts on register bit r (a count group's header carries no bits: its members do)
  auto touches = [](const Desc& d, int r) {
    if (!d.diag) return d.rb[0] == r || (d.n == 2 && d.rb[1] == r);
    if (group_header(d)) return false;
    return d.kreg[0] == r || (d.n == 2 && d.kreg[1] == r);
  };
  const std::vector<Desc> v(g, g + n);
  std::vector<char> used(n, 0);
  int o = 0;
  for (int i = 0; i < n; ++i) {
    if (used[i]) continue;
    const Desc& d = v[i];
    if (!d.diag && d.n == 1 && d.rb[0] >= 0 && d.rb[0] < 4) {
      int pick[4] = {-1, -1, -1, -1};
      pick[d.rb[0]] = i;
      int mask = 1 << d.rb[0];
      for (int r = 0; r < 4; ++r) {
        if (r == d.rb[0]) continue;
        for (int j = i + 1; j < n; ++j) {
          if (used[j]) continue;
          const Desc& e = v[j];
          if (!e.diag && e.n == 1 && e.rb[0] == r && run_form(e) == run_form(d)) {
            pick[r] = j;
            mask |= 1 << r;
            break;
          }
          if (touches(e, r)) break;
        }
      }
      if (mask != (1 << d.rb[0])) {
        bool first = true;
        for (int r = 0; r < 4; ++r) {
          if (pick[r] < 0) continue;
          g[o] = v[pick[r]];
          g[o].run_mask = first ? mask : 0;
          first = false;
          used[pick[r]] = 1;
          ++o;
        }
        continue;
      }
    }
    g[o] = v[i];
    g[o].run_mask = 0;
    used[i] = 1;
    ++o;
  }
}

void build_chains(tn_path* path, int T) {
  path->chains.clear();
  path->passes.clear();
  path->segments.clear();
  path->sweep_gates.clear();
  path->sweep_val_src.clear();
  const int S = (int)path->steps.size();
  auto sweepable = [&](int s) {
    const StepProgram& P = path->steps[s];
    if (P.kind != SK_SKINNY || P.sk.c_mode != 0 || P.sk.t_bits < 16 || !P.pre.empty()) return false;
    const SkinnyDesc& d = P.sk;
    if (d.nb == 0) return d.nk == d.nm && d.nk >= 1 && d.nk <= 2;
    return d.nk == 0 && d.nm == 0 && d.nb <= 2;
  };
  for (int s = path->n_small; s < S;) {
    if (!sweepable(s)) { ++s; continue; }
    int e = s + 1;
    while (e < S && sweepable(e)) {
      // the next step must act on this step's result
      const int ia = path->pairs[2 * e], ib = path->pairs[2 * e + 1];
      if (ia != T + e - 1 && ib != T + e - 1) break;
      const StepProgram& Q = path->steps[e];
      const StepProgram& P = path->steps[e - 1];
      if (Q.sk.t.buf != P.sk.c.buf || Q.sk.t.off != P.sk.c.off || Q.sk.t_bits != P.sk.t_bits) break;
      ++e;
    }
    if (e - s < 2) { s = e; continue; }
    SweepChain ch;
    ch.in = path->steps[s].sk.t;
    ch.out = path->steps[e - 1].sk.c;
    ch.bits = path->steps[s].sk.t_bits;
    ch.first_pass = (int32_t)path->passes.size();
    ch.n_steps = e - s;
    ch.first_val = (int32_t)path->sweep_val_src.size();
    ch.n_vals = 0;
    const int R = ch.bits;
    std::vector<PassItem> items;
    for (int i = s; i < e; ++i) {
      const SkinnyDesc& d = path->steps[i].sk;
      PassItem it;
      it.diag = d.nb > 0;
      it.movable = path->steps[i].zz_param == -2;  // ZZ phases stay together for count groups
      if (d.nb == 0) for (int j = 0; j < d.nk; ++j) it.pos.push_back(d.k_pos[j]);
      else for (int j = 0; j < d.nb; ++j) it.pos.push_back(d.bt_pos[j]);
      items.push_back(it);
    }
    std::vector<PlannedPass> planned;
    if (!plan_passes(R, items, planned)) {  // leave the chain to the per-step kernels
      s = e;
      continue;
    }
    for (const PlannedPass& pp : planned) {
      SweepPass ps;
      ps.l = pp.l;
      for (int j = 0; j < kSweepMaxLocal; ++j) ps.lpos[j] = j < ps.l ? (int8_t)pp.lpos[j] : 0;
      ps.first_gate = (int32_t)path->sweep_gates.size();
      ps.n_red = 0;
      ps.val_off = (int32_t)path->sweep_val_src.size() - ch.first_val;
      std::vector<int64_t> ctab;  // the pass's power tables
      // the descriptor of planned gate gi, its diagonal bits resolved for segment sg
      // (values: appended to the chain's value table unless `with_vals` is false)
      auto make_gd = [&](int gi, const PlannedSeg& sg, bool with_vals) {
        const PlannedGate& pg = pp.gates[gi];
        const SkinnyDesc& d = path->steps[s + pg.item].sk;
        SweepGateDesc gd;
        gd.diag = pg.diag;
        gd.n = pg.n;
        for (int j = 0; j < 2; ++j) {
          gd.lidx[j] = pg.lidx[j];
          gd.rb[j] = pg.rb[j];
        }
        gd.g_buf = d.g.buf;
        gd.unit = gd.diag ? d.g_unit : 0;
        gd.form = d.g_form;
        gd.g_off = d.g.off;
        for (int j = 0; j < 16; ++j) gd.gidx[j] = 0;
        const int ne = gd.diag ? (1 << gd.n) : (1 << (2 * gd.n));
        for (int j = 0; j < ne; ++j) gd.gidx[j] = d.gidx[j];
        // the gate's values, in the order the kernel reads them
        gd.voff = (int32_t)path->sweep_val_src.size() - ch.first_val;
        if (with_vals)
          for (int j = 0; j < ne; ++j)
            path->sweep_val_src.push_back((d.g.off + d.gidx[j]) | ((int64_t)d.g.buf << 56));
        gd.kreg[0] = gd.kreg[1] = -1;
        gd.csrc[0] = gd.csrc[1] = 0;
        if (gd.diag) {
          for (int j = 0; j < gd.n; ++j) {
            const int lj = gd.lidx[j];
            if (lj < 0) {
              gd.csrc[j] = 64 + (-lj - 1);
              continue;
            }
            for (int r = 0; r < 4; ++r)
              if (sg.rbits[r] == lj) gd.kreg[j] = r;
            if (gd.kreg[j] < 0) gd.csrc[j] = lj;
          }
        }
        return gd;
      };
      ps.first_seg = (int32_t)path->segments.size();
      for (const PlannedSeg& sg : pp.segs) {
        SweepSegment seg;
        for (int j = 0; j < 4; ++j) seg.rbits[j] = sg.rbits[j];
        seg.first_gate = (int32_t)path->sweep_gates.size();
        const int g_end = sg.first + sg.count;
        for (int g = sg.first; g < g_end;) {
          if (!pp.gates[g].diag) {
            path->sweep_gates.push_back(make_gd(g, sg, true));
            ++g;
            continue;
          }
          // a run of consecutive diagonal gates commutes: its ZZ phases that share one angle
          // become count groups, the rest keep their order
          int g2 = g;
          while (g2 < g_end && pp.gates[g2].diag) ++g2;
          std::vector<std::pair<std::pair<int32_t, double>, std::vector<int>>> groups;
          std::vector<int> rest;
          for (int q = g; q < g2; ++q) {
            const StepProgram& P = path->steps[s + pp.gates[q].item];
            if (P.zz_param == -2) {
              rest.push_back(q);
              continue;
            }
            const std::pair<int32_t, double> key(P.zz_param, P.zz_angle);
            size_t k = 0;
            while (k < groups.size() && (groups[k].first != key || groups[k].second.size() >= (size_t)kCountMaxEdges))
              ++k;
            if (k == groups.size()) groups.push_back({key, {}});
            groups[k].second.push_back(q);
          }
          for (auto& gr : groups)
            if (gr.second.size() < 2 || ctab.size() + gr.second.size() + 1 > (size_t)kCountTabMax) {
              rest.insert(rest.end(), gr.second.begin(), gr.second.end());
              gr.second.clear();
            }
          std::sort(rest.begin(), rest.end());
          for (int q : rest) path->sweep_gates.push_back(make_gd(q, sg, true));
          for (const auto& gr : groups) {
            if (gr.second.empty()) continue;
            const int E = (int)gr.second.size();
            const SkinnyDesc& d0 = path->steps[s + pp.gates[gr.second[0]].item].sk;
            SweepGateDesc h = make_gd(gr.second[0], sg, false);
            h.form = kFormCount;
            h.n = E;
            h.voff = (int32_t)ctab.size();  // index in the pass's tables
            const int64_t w_src = (d0.g.off + d0.gidx[1]) | ((int64_t)d0.g.buf << 56);  // entry of differing bits
            for (int c = 0; c <= E; ++c) ctab.push_back(w_src | kValPow | ((int64_t)c << kValExpShift));
            path->sweep_gates.push_back(h);
            for (int q : gr.second) {
              SweepGateDesc m = make_gd(q, sg, false);
              m.form = kFormCountMember;
              path->sweep_gates.push_back(m);
            }
          }
          g = g2;
        }
        seg.n_gates = (int32_t)path->sweep_gates.size() - seg.first_gate;
        // the segment's diagonal gates on bits outside its registers first: they commute with
        // every other gate of the segment and change only a per-thread factor, so the kernel
        // runs them in a loop of their own that leaves the register elements alone
        std::stable_partition(path->sweep_gates.begin() + seg.first_gate, path->sweep_gates.end(),
                              [](const SweepGateDesc& gd) {
                                return gd.diag && gd.form != kFormCount && gd.form != kFormCountMember &&
                                       gd.kreg[0] < 0 && (gd.n == 1 || gd.kreg[1] < 0);
                              });
        mark_runs(path->sweep_gates.data() + seg.first_gate, seg.n_gates);
        mark_diag_runs(path->sweep_gates.data() + seg.first_gate, seg.n_gates);
        mark_sign_runs(path->sweep_gates.data() + seg.first_gate, seg.n_gates);
        fill_segment_tables(seg, ps.l);
        path->segments.push_back(seg);
      }
      ps.n_segs = (int32_t)pp.segs.size();
      ps.n_gates = (int32_t)path->sweep_gates.size() - ps.first_gate;
      ps.ctab_off = (int32_t)path->sweep_val_src.size() - ch.first_val;
      ps.ctab_n = (int32_t)ctab.size();
      path->sweep_val_src.insert(path->sweep_val_src.end(), ctab.begin(), ctab.end());
      path->passes.push_back(ps);
    }
    ch.n_passes = (int32_t)path->passes.size() - ch.first_pass;
    ch.n_vals = (int32_t)path->sweep_val_src.size() - ch.first_val;
    path->steps[s].chain = (int32_t)path->chains.size();
    for (int i = s + 1; i < e; ++i) path->steps[i].chain = -2;
    path->chains.push_back(ch);
    s = e;
  }
}

}  // namespace

std::vector<int32_t> output_layout(const tn_network* net) {
  std::vector<int32_t> to;
  if (net->output_kind == TN_OUT_STATEVECTOR) {
    for (int q = 0; q < net->n_qubits; ++q) to.push_back(label(net->wire_final[q], 0));
  } else {
    for (int j = net->batch_log2 - 1; j >= 0; --j) to.push_back(label(net->batch_mode, j));
  }
  return to;
}

// Runs of outer products with one-qubit vectors (see OuterChain), e.g. a
// product state growing one qubit at a time before the gates act on it.
void build_outer_chains(tn_path* path, int T) {
  path->outers.clear();
  const int S = (int)path->steps.size();
  auto outer_step = [&](int s) {
    const StepProgram& P = path->steps[s];
    const SkinnyDesc& d = P.sk;
    return P.kind == SK_SKINNY && P.chain == -1 && P.pre.empty() && d.nk == 0 && d.nm == 1 && d.nb == 0 &&
           d.c_mode == 1 && d.mofs[0] == 0 && d.mofs[1] == ((int64_t)1 << d.t_bits);
  };
  for (int s = path->n_small; s < S;) {
    if (!outer_step(s)) {
      ++s;
      continue;
    }
    int e = s + 1;
    while (e < S && e - s < kOuterMax && outer_step(e)) {
      // the next step must act on this step's result
      const int ia = path->pairs[2 * e], ib = path->pairs[2 * e + 1];
      if (ia != T + e - 1 && ib != T + e - 1) break;
      const SkinnyDesc& q = path->steps[e].sk;
      const SkinnyDesc& p = path->steps[e - 1].sk;
      if (q.t.buf != p.c.buf || q.t.off != p.c.off || q.t_bits != p.t_bits + 1) break;
      ++e;
    }
    const SkinnyDesc& first = path->steps[s].sk;
    const SkinnyDesc& last = path->steps[e - 1].sk;
    // the launch reads T while it writes C: they may not overlap; a block per value of the
    // vector bits writes T's 2^t_bits elements, so T should not be tiny
    const int64_t tn = (int64_t)1 << first.t_bits, cn = (int64_t)1 << (last.t_bits + 1);
    const bool overlap = first.t.buf == last.c.buf && first.t.off < last.c.off + cn && last.c.off < first.t.off + tn;
    if (e - s < 2 || overlap || first.t_bits < 8) {
      s = e;
      continue;
    }
    OuterChain oc;
    oc.t = first.t;
    oc.c = last.c;
    oc.t_bits = first.t_bits;
    oc.k = e - s;
    oc.bytes = 8.0 * (double)(tn + cn);
    for (int i = 0; i < oc.k; ++i) {
      StepProgram& P = path->steps[s + i];
      for (int m = 0; m < 2; ++m) oc.vsrc[i][m] = (P.sk.g.off + P.sk.gidx[m]) | ((int64_t)P.sk.g.buf << 56);
      oc.flops += P.flops;
      P.outer = i == 0 ? (int32_t)path->outers.size() : -2;
    }
    path->outers.push_back(oc);
    s = e;
  }
}

tn_status compile_program(const tn_network* net, tn_path* path, const std::vector<int32_t>* final_layout) {
  const int T = (int)net->tensors.size();
  const int S = (int)path->pairs.size() / 2;
  std::vector<Loc> loc(T + S);
  std::vector<std::vector<int32_t>> modes(T + S);
  for (int t = 0; t < T; ++t) {
    loc[t].ref.buf = BUF_IN;
    loc[t].ref.off = net->tensors[t].offset;
    loc[t].bits = bits_of_modes(net, net->tensors[t].modes);
    loc[t].elems = net->tensors[t].size;
    loc[t].input = true;
    modes[t] = net->tensors[t].modes;
  }
  for (int s = 0; s < S; ++s) {
    loc[path->pairs[2 * s]].last_use = s;
    loc[path->pairs[2 * s + 1]].last_use = s;
  }
  // holder counts, replayed along the path
  std::vector<int> holders(net->mode_log2.size(), 0);
  std::vector<char> is_out(net->mode_log2.size(), 0);
  for (int m : net->output_modes) is_out[m] = 1;
  for (int t = 0; t < T; ++t)
    for (int m : modes[t]) holders[m]++;

  // workspace ranges each step reads and writes (for grouping steps into one launch)
  struct Foot {
    BufRef rd[2], wr[2];
    int64_t n_rd[2] = {0, 0}, n_wr[2] = {0, 0};
  };
  std::vector<Foot> foot(S);
  std::vector<std::pair<int64_t, int64_t>> deferred;  // frees held back until the current run ends
  std::vector<int> run;
  std::vector<char> in_run(S, 0);
  int run_len = 0;
  Alloc alloc;
  alloc.top = alloc.peak = path->small_region;  // [0, small_region): results of the interpreter's steps
  int64_t small_bump = 0;
  path->steps.assign(S, StepProgram());
  path->step_modes.assign(S, {});
  tn_path_stats& st = path->stats;
  st.flops = st.bytes = st.max_intermediate_elems = st.large_step_flops = 0;
  st.n_steps = S;
  st.n_permutes = st.n_gemm_steps = st.n_skinny_steps = 0;
  for (int t = 0; t < T; ++t) st.max_intermediate_elems = std::max(st.max_intermediate_elems, (double)loc[t].elems);

  for (int s = 0; s < S; ++s) {
    const int ia = path->pairs[2 * s], ib = path->pairs[2 * s + 1];
    const int ic = T + s;
    Loc& A = loc[ia];
    Loc& B = loc[ib];
    StepProgram& P = path->steps[s];
    foot[s].rd[0] = A.ref;
    foot[s].rd[1] = B.ref;
    foot[s].n_rd[0] = A.elems;
    foot[s].n_rd[1] = B.elems;
    // ---- classify modes
    std::map<int, int> mcls;
    auto in = [](const std::vector<int32_t>& v, int m) { return std::find(v.begin(), v.end(), m) != v.end(); };
    std::vector<int32_t> cmodes;
    for (int m : modes[ia]) {
      if (in(modes[ib], m)) {
        const bool kept = is_out[m] || holders[m] > 2;
        mcls[m] = kept ? C_BATCH : C_K;
      } else {
        if (!(is_out[m] || holders[m] > 1)) return set_error(TN_EINVAL, "mode held by a single tensor");
        mcls[m] = C_M;
      }
    }
    for (int m : modes[ib])
      if (!in(modes[ia], m)) {
        if (!(is_out[m] || holders[m] > 1)) return set_error(TN_EINVAL, "mode held by a single tensor");
        mcls[m] = C_N;
      }
    std::map<int32_t, int> cls;
    for (int32_t b : A.bits) cls[b] = mcls[mode_of(b)];
    for (int32_t b : B.bits) cls[b] = mcls[mode_of(b)];
    int nbits[4] = {0, 0, 0, 0};
    for (auto& kv : cls) nbits[kv.second]++;
    const int64_t bsz = (int64_t)1 << nbits[C_BATCH], msz = (int64_t)1 << nbits[C_M];
    const int64_t nsz = (int64_t)1 << nbits[C_N], ksz = (int64_t)1 << nbits[C_K];
    const double flops = 8.0 * (double)bsz * (double)msz * (double)nsz * (double)ksz;
    const int64_t c_elems = bsz * msz * nsz;
    P.flops = flops;
    P.gemm_bmnk[0] = bsz; P.gemm_bmnk[1] = msz; P.gemm_bmnk[2] = nsz; P.gemm_bmnk[3] = ksz;
    P.bytes = 8.0 * (double)(A.elems + B.elems + c_elems);

    // ---- choose the kernel
    const bool a_small = A.elems <= B.elems;
    Loc& G = a_small ? A : B;
    Loc& Tt = a_small ? B : A;
    const int g_only = a_small ? C_M : C_N;   // class of G's private bits
    const int g_bits = (int)G.bits.size();
    const int nk = nbits[C_K], nm = nbits[g_only], nb = nbits[C_BATCH];
    Loc& C = loc[ic];
    C.elems = c_elems;
    const bool skinny_kind = g_bits <= kSkinnyMaxG && nk <= kSkinnyMaxK && nm <= kSkinnyMaxM &&
                             c_elems > ((int64_t)1 << kElemSkinnyBits);
    // products that may share a launch with the run before them: what they
    // free stays reserved until the run ends, so no member overwrites another's operand
    const bool cand = s >= path->n_small && !skinny_kind &&
                      elem_group_shape(nbits[C_BATCH] + nbits[C_M] + nbits[C_N], nbits[C_M], nbits[C_N], nbits[C_K]);
    {
      bool joins = cand && run_len > 0 && run_len < kElemGroupMax;
      for (int k = 0; k < 2 && joins; ++k)
        if (path->pairs[2 * s + k] >= T && in_run[path->pairs[2 * s + k] - T]) joins = false;
      if (!joins) {
        for (const auto& f : deferred) alloc.put(f.first, f.second);
        deferred.clear();
        for (int m : run) in_run[m] = 0;
        run.clear();
        run_len = 0;
      }
      if (cand) {
        run.push_back(s);
        in_run[s] = 1;
        ++run_len;
      }
    }
    // result layout of a gate-sized product, as the streaming kernel writes it:
    // the large operand's layout with the small operand's own bits at the summed
    // positions when the counts match, else [G's own bits | T's other bits]
    const bool skinny_shape = g_bits <= kSkinnyMaxG && nk <= kSkinnyMaxK && nm <= kSkinnyMaxM;
    auto skinny_layout = [&]() {
      const int tb = (int)Tt.bits.size();
      std::vector<int32_t> klab, outer;  // by ascending position in T
      for (int p = 0; p < tb; ++p) {
        const int32_t lab = Tt.bits[tb - 1 - p];
        if (cls[lab] == C_K) klab.push_back(lab); else outer.push_back(lab);
      }
      std::vector<int32_t> mlab = filter(G.bits, cls, g_only);
      std::reverse(mlab.begin(), mlab.end());
      std::vector<int32_t> out;
      if (nm == nk) {
        out = Tt.bits;
        for (int j = 0; j < nk; ++j) out[tb - 1 - pos_of(Tt.bits, klab[j])] = mlab[j];
      } else {
        out.assign(mlab.rbegin(), mlab.rend());
        out.insert(out.end(), outer.rbegin(), outer.rend());
      }
      return out;
    };
    if (s < path->n_small) {
      P.kind = SK_SMALL;
      // C's layout: the large operand's, with a gate-sized operand's output bits at the summed
      // positions when the counts match; else [batch | M | N]
      const bool skinny_like = g_bits <= kSkinnyMaxG && nk == nm && nk <= kSkinnyMaxK;
      if (skinny_like) {
        std::vector<int32_t> klab;
        for (int p = 0; p < (int)Tt.bits.size(); ++p) {
          int32_t lab = Tt.bits[Tt.bits.size() - 1 - p];
          if (cls[lab] == C_K) klab.push_back(lab);
        }
        std::vector<int32_t> mlab = filter(G.bits, cls, g_only);
        std::reverse(mlab.begin(), mlab.end());
        C.bits = Tt.bits;
        for (int j = 0; j < nk; ++j) C.bits[Tt.bits.size() - 1 - pos_of(Tt.bits, klab[j])] = mlab[j];
      } else {
        C.bits = cat(filter(A.bits, cls, C_BATCH), filter(A.bits, cls, C_M), filter(B.bits, cls, C_N));
      }
      // every result of the interpreter gets a buffer of its own: independent steps of a
      // level run concurrently, so none may overwrite another's operand
      C.ref.buf = BUF_WS;
      C.ref.off = small_bump;
      small_bump += Alloc::round(C.elems);
      SmallStep& d = P.sm;
      d.a_buf = A.ref.buf == -1 ? BUF_WS : A.ref.buf;
      d.b_buf = B.ref.buf == -1 ? BUF_WS : B.ref.buf;
      d.a_off = A.ref.off;
      d.b_off = B.ref.off;
      d.c_buf = C.ref.buf;
      d.c_off = C.ref.off;
      d.c_bits = (int32_t)C.bits.size();
      d.a_bits = (int16_t)A.bits.size();
      d.b_bits = (int16_t)B.bits.size();
      for (int p = 0; p < kSmallMaxBits; ++p) d.apos[p] = d.bpos[p] = d.ka[p] = d.kb[p] = -1;
      for (int p = 0; p < d.c_bits; ++p) {
        const int32_t lab = C.bits[C.bits.size() - 1 - p];
        d.apos[p] = (int8_t)pos_of(A.bits, lab);
        d.bpos[p] = (int8_t)pos_of(B.bits, lab);
      }
      int j = 0;
      for (int32_t lab : A.bits)
        if (cls[lab] == C_K) {
          d.ka[j] = (int8_t)pos_of(A.bits, lab);
          d.kb[j] = (int8_t)pos_of(B.bits, lab);
          ++j;
        }
      d.k_bits = j;
    } else if (skinny_kind) {
      P.kind = SK_SKINNY;
      st.n_skinny_steps++;
      SkinnyDesc& d = P.sk;
      d.t_bits = (int32_t)Tt.bits.size();
      d.nk = nk; d.nm = nm; d.nb = nb;
      // K labels by ascending position in T
      std::vector<int32_t> klab, outer;  // outer: ascending positions
      for (int p = 0; p < d.t_bits; ++p) {
        int32_t lab = Tt.bits[d.t_bits - 1 - p];
        if (cls[lab] == C_K) klab.push_back(lab); else outer.push_back(lab);
      }
      for (int j = 0; j < nk; ++j) d.k_pos[j] = pos_of(Tt.bits, klab[j]);
      std::vector<int32_t> mlab = filter(G.bits, cls, g_only);  // MSB first
      std::reverse(mlab.begin(), mlab.end());                  // m bit j = mlab[j]
      std::vector<int32_t> blab = filter(G.bits, cls, C_BATCH);
      std::reverse(blab.begin(), blab.end());
      for (int j = 0; j < nb; ++j) {
        int p = (int)(std::find(outer.begin(), outer.end(), blab[j]) - outer.begin());
        d.b_pos[j] = p;
        d.bt_pos[j] = pos_of(Tt.bits, blab[j]);
      }
      // C layout
      d.c_mode = nm == nk ? 0 : 1;
      C.bits = skinny_layout();
      for (int k = 0; k < (1 << nk); ++k) {
        int64_t o = 0;
        for (int j = 0; j < nk; ++j)
          if ((k >> j) & 1) o |= (int64_t)1 << d.k_pos[j];
        d.kofs[k] = o;
      }
      for (int m = 0; m < (1 << nm); ++m) {
        int64_t o = 0;
        for (int j = 0; j < nm; ++j)
          if ((m >> j) & 1) o |= (int64_t)1 << pos_of(C.bits, mlab[j]);
        d.mofs[m] = o;
      }
      std::vector<int32_t> klab_g = klab;  // k bit j = klab[j]
      for (int b = 0; b < (1 << nb); ++b)
        for (int m = 0; m < (1 << nm); ++m)
          for (int k = 0; k < (1 << nk); ++k) {
            int64_t a = 0;
            for (int j = 0; j < nb; ++j)
              if ((b >> j) & 1) a |= (int64_t)1 << pos_of(G.bits, blab[j]);
            for (int j = 0; j < nm; ++j)
              if ((m >> j) & 1) a |= (int64_t)1 << pos_of(G.bits, mlab[j]);
            for (int j = 0; j < nk; ++j)
              if ((k >> j) & 1) a |= (int64_t)1 << pos_of(G.bits, klab_g[j]);
            d.gidx[((b << nm) + m) * (1 << nk) + k] = (int32_t)a;
          }
      d.g = G.ref;
      // the gate tensor's value shape, from its gate kinds: unit-modulus or +-1 diagonals; real or
      // RX-like one-qubit matrices (products of real matrices are real, of RX-like ones RX-like)
      d.g_unit = 0;
      d.g_form = kFormGeneric;
      {
        const int gid = a_small ? ia : ib;
        if (gid < T && net->tensors[gid].kind == TK_GATE && net->tensors[gid].recipe >= 0) {
          const Recipe& r = net->recipes[net->tensors[gid].recipe];
          bool unit = true, signs = true, real = true, rxl = true;
          for (int o = r.op_begin; o < r.op_end; ++o) {
            const int k = net->ops[o].kind;
            unit &= k == TN_GATE_Z || k == TN_GATE_S || k == TN_GATE_T || k == TN_GATE_RZ || k == TN_GATE_CZ ||
                    k == TN_GATE_CPHASE || k == TN_GATE_ZZPHASE;
            signs &= k == TN_GATE_Z || k == TN_GATE_CZ;
            real &= k == TN_GATE_H || k == TN_GATE_X || k == TN_GATE_Z || k == TN_GATE_RY || k == TN_GATE_CZ ||
                    k == TN_GATE_CNOT || k == TN_GATE_SWAP;
            rxl &= k == TN_GATE_RX || k == TN_GATE_MIXER || k == TN_GATE_Y;
          }
          const bool whole = r.split_side < 0 && r.op_end > r.op_begin;
          if (d.nk == 0 && d.nm == 0 && r.diag && whole) {
            d.g_unit = unit ? 1 : 0;
            d.g_form = signs ? kFormSigns : unit ? kFormUnit : kFormGeneric;
            if (d.nb == 2 && r.nq == 2 && r.op_end - r.op_begin == 1 && net->ops[r.op_begin].kind == TN_GATE_ZZPHASE) {
              P.zz_param = net->ops[r.op_begin].param[0];
              P.zz_angle = P.zz_param >= 0 ? 0.0 : net->ops[r.op_begin].angle[0];
            }
          } else if (d.nb == 0 && d.nk == 1 && d.nm == 1 && !r.diag && whole && r.nq == 1) {
            d.g_form = real ? kFormReal : rxl ? kFormRxLike : kFormGeneric;
          }
        }
      }
      d.t = Tt.ref;
      // output buffer: in place over T when T dies here and the layout positions coincide
      if (d.c_mode == 0 && !Tt.input && Tt.last_use == s && Tt.elems == C.elems) {
        C.ref = Tt.ref;
        Tt.ref.buf = -1;  // ownership moved
      } else {
        C.ref.buf = BUF_WS;
        C.ref.off = alloc.get(C.elems);
      }
      d.c = C.ref;
    } else {
      P.kind = SK_GEMM;
      st.n_gemm_steps++;
      // C: the requested output layout for the last step, else [batch | M | N] in the operands' orders
      if (s == S - 1 && final_layout && final_layout->size() == (size_t)nbits[0] + nbits[1] + nbits[2]) {
        C.bits = *final_layout;
      } else if (skinny_shape) {
        C.bits = skinny_layout();  // a small gate-sized product keeps the streaming kernel's layout
      } else {
        C.bits = cat(filter(A.bits, cls, C_BATCH), filter(A.bits, cls, C_M), filter(B.bits, cls, C_N));
      }
      C.ref.buf = BUF_WS;
      C.ref.off = alloc.get(C.elems);
      // Two orientations: C = A B, or C = B^T A^T (operands trade places, m and
      // n trade roles).  The kernel stores its result tile with consecutive
      // lanes along n, so the transposed form suits a result whose lowest
      // address bits are m bits; which one runs is a launch-shape choice.
      for (int o = 0; o < 2; ++o) {
        const bool swap = o == 1;
        Loc& GA = swap ? B : A;
        Loc& GB = swap ? A : B;
        const int CM = swap ? C_N : C_M, CN = swap ? C_M : C_N;
        // logical bit orders: batch, m, n by ascending position in C; k by ascending position in A
        auto by_pos = [&](const std::vector<int32_t>& layout, int c) {
          std::vector<int32_t> v;
          for (int p = 0; p < (int)layout.size(); ++p) {
            const int32_t lab = layout[layout.size() - 1 - p];
            if (cls[lab] == c) v.push_back(lab);
          }
          return v;
        };
        const std::vector<int32_t> lb_ = by_pos(C.bits, C_BATCH), lm = by_pos(C.bits, CM), ln = by_pos(C.bits, CN),
                                   lk = by_pos(GA.bits, C_K);
        GemmDesc& g = P.gm[o];
        g.swapped = o;
        g.batch = bsz; g.M = swap ? nsz : msz; g.N = swap ? msz : nsz; g.K = ksz;
        g.nbb = (int32_t)lb_.size(); g.nbm = (int32_t)lm.size(); g.nbn = (int32_t)ln.size();
        g.nbk = (int32_t)lk.size();
        if (g.nbb > kGemmMaxBits || g.nbm > kGemmMaxBits || g.nbn > kGemmMaxBits || g.nbk > kGemmMaxBits)
          return set_error(TN_EUNSUPPORTED, "contraction index wider than 2^40");
        for (int j = 0; j < kGemmMaxBits; ++j)
          g.a_b[j] = g.a_m[j] = g.a_k[j] = g.b_b[j] = g.b_k[j] = g.b_n[j] = g.c_b[j] = g.c_m[j] = g.c_n[j] = 0;
        for (int j = 0; j < g.nbb; ++j) {
          g.a_b[j] = (int8_t)pos_of(GA.bits, lb_[j]);
          g.b_b[j] = (int8_t)pos_of(GB.bits, lb_[j]);
          g.c_b[j] = (int8_t)pos_of(C.bits, lb_[j]);
        }
        for (int j = 0; j < g.nbm; ++j) {
          g.a_m[j] = (int8_t)pos_of(GA.bits, lm[j]);
          g.c_m[j] = (int8_t)pos_of(C.bits, lm[j]);
        }
        for (int j = 0; j < g.nbn; ++j) {
          g.b_n[j] = (int8_t)pos_of(GB.bits, ln[j]);
          g.c_n[j] = (int8_t)pos_of(C.bits, ln[j]);
        }
        for (int j = 0; j < g.nbk; ++j) {
          g.a_k[j] = (int8_t)pos_of(GA.bits, lk[j]);
          g.b_k[j] = (int8_t)pos_of(GB.bits, lk[j]);
        }
        // tile-load orientation: walk the index owning the operand's lowest m/k (k/n) address bit fastest
        auto lowest_cls = [&](const std::vector<int32_t>& layout, int c1, int c2) {
          for (int p = 0; p < (int)layout.size(); ++p) {
            const int c = cls[layout[layout.size() - 1 - p]];
            if (c == c1 || c == c2) return c;
          }
          return c2;
        };
        g.a_kfast = lowest_cls(GA.bits, CM, C_K) == C_K ? 1 : 0;
        g.b_nfast = lowest_cls(GB.bits, C_K, CN) == CN ? 1 : 0;
        g.a = GA.ref;
        g.b = GB.ref;
        g.c = C.ref;
        int tile, split;
        gemm_default_launch(g, &tile, &split);
        g.tile[0] = g.tile[1] = tile;
        g.split[0] = g.split[1] = split;
        // FP32: the three-product form where its 64-column tiles fit
        if ((tile == 0 || tile == 2) && g.N >= 64) g.tile[TN_PREC_C64] = tile == 0 ? 5 : 6;
        // room for the autotuner to try K splits of products with a small result
        g.max_split = split;
        if (tile != kGemmVector && C.elems * kGemmMaxSplit <= ((int64_t)1 << 22) && g.K >= 64)
          g.max_split = kGemmMaxSplit;
      }
      // a matrix-core tile stores each row of its result as 32 consecutive columns per wave:
      // for a short sum the stores are the product's time, so take the orientation whose
      // columns are the result's lowest address bits (the tuner may still choose otherwise)
      P.orient[0] = P.orient[1] = 0;
      {
        auto low_n = [](const GemmDesc& g) {
          int c = 0;
          while (c < g.nbn && c < 5 && g.c_n[c] == c) ++c;
          return c;
        };
        for (int prec = 0; prec < 2; ++prec)
          if (P.gm[0].K <= 32 && P.gm[0].tile[prec] != kGemmVector && P.gm[1].tile[prec] != kGemmVector &&
              low_n(P.gm[1]) > low_n(P.gm[0]))
            P.orient[prec] = 1;
      }
      const int max_split = std::max(P.gm[0].max_split, P.gm[1].max_split);
      if (max_split > 1) {
        BufRef tmp;
        tmp.buf = BUF_WS;
        tmp.off = alloc.get((int64_t)max_split * C.elems);
        alloc.put(tmp.off, (int64_t)max_split * C.elems);  // scratch for this step only
        for (GemmDesc& g : P.gm) g.tmp = tmp;
      }
      P.gemm_bmnk[1] = P.gm[0].M;
      P.gemm_bmnk[2] = P.gm[0].N;
    }
    foot[s].wr[0] = C.ref;
    foot[s].n_wr[0] = C.elems;
    if (P.kind == SK_GEMM && P.gm[0].max_split > 1) {
      foot[s].wr[1] = P.gm[0].tmp;
      foot[s].n_wr[1] = (int64_t)std::max(P.gm[0].max_split, P.gm[1].max_split) * C.elems;
    }
    // ---- bookkeeping
    for (int m : modes[ia]) holders[m]--;
    for (int m : modes[ib]) holders[m]--;
    std::vector<int32_t> cm;
    for (size_t i = 0; i < C.bits.size(); ++i) {
      int m = mode_of(C.bits[i]);
      if (cm.empty() || cm.back() != m) cm.push_back(m);
    }
    modes[ic] = cm;
    for (int m : cm) holders[m]++;
    path->step_modes[s] = cm;
    for (Loc* X : {&A, &B})
      if (!X->input && X->last_use == s && X->ref.buf == BUF_WS) {
        // buffers of the interpreter's results are released only once the interpreter has run
        if (s >= path->n_small) {
          if (cand) deferred.emplace_back(X->ref.off, X->elems);
          else alloc.put(X->ref.off, X->elems);
        }
        X->ref.buf = -1;
      }
    if (s == path->n_small - 1) {
      // the interpreter's results that later steps read stay where they are; the rest of
      // the small region becomes free
      if (small_bump > path->small_region) return set_error(TN_EINVAL, "internal: small region overflow");
    }
    st.flops += P.flops;
    st.bytes += P.bytes;
    st.max_intermediate_elems = std::max(st.max_intermediate_elems, (double)C.elems);
    const double inten = P.flops / (8.0 * (double)(A.elems + B.elems + C.elems));
    if (P.flops >= 1e9 && inten >= 40.0) st.large_step_flops += P.flops;
  }
  // ---- consistency checks of every descriptor before anything can reach a GPU
  auto ref_ok = [&](const BufRef& r, int64_t elems) {
    if (r.buf == BUF_IN) return r.off >= 0 && r.off + elems <= net->input_elems;
    if (r.buf == BUF_WS) return r.off >= 0 && r.off + elems <= alloc.peak;
    return false;
  };
  for (int s = path->n_small; s < S; ++s) {
    const StepProgram& P = path->steps[s];
    const int ia = path->pairs[2 * s], ib = path->pairs[2 * s + 1];
    const int64_t ea = loc[ia].elems, eb = loc[ib].elems, ec = loc[T + s].elems;
    for (const PermuteDesc& pd : P.pre) {
      const int64_t e = (int64_t)1 << pd.bits;
      if (!ref_ok(pd.in, e) || !ref_ok(pd.out, e)) return set_error(TN_EINVAL, "internal: permute buffer out of range");
      std::vector<char> seen(pd.bits, 0);
      for (int p = 0; p < pd.bits; ++p) {
        if (pd.dst[p] < 0 || pd.dst[p] >= pd.bits || seen[pd.dst[p]]) return set_error(TN_EINVAL, "internal: bad permutation");
        seen[pd.dst[p]] = 1;
      }
    }
    if (P.kind == SK_SKINNY) {
      const SkinnyDesc& d = P.sk;
      const int64_t te = (int64_t)1 << d.t_bits;
      const int64_t ge = std::min(ea, eb);
      if (te != std::max(ea, eb) || !ref_ok(d.g, ge) || !ref_ok(d.t, te) || !ref_ok(d.c, ec))
        return set_error(TN_EINVAL, "internal: skinny buffer out of range");
      const int outer_bits = d.t_bits - d.nk;
      for (int j = 0; j < d.nk; ++j)
        if (d.k_pos[j] < 0 || d.k_pos[j] >= d.t_bits || (j && d.k_pos[j] <= d.k_pos[j - 1]))
          return set_error(TN_EINVAL, "internal: bad summed-bit positions");
      for (int j = 0; j < d.nb; ++j)
        if (d.b_pos[j] < 0 || d.b_pos[j] >= outer_bits) return set_error(TN_EINVAL, "internal: bad batch-bit positions");
      for (int i = 0; i < (1 << (d.nb + d.nm + d.nk)); ++i)
        if (d.gidx[i] < 0 || d.gidx[i] >= ge) return set_error(TN_EINVAL, "internal: bad small-operand index");
      for (int k = 0; k < (1 << d.nk); ++k)
        if (d.kofs[k] < 0 || d.kofs[k] >= te) return set_error(TN_EINVAL, "internal: bad operand offset");
      const int64_t cmax = d.c_mode ? ((int64_t)1 << outer_bits) : te;
      for (int m = 0; m < (1 << d.nm); ++m)
        if (d.mofs[m] < 0 || (d.mofs[m] | (cmax - 1)) >= ec) return set_error(TN_EINVAL, "internal: bad output offset");
      if (d.c_mode == 0 && ec != te) return set_error(TN_EINVAL, "internal: in-layout output size mismatch");
      if (d.c_mode == 1 && ec != ((int64_t)1 << (outer_bits + d.nm))) return set_error(TN_EINVAL, "internal: output size");
    } else {
     for (const GemmDesc& g : P.gm) {
      const int xa = g.swapped ? ib : ia, xb = g.swapped ? ia : ib;  // the kernel's A and B
      const int64_t ea = loc[xa].elems, eb = loc[xb].elems;
      if (g.batch * g.M * g.K != ea || g.batch * g.K * g.N != eb || g.batch * g.M * g.N != ec)
        return set_error(TN_EINVAL, "internal: GEMM shape mismatch");
      const int ra = (int)loc[xa].bits.size(), rb = (int)loc[xb].bits.size(), rc = (int)loc[T + s].bits.size();
      if (g.nbb + g.nbm + g.nbk != ra || g.nbb + g.nbk + g.nbn != rb || g.nbb + g.nbm + g.nbn != rc)
        return set_error(TN_EINVAL, "internal: GEMM bit counts");
      auto perm_ok = [](int r, std::initializer_list<std::pair<const int8_t*, int>> parts) {
        std::vector<char> seen(r, 0);
        for (auto& pr : parts)
          for (int j = 0; j < pr.second; ++j) {
            const int p = pr.first[j];
            if (p < 0 || p >= r || seen[p]) return false;
            seen[p] = 1;
          }
        return true;
      };
      if (g.max_split > 1 && !ref_ok(g.tmp, (int64_t)g.max_split * ec))
        return set_error(TN_EINVAL, "internal: split-K scratch out of range");
      if (!perm_ok(ra, {{g.a_b, g.nbb}, {g.a_m, g.nbm}, {g.a_k, g.nbk}}) ||
          !perm_ok(rb, {{g.b_b, g.nbb}, {g.b_k, g.nbk}, {g.b_n, g.nbn}}) ||
          !perm_ok(rc, {{g.c_b, g.nbb}, {g.c_m, g.nbm}, {g.c_n, g.nbn}}))
        return set_error(TN_EINVAL, "internal: GEMM bit positions");
      if (!ref_ok(g.a, ea) || !ref_ok(g.b, eb) || !ref_ok(g.c, ec))
        return set_error(TN_EINVAL, "internal: GEMM buffer out of range");
     }
    }
  }
  for (int s = 0; s < path->n_small; ++s) {
    const SmallStep& d = path->steps[s].sm;
    const int ia = path->pairs[2 * s], ib = path->pairs[2 * s + 1];
    auto buf_ok = [&](int buf, int64_t off, int64_t elems) {
      if (buf == BUF_IN) return off >= 0 && off + elems <= net->input_elems;
      if (buf == BUF_WS) return off >= 0 && off + elems <= alloc.peak;
      return false;
    };
    if (d.c_bits > kSmallMaxBits || d.k_bits > kSmallMaxBits || !buf_ok(d.a_buf, d.a_off, loc[ia].elems) ||
        !buf_ok(d.b_buf, d.b_off, loc[ib].elems) || !buf_ok(d.c_buf, d.c_off, loc[T + s].elems) ||
        ((int64_t)1 << d.c_bits) != loc[T + s].elems)
      return set_error(TN_EINVAL, "internal: bad small step");
    const int abits = (int)loc[ia].bits.size(), bbits = (int)loc[ib].bits.size();
    for (int p = 0; p < d.c_bits; ++p)
      if (d.apos[p] >= abits || d.bpos[p] >= bbits || (d.apos[p] < 0 && d.bpos[p] < 0))
        return set_error(TN_EINVAL, "internal: bad small-step bit map");
    for (int j = 0; j < d.k_bits; ++j)
      if (d.ka[j] < 0 || d.ka[j] >= abits || d.kb[j] < 0 || d.kb[j] >= bbits)
        return set_error(TN_EINVAL, "internal: bad small-step summed bits");
  }
  // steps that may share a launch: pairwise independent, and no step writes a
  // workspace range another one reads or writes
  {
    auto overlap = [](const BufRef& x, int64_t nx, const BufRef& y, int64_t ny) {
      return nx > 0 && ny > 0 && x.buf == y.buf && x.off < y.off + ny && y.off < x.off + nx;
    };
    auto compatible = [&](int i, int j) {
      for (int k = 0; k < 2; ++k)
        if (path->pairs[2 * j + k] == T + i || path->pairs[2 * i + k] == T + j) return false;
      const Foot &fi = foot[i], &fj = foot[j];
      for (int w = 0; w < 2; ++w)
        for (int k = 0; k < 2; ++k)
          if (overlap(fi.wr[w], fi.n_wr[w], fj.rd[k], fj.n_rd[k]) ||
              overlap(fj.wr[w], fj.n_wr[w], fi.rd[k], fi.n_rd[k]) ||
              overlap(fi.wr[w], fi.n_wr[w], fj.wr[k], fj.n_wr[k]))
            return false;
      return true;
    };
    for (int s = path->n_small; s < S; ++s) {
      StepProgram& P = path->steps[s];
      P.grp_from = s;
      if (P.kind != SK_GEMM) continue;
      for (int g = s - 1; g >= path->n_small && s - g < kElemGroupMax; --g) {
        if (path->steps[g].kind != SK_GEMM) break;
        bool ok = true;
        for (int t = g + 1; t <= s && ok; ++t) ok = compatible(g, t);
        if (!ok) break;
        P.grp_from = g;
      }
    }
  }
  // independent sub-trees of the interpreter's steps -> one work list each
  path->small_steps.clear();
  path->small_lists.clear();
  if (path->n_small > 0) {
    std::vector<int> consumer(S, -1);
    for (int s = 0; s < S; ++s)
      for (int k = 0; k < 2; ++k) {
        const int id = path->pairs[2 * s + k];
        if (id >= T) consumer[id - T] = s;
      }
    std::vector<int> root(path->n_small);
    for (int s = path->n_small - 1; s >= 0; --s) {
      const int c = consumer[s];
      root[s] = (c >= 0 && c < path->n_small) ? root[c] : s;
    }
    // level of a step = 1 + the deepest level among the steps producing its operands;
    // steps of one level are independent
    std::vector<int> level(path->n_small, 0);
    for (int s = 0; s < path->n_small; ++s) {
      int lv = 0;
      for (int k = 0; k < 2; ++k) {
        const int id = path->pairs[2 * s + k];
        if (id >= T) lv = std::max(lv, level[id - T] + 1);
      }
      level[s] = lv;
    }
    std::map<int, std::vector<int>> trees;
    for (int s = 0; s < path->n_small; ++s) trees[root[s]].push_back(s);
    path->small_levels.clear();
    path->small_items.clear();
    path->small_lists.push_back(0);
    for (auto& kv : trees) {
      std::vector<int> lst = kv.second;
      std::stable_sort(lst.begin(), lst.end(), [&](int x, int y) { return level[x] < level[y]; });
      for (size_t i = 0; i < lst.size(); ++i) {
        if (i == 0 || level[lst[i]] != level[lst[i - 1]])
          path->small_levels.push_back((int32_t)path->small_steps.size());
        path->small_steps.push_back(path->steps[lst[i]].sm);
      }
      path->small_lists.push_back((int32_t)path->small_levels.size());
    }
    path->small_levels.push_back((int32_t)path->small_steps.size());
    // rounds of each level (in chunks of kSmallDescCache steps, as the kernel
    // reads them): consecutive steps while their operands fit the stage
    for (size_t lv = 0; lv + 1 < path->small_levels.size(); ++lv) {
      const int l0 = path->small_levels[lv], l1 = path->small_levels[lv + 1];
      for (int cb = l0; cb < l1; cb += kSmallDescCache) {
        const int ce = std::min(l1, cb + kSmallDescCache);
        for (int r0 = cb; r0 < ce;) {
          int used = 0, outs = 0, i = r0;
          for (; i < ce; ++i) {
            SmallStep& d = path->small_steps[i];
            const int need = (1 << d.a_bits) + (1 << d.b_bits);
            if (i > r0 && used + need > kSmallStage) break;
            d.stage_a = used;
            d.stage_b = used + (1 << d.a_bits);
            d.out0 = outs;
            d.round_end = 0;
            d.item0 = d.n_items = d.pad2[0] = d.pad2[1] = 0;
            used += need;
            outs += 1 << d.c_bits;
          }
          path->small_steps[r0].round_end = i - cb;
          // work items: about equal work (outputs times summed terms, plus the
          // store) per thread, each a run of consecutive outputs of one step
          int64_t total = 0;
          for (int q = r0; q < i; ++q) {
            const SmallStep& d = path->small_steps[q];
            total += ((int64_t)1 << d.c_bits) * (((int64_t)1 << d.k_bits) + 4);
          }
          for (int64_t target = std::max<int64_t>(1, (total + kSmallThreads - 1) / kSmallThreads);; target *= 2) {
            std::vector<uint32_t> items;
            for (int q = r0; q < i; ++q) {
              const SmallStep& d = path->small_steps[q];
              const int64_t per = ((int64_t)1 << d.k_bits) + 4;
              int lc = 0;  // log2 of the outputs per item
              while (lc < d.c_bits && ((int64_t)2 << lc) * per <= target) ++lc;
              const int qb = d.c_bits - lc;
              for (int64_t j = 0; j < ((int64_t)1 << qb); ++j)
                items.push_back((uint32_t)(q - cb) | ((uint32_t)j << 8) | ((uint32_t)qb << 20));
            }
            if ((int)items.size() <= kSmallMaxItems) {
              // every output of every step of the round exactly once, in range
              std::vector<int64_t> covered(i - r0, 0);
              for (uint32_t it : items) {
                const int q = (int)(it & 255u) + cb, j = (int)((it >> 8) & 4095u), qb = (int)(it >> 20);
                if (q < r0 || q >= i || qb > path->small_steps[q].c_bits || j >= (1 << qb))
                  return set_error(TN_EINVAL, "internal: bad interpreter work item");
                covered[q - r0] += (int64_t)1 << (path->small_steps[q].c_bits - qb);
              }
              for (int q = r0; q < i; ++q)
                if (covered[q - r0] != ((int64_t)1 << path->small_steps[q].c_bits))
                  return set_error(TN_EINVAL, "internal: interpreter work items miss outputs");
              path->small_steps[r0].item0 = (int32_t)path->small_items.size();
              path->small_steps[r0].n_items = (int32_t)items.size();
              path->small_items.insert(path->small_items.end(), items.begin(), items.end());
              break;
            }
          }
          r0 = i;
        }
      }
    }
  }
  build_chains(path, T);
  build_outer_chains(path, T);
  st.n_product_launches = 0;
  for (int s = path->n_small, run0 = -1, run_len = 0; s < S; ++s) {
    const StepProgram& P = path->steps[s];
    if (P.chain != -1) {
      run0 = -1;
      continue;
    }
    if (elem_groupable(P, TN_PREC_C64) && run0 >= 0 && P.grp_from <= run0 && run_len < kElemGroupMax) {
      ++run_len;
    } else {
      st.n_product_launches++;
      run0 = elem_groupable(P, TN_PREC_C64) ? s : -1;
      run_len = 1;
    }
  }
  st.n_sweep_steps = st.n_sweep_passes = 0;
  for (const SweepChain& ch : path->chains) {
    st.n_sweep_steps += ch.n_steps;
    st.n_sweep_passes += ch.n_passes;
  }
  st.n_sweep_gate_runs = 0;
  for (const SweepGateDesc& gd : path->sweep_gates) st.n_sweep_gate_runs += gd.run_mask != 0;
  st.n_small_steps = path->n_small;
  st.n_small_lists = path->small_lists.empty() ? 0 : (int32_t)path->small_lists.size() - 1;
  const int last = S > 0 ? T + S - 1 : 0;
  if (S == 0 && T != 1) return set_error(TN_EINVAL, "empty path for a network of several tensors");
  if (S == 0) {
    // a single input tensor: copy it into the workspace so the result lives there
    loc[0].ref = loc[0].ref;
  }
  path->final_bits = loc[last].bits;
  path->final_ref = loc[last].ref;
  path->final_elems = loc[last].elems;
  // the chains' gathered gate values sit above every other buffer (chains run one at a time)
  int64_t max_vals = 0;
  for (const SweepChain& ch : path->chains) max_vals = std::max<int64_t>(max_vals, ch.n_vals);
  if (max_vals > 0) {
    const int64_t off = (alloc.peak + 31) & ~(int64_t)31;
    for (SweepChain& ch : path->chains) {
      ch.vals.buf = BUF_WS;
      ch.vals.off = off;
    }
    alloc.peak = off + max_vals;
  }
  path->ws_elems = std::max<int64_t>(alloc.peak, 32);
  path->n_inputs = T;
  build_q328_program(net, path);
  return TN_OK;
}

// A coarse model of the program's run time on MI355X, used to choose between
// orders: launch overhead per kernel, streaming kernels at a sustained HBM rate,
// permutes at their measured rate, matrix products at the sustained FP32
// matrix-core rate scaled down for tiles the shape leaves partly empty.
void build_adjoint_plan(const tn_network* net, tn_path* path, const std::vector<int32_t>& slot_of_gate) {
  path->adj_passes.clear();
  path->adj_segments.clear();
  path->adj_gates.clear();
  path->adj_state = -1;
  const int R = (int)path->final_bits.size();
  // whole waves for the gradient reductions need chunks of 2^10 elements at least
  if (R < 18 || path->final_elems != ((int64_t)1 << R) || path->final_ref.buf != BUF_WS) return;
  const int G = (int)net->sweep.size();
  if ((int)slot_of_gate.size() != G) return;
  // the passes' operations in a layout (-1: a gate the passes cannot take)
  auto make_items = [&](const std::vector<int32_t>& bits, std::vector<PassItem>& items) {
    items.clear();
    for (int gi = G - 1; gi >= 0; --gi) {  // the reverse sweep undoes the gates last to first
      const SweepGate& g = net->sweep[gi];
      if (g.nq == 2 && !g.diag && g.gen != GEN_NONE) return false;
      PassItem it;
      it.diag = g.diag != 0;
      it.grad = slot_of_gate[gi] >= 0;
      const int p0 = pos_of(bits, net->wire_final[g.q[0]] * 64);
      const int p1 = g.nq == 2 ? pos_of(bits, net->wire_final[g.q[1]] * 64) : 0;
      if (p0 < 0 || p1 < 0) return false;
      // bit 0 of the gate's own index is its second qubit (the first is the more significant)
      if (g.nq == 2) it.pos = {p1, p0};
      else it.pos = {p0};
      items.push_back(it);
    }
    return true;
  };
  std::vector<PassItem> items;
  std::vector<PlannedPass> planned;
  if (!make_items(path->final_bits, items) || !plan_passes(R, items, planned, kAdjPreGates, kAdjMaxRed)) return;
  path->adj_bits = path->final_bits;
  path->adj_perm = 0;
  // the qubit order (qubit 0 most significant) keeps neighbouring qubits on neighbouring bits, the
  // layout a contraction leaves need not; take it when its light cones need fewer passes (one
  // permute of the state costs about a pass's traffic on one state)
  if (R == net->n_qubits) {
    std::vector<int32_t> nat(R);
    for (int q = 0; q < R; ++q) nat[q] = net->wire_final[q] * 64;
    std::vector<PassItem> items2;
    std::vector<PlannedPass> planned2;
    if (nat != path->final_bits && make_items(nat, items2) &&
        plan_passes(R, items2, planned2, kAdjPreGates, kAdjMaxRed) && planned2.size() < planned.size()) {
      planned.swap(planned2);
      path->adj_bits = nat;
      path->adj_perm = 1;
    }
  }
  for (const PlannedPass& pp : planned) {
    SweepPass ps;
    ps.l = pp.l;
    for (int j = 0; j < kSweepMaxLocal; ++j) ps.lpos[j] = j < ps.l ? (int8_t)pp.lpos[j] : 0;
    ps.first_gate = (int32_t)path->adj_gates.size();
    ps.n_gates = (int32_t)pp.gates.size();
    ps.n_red = 0;
    for (const PlannedGate& pg : pp.gates) {
      const int gi = G - 1 - pg.item;
      const SweepGate& g = net->sweep[gi];
      AdjGateDesc gd;
      gd.diag = pg.diag;
      gd.n = pg.n;
      for (int j = 0; j < 2; ++j) {
        gd.lidx[j] = pg.lidx[j];
        gd.rb[j] = pg.rb[j];
      }
      gd.gate = gi;
      gd.slot = slot_of_gate[gi];
      gd.red = gd.slot >= 0 ? ps.n_red++ : -1;
      gd.form = ADJ_GENERIC;
      // generator G with g = Im<lambda|G|psi> (the derivative of the gate is -i G / 2 or -i G)
      for (float& x : gd.gen) x = 0.f;
      auto set = [&](int k, float re, float im) { gd.gen[2 * k] = re; gd.gen[2 * k + 1] = im; };
      switch (gd.slot >= 0 ? g.gen : GEN_NONE) {
        case GEN_X_HALF: set(1, 1, 0); set(2, 1, 0); break;            // X
        case GEN_X: set(1, 2, 0); set(2, 2, 0); break;                 // 2 X
        case GEN_Y_HALF: set(1, 0, -1); set(2, 0, 1); break;           // Y
        case GEN_Z_HALF: set(0, 1, 0); set(1, -1, 0); break;           // Z (diagonal)
        case GEN_ZZ_PHASE: set(1, 2, 0); set(2, 2, 0); break;          // 1 - Z Z (diagonal)
        case GEN_CPHASE: set(3, -2, 0); break;                         // -2 |11><11| (diagonal)
        default: break;
      }
      if (gd.slot >= 0 && g.gen == GEN_NONE) return;
      if (gd.slot >= 0 && (g.gen == GEN_X_HALF || g.gen == GEN_X)) gd.form = ADJ_GEN_X;  // gen[2] holds c
      if (gd.slot >= 0 && g.gen == GEN_Y_HALF) gd.form = ADJ_GEN_Y;
      // fixed diagonal gates of +-1 entries (Z, CZ) are sign flips
      const Recipe& rc = net->sweep_recipes[g.recipe];
      const int kind0 = rc.op_end > rc.op_begin ? net->sweep_ops[rc.op_begin].kind : -1;
      const bool single = rc.op_end - rc.op_begin == 1;
      if (g.diag && gd.slot < 0 && (kind0 == TN_GATE_Z || kind0 == TN_GATE_CZ))
        gd.form = ADJ_DIAG_SIGNS | ((g.nq == 2 ? 8 : 2) << 8);  // the -1 entry: |11> (b = 3) or |1> (b = 1)
      // U^dagger of a real matrix is real, of an RX-like one RX-like
      gd.uform = kFormGeneric;
      if (!g.diag && g.nq == 1 && single) {
        if (kind0 == TN_GATE_RY || kind0 == TN_GATE_H || kind0 == TN_GATE_X || kind0 == TN_GATE_Z) gd.uform = kFormReal;
        if (kind0 == TN_GATE_RX || kind0 == TN_GATE_MIXER || kind0 == TN_GATE_Y) gd.uform = kFormRxLike;
      }
      // resolve a diagonal's bits for its segment
      gd.kreg[0] = gd.kreg[1] = -1;
      gd.csrc[0] = gd.csrc[1] = 0;
      if (g.diag) {
        const PlannedSeg* segp = nullptr;
        const int gi_in_pass = (int)(&pg - &pp.gates[0]);
        for (const PlannedSeg& sg : pp.segs)
          if (gi_in_pass >= sg.first && gi_in_pass < sg.first + sg.count) segp = &sg;
        for (int j = 0; j < gd.n && segp; ++j) {
          const int lj = gd.lidx[j];
          if (lj < 0) {
            gd.csrc[j] = (int8_t)(64 + (-lj - 1));
            continue;
          }
          for (int r = 0; r < 4; ++r)
            if (segp->rbits[r] == lj) gd.kreg[j] = (int8_t)r;
          if (gd.kreg[j] < 0) gd.csrc[j] = (int8_t)lj;
        }
      }
      path->adj_gates.push_back(gd);
    }
    if (ps.n_red > kAdjMaxRed) {
      path->adj_passes.clear();
      path->adj_segments.clear();
      path->adj_gates.clear();
      return;
    }
    ps.first_seg = (int32_t)path->adj_segments.size();
    for (const PlannedSeg& sg : pp.segs) {
      SweepSegment seg;
      for (int j = 0; j < 4; ++j) seg.rbits[j] = sg.rbits[j];
      seg.first_gate = ps.first_gate + sg.first;
      seg.n_gates = sg.count;
      // diagonal gates on bits outside the registers first (as in the forward passes; their
      // gradient terms do not depend on where in the segment they are taken)
      std::stable_partition(path->adj_gates.begin() + seg.first_gate,
                            path->adj_gates.begin() + seg.first_gate + seg.n_gates, [](const AdjGateDesc& gd) {
                              return gd.diag && gd.kreg[0] < 0 && (gd.n == 1 || gd.kreg[1] < 0);
                            });
      mark_runs(path->adj_gates.data() + seg.first_gate, seg.n_gates);
      mark_diag_runs(path->adj_gates.data() + seg.first_gate, seg.n_gates);
      mark_sign_runs(path->adj_gates.data() + seg.first_gate, seg.n_gates);
      fill_segment_tables(seg, ps.l);
      path->adj_segments.push_back(seg);
    }
    ps.n_segs = (int32_t)pp.segs.size();
    path->adj_passes.push_back(ps);
  }
  path->adj_state = 1;
}

void gemm_default_launch(const GemmDesc& g, int* tile, int* split) {
  *split = 1;
  // narrow products, and small ones with a short sum (latency-bound either way;
  // on the per-output kernel they can share a launch)
  if (((g.M < 64 || g.N < 32) && g.K <= kElemMaxK) ||
      (g.batch * g.M * g.N <= ((int64_t)1 << kElemSmallBits) && g.K <= 32)) {
    *tile = kGemmVector;
    return;
  }
  // the largest tile that still gives two blocks per compute unit
  for (int t = 0; t < kGemmVector; ++t) {
    const int64_t blocks =
        ((g.M + kGemmTileM[t] - 1) / kGemmTileM[t]) * ((g.N + kGemmTileN[t] - 1) / kGemmTileN[t]) * g.batch;
    if (blocks >= 512) {
      *tile = t;
      return;
    }
  }
  // else the smallest tile, and K cut into ranges while that adds blocks
  *tile = kGemmVector - 1;
  const int64_t blocks = ((g.M + 63) / 64) * ((g.N + 31) / 32) * g.batch;
  int sp = 1;
  while (sp < kGemmMaxSplit && blocks * sp * 2 <= 1024 && g.K / (sp * 2) >= 32 && g.K % (sp * 2) == 0) sp *= 2;
  *split = sp;
}

double modeled_seconds(const tn_path* path) {
  constexpr double kLaunch = 5e-6, kHbm = 6.0e12, kPerm = 1.6e12, kMfma = 95e12;
  double t = 0;
  if (path->n_small > 0) {
    size_t deepest = 0;  // levels of the deepest work list
    for (size_t i = 0; i + 1 < path->small_lists.size(); ++i)
      deepest = std::max(deepest, (size_t)(path->small_lists[i + 1] - path->small_lists[i]));
    t += kLaunch + 2.0e-6 * (double)deepest;
  }
  constexpr double kLds = 40e12;  // sustained LDS traffic of the fused passes, bytes/s
  for (const SweepChain& ch : path->chains)
    for (int i = 0; i < ch.n_passes; ++i) {
      const SweepPass& ps = path->passes[ch.first_pass + i];
      const double e = std::ldexp(1.0, ch.bits);
      // measured: about 20 vector instructions per element and gate on 64 lanes per CU
      t += kLaunch + 16.0 * e / kHbm + 16.0 * e * ps.n_segs / kLds + 5.0e-13 * e * ps.n_gates;
    }
  int run0 = -1, run_len = 0;  // current run of products that share one launch
  for (int s = 0; s < (int)path->steps.size(); ++s) {
    const StepProgram& P = path->steps[s];
    if (P.kind == SK_SMALL || P.chain != -1) continue;
    if (elem_groupable(P, TN_PREC_C64) && run0 >= 0 && P.grp_from <= run0 && run_len < kElemGroupMax) {
      ++run_len;  // joins the previous launch
    } else {
      t += kLaunch;
      run0 = elem_groupable(P, TN_PREC_C64) ? s : -1;
      run_len = 1;
    }
    for (const PermuteDesc& pd : P.pre) t += kLaunch + 16.0 * std::ldexp(1.0, pd.bits) / kPerm;
    if (P.kind == SK_SKINNY) {
      t += P.bytes / kHbm;
    } else {
      const GemmDesc& g = P.gm[P.orient[0]];
      const double bytes = 8.0 * (double)g.batch * (double)(g.M * g.K + g.K * g.N + g.M * g.N);
      const int tl = g.tile[0];
      if (tl == kGemmVector) {  // per-output vector kernel
        t += std::max(P.flops / 20e12, bytes / kHbm);
        continue;
      }
      const double tm = kGemmTileM[tl], tn = kGemmTileN[tl];
      const double tiles = std::ceil(g.M / tm) * std::ceil(g.N / tn) * (double)g.batch * g.split[0];
      // the 3M tiles do three real products where the real embedding does four
      const double form = tl > kGemmVector ? 4.0 / 3.0 : 1.0;
      const double eff = form * std::min(1.0, g.M / tm) * std::min(1.0, g.N / tn) * std::min(1.0, g.K / 32.0) *
                         std::min(1.0, tiles / 256.0) * (tm * tn >= 8192 ? 1.0 : 0.8);
      t += std::max(P.flops / (kMfma * std::max(eff, 1e-3)), bytes / kHbm) + (g.split[0] > 1 ? kLaunch : 0.0);
    }
  }
  return t;
}

}  // namespace tnq

using namespace tnq;

// An order of kind o.kind within the cap and its compiled program (TN_ELIMIT if none fits).
static tn_status plan_path_impl(const tn_network* net, const tn_plan_opts& o, tn_path** path_out) {
  tn_path* p = nullptr;
  double max_log2 = 0;
  const std::string cap_msg =
      " exceeds the cap 2^" + std::to_string(o.max_log2_intermediate > 0 ? o.max_log2_intermediate : 40);
  if (o.kind != TN_PATH_SEARCH) {
    p = new tn_path();
    tn_status s = plan_order(net, o, p->pairs, &max_log2);
    if (s != TN_OK) {
      delete p;
      return set_error(s, "largest intermediate 2^" + std::to_string((int)max_log2) + cap_msg);
    }
    p->pairs = reorder_small_first(net, p->pairs, &p->n_small, &p->small_region);
    const std::vector<int32_t> fl = output_layout(net);
    s = compile_program(net, p, &fl);
    if (s != TN_OK) { delete p; return s; }
    p->stats.modeled_seconds = modeled_seconds(p);
  } else {
    const int trials = o.trials > 0 ? o.trials : 64;
    // the candidates (greedy, sequential, then randomised greedy orders) are
    // drawn up front from one generator, so the result does not depend on
    // how the trials are spread over host threads
    struct Trial {
      tn_plan_opts o;
      double alpha, temp;
      uint64_t seed;
    };
    std::vector<Trial> cand;
    uint64_t rng = o.seed ^ 0x3f5a1c0de2108ull;
    for (int trial = -2; trial < trials; ++trial) {
      Trial c{o, 1.0, 0.0, splitmix(rng)};
      if (trial == -2) {
        c.o.kind = TN_PATH_GREEDY;
      } else if (trial == -1) {
        c.o.kind = TN_PATH_SEQUENTIAL;
      } else {
        c.o.kind = TN_PATH_GREEDY;
        c.alpha = 0.25 + 1.75 * (double)(splitmix(rng) >> 11) / 9007199254740992.0;
        const double u = (double)(splitmix(rng) >> 11) / 9007199254740992.0;
        c.temp = u * u;
      }
      cand.push_back(c);
    }
    struct Best {
      tn_path* p = nullptr;
      double t = 0;
      size_t idx = 0;
      int min_log2 = 1 << 20;
      tn_status hard = TN_OK;  // an error other than the size cap
      std::string msg;
    };
    const std::vector<int32_t> fl = output_layout(net);
    auto worker = [&](std::atomic<size_t>* next, Best* b) {
      for (size_t i = (*next)++; i < cand.size(); i = (*next)++) {
        const Trial& c = cand[i];
        tn_path* q = new tn_path();
        double ml = 0;
        tn_status s = plan_order(net, c.o, q->pairs, &ml, c.alpha, c.temp, c.seed);
        b->min_log2 = std::min(b->min_log2, (int)ml);
        if (s == TN_OK) {
          q->pairs = reorder_small_first(net, q->pairs, &q->n_small, &q->small_region);
          s = compile_program(net, q, &fl);
        }
        if (s != TN_OK) {
          delete q;
          if (s != TN_ELIMIT && b->hard == TN_OK) {
            b->hard = s;
            b->msg = tn_last_error();
          }
          continue;
        }
        const double t = modeled_seconds(q);
        q->stats.modeled_seconds = t;
        if (!b->p || t < b->t || (t == b->t && i < b->idx)) {
          delete b->p;
          b->p = q;
          b->t = t;
          b->idx = i;
        } else {
          delete q;
        }
      }
    };
    int nth = (int)std::thread::hardware_concurrency();
    if (const char* e = std::getenv("TNQ_PLAN_THREADS")) nth = std::atoi(e);
    nth = std::max(1, std::min({nth, 16, (int)cand.size()}));
    std::atomic<size_t> next{0};
    std::vector<Best> bests(nth);
    std::vector<std::thread> pool;
    for (int k = 1; k < nth; ++k) pool.emplace_back(worker, &next, &bests[k]);
    worker(&next, &bests[0]);
    for (std::thread& th : pool) th.join();
    int min_log2 = 1 << 20;
    for (Best& b : bests) {
      min_log2 = std::min(min_log2, b.min_log2);
      if (b.hard != TN_OK) {
        for (Best& x : bests) delete x.p;
        return set_error(b.hard, b.msg);
      }
    }
    // the lowest modelled time wins, ties go to the earliest candidate
    size_t best_i = SIZE_MAX;
    for (size_t k = 0; k < bests.size(); ++k) {
      if (!bests[k].p) continue;
      if (best_i == SIZE_MAX || bests[k].t < bests[best_i].t ||
          (bests[k].t == bests[best_i].t && bests[k].idx < bests[best_i].idx))
        best_i = k;
    }
    for (size_t k = 0; k < bests.size(); ++k)
      if (k != best_i) delete bests[k].p;
    if (best_i != SIZE_MAX) p = bests[best_i].p;
    if (!p) return set_error(TN_ELIMIT, "every searched order's largest intermediate (at best 2^" +
                                            std::to_string(min_log2) + ")" + cap_msg);
    clear_error();
  }
  *path_out = p;
  return TN_OK;
}

extern "C" tn_status tn_plan_path(const tn_network* net, const tn_plan_opts* opts, tn_path** path_out,
                                  tn_path_stats* stats_out) {
  clear_error();
  if (!net || !path_out) return set_error(TN_EINVAL, "NULL argument");
  *path_out = nullptr;
  tn_plan_opts o{};
  o.kind = TN_PATH_GREEDY;
  o.max_log2_intermediate = 0;
  o.seed = 0;
  if (opts) o = *opts;
  if (o.kind < TN_PATH_GREEDY || o.kind > TN_PATH_SEARCH) return set_error(TN_EINVAL, "unknown path kind");
  if (o.max_slice_bits < 0 || o.max_slice_bits > kSliceMaxCut)
    return set_error(TN_EINVAL, "max_slice_bits must be in 0.." + std::to_string(kSliceMaxCut));
  auto t0 = std::chrono::steady_clock::now();
  tn_path* p = nullptr;
  tn_status st = plan_path_impl(net, o, &p);
  if (st == TN_ELIMIT && o.max_slice_bits > 0) {
    // index slicing: bond indices chosen on an uncapped greedy order, then the sliced network planned
    const int cap = o.max_log2_intermediate > 0 ? o.max_log2_intermediate : 40;
    tn_plan_opts g = o;
    g.kind = TN_PATH_GREEDY;
    g.max_log2_intermediate = 62;
    std::vector<int32_t> pairs, smodes;
    double ml = 0;
    if ((st = plan_order(net, g, pairs, &ml)) != TN_OK) return st;
    if ((st = choose_slices(net, pairs, cap, o.max_slice_bits, &smodes)) != TN_OK) return st;
    std::shared_ptr<tn_network> sn = sliced_network(net, smodes);
    st = plan_path_impl(sn.get(), o, &p);
    if (st == TN_ELIMIT) {  // the uncapped greedy order fits once sliced
      p = new tn_path();
      p->pairs = reorder_small_first(sn.get(), pairs, &p->n_small, &p->small_region);
      const std::vector<int32_t> fl = output_layout(sn.get());
      if ((st = compile_program(sn.get(), p, &fl)) != TN_OK) {
        delete p;
        return st;
      }
      p->stats.modeled_seconds = modeled_seconds(p);
    }
    if (st != TN_OK) return st;
    if ((st = slice_gather_tables(net, sn.get(), smodes, &p->slice_tensors)) != TN_OK) {
      delete p;
      return st;
    }
    int bits = 0;
    for (int m : smodes) bits += net->mode_log2[m];
    p->slice_bits = bits;
    p->slice_modes = smodes;
    p->sliced_net = sn;
    p->q_state = -1;  // the fixed-point mode runs unsliced paths only
    p->stats.n_slice_bits = bits;
    clear_error();
  }
  if (st != TN_OK) return st;
  auto t1 = std::chrono::steady_clock::now();
  p->stats.plan_seconds = std::chrono::duration<double>(t1 - t0).count();
  if (stats_out) *stats_out = p->stats;
  *path_out = p;
  return TN_OK;
}

extern "C" void tn_path_destroy(tn_path* path) {
  if (!path) return;
  device_release_path(path);
  delete path;
}

extern "C" tn_status tn_path_pairs(const tn_path* path, int32_t* n_steps, int32_t* pairs, int32_t capacity) {
  clear_error();
  if (!path) return set_error(TN_EINVAL, "path is NULL");
  const int S = (int)path->pairs.size() / 2;
  if (n_steps) *n_steps = S;
  if (pairs) {
    if (capacity < 2 * S) return set_error(TN_EINVAL, "capacity too small");
    for (int i = 0; i < 2 * S; ++i) pairs[i] = path->pairs[i];
  }
  return TN_OK;
}

extern "C" tn_status tn_path_slices(const tn_path* path, int32_t* n_modes, int32_t* modes, int32_t capacity) {
  clear_error();
  if (!path) return set_error(TN_EINVAL, "path is NULL");
  const int n = (int)path->slice_modes.size();
  if (n_modes) *n_modes = n;
  if (modes) {
    if (capacity < n) return set_error(TN_EINVAL, "capacity too small");
    for (int i = 0; i < n; ++i) modes[i] = path->slice_modes[i];
  }
  return TN_OK;
}

extern "C" tn_status tn_path_step(const tn_path* path, int32_t s, int32_t* rank, int32_t* modes, int64_t* gemm_bmnk,
                                  int32_t* kind) {
  clear_error();
  if (!path || s < 0 || s >= (int32_t)path->steps.size()) return set_error(TN_EINVAL, "bad step index");
  const auto& m = path->step_modes[s];
  if (rank) *rank = (int32_t)m.size();
  if (modes)
    for (size_t i = 0; i < m.size(); ++i) modes[i] = m[i];
  if (gemm_bmnk)
    for (int i = 0; i < 4; ++i) gemm_bmnk[i] = path->steps[s].gemm_bmnk[i];
  if (kind) *kind = path->steps[s].kind;
  return TN_OK;
}
