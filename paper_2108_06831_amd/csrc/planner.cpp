// Contraction-order search (Sec. 2.2.3: the order is a free hyperparameter
// since contraction is associative; Sec. 3 and Sec. 4: greedy search).
//
// Greedy objective: the pair of live tensors sharing a mode that minimises
// |C| - |A| - |B| (elements), ties by smaller |C|, then fewer flops, then the
// smaller (min id, max id).  A mode is summed only when no other live tensor
// and no output holds it, so hyper-indices (diagonal gates, the amplitude
// batch index) stay open until their last holder.  All extents are powers of
// two, so sizes are exact integers kept as log2.
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "internal.h"

namespace tnq {

namespace {

struct LiveTensor {
  std::vector<int32_t> modes;
  int32_t log2size = 0;
  bool live = false;
};

using i128 = __int128;

i128 pow2(int e) { return e >= 120 ? ((i128)1 << 120) : ((i128)1 << e); }

struct Cost {
  double score;   // randomised objective of the search trials (0 for the plain greedy)
  i128 delta;     // |C| - |A| - |B|
  int32_t c_log2; // log2 |C|
  int32_t f_log2; // log2 of the multiply-add count
  int32_t lo, hi; // ids
  bool operator<(const Cost& o) const {
    return std::tie(score, delta, c_log2, f_log2, lo, hi) < std::tie(o.score, o.delta, o.c_log2, o.f_log2, o.lo, o.hi);
  }
};

struct State {
  const tn_network* net;
  double alpha = 1.0, temp = 0.0;  // search trials: |C| - alpha (|A| + |B|) with Gumbel noise of scale temp
  mutable uint64_t rng = 0;
  std::vector<LiveTensor> ts;
  std::vector<std::vector<int32_t>> holders;  // per mode: live tensors holding it
  std::vector<char> is_output;

  void add(int id, const std::vector<int32_t>& modes) {
    if ((int)ts.size() <= id) ts.resize(id + 1);
    LiveTensor& t = ts[id];
    t.modes = modes;
    t.log2size = 0;
    for (int m : modes) t.log2size += net->mode_log2[m];
    t.live = true;
    for (int m : modes) holders[m].push_back(id);
  }
  void remove(int id) {
    ts[id].live = false;
    for (int m : ts[id].modes) {
      auto& h = holders[m];
      h.erase(std::find(h.begin(), h.end(), id));
    }
  }
  // modes of the result of contracting a and b, A's order then B's new ones
  void result(int a, int b, std::vector<int32_t>& out, int* c_log2, int* f_log2) const {
    out.clear();
    int f = 0, c = 0;
    const auto& ma = ts[a].modes;
    const auto& mb = ts[b].modes;
    auto inb = [&](int m) { return std::find(mb.begin(), mb.end(), m) != mb.end(); };
    auto ina = [&](int m) { return std::find(ma.begin(), ma.end(), m) != ma.end(); };
    for (int m : ma) {
      const bool shared = inb(m);
      const size_t others = holders[m].size() - (shared ? 2 : 1);
      f += net->mode_log2[m];
      if (is_output[m] || others > 0) { out.push_back(m); c += net->mode_log2[m]; }
    }
    for (int m : mb) {
      if (ina(m)) continue;
      f += net->mode_log2[m];
      out.push_back(m);  // a mode of B only always survives (it has another holder or is an output)
      c += net->mode_log2[m];
    }
    *c_log2 = c;
    *f_log2 = f;
  }
  Cost cost(int a, int b) const {
    std::vector<int32_t> tmp;
    Cost k;
    result(a, b, tmp, &k.c_log2, &k.f_log2);
    k.delta = pow2(k.c_log2) - pow2(ts[a].log2size) - pow2(ts[b].log2size);
    k.score = 0.0;
    if (alpha != 1.0 || temp != 0.0) {
      const double sa = std::ldexp(1.0, ts[a].log2size), sb = std::ldexp(1.0, ts[b].log2size);
      const double u = ((double)(splitmix(rng) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      const double gumbel = -std::log(-std::log(u));
      k.score = std::ldexp(1.0, k.c_log2) - alpha * (sa + sb) - temp * (sa + sb) * gumbel;
    }
    k.lo = std::min(a, b);
    k.hi = std::max(a, b);
    return k;
  }
};

}  // namespace

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

tn_status plan_order(const tn_network* net, const tn_plan_opts& opts, std::vector<int32_t>& pairs,
                     double* max_log2_out, double alpha, double temp, uint64_t seed) {
  const int T = (int)net->tensors.size();
  State st;
  st.net = net;
  st.alpha = alpha;
  st.temp = temp;
  st.rng = seed;
  st.holders.assign(net->mode_log2.size(), {});
  st.is_output.assign(net->mode_log2.size(), 0);
  for (int m : net->output_modes) st.is_output[m] = 1;
  for (int t = 0; t < T; ++t) st.add(t, net->tensors[t].modes);
  int next_id = T;
  int n_live = T;
  int max_log2 = 0;
  for (int t = 0; t < T; ++t) max_log2 = std::max(max_log2, st.ts[t].log2size);
  pairs.clear();
  const int cap = opts.max_log2_intermediate > 0 ? opts.max_log2_intermediate : 40;

  auto contract = [&](int a, int b) {
    std::vector<int32_t> modes;
    int c_log2, f_log2;
    st.result(a, b, modes, &c_log2, &f_log2);
    st.remove(a);
    st.remove(b);
    const int id = next_id++;
    st.add(id, modes);
    pairs.push_back(a);
    pairs.push_back(b);
    --n_live;
    max_log2 = std::max(max_log2, c_log2);
    return id;
  };

  if (opts.kind == TN_PATH_SEQUENTIAL) {
    int acc = 0;
    for (int t = 1; t < T; ++t) {
      acc = contract(acc, t);
      if (max_log2 > cap) break;
    }
  } else if (opts.kind == TN_PATH_RANDOM) {
    uint64_t seed = opts.seed ^ 0x2108068310ull;
    while (n_live > 1) {
      std::vector<std::pair<int, int>> cand;
      for (size_t m = 0; m < st.holders.size(); ++m) {
        const auto& h = st.holders[m];
        for (size_t i = 0; i < h.size(); ++i)
          for (size_t j = i + 1; j < h.size(); ++j) cand.push_back({std::min(h[i], h[j]), std::max(h[i], h[j])});
      }
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      if (cand.empty()) {
        std::vector<int> live;
        for (int i = 0; i < (int)st.ts.size(); ++i)
          if (st.ts[i].live) live.push_back(i);
        int i = (int)(splitmix(seed) % live.size());
        int j = (int)(splitmix(seed) % (live.size() - 1));
        if (j >= i) ++j;
        contract(live[i], live[j]);
      } else {
        auto p = cand[splitmix(seed) % cand.size()];
        contract(p.first, p.second);
      }
      if (max_log2 > cap) break;
    }
  } else {
    // greedy with an ordered candidate set, recomputing only affected pairs
    std::set<Cost> heap;
    std::map<std::pair<int, int>, Cost> cur;
    auto upsert = [&](int a, int b) {
      const std::pair<int, int> key{std::min(a, b), std::max(a, b)};
      auto it = cur.find(key);
      if (it != cur.end()) { heap.erase(it->second); cur.erase(it); }
      Cost c = st.cost(key.first, key.second);
      heap.insert(c);
      cur[key] = c;
    };
    auto drop_all = [&](int a) {
      for (auto it = cur.begin(); it != cur.end();) {
        if (it->first.first == a || it->first.second == a) { heap.erase(it->second); it = cur.erase(it); }
        else ++it;
      }
    };
    for (size_t m = 0; m < st.holders.size(); ++m) {
      const auto& h = st.holders[m];
      for (size_t i = 0; i < h.size(); ++i)
        for (size_t j = i + 1; j < h.size(); ++j) {
          std::pair<int, int> key{std::min(h[i], h[j]), std::max(h[i], h[j])};
          if (!cur.count(key)) upsert(key.first, key.second);
        }
    }
    while (n_live > 1) {
      int a, b;
      if (!heap.empty()) {
        a = heap.begin()->lo;
        b = heap.begin()->hi;
      } else {
        // no shared mode: outer product of the two smallest
        std::vector<std::pair<int, int>> live;
        for (int i = 0; i < (int)st.ts.size(); ++i)
          if (st.ts[i].live) live.push_back({st.ts[i].log2size, i});
        std::sort(live.begin(), live.end());
        a = std::min(live[0].second, live[1].second);
        b = std::max(live[0].second, live[1].second);
      }
      // modes whose holder count drops (shared and kept): pairs among their holders change cost
      std::vector<int32_t> changed;
      {
        const auto& ma = st.ts[a].modes;
        const auto& mb = st.ts[b].modes;
        for (int m : ma)
          if (std::find(mb.begin(), mb.end(), m) != mb.end()) changed.push_back(m);
      }
      drop_all(a);
      drop_all(b);
      const int c = contract(a, b);
      if (max_log2 > cap) break;
      std::set<int> nbrs;
      for (int m : st.ts[c].modes)
        for (int h : st.holders[m])
          if (h != c) nbrs.insert(h);
      for (int x : nbrs) upsert(x, c);
      for (int m : changed) {
        const auto& h = st.holders[m];
        for (size_t i = 0; i < h.size(); ++i)
          for (size_t j = i + 1; j < h.size(); ++j)
            if (h[i] != c && h[j] != c) upsert(h[i], h[j]);
      }
    }
  }
  if (max_log2_out) *max_log2_out = max_log2;
  if (max_log2 > cap) return TN_ELIMIT;
  return TN_OK;
}

}  // namespace tnq
