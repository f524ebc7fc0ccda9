// The Q3.28 fixed-point program of a contraction path (TN_PREC_Q3_28).
//
// Sec. 3 of the paper runs its contractions in 32-bit fixed point with 28 bits
// behind the binary point.  This mode reproduces that arithmetic: the steps of
// the path are executed in order, each as one launch of a per-output product
// (every result element a sum over the shared indices, eq. (2.2)) whose real
// products are rounded to Q3.28.  Every intermediate is C-ordered over its
// modes in a workspace arena planned here with the same liveness rule as the
// floating-point program: a buffer is free after the step that reads it last.
#include <algorithm>
#include <map>
#include <vector>

#include "internal.h"

namespace tnq {

namespace {

// first-fit arena in 256-byte granules (32 complex elements)
struct QArena {
  std::map<int64_t, int64_t> free_;  // offset -> size
  int64_t top = 0;
  static int64_t round(int64_t n) { return (n + 31) & ~(int64_t)31; }
  int64_t get(int64_t n) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        const int64_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > n) free_[off + n] = sz - n;
        return off;
      }
    const int64_t off = top;
    top += n;
    return off;
  }
  void put(int64_t off, int64_t n) {
    n = round(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {  // merge with the next block
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {  // and with the previous one
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// address position of bit j of mode m in a tensor C-ordered over `modes`
int bit_pos(const tn_network* net, const std::vector<int32_t>& modes, int m, int j) {
  int below = 0;
  for (size_t i = modes.size(); i-- > 0;) {
    if (modes[i] == m) return below + j;
    below += net->mode_log2[modes[i]];
  }
  return -1;
}

int total_bits(const tn_network* net, const std::vector<int32_t>& modes) {
  int b = 0;
  for (int m : modes) b += net->mode_log2[m];
  return b;
}

}  // namespace

void build_q328_program(const tn_network* net, tn_path* path) {
  path->q_steps.clear();
  path->q_final_modes.clear();
  path->q_ws_elems = 0;
  path->q_state = -1;
  const int T = (int)net->tensors.size();
  const int S = (int)path->pairs.size() / 2;
  if ((int)path->step_modes.size() != S) return;
  std::vector<std::vector<int32_t>> modes(T + S);
  std::vector<BufRef> ref(T + S);
  std::vector<int> last_use(T + S, -1);
  for (int t = 0; t < T; ++t) {
    modes[t] = net->tensors[t].modes;
    ref[t].buf = BUF_IN;
    ref[t].off = net->tensors[t].offset;
  }
  for (int s = 0; s < S; ++s) {
    last_use[path->pairs[2 * s]] = s;
    last_use[path->pairs[2 * s + 1]] = s;
  }
  QArena arena;
  for (int s = 0; s < S; ++s) {
    const int ia = path->pairs[2 * s], ib = path->pairs[2 * s + 1], ic = T + s;
    // the result's modes, each once, in the order the path records them
    std::vector<int32_t> cm;
    for (int m : path->step_modes[s])
      if (std::find(cm.begin(), cm.end(), m) == cm.end()) cm.push_back(m);
    modes[ic] = cm;
    const std::vector<int32_t>& ma = modes[ia];
    const std::vector<int32_t>& mb = modes[ib];
    auto has = [](const std::vector<int32_t>& v, int m) { return std::find(v.begin(), v.end(), m) != v.end(); };
    QStep q{};
    q.a_buf = ref[ia].buf;
    q.b_buf = ref[ib].buf;
    q.a_off = ref[ia].off;
    q.b_off = ref[ib].off;
    q.n_out = total_bits(net, cm);
    if (q.n_out > kQMaxOutBits) return;
    for (int i = 0; i < kQMaxOutBits; ++i) q.a_o[i] = q.b_o[i] = -1;
    for (int i = 0; i < kQMaxKBits; ++i) q.a_k[i] = q.b_k[i] = 0;
    for (int m : cm) {
      if (!has(ma, m) && !has(mb, m)) return;  // a result mode must come from an operand
      for (int j = 0; j < net->mode_log2[m]; ++j) {
        const int c = bit_pos(net, cm, m, j);
        q.a_o[c] = (int8_t)(has(ma, m) ? bit_pos(net, ma, m, j) : -1);
        q.b_o[c] = (int8_t)(has(mb, m) ? bit_pos(net, mb, m, j) : -1);
      }
    }
    int nk = 0;
    for (int m : ma) {
      if (!has(mb, m) || has(cm, m)) continue;  // shared and not kept: summed
      for (int j = 0; j < net->mode_log2[m]; ++j) {
        if (nk >= kQMaxKBits) return;
        q.a_k[nk] = (int8_t)bit_pos(net, ma, m, j);
        q.b_k[nk] = (int8_t)bit_pos(net, mb, m, j);
        ++nk;
      }
    }
    q.n_k = nk;
    // a mode of one operand only that the result drops would be a sum over a free index
    // (harmless for a mode of extent 1, which has no address bits)
    for (int m : ma)
      if (!has(mb, m) && !has(cm, m) && net->mode_log2[m] > 0) return;
    for (int m : mb)
      if (!has(ma, m) && !has(cm, m) && net->mode_log2[m] > 0) return;
    const int64_t c_elems = (int64_t)1 << q.n_out;
    q.c_off = arena.get(c_elems);
    ref[ic].buf = BUF_WS;
    ref[ic].off = q.c_off;
    for (int x : {ia, ib})
      if (x >= T && last_use[x] == s) arena.put(ref[x].off, (int64_t)1 << total_bits(net, modes[x]));
    path->q_steps.push_back(q);
  }
  const int last = S > 0 ? T + S - 1 : 0;
  path->q_final = ref[last];
  path->q_final_modes = modes[last];
  path->q_ws_elems = std::max<int64_t>(arena.top, 32);
  path->q_state = 1;
}

}  // namespace tnq
