// Index slicing of a contraction whose intermediates exceed the size cap.
//
// Contraction is a sum over the values of every summed index (eq. (2.2)), so
// fixing a bond index to each of its values and adding up the resulting
// contractions gives the full result.  The order is a free hyperparameter
// (Sec. 2.2.3) and the size of the intermediates is what bounds a device
// (Sec. 3's footnote): slicing trades a cap on that size for repeated work.
// Bond indices are picked greedily: each time the index whose removal most
// lowers the largest intermediate of the current order (ties: the smallest sum
// of intermediate sizes), until the order fits the cap.  The network with
// those indices fixed (their modes take no address bits) is then planned again
// under the cap, and its program is what each slice executes.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace tnq {

namespace {

// log2 sizes of the results along `pairs` on `net`, with the modes in `cut`
// taking no bits, using the planner's rule for which modes survive a step (a
// shared mode is kept while another live tensor or the output holds it).
void path_sizes(const tn_network* net, const std::vector<int32_t>& pairs, const std::vector<char>& cut,
                std::vector<int>& out, double* sum_sizes) {
  const int T = (int)net->tensors.size();
  const int S = (int)pairs.size() / 2;
  const int nm = (int)net->mode_log2.size();
  std::vector<std::vector<int32_t>> modes(T + S);
  std::vector<int> holders(nm, 0);
  std::vector<char> is_out(nm, 0);
  for (int m : net->output_modes) is_out[m] = 1;
  for (int t = 0; t < T; ++t) {
    modes[t] = net->tensors[t].modes;
    for (int m : modes[t]) holders[m]++;
  }
  out.assign(S, 0);
  *sum_sizes = 0;
  for (int s = 0; s < S; ++s) {
    const int a = pairs[2 * s], b = pairs[2 * s + 1];
    std::vector<int32_t> c;
    for (int m : modes[a]) {
      const bool shared = std::find(modes[b].begin(), modes[b].end(), m) != modes[b].end();
      if (is_out[m] || holders[m] > (shared ? 2 : 1)) c.push_back(m);
    }
    for (int m : modes[b])
      if (std::find(modes[a].begin(), modes[a].end(), m) == modes[a].end() && (is_out[m] || holders[m] > 1))
        c.push_back(m);
    for (int m : modes[a]) holders[m]--;
    for (int m : modes[b]) holders[m]--;
    for (int m : c) holders[m]++;
    int lg = 0;
    for (int m : c) lg += cut[m] ? 0 : net->mode_log2[m];
    out[s] = lg;
    *sum_sizes += std::ldexp(1.0, lg);
    modes[T + s] = std::move(c);
  }
}

int bit_pos(const tn_network* net, const std::vector<int32_t>& modes, int m, int j) {
  int below = 0;
  for (size_t i = modes.size(); i-- > 0;) {
    if (modes[i] == m) return below + j;
    below += net->mode_log2[modes[i]];
  }
  return -1;
}

}  // namespace

tn_status choose_slices(const tn_network* net, const std::vector<int32_t>& pairs, int cap_log2, int max_bits,
                        std::vector<int32_t>* slice_modes) {
  const int nm = (int)net->mode_log2.size();
  std::vector<char> cut(nm, 0), is_out(nm, 0);
  for (int m : net->output_modes) is_out[m] = 1;
  int bits = 0;
  slice_modes->clear();
  std::vector<int> sizes;
  double sum = 0;
  for (;;) {
    path_sizes(net, pairs, cut, sizes, &sum);
    const int mx = sizes.empty() ? 0 : *std::max_element(sizes.begin(), sizes.end());
    if (mx <= cap_log2) return TN_OK;
    // candidates: bond modes held by an intermediate above the cap (the others cannot lower the maximum)
    std::vector<char> cand(nm, 0);
    {
      const int T = (int)net->tensors.size();
      std::vector<std::vector<int32_t>> modes(T + (int)sizes.size());
      std::vector<int> holders(nm, 0);
      for (int t = 0; t < T; ++t) {
        modes[t] = net->tensors[t].modes;
        for (int m : modes[t]) holders[m]++;
      }
      for (size_t s = 0; s < sizes.size(); ++s) {
        const int a = pairs[2 * s], b = pairs[2 * s + 1];
        std::vector<int32_t> c;
        for (int m : modes[a]) {
          const bool shared = std::find(modes[b].begin(), modes[b].end(), m) != modes[b].end();
          if (is_out[m] || holders[m] > (shared ? 2 : 1)) c.push_back(m);
        }
        for (int m : modes[b])
          if (std::find(modes[a].begin(), modes[a].end(), m) == modes[a].end() && (is_out[m] || holders[m] > 1))
            c.push_back(m);
        for (int m : modes[a]) holders[m]--;
        for (int m : modes[b]) holders[m]--;
        for (int m : c) holders[m]++;
        if (sizes[s] > cap_log2)
          for (int m : c) cand[m] = !is_out[m] && !cut[m] && net->mode_log2[m] > 0;
        modes[T + s] = std::move(c);
      }
    }
    int best = -1, best_mx = 1 << 30;
    double best_sum = 0;
    for (int m = 0; m < nm; ++m) {
      if (!cand[m] || bits + net->mode_log2[m] > max_bits) continue;
      cut[m] = 1;
      std::vector<int> sz;
      double sm = 0;
      path_sizes(net, pairs, cut, sz, &sm);
      cut[m] = 0;
      const int m2 = sz.empty() ? 0 : *std::max_element(sz.begin(), sz.end());
      if (best < 0 || m2 < best_mx || (m2 == best_mx && sm < best_sum)) {
        best = m;
        best_mx = m2;
        best_sum = sm;
      }
    }
    if (best < 0)
      return set_error(TN_ELIMIT, "slicing " + std::to_string(max_bits) + " bond-index bits does not bring the largest "
                                  "intermediate (2^" + std::to_string(mx) + ") within the cap 2^" +
                                  std::to_string(cap_log2));
    cut[best] = 1;
    bits += net->mode_log2[best];
    slice_modes->push_back(best);
  }
}

std::shared_ptr<tn_network> sliced_network(const tn_network* net, const std::vector<int32_t>& slice_modes) {
  auto sn = std::make_shared<tn_network>(*net);
  sn->dev = nullptr;
  std::vector<char> cut(net->mode_log2.size(), 0);
  for (int m : slice_modes) {
    sn->mode_log2[m] = 0;
    cut[m] = 1;
  }
  int64_t off = 0;
  for (TensorDef& t : sn->tensors) {
    // a fixed index is no longer a mode of any tensor
    t.modes.erase(std::remove_if(t.modes.begin(), t.modes.end(), [&](int32_t m) { return cut[m] != 0; }),
                  t.modes.end());
    int64_t sz = 1;
    for (int m : t.modes) sz <<= sn->mode_log2[m];
    t.size = sz;
    t.offset = off;
    off += sz;
  }
  sn->input_elems = off;
  return sn;
}

tn_status slice_gather_tables(const tn_network* net, const tn_network* sliced, const std::vector<int32_t>& slice_modes,
                              std::vector<SliceTensor>* out) {
  out->clear();
  // slice-index bit of (mode, bit): the modes in order, each mode's bits low to high
  std::vector<int> first(net->mode_log2.size(), -1);
  int nb = 0;
  for (int m : slice_modes) {
    first[m] = nb;
    nb += net->mode_log2[m];
  }
  for (size_t t = 0; t < net->tensors.size(); ++t) {
    const TensorDef& full = net->tensors[t];
    SliceTensor st{};
    st.src_off = full.offset;
    st.dst_off = sliced->tensors[t].offset;
    int nk = 0, nc = 0;
    // sliced address bits from the least significant: the modes in reverse, each mode's bits low to high
    for (size_t i = full.modes.size(); i-- > 0;) {
      const int m = full.modes[i];
      for (int j = 0; j < net->mode_log2[m]; ++j) {
        const int p = bit_pos(net, full.modes, m, j);
        if (first[m] >= 0) {
          if (nc >= kSliceMaxCut) return set_error(TN_EUNSUPPORTED, "too many sliced bits in one tensor");
          st.cut_pos[nc] = (int8_t)p;
          st.cut_src[nc] = (int8_t)(first[m] + j);
          ++nc;
        } else {
          if (nk >= kSliceMaxKeep) return set_error(TN_EUNSUPPORTED, "input tensor too large to slice");
          st.keep_pos[nk++] = (int8_t)p;
        }
      }
    }
    st.n_keep = nk;
    st.n_cut = nc;
    if (((int64_t)1 << nk) != sliced->tensors[t].size) return set_error(TN_EINVAL, "internal: sliced tensor size");
    out->push_back(st);
  }
  return TN_OK;
}

}  // namespace tnq
