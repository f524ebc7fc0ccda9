// Grouping of a sequence of gate-sized operations on one large tensor into
// fused streaming passes (see SweepPass / SweepSegment).
//
// Light-cone rule: walking the operations in order, an operation joins the
// current pass if no earlier operation left out of the pass touches its bits
// (operations on disjoint bits commute); a dense operation must also have all
// its bits in the pass's local set (at most lmax bits, always including the
// five lowest so that chunk loads move 256-byte runs).  Diagonal operations
// commute with each other and need no local bits: outside the chunk a bit is
// constant and comes from the chunk's base address.
#include <algorithm>
#include <vector>

#include "passes.h"

namespace tnq {

bool plan_passes(int R, const std::vector<PassItem>& items, std::vector<PlannedPass>& out, int max_items,
                 int max_grads) {
  out.clear();
  if (R < 16 || max_items < 1 || max_grads < 1) return false;
  // Every pass takes the widest local set: passes on states of 2^16..2^19 elements are
  // launch-bound, so fewer of them beat more blocks per pass.
  const int lmax = std::min(kSweepMaxLocal, R - 4);
  const int low = 5;
  std::vector<char> done(items.size(), 0);
  size_t remaining = items.size();
  while (remaining > 0) {
    // blk_any[p]: an operation left out touches p (later dense ones on p wait);
    // blk_dense[p]: a dense operation left out touches p (later diagonal ones on p wait too)
    std::vector<char> local(R, 0), blk_any(R, 0), blk_dense(R, 0);
    int nl = 0;
    for (int p = 0; p < low; ++p) { local[p] = 1; ++nl; }
    std::vector<int> members;
    int n_grads = 0;
    for (size_t i = 0; i < items.size(); ++i) {
      if (done[i]) continue;
      const PassItem& it = items[i];
      // a full pass takes nothing more: the rest waits for the next ones
      if ((int)members.size() == max_items || (it.grad && n_grads == max_grads)) break;
      bool take = true;
      if (it.diag) {
        for (int p : it.pos) take &= !blk_dense[p];
      } else {
        int extra = 0;
        for (int p : it.pos) { take &= !blk_any[p]; extra += !local[p]; }
        take &= nl + extra <= lmax;
      }
      if (take) {
        if (!it.diag)
          for (int p : it.pos) if (!local[p]) { local[p] = 1; ++nl; }
        members.push_back((int)i);
        n_grads += it.grad;
        done[i] = 1;
        --remaining;
      } else {
        for (int p : it.pos) {
          blk_any[p] = 1;
          if (!it.diag) blk_dense[p] = 1;
        }
      }
    }
    if (members.empty()) return false;
    // fill the local set up to lmax with the lowest remaining bits (longer contiguous runs)
    for (int p = 0; p < R && nl < lmax; ++p) if (!local[p]) { local[p] = 1; ++nl; }
    PlannedPass ps;
    for (int p = 0; p < R; ++p) if (local[p]) ps.lpos.push_back(p);
    ps.l = (int)ps.lpos.size();
    auto lidx_of = [&](int p) { return (int32_t)(std::find(ps.lpos.begin(), ps.lpos.end(), p) - ps.lpos.begin()); };
    for (int i : members) {
      PlannedGate g;
      g.item = i;
      g.n = (int32_t)items[i].pos.size();
      g.diag = items[i].diag;
      for (int j = 0; j < 2; ++j) {
        g.lidx[j] = 0;
        g.rb[j] = 0;
        if (j >= g.n) continue;
        const int p = items[i].pos[j];
        g.lidx[j] = local[p] ? lidx_of(p) : -(p + 1);
      }
      ps.gates.push_back(g);
    }
    // segments: consecutive runs whose dense gates' local bits fit in four register bits
    std::vector<std::vector<int>> sg_gates, sg_dense;  // per segment: its gates, its dense gates' bits
    {
      std::vector<int> cur, dset;
      for (int g = 0; g < (int)ps.gates.size(); ++g) {
        const PlannedGate& pg = ps.gates[g];
        if (!pg.diag) {
          std::vector<int> u = dset;
          for (int j = 0; j < pg.n; ++j)
            if (std::find(u.begin(), u.end(), pg.lidx[j]) == u.end()) u.push_back(pg.lidx[j]);
          if ((int)u.size() > 4) {
            sg_gates.push_back(cur);
            sg_dense.push_back(dset);
            cur.clear();
            u.clear();
            for (int j = 0; j < pg.n; ++j) u.push_back(pg.lidx[j]);
          }
          dset = u;
        }
        cur.push_back(g);
      }
      sg_gates.push_back(cur);
      sg_dense.push_back(dset);
    }
    const int n_sg = (int)sg_gates.size();
    auto local_bits = [&](int g) {
      std::vector<int> b;
      for (int j = 0; j < ps.gates[g].n; ++j)
        if (ps.gates[g].lidx[j] >= 0) b.push_back(ps.gates[g].lidx[j]);
      return b;
    };
    auto meets = [](const std::vector<int>& a, const std::vector<int>& b) {
      for (int x : a)
        if (std::find(b.begin(), b.end(), x) != b.end()) return true;
      return false;
    };
    auto dense_on = [&](int g, const std::vector<int>& b) { return !ps.gates[g].diag && meets(local_bits(g), b); };
    // A diagonal gate on a register bit multiplies each of a thread's elements;
    // on bits outside the registers it is one factor per thread.  So a diagonal
    // gate whose bits its segment's dense gates hold in registers moves to the
    // next (or else the previous) segment when that one's dense gates leave its
    // bits alone and no dense gate on its bits lies in between.
    for (int sg = 0; sg < n_sg; ++sg) {
      for (size_t i = 0; i < sg_gates[sg].size();) {
        const int g = sg_gates[sg][i];
        const std::vector<int> b = local_bits(g);
        if (!ps.gates[g].diag || !items[ps.gates[g].item].movable || !meets(b, sg_dense[sg])) {
          ++i;
          continue;
        }
        bool fwd = sg + 1 < n_sg && !meets(b, sg_dense[sg + 1]);
        for (size_t j = i + 1; fwd && j < sg_gates[sg].size(); ++j) fwd = !dense_on(sg_gates[sg][j], b);
        bool back = !fwd && sg > 0 && !meets(b, sg_dense[sg - 1]);
        for (size_t j = 0; back && j < i; ++j) back = !dense_on(sg_gates[sg][j], b);
        if (!fwd && !back) {
          ++i;
          continue;
        }
        sg_gates[sg].erase(sg_gates[sg].begin() + i);
        if (fwd) sg_gates[sg + 1].insert(sg_gates[sg + 1].begin(), g);
        else sg_gates[sg - 1].push_back(g);
      }
    }
    // the pass's gates in their new order, and each segment's register bits: its
    // dense gates' bits, then the lowest other local bits, those of the
    // segment's diagonal gates last
    std::vector<PlannedGate> order;
    for (int sg = 0; sg < n_sg; ++sg) {
      PlannedSeg seg;
      seg.first = (int)order.size();
      seg.count = (int)sg_gates[sg].size();
      std::vector<int> diag_bits;
      for (int g : sg_gates[sg]) {
        order.push_back(ps.gates[g]);
        if (ps.gates[g].diag)
          for (int x : local_bits(g)) diag_bits.push_back(x);
      }
      std::vector<int> rset = sg_dense[sg];
      for (int pass2 = 0; pass2 < 2; ++pass2)
        for (int x = 0; x < ps.l && (int)rset.size() < 4; ++x) {
          if (std::find(rset.begin(), rset.end(), x) != rset.end()) continue;
          const bool dg = std::find(diag_bits.begin(), diag_bits.end(), x) != diag_bits.end();
          if (dg == (pass2 == 1)) rset.push_back(x);
        }
      std::sort(rset.begin(), rset.end());
      for (int j = 0; j < 4; ++j) seg.rbits[j] = (int8_t)rset[j];
      for (int g = seg.first; g < seg.first + seg.count; ++g) {
        PlannedGate& pg = order[g];
        if (pg.diag) continue;
        for (int j = 0; j < pg.n; ++j)
          pg.rb[j] = (int32_t)(std::find(rset.begin(), rset.end(), pg.lidx[j]) - rset.begin());
      }
      ps.segs.push_back(seg);
    }
    // the new order keeps every pair of gates that share a bit, one of them
    // dense, in their old order
    for (size_t x = 0; x < order.size(); ++x)
      for (size_t y = x + 1; y < order.size(); ++y) {
        if (order[x].diag && order[y].diag) continue;
        bool share = false;
        for (int j = 0; j < order[x].n; ++j)
          for (int k = 0; k < order[y].n; ++k) share |= order[x].lidx[j] == order[y].lidx[k];
        if (share && order[x].item > order[y].item) return false;
      }
    ps.gates = order;
    out.push_back(ps);
  }
  return true;
}

}  // namespace tnq
