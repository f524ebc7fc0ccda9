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

bool plan_passes(int R, const std::vector<PassItem>& items, std::vector<PlannedPass>& out) {
  out.clear();
  if (R < 16) return false;
  const int lmax = std::min(kSweepMaxLocal, R - 8);  // >= 8, enough for the low bits plus two more
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
    for (size_t i = 0; i < items.size(); ++i) {
      if (done[i]) continue;
      const PassItem& it = items[i];
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
    std::vector<int> rset;
    PlannedSeg seg;
    seg.first = 0;
    seg.count = 0;
    auto close = [&]() {
      for (int b = 0; b < ps.l && (int)rset.size() < 4; ++b)
        if (std::find(rset.begin(), rset.end(), b) == rset.end()) rset.push_back(b);
      std::sort(rset.begin(), rset.end());
      for (int j = 0; j < 4; ++j) seg.rbits[j] = (int8_t)rset[j];
      for (int g = seg.first; g < seg.first + seg.count; ++g) {
        PlannedGate& pg = ps.gates[g];
        if (pg.diag) continue;
        for (int j = 0; j < pg.n; ++j)
          pg.rb[j] = (int32_t)(std::find(rset.begin(), rset.end(), pg.lidx[j]) - rset.begin());
      }
      ps.segs.push_back(seg);
    };
    for (int g = 0; g < (int)ps.gates.size(); ++g) {
      const PlannedGate& pg = ps.gates[g];
      if (!pg.diag) {
        std::vector<int> u = rset;
        for (int j = 0; j < pg.n; ++j)
          if (std::find(u.begin(), u.end(), pg.lidx[j]) == u.end()) u.push_back(pg.lidx[j]);
        if ((int)u.size() > 4) {
          close();
          rset.clear();
          seg.first = g;
          seg.count = 0;
          u.clear();
          for (int j = 0; j < pg.n; ++j) u.push_back(pg.lidx[j]);
        }
        rset = u;
      }
      seg.count++;
    }
    close();
    out.push_back(ps);
  }
  return true;
}

}  // namespace tnq
