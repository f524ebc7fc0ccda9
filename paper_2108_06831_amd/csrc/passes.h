// Planning of fused streaming passes over one large tensor (passes.cpp).
#pragma once
#include <stdint.h>

#include <vector>

#include "internal.h"

namespace tnq {

struct PassItem {
  std::vector<int> pos;  // address positions of bit 0 and bit 1 of the operation's own index (1 or 2 of them)
  bool diag;             // diagonal: commutes with other diagonal operations, needs no local bits
  bool movable = true;   // diagonal: may move to a neighbouring segment (see plan_passes)
  bool grad = false;     // has a gradient term (counts against a pass's max_grads)
};

struct PlannedGate {
  int item;
  int32_t n;
  bool diag;
  int32_t lidx[2];  // local bit index, or -(position + 1) for a diagonal operation's bit outside the chunk
  int32_t rb[2];    // dense: index of lidx[j] in its segment's register bits
};

struct PlannedSeg {
  int8_t rbits[4];
  int first, count;  // range of the pass's gates
};

struct PlannedPass {
  int l;
  std::vector<int> lpos;
  std::vector<PlannedGate> gates;
  std::vector<PlannedSeg> segs;
};

// Splits `items` (in order) on a 2^R tensor into passes of at most max_items
// operations, max_grads of them with a gradient term.  Returns false if the
// tensor is too small for fused passes (R < 16).
bool plan_passes(int R, const std::vector<PassItem>& items, std::vector<PlannedPass>& out, int max_items = 1 << 30,
                 int max_grads = 1 << 30);

}  // namespace tnq
