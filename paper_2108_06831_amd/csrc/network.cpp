// Circuit -> tensor network (Sec. 2.2.2-2.2.3), with optional pre-contraction
// of one-qubit gates into the adjacent two-qubit gates (Sec. 3).
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "internal.h"

namespace tnq {

namespace {

struct Block {
  int nq;
  int q[2];
  std::vector<RecipeOp> ops;
};

RecipeOp make_op(const tn_gate& g, int pos, int mat) {
  RecipeOp op;
  op.kind = g.kind;
  op.pos = pos;
  op.mat = mat;
  for (int j = 0; j < 3; ++j) {
    op.angle[j] = g.angle[j];
    op.param[j] = j < gate_n_angles(g.kind) ? g.param[j] : -1;
  }
  return op;
}

bool ops_diagonal(const std::vector<RecipeOp>& ops, const std::vector<double>& mats) {
  for (const RecipeOp& op : ops) {
    if (op.kind == TN_GATE_MATRIX1 || op.kind == TN_GATE_MATRIX2) {
      const int d = op.kind == TN_GATE_MATRIX2 ? 4 : 2;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
          if (i != j && (mats[32 * op.mat + 2 * (d * i + j)] != 0.0 || mats[32 * op.mat + 2 * (d * i + j) + 1] != 0.0))
            return false;
      continue;
    }
    if (!gate_is_diagonal(op.kind)) return false;
  }
  return true;
}

// block qubit (0 or 1) in whose value the block's two-qubit gate is
// block-diagonal, or -1
int split_qubit(const std::vector<RecipeOp>& ops, const std::vector<double>& mats) {
  for (const RecipeOp& op : ops) {
    if (!gate_is_two_qubit(op.kind)) continue;
    if (op.kind == TN_GATE_CZ || op.kind == TN_GATE_CPHASE || op.kind == TN_GATE_ZZPHASE) return 0;
    if (op.kind == TN_GATE_CNOT) return op.pos;  // the control
    if (op.kind == TN_GATE_MATRIX2) {
      const double* m = &mats[32 * op.mat];
      auto zero = [&](int x, int y) { return m[2 * (4 * x + y)] == 0.0 && m[2 * (4 * x + y) + 1] == 0.0; };
      for (int q = 0; q < 2; ++q) {  // q: gate-order qubit tested for block-diagonality
        bool ok = true;
        for (int x = 0; x < 4 && ok; ++x)
          for (int y = 0; y < 4 && ok; ++y) {
            const int bx = q == 0 ? (x >> 1) : (x & 1), by = q == 0 ? (y >> 1) : (y & 1);
            if (bx != by && !zero(x, y)) ok = false;
          }
        if (ok) return op.pos ? 1 - q : q;
      }
    }
    return -1;
  }
  return -1;
}

int gen_of(int kind) {
  switch (kind) {
    case TN_GATE_RX: return GEN_X_HALF;
    case TN_GATE_RY: return GEN_Y_HALF;
    case TN_GATE_RZ: return GEN_Z_HALF;
    case TN_GATE_MIXER: return GEN_X;
    case TN_GATE_ZZPHASE: return GEN_ZZ_PHASE;
    case TN_GATE_CPHASE: return GEN_CPHASE;
    default: return GEN_NONE;
  }
}

}  // namespace

void network_values_host(const tn_network* net, const double* params, const uint64_t* bits, double* out) {
  for (const TensorDef& t : net->tensors) {
    double* o = out + 2 * t.offset;
    if (t.kind == TK_KET0) {
      o[0] = 1; o[1] = 0; o[2] = 0; o[3] = 0;
    } else if (t.kind == TK_PROJ) {
      const int shift = net->n_qubits - 1 - t.qubit;
      for (int64_t s = 0; s < ((int64_t)1 << net->batch_log2); ++s) {
        int bit = s < net->n_bitstrings ? (int)((bits[s] >> shift) & 1) : 0;
        for (int w = 0; w < 2; ++w) {
          o[2 * (2 * s + w)] = (w == bit) ? 1.0 : 0.0;
          o[2 * (2 * s + w) + 1] = 0.0;
        }
      }
    } else {
      const Recipe& r = net->recipes[t.recipe];
      c128 M[16];
      if (r.split_side >= 0) {
        recipe_split_half(r, net->ops.data(), net->matrices.data(), params, M);
        for (int i = 0; i < 8; ++i) { o[2 * i] = M[i].re; o[2 * i + 1] = M[i].im; }
        continue;
      }
      recipe_matrix(r, net->ops.data(), net->matrices.data(), params, M);
      const int d = r.nq == 2 ? 4 : 2;
      if (r.diag) {
        for (int i = 0; i < d; ++i) { o[2 * i] = M[d * i + i].re; o[2 * i + 1] = M[d * i + i].im; }
      } else {
        for (int i = 0; i < d * d; ++i) { o[2 * i] = M[i].re; o[2 * i + 1] = M[i].im; }
      }
    }
  }
}

}  // namespace tnq

using namespace tnq;

extern "C" tn_status tn_build_network(int32_t n_qubits, const tn_gate* gates, int32_t n_gates, int32_t n_params,
                                      int32_t output_kind, int64_t n_bitstrings, int32_t flags,
                                      tn_network** net_out) {
  clear_error();
  if (!net_out) return set_error(TN_EINVAL, "net_out is NULL");
  *net_out = nullptr;
  if (n_qubits < 1 || n_qubits > 62) return set_error(TN_EINVAL, "n_qubits must be in 1..62");
  if (n_gates < 0 || (n_gates > 0 && !gates)) return set_error(TN_EINVAL, "bad gate array");
  if (n_params < 0) return set_error(TN_EINVAL, "n_params < 0");
  if (output_kind != TN_OUT_STATEVECTOR && output_kind != TN_OUT_AMPLITUDES)
    return set_error(TN_EINVAL, "unknown output kind");
  if (output_kind == TN_OUT_AMPLITUDES && (n_bitstrings < 1 || n_bitstrings > ((int64_t)1 << 24)))
    return set_error(TN_EINVAL, "n_bitstrings must be in 1..2^24");

  tn_network* net = new tn_network();
  net->n_qubits = n_qubits;
  net->n_params = n_params;
  net->output_kind = output_kind;
  net->flags = flags;

  // ---- validate gates, collect explicit matrices, build blocks (pass 1)
  std::vector<int> gate_mat(n_gates, -1);
  for (int g = 0; g < n_gates; ++g) {
    const tn_gate& G = gates[g];
    const bool known = (G.kind >= TN_GATE_H && G.kind <= TN_GATE_MATRIX2);
    if (!known) { delete net; return set_error(TN_EINVAL, "gate " + std::to_string(g) + ": unknown kind"); }
    const bool two = gate_is_two_qubit(G.kind);
    if (G.q[0] < 0 || G.q[0] >= n_qubits || (two && (G.q[1] < 0 || G.q[1] >= n_qubits || G.q[1] == G.q[0]))) {
      delete net;
      return set_error(TN_EINVAL, "gate " + std::to_string(g) + ": bad qubit index");
    }
    for (int j = 0; j < gate_n_angles(G.kind); ++j)
      if (G.param[j] >= n_params || G.param[j] < -1) {
        delete net;
        return set_error(TN_EINVAL, "gate " + std::to_string(g) + ": parameter index out of range");
      }
    if (G.kind == TN_GATE_MATRIX1 || G.kind == TN_GATE_MATRIX2) {
      if (!G.matrix) { delete net; return set_error(TN_EINVAL, "gate " + std::to_string(g) + ": NULL matrix"); }
      const int d = G.kind == TN_GATE_MATRIX2 ? 4 : 2;
      gate_mat[g] = (int)(net->matrices.size() / 32);
      net->matrices.resize(net->matrices.size() + 32, 0.0);
      memcpy(&net->matrices[32 * gate_mat[g]], G.matrix, sizeof(double) * 2 * d * d);
    }
  }

  std::vector<Block> blocks;
  if (flags & TN_FUSE_2Q) {
    std::vector<std::vector<RecipeOp>> pending(n_qubits);
    std::vector<int> last_block(n_qubits, -1);
    for (int g = 0; g < n_gates; ++g) {
      const tn_gate& G = gates[g];
      if (!gate_is_two_qubit(G.kind)) {
        pending[G.q[0]].push_back(make_op(G, 0, gate_mat[g]));
        continue;
      }
      Block b;
      b.nq = 2;
      b.q[0] = G.q[0];
      b.q[1] = G.q[1];
      for (RecipeOp op : pending[G.q[0]]) { op.pos = 0; b.ops.push_back(op); }
      for (RecipeOp op : pending[G.q[1]]) { op.pos = 1; b.ops.push_back(op); }
      pending[G.q[0]].clear();
      pending[G.q[1]].clear();
      b.ops.push_back(make_op(G, 0, gate_mat[g]));
      last_block[G.q[0]] = last_block[G.q[1]] = (int)blocks.size();
      blocks.push_back(b);
    }
    for (int q = 0; q < n_qubits; ++q) {
      if (pending[q].empty()) continue;
      if (last_block[q] >= 0) {
        Block& b = blocks[last_block[q]];
        const int pos = (b.q[0] == q) ? 0 : 1;
        for (RecipeOp op : pending[q]) { op.pos = pos; b.ops.push_back(op); }
      } else {
        Block b;
        b.nq = 1;
        b.q[0] = q;
        b.q[1] = -1;
        b.ops = pending[q];
        blocks.push_back(b);
      }
    }
  } else {
    for (int g = 0; g < n_gates; ++g) {
      const tn_gate& G = gates[g];
      Block b;
      b.nq = gate_is_two_qubit(G.kind) ? 2 : 1;
      b.q[0] = G.q[0];
      b.q[1] = b.nq == 2 ? G.q[1] : -1;
      b.ops.push_back(make_op(G, 0, gate_mat[g]));
      blocks.push_back(b);
    }
  }

  // ---- tensors (pass 2)
  auto new_mode = [&](int log2) {
    net->mode_log2.push_back(log2);
    return (int32_t)net->mode_log2.size() - 1;
  };
  int64_t offset = 0;
  auto add_tensor = [&](TensorDef t) {
    int64_t sz = 1;
    for (int m : t.modes) sz <<= net->mode_log2[m];
    t.size = sz;
    t.offset = offset;
    offset += sz;
    net->tensors.push_back(t);
  };
  std::vector<int32_t> cur(n_qubits);
  for (int q = 0; q < n_qubits; ++q) {
    cur[q] = new_mode(1);
    TensorDef t;
    t.modes = {cur[q]};
    t.kind = TK_KET0;
    t.recipe = -1;
    t.qubit = q;
    add_tensor(t);
  }
  for (const Block& b : blocks) {
    Recipe r;
    r.nq = b.nq;
    r.diag = ops_diagonal(b.ops, net->matrices) ? 1 : 0;
    r.split_side = -1;
    r.split_on = 0;
    r.op_begin = (int32_t)net->ops.size();
    for (const RecipeOp& op : b.ops) net->ops.push_back(op);
    r.op_end = (int32_t)net->ops.size();
    const int on = (b.nq == 2 && !r.diag && (flags & TN_FUSE_SPLIT)) ? split_qubit(b.ops, net->matrices) : -1;
    if (on >= 0) {
      // operator-Schmidt form: two 3-leg tensors [k][o][i] joined by the bond k
      const int32_t k = new_mode(1);
      for (int side = 0; side < 2; ++side) {
        Recipe h = r;
        h.split_side = side;
        h.split_on = on;
        TensorDef t;
        t.kind = TK_GATE;
        t.qubit = b.q[side];
        t.recipe = (int32_t)net->recipes.size();
        const int32_t o = new_mode(1);
        t.modes = {k, o, cur[b.q[side]]};
        cur[b.q[side]] = o;
        h.offset = offset;
        net->recipes.push_back(h);
        add_tensor(t);
      }
      continue;
    }
    TensorDef t;
    t.kind = TK_GATE;
    t.qubit = b.q[0];
    t.recipe = (int32_t)net->recipes.size();
    if (b.nq == 1) {
      if (r.diag) {
        t.modes = {cur[b.q[0]]};
      } else {
        int32_t o = new_mode(1);
        t.modes = {o, cur[b.q[0]]};
        cur[b.q[0]] = o;
      }
    } else {
      if (r.diag) {
        t.modes = {cur[b.q[0]], cur[b.q[1]]};
      } else {
        int32_t oa = new_mode(1), ob = new_mode(1);
        t.modes = {oa, ob, cur[b.q[0]], cur[b.q[1]]};
        cur[b.q[0]] = oa;
        cur[b.q[1]] = ob;
      }
    }
    r.offset = offset;
    net->recipes.push_back(r);
    add_tensor(t);
  }
  net->wire_final = cur;
  if (output_kind == TN_OUT_STATEVECTOR) {
    net->output_modes = cur;
  } else {
    int lg = 0;
    while (((int64_t)1 << lg) < n_bitstrings) ++lg;
    net->batch_log2 = lg;
    net->n_bitstrings = n_bitstrings;
    net->batch_mode = new_mode(lg);
    for (int q = 0; q < n_qubits; ++q) {
      TensorDef t;
      t.modes = {net->batch_mode, cur[q]};
      t.kind = TK_PROJ;
      t.recipe = -1;
      t.qubit = q;
      add_tensor(t);
    }
    net->output_modes = {net->batch_mode};
  }
  net->input_elems = offset;

  // ---- adjoint sweep description (unfused gates, circuit order)
  for (int g = 0; g < n_gates; ++g) {
    const tn_gate& G = gates[g];
    const bool two = gate_is_two_qubit(G.kind);
    auto push = [&](int kind, double angle, int param) {
      SweepGate s;
      s.nq = two ? 2 : 1;
      s.q[0] = G.q[0];
      s.q[1] = two ? G.q[1] : -1;
      Recipe r;
      r.nq = s.nq;
      r.diag = 0;
      r.split_side = -1;
      r.split_on = 0;
      r.op_begin = (int32_t)net->sweep_ops.size();
      RecipeOp op;
      op.kind = kind;
      op.pos = 0;
      op.mat = gate_mat[g];
      op.angle[0] = angle;
      op.angle[1] = op.angle[2] = 0;
      op.param[0] = param;
      op.param[1] = op.param[2] = -1;
      if (kind == G.kind) {  // keep every angle of the original gate
        for (int j = 0; j < 3; ++j) { op.angle[j] = G.angle[j]; op.param[j] = j < gate_n_angles(kind) ? G.param[j] : -1; }
      }
      net->sweep_ops.push_back(op);
      r.op_end = (int32_t)net->sweep_ops.size();
      r.offset = 0;
      s.recipe = (int32_t)net->sweep_recipes.size();
      net->sweep_recipes.push_back(r);
      s.param = op.param[0];
      s.gen = s.param >= 0 ? gen_of(kind) : GEN_NONE;
      s.diag = gate_is_diagonal(kind) ? 1 : 0;
      net->sweep.push_back(s);
    };
    if (G.kind == TN_GATE_U3 && (G.param[0] >= 0 || G.param[1] >= 0 || G.param[2] >= 0)) {
      // U3(t, f, l) = e^{i(f+l)/2} RZ(f) RY(t) RZ(l): in circuit order RZ(l), RY(t), RZ(f)
      push(TN_GATE_RZ, G.angle[2], G.param[2]);
      push(TN_GATE_RY, G.angle[0], G.param[0]);
      push(TN_GATE_RZ, G.angle[1], G.param[1]);
    } else {
      push(G.kind, G.angle[0], gate_n_angles(G.kind) ? G.param[0] : -1);
    }
  }
  *net_out = net;
  return TN_OK;
}

extern "C" void tn_network_destroy(tn_network* net) {
  if (!net) return;
  device_release_network(net);
  delete net;
}

extern "C" tn_status tn_network_info(const tn_network* net, int32_t* n_tensors, int32_t* n_modes, int32_t* n_qubits,
                                     int32_t* n_output_modes) {
  clear_error();
  if (!net) return set_error(TN_EINVAL, "net is NULL");
  if (n_tensors) *n_tensors = (int32_t)net->tensors.size();
  if (n_modes) *n_modes = (int32_t)net->mode_log2.size();
  if (n_qubits) *n_qubits = net->n_qubits;
  if (n_output_modes) *n_output_modes = (int32_t)net->output_modes.size();
  return TN_OK;
}

extern "C" tn_status tn_network_tensor(const tn_network* net, int32_t t, int32_t* rank, int32_t* modes,
                                       int64_t* extents) {
  clear_error();
  if (!net || t < 0 || t >= (int32_t)net->tensors.size()) return set_error(TN_EINVAL, "bad tensor index");
  const TensorDef& T = net->tensors[t];
  if (rank) *rank = (int32_t)T.modes.size();
  for (size_t i = 0; i < T.modes.size(); ++i) {
    if (modes) modes[i] = T.modes[i];
    if (extents) extents[i] = (int64_t)1 << net->mode_log2[T.modes[i]];
  }
  return TN_OK;
}

extern "C" tn_status tn_network_output(const tn_network* net, int32_t* modes, int64_t* extents) {
  clear_error();
  if (!net) return set_error(TN_EINVAL, "net is NULL");
  for (size_t i = 0; i < net->output_modes.size(); ++i) {
    if (modes) modes[i] = net->output_modes[i];
    if (extents) extents[i] = (int64_t)1 << net->mode_log2[net->output_modes[i]];
  }
  return TN_OK;
}

extern "C" tn_status tn_network_values(const tn_network* net, const double* params, const uint64_t* bitstrings,
                                       double* out, int64_t out_len_doubles) {
  clear_error();
  if (!net || !out) return set_error(TN_EINVAL, "NULL argument");
  if (out_len_doubles < 2 * net->input_elems) return set_error(TN_EINVAL, "output array too short");
  if (net->n_params > 0 && !params) return set_error(TN_EINVAL, "params required");
  if (net->output_kind == TN_OUT_AMPLITUDES && !bitstrings) return set_error(TN_EINVAL, "bitstrings required");
  std::vector<double> zero(1, 0.0);
  network_values_host(net, params ? params : zero.data(), bitstrings, out);
  return TN_OK;
}
