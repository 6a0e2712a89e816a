// Host planner for the register-resident engine.
//
// A sample's 2^n amplitudes are spread over 2^t threads holding 2^r
// amplitudes each (n = r + t). Single-qubit gates are applied in registers:
// the runs of them on each register-resident qubit are multiplied into one
// 2x2 block per qubit, and one layer op (L1Q) applies the blocks of all r
// register bits in one pass. CZs act on any bits (a sign pattern). The
// planner cuts the gate list into segments with one qubit placement each;
// between segments the engine re-places the state through LDS (a "remap").
//
// Gates on disjoint qubits commute, so the planner list-schedules the gate
// dependency DAG (only the order of gates sharing a qubit is kept), in
// rounds: every ready CZ, then the ready single-qubit runs of the register
// qubits as one L1Q round. It re-places when no round can start. At a
// re-placement the register bits receive the r qubits whose next pending
// single-qubit gate is soonest (ties: lower qubit). A round that finds fewer
// than r runs ready costs as much as a full one; the planner also plans with
// such partial rounds deferred (to a later segment holding their qubits) once
// a segment has made progress, and keeps the cheaper plan. Checkpoint
// positions are scheduling barriers.
//
// CNOTs are never applied as engine ops. A CNOT maps the amplitude index
// x -> x ^ (x_c << t), a linear map over GF(2); so is the LDS slot of a remap.
// Every ready CNOT is therefore folded, at the next re-placement, into the
// write addresses of the closing segment: its write masks are the closing
// placement's unit vectors mapped through the folded CNOTs (in order).
#include <algorithm>
#include <climits>
#include <cstring>

#include "qs_internal.h"

namespace qs {

namespace {

// The qubit a gate needs on a register bit: every single-qubit gate runs in
// registers as part of a block; CZs act on any bits; CNOTs are folded into
// remaps.
int register_target(const qs_gate& g) {
  return g.op <= QS_OP_H ? g.q0 : -1;
}

// x -> x ^ (bit c of x) << t on a logical index mask.
uint16_t apply_cnot(uint16_t x, int c, int t) {
  return (uint16_t)(x ^ (((x >> c) & 1u) << t));
}

struct Placement {
  uint8_t phys2log[kMapStride];
  uint8_t log2phys[32];
};

// Registers: the r qubits used soonest from gate g on. Threads: the rest,
// ordered so that the lowest thread bits carry qubits with distinct q mod 5
// (the LDS slot swizzle folds logical bits in groups of 5, so distinct
// residues give distinct banks for lanes that differ in those bits).
Placement choose(int n, int r, const std::vector<int>& next_use) {
  std::vector<int> q(n);
  for (int i = 0; i < n; ++i) q[i] = i;
  std::stable_sort(q.begin(), q.end(), [&](int a, int b) {
    return next_use[a] < next_use[b];
  });
  std::vector<int> regs(q.begin(), q.begin() + r);
  std::sort(regs.begin(), regs.end());
  std::vector<int> rest(q.begin() + r, q.end());
  std::sort(rest.begin(), rest.end());
  std::vector<int> thr;
  bool used_res[5] = {false, false, false, false, false};
  std::vector<bool> taken(rest.size(), false);
  for (size_t pass = 0; pass < rest.size(); ++pass) {
    int pick = -1;
    for (size_t i = 0; i < rest.size(); ++i)
      if (!taken[i] && !used_res[rest[i] % 5]) { pick = (int)i; break; }
    if (pick < 0)
      for (size_t i = 0; i < rest.size(); ++i)
        if (!taken[i]) { pick = (int)i; break; }
    taken[pick] = true;
    used_res[rest[pick] % 5] = true;
    thr.push_back(rest[pick]);
    if (thr.size() % 5 == 0) std::fill(used_res, used_res + 5, false);
  }
  Placement p;
  std::memset(&p, 0xff, sizeof(p));
  for (int j = 0; j < r; ++j) p.phys2log[j] = (uint8_t)regs[j];
  for (int i = 0; i < (int)thr.size(); ++i) p.phys2log[r + i] = (uint8_t)thr[i];
  for (int i = 0; i < n; ++i) p.log2phys[p.phys2log[i]] = (uint8_t)i;
  return p;
}

bool is_rotation(int op) {
  return op == QS_OP_RX || op == QS_OP_RY || op == QS_OP_RZ;
}

bool is_one_qubit(int op) { return op <= QS_OP_H; }

// Regroups the single-gate ops of each segment into layer ops. Inside a
// segment the placement is fixed, and only the order of gates sharing a
// qubit matters. Alternately (a) every register bit takes the run of
// single-qubit gates at the head of its qubit's pending list as one block,
// and all blocks go into one L1Q op; (b) every CZ whose two qubits have it at
// the head of their pending lists joins one sign pattern (a DIAG record)
// that the same L1Q op applies after its blocks. CZs ready before the
// segment's first round form a pattern applied before its blocks. The
// earliest pending gate is always at the head of its lists, so every round
// makes progress. Any other op (which the scheduler never emits) marks the
// plan as not layered.
void build_layers(SvPlan& P, const qs_circuit& c, bool per_sample_angles_all) {
  const int r = P.r, R = 1 << r;
  std::vector<SvOp> in = std::move(P.ops);
  std::vector<int32_t> seg_in = P.seg_begin;
  P.ops.clear();
  P.exec.clear();
  P.exec_seg.assign(1, 0);
  auto per_sample = [&](const qs_gate& g) {
    if (!is_rotation(g.op)) return false;
    return per_sample_angles_all ? (g.p_w >= 0 || g.p_b >= 0 || g.feat >= 0)
                                 : g.feat >= 0;
  };
  for (int s = 0; s + 1 < (int)seg_in.size(); ++s) {
    const int beg = seg_in[s], end = seg_in[s + 1];
    P.seg_begin[s] = (int32_t)P.ops.size();
    std::vector<std::vector<int>> q(P.n);  // pending ops per physical position
    std::vector<size_t> head(P.n, 0);
    for (int o = beg; o < end; ++o) {
      q[in[o].a].push_back(o);
      if (in[o].kind == QS_OP_CNOT || in[o].kind == QS_OP_CZ) q[in[o].b].push_back(o);
    }
    auto at_head = [&](int pos, int o) {
      return head[pos] < q[pos].size() && q[pos][head[pos]] == o;
    };
    auto is_u = [&](int o) { return is_one_qubit(in[o].kind) && in[o].a < r; };
    std::vector<char> done(end - beg, 0);
    int left = end - beg;
    // (b) the ready CZs as one sign pattern: its DIAG record, or -1.
    auto take_czs = [&]() {
      int rec = -1;
      bool progress = true;
      while (progress) {
        progress = false;
        for (int o = beg; o < end; ++o) {
          if (done[o - beg] || is_u(o)) continue;
          const SvOp& x = in[o];
          const bool two = x.kind == QS_OP_CNOT || x.kind == QS_OP_CZ;
          if (!at_head(x.a, o) || (two && !at_head(x.b, o))) continue;
          head[x.a]++;
          if (two) head[x.b]++;
          done[o - beg] = 1;
          --left;
          progress = true;
          P.exec.insert(P.exec.end(), {x.gate, x.a, two ? x.b : 0});
          if (x.kind != QS_OP_CZ) {
            P.layered = false;
            continue;
          }
          if (rec < 0) {
            rec = (int)(P.diag.size() / kDiagWords);
            P.diag.resize(P.diag.size() + kDiagWords, 0u);
          }
          uint32_t* d = &P.diag[(size_t)rec * kDiagWords];
          const int lo = x.a < x.b ? x.a : x.b, hi = x.a < x.b ? x.b : x.a;
          if (hi < r) {
            for (int k = 0; k < R; ++k)
              if (((k >> lo) & 1) && ((k >> hi) & 1)) d[0] ^= 1u << k;
          } else if (lo < r) {
            d[2 + lo] ^= 1u << (hi - r);
          } else {
            d[7 + (lo - r)] ^= 1u << (hi - r);
          }
        }
      }
      return rec;
    };
    auto new_op = [&](uint8_t mask, uint8_t ps, const int32_t* rec) {
      const int id = (int)(P.l1q.size() / kL1QWords);
      P.ops.push_back(SvOp{kOpL1Q, mask, 0, ps, id});
      P.l1q.insert(P.l1q.end(), rec, rec + kL1QWords);
      return id;
    };
    int pre = take_czs();
    while (left > 0 || pre >= 0) {
      // (a) one block per register bit
      int32_t rec[kL1QWords];
      for (int j = 0; j < kL1QWords; ++j) rec[j] = -1;
      uint8_t mask = 0, ps = 0;
      for (int j = 0; j < r; ++j) {
        std::vector<int> gl;
        while (head[j] < q[j].size() && is_u(q[j][head[j]])) {
          const int o = q[j][head[j]++];
          gl.push_back(in[o].gate);
          done[o - beg] = 1;
          --left;
        }
        if (gl.empty()) continue;
        uint8_t bps = 0;
        for (int g : gl) {
          bps |= per_sample(c.gates[g]) ? 1 : 0;
          P.exec.insert(P.exec.end(), {g, j, 0});
        }
        rec[j] = (int32_t)P.blk_fu.size();
        P.blk_gates.insert(P.blk_gates.end(), gl.begin(), gl.end());
        P.blk_begin.push_back((int32_t)P.blk_gates.size());
        rec[kL1QFused + j] = bps ? -1 : P.n_fu;
        P.blk_fu.push_back(bps ? -1 : P.n_fu++);
        P.blk_gen.push_back(bps ? -1 : P.n_gen);
        if (!bps) P.n_gen += (int)gl.size();
        mask |= (uint8_t)(1u << j);
        ps |= bps;
      }
      int id = -1;  // this round's L1Q record
      if (mask || pre >= 0) {
        rec[kL1QPreDiag] = pre;
        pre = -1;
        id = new_op(mask, ps, rec);
      }
      // (b) the CZs this round made ready, applied after its blocks
      const int post = take_czs();
      if (post >= 0) {
        if (id < 0) {
          for (int j = 0; j < kL1QWords; ++j) rec[j] = -1;
          id = new_op(0, 0, rec);
        }
        P.l1q[(size_t)id * kL1QWords + kL1QPostDiag] = post;
      }
    }
    for (int g : P.seg_folded[s]) P.exec.insert(P.exec.end(), {g, -1, -1});
    P.exec_seg.push_back((int32_t)(P.exec.size() / 3));
  }
  P.seg_begin.back() = (int32_t)P.ops.size();
  // Register bits without a block read the identity from the slot after the
  // fused matrices.
  for (size_t o = 0; o < P.l1q.size() / kL1QWords; ++o)
    for (int j = 0; j < r; ++j)
      if (P.l1q[o * kL1QWords + j] < 0) P.l1q[o * kL1QWords + kL1QFused + j] = P.n_fu;
}

}  // namespace

namespace {

// One scheduling pass (see the file comment); `defer` holds back partial
// L1Q rounds once the segment has made progress.
SvPlan plan_once(const qs_circuit& c, int r, bool per_sample_angles_all,
                 const int32_t* ckpt_gates, int n_ckpt, bool defer) {
  SvPlan P;
  const int n = c.n_qubits, G = c.n_gates;
  P.n = n;
  P.r = r;
  P.t = n - r;
  P.n_gates = G;

  // Epochs: checkpoint boundaries are scheduling barriers.
  std::vector<int> bounds;
  for (int i = 0; i < n_ckpt; ++i) bounds.push_back(ckpt_gates[i]);
  bounds.push_back(G);

  // Per-qubit gate sequences (the dependency DAG of the gate list: gates on
  // disjoint qubits commute, so only the per-qubit order must be kept).
  std::vector<std::vector<int>> seq(n);
  for (int g = 0; g < G; ++g) {
    seq[c.gates[g].q0].push_back(g);
    if (c.gates[g].q1 >= 0) seq[c.gates[g].q1].push_back(g);
  }
  std::vector<size_t> head(n, 0);   // next unscheduled position per qubit
  std::vector<char> done(G, 0);

  auto ready = [&](int g) {
    const qs_gate& x = c.gates[g];
    if (seq[x.q0][head[x.q0]] != g) return false;
    if (x.q1 >= 0 && seq[x.q1][head[x.q1]] != g) return false;
    return true;
  };
  // Soonest pending single-qubit gate of each qubit, counted in gate order.
  auto next_use_from_heads = [&]() {
    std::vector<int> nu(n, INT_MAX);
    for (int q = 0; q < n; ++q)
      for (size_t i = head[q]; i < seq[q].size(); ++i) {
        int g = seq[q][i];
        if (register_target(c.gates[g]) == q) { nu[q] = g; break; }
      }
    return nu;
  };

  std::vector<SvOp> ops;
  Placement cur = choose(n, r, next_use_from_heads());
  auto open_segment = [&](const Placement& pl) {
    P.seg_begin.push_back((int32_t)ops.size());
    P.seg_map.insert(P.seg_map.end(), pl.phys2log, pl.phys2log + kMapStride);
    P.seg_ckpt.push_back(-1);
    P.seg_folded.emplace_back();
  };
  auto seg_empty = [&]() {
    return P.seg_begin.back() == (int32_t)ops.size() && P.seg_ckpt.back() < 0 &&
           P.seg_folded.back().empty();
  };
  auto emit = [&](int g, int& remaining) {
    const qs_gate& x = c.gates[g];
    SvOp op;
    op.kind = (uint8_t)x.op;
    op.aux = 0;
    op.gate = g;
    op.a = cur.log2phys[x.q0];
    op.b = x.q1 >= 0 ? cur.log2phys[x.q1] : 0;
    ops.push_back(op);
    done[g] = 1;
    head[x.q0]++;
    if (x.q1 >= 0) head[x.q1]++;
    --remaining;
  };
  // Folds every ready CNOT of [lo, hi) (repeatedly: a chain folds whole) into
  // the current segment's closing remap.
  auto fold_cnots = [&](int lo, int hi, int& remaining) {
    bool any = false, more = true;
    while (more) {
      more = false;
      for (int g = lo; g < hi; ++g) {
        if (done[g] || c.gates[g].op != QS_OP_CNOT || !ready(g)) continue;
        P.seg_folded.back().push_back(g);
        done[g] = 1;
        head[c.gates[g].q0]++;
        head[c.gates[g].q1]++;
        --remaining;
        more = any = true;
      }
    }
    return any;
  };
  open_segment(cur);
  int lo = 0;
  for (size_t ep = 0; ep < bounds.size(); ++ep) {
    const int hi = bounds[ep];  // gates [lo, hi) form this epoch
    int remaining = hi - lo;
    while (remaining > 0) {
      // Rounds: every ready CZ of the epoch, then the ready single-qubit
      // runs of the register qubits, until no round can start.
      for (;;) {
        bool more = true;
        while (more) {
          more = false;
          for (int g = lo; g < hi; ++g)
            if (!done[g] && c.gates[g].op == QS_OP_CZ && ready(g)) {
              emit(g, remaining);
              more = true;
            }
        }
        int runs = 0;
        for (int j = 0; j < r; ++j) {
          const int q = cur.phys2log[j];
          if (head[q] < seq[q].size()) {
            const int g = seq[q][head[q]];
            if (g >= lo && g < hi && register_target(c.gates[g]) == q) ++runs;
          }
        }
        if (runs == 0) break;
        if (defer && runs < r && P.seg_begin.back() < (int32_t)ops.size()) break;
        for (int j = 0; j < r; ++j) {
          const int q = cur.phys2log[j];
          while (head[q] < seq[q].size()) {
            const int g = seq[q][head[q]];
            if (g < lo || g >= hi || register_target(c.gates[g]) != q) break;
            emit(g, remaining);
          }
        }
      }
      // Stuck: every ready gate needs a thread-resident qubit in a register
      // or is a CNOT (or a partial round was held back). Fold the ready
      // CNOTs into this segment's closing remap and re-place (an epoch
      // ending in CNOTs gets a remap to the same placement, so every
      // checkpoint and the last segment end in a plain placement).
      const bool folded = remaining > 0 && fold_cnots(lo, hi, remaining);
      if (remaining == 0) {
        if (folded) open_segment(cur);
        break;
      }
      Placement nxt = choose(n, r, next_use_from_heads());
      if (seg_empty())
        std::memcpy(&P.seg_map[P.seg_map.size() - kMapStride], nxt.phys2log,
                    kMapStride);
      else
        open_segment(nxt);
      cur = nxt;
    }
    if (ep + 1 < bounds.size()) {  // checkpoint after the first hi gates
      P.seg_ckpt.back() = (int32_t)ep;
      open_segment(cur);
    }
    lo = hi;
  }
  P.seg_begin.push_back((int32_t)ops.size());

  // Angle slots, by gate: rotations whose angle differs per sample.
  P.gate_slot.assign(G, -1);
  for (int g = 0; g < G; ++g) {
    const qs_gate& gt = c.gates[g];
    if (!is_rotation(gt.op)) continue;
    bool per_sample = per_sample_angles_all
                          ? (gt.p_w >= 0 || gt.p_b >= 0 || gt.feat >= 0)
                          : (gt.feat >= 0);
    if (per_sample) {
      P.gate_slot[g] = (int)P.slot_gate.size();
      P.slot_gate.push_back(g);
    }
  }
  P.ops = std::move(ops);
  P.blk_begin.assign(1, 0);
  build_layers(P, c, per_sample_angles_all);

  // Read masks (a segment's placement) and write masks (its placement mapped
  // through the CNOTs folded at its end).
  const int nseg = P.nseg();
  P.seg_lay.assign((size_t)nseg * kLayWords, 0);
  for (int s = 0; s < nseg; ++s) {
    uint16_t* rd = &P.seg_lay[(size_t)s * kLayWords];
    uint16_t* wr = rd + kMapStride;
    for (int p = 0; p < n; ++p) {
      uint16_t v = (uint16_t)(1u << P.seg_map[(size_t)s * kMapStride + p]);
      rd[p] = v;
      for (int g : P.seg_folded[s]) v = apply_cnot(v, c.gates[g].q0, c.gates[g].q1);
      wr[p] = v;
    }
  }
  int changes = 0;
  for (int s = 1; s < nseg; ++s)
    if (std::memcmp(&P.seg_lay[(size_t)(s - 1) * kLayWords + kMapStride],
                    &P.seg_lay[(size_t)s * kLayWords], kMapStride * 2) != 0)
      ++changes;
  P.n_remaps = changes;
  return P;
}

}  // namespace

SvPlan plan_sv(const qs_circuit& c, int r, bool per_sample_angles_all,
               const int32_t* ckpt_gates, int n_ckpt) {
  // Cost of a plan: an L1Q op does about 30 times the work of a remap.
  auto cost = [](const SvPlan& p) { return 32 * (int64_t)p.ops.size() + p.n_remaps; };
  SvPlan P = plan_once(c, r, per_sample_angles_all, ckpt_gates, n_ckpt, false);
  SvPlan D = plan_once(c, r, per_sample_angles_all, ckpt_gates, n_ckpt, true);
  if (D.layered && (!P.layered || cost(D) < cost(P))) P = std::move(D);

  // Gradient columns of the shared parameters, and each rotation's columns.
  const int G = c.n_gates;
  P.grad_cols = grad_columns(c, per_sample_angles_all);
  if (!per_sample_angles_all) {
    std::vector<int32_t> col(c.n_params > 0 ? c.n_params : 1, -1);
    for (size_t j = 0; j < P.grad_cols.size(); ++j) col[P.grad_cols[j]] = (int32_t)j;
    P.gate_cols.assign(2 * (size_t)G, -1);
    for (int g = 0; g < G; ++g) {
      const qs_gate& x = c.gates[g];
      if (!is_rotation(x.op)) continue;
      if (x.p_w >= 0) P.gate_cols[2 * (size_t)g] = col[x.p_w];
      if (x.p_b >= 0) P.gate_cols[2 * (size_t)g + 1] = col[x.p_b];
    }
  }
  return P;
}

std::vector<int32_t> grad_columns(const qs_circuit& c, bool per_sample_params) {
  std::vector<int32_t> cols;
  if (per_sample_params || c.n_params <= 0) return cols;
  std::vector<char> used(c.n_params, 0);
  for (int g = 0; g < c.n_gates; ++g) {
    const qs_gate& x = c.gates[g];
    if (!is_rotation(x.op)) continue;
    if (x.p_w >= 0) used[x.p_w] = 1;
    if (x.p_b >= 0) used[x.p_b] = 1;
  }
  for (int p = 0; p < c.n_params; ++p)
    if (used[p]) cols.push_back(p);
  return cols;
}

std::vector<TiledEpoch> plan_tiled(const qs_circuit& c, int m, int low_keep,
                                   const int32_t* ckpt_gates, int n_ckpt) {
  const int n = c.n_qubits, G = c.n_gates;
  if (m > n) m = n;
  if (low_keep > m) low_keep = m;
  std::vector<std::vector<int>> seq(n);
  for (int g = 0; g < G; ++g) {
    seq[c.gates[g].q0].push_back(g);
    if (c.gates[g].q1 >= 0) seq[c.gates[g].q1].push_back(g);
  }
  std::vector<size_t> head(n, 0);
  std::vector<char> done(G, 0);
  auto ready = [&](int g) {
    const qs_gate& x = c.gates[g];
    if (seq[x.q0][head[x.q0]] != g) return false;
    if (x.q1 >= 0 && seq[x.q1][head[x.q1]] != g) return false;
    return true;
  };
  std::vector<int> bounds;
  for (int i = 0; i < n_ckpt; ++i) bounds.push_back(ckpt_gates[i]);
  bounds.push_back(G);

  std::vector<TiledEpoch> out;
  int lo = 0;
  for (size_t ep = 0; ep < bounds.size(); ++ep) {
    const int hi = bounds[ep];
    int remaining = hi - lo;
    while (remaining > 0) {
      // Tile: the low_keep lowest qubits, then the qubits whose next
      // unscheduled gate comes soonest.
      std::vector<int> nxt(n, INT_MAX);
      for (int q = 0; q < n; ++q)
        if (head[q] < seq[q].size()) nxt[q] = seq[q][head[q]];
      std::vector<int> cand;
      for (int q = low_keep; q < n; ++q) cand.push_back(q);
      std::stable_sort(cand.begin(), cand.end(),
                       [&](int a, int b) { return nxt[a] < nxt[b]; });
      std::vector<int> L;
      for (int q = 0; q < low_keep; ++q) L.push_back(q);
      for (int i = 0; (int)L.size() < m && i < (int)cand.size(); ++i)
        L.push_back(cand[i]);
      std::sort(L.begin(), L.end());
      std::vector<int> local(n, -1);
      for (int j = 0; j < (int)L.size(); ++j) local[L[j]] = j;
      TiledEpoch e;
      e.L = L;
      bool progress = true;
      while (progress) {
        progress = false;
        for (int g = lo; g < hi; ++g) {
          if (done[g] || !ready(g)) continue;
          const qs_gate& x = c.gates[g];
          if (local[x.q0] < 0 || (x.q1 >= 0 && local[x.q1] < 0)) continue;
          qs_gate y = x;
          y.q0 = local[x.q0];
          y.q1 = x.q1 >= 0 ? local[x.q1] : -1;
          e.gates.push_back(y);
          e.gate_index.push_back(g);
          done[g] = 1;
          head[x.q0]++;
          if (x.q1 >= 0) head[x.q1]++;
          --remaining;
          progress = true;
        }
      }
      out.push_back(std::move(e));
    }
    if (ep + 1 < bounds.size() && !out.empty()) out.back().ckpt_after = (int)ep;
    lo = hi;
  }
  return out;
}

}  // namespace qs
