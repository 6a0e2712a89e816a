// Host planner for the dense-block path of large states.
//
// The gate list is cut into blocks, each acting on a set of K qubits
// (K = 4 or 5): the block's gates multiply into one 2^K x 2^K unitary, which
// the MFMA kernels apply to the whole state as a complex matrix product in
// its real embedding (one HBM pass per block). Gates on disjoint qubits
// commute, so a block takes every gate it can reach in the dependency DAG
// (only the order of gates sharing a qubit is kept): a gate is ready when it
// heads the pending list of each of its qubits, and a block absorbs ready
// gates whose qubits it holds until none is left.
//
// A block's qubit set is grown one qubit at a time from a seed, each step
// adding the qubit that lets the block absorb the most gates; every qubit
// that heads some pending gate is tried as the seed and the block absorbing
// the most gates is kept (ties: the block holding the earliest pending gate).
// A set still smaller than K is padded with the highest unused qubits (so
// the low, contiguous address bits stay outside the block and the kernels'
// column loads stay coalesced) and absorbs again. Checkpoint positions are
// barriers: the gates before a checkpoint are blocked on their own.
#include <algorithm>
#include <climits>

#include "qs_internal.h"

namespace qs {

namespace {

struct Frontier {
  const qs_circuit* c;
  std::vector<std::vector<int>> seq;  // gates of each qubit, in order
  std::vector<size_t> head;           // next pending position per qubit
};

bool two_qubit(const qs_gate& g) { return g.q1 >= 0; }

// Gates absorbed by a block on qubit set `in` (a mask over qubits), taken
// from a copy of the heads; their indices are appended to `out` when given.
int absorb(const Frontier& f, const std::vector<char>& in, std::vector<size_t>& head,
           std::vector<int>* out) {
  const int n = f.c->n_qubits;
  int taken = 0;
  bool progress = true;
  while (progress) {
    progress = false;
    for (int q = 0; q < n; ++q) {
      if (!in[q]) continue;
      while (head[q] < f.seq[q].size()) {
        const int g = f.seq[q][head[q]];
        const qs_gate& x = f.c->gates[g];
        if (two_qubit(x)) {
          const int o = x.q0 == q ? x.q1 : x.q0;
          if (!in[o] || head[o] >= f.seq[o].size() || f.seq[o][head[o]] != g) break;
          ++head[o];
        }
        ++head[q];
        ++taken;
        progress = true;
        if (out) out->push_back(g);
      }
    }
  }
  return taken;
}

int count_in(const std::vector<char>& in) {
  int k = 0;
  for (char v : in) k += v;
  return k;
}

// Grows a qubit set from `seed` to at most K qubits, greedily by absorbed
// gates; returns the absorbed count.
int grow(const Frontier& f, int K, int seed, std::vector<char>& in) {
  const int n = f.c->n_qubits;
  in.assign(n, 0);
  in[seed] = 1;
  std::vector<size_t> h = f.head;
  int best = absorb(f, in, h, nullptr);
  while (count_in(in) < K) {
    int pick = -1, pick_score = -1;
    for (int q = 0; q < n; ++q) {
      if (in[q] || f.head[q] >= f.seq[q].size()) continue;
      in[q] = 1;
      std::vector<size_t> hh = f.head;
      const int s = absorb(f, in, hh, nullptr);
      in[q] = 0;
      if (s > pick_score) {
        pick_score = s;
        pick = q;
      }
    }
    if (pick < 0 || pick_score <= best) {
      // no qubit adds a gate by itself; a 2-qubit gate may still need both
      // of its qubits: take the partner of the earliest pending 2-qubit gate
      // that touches the set, if there is room.
      int partner = -1, first = INT_MAX;
      for (int q = 0; q < n; ++q) {
        if (!in[q] || h[q] >= f.seq[q].size()) continue;
        const int g = f.seq[q][h[q]];
        const qs_gate& x = f.c->gates[g];
        if (!two_qubit(x) || g >= first) continue;
        const int o = x.q0 == q ? x.q1 : x.q0;
        if (!in[o]) {
          partner = o;
          first = g;
        }
      }
      if (partner < 0) break;
      in[partner] = 1;
      std::vector<size_t> hh = f.head;
      const int s = absorb(f, in, hh, nullptr);
      if (s <= best && count_in(in) >= K) {
        in[partner] = 0;
        break;
      }
      best = s;
      continue;
    }
    in[pick] = 1;
    best = pick_score;
  }
  return best;
}

}  // namespace

std::vector<DenseBlock> plan_blocks(const qs_circuit& c, int K, const int32_t* ckpt_gates,
                                    int n_ckpt) {
  const int n = c.n_qubits, G = c.n_gates;
  if (K > n) K = n;
  std::vector<DenseBlock> out;
  std::vector<int> bounds;
  for (int i = 0; i < n_ckpt; ++i) bounds.push_back(ckpt_gates[i]);
  bounds.push_back(G);
  int lo = 0;
  for (size_t seg = 0; seg < bounds.size(); ++seg) {
    const int hi = bounds[seg];
    // The segment's own dependency lists.
    qs_circuit sub = c;
    Frontier f;
    f.c = &c;
    f.seq.assign(n, {});
    for (int g = lo; g < hi; ++g) {
      f.seq[c.gates[g].q0].push_back(g);
      if (c.gates[g].q1 >= 0) f.seq[c.gates[g].q1].push_back(g);
    }
    f.head.assign(n, 0);
    (void)sub;
    int remaining = hi - lo;
    while (remaining > 0) {
      std::vector<char> best_in;
      int best = -1, best_first = INT_MAX;
      for (int s = 0; s < n; ++s) {
        if (f.head[s] >= f.seq[s].size()) continue;
        std::vector<char> in;
        const int got = grow(f, K, s, in);
        // earliest pending gate the block holds, for ties
        int first = INT_MAX;
        for (int q = 0; q < n; ++q)
          if (in[q] && f.head[q] < f.seq[q].size()) first = std::min(first, f.seq[q][f.head[q]]);
        if (got > best || (got == best && first < best_first)) {
          best = got;
          best_first = first;
          best_in = in;
        }
      }
      // pad with the highest unused qubits
      for (int q = n - 1; q >= 0 && count_in(best_in) < K; --q)
        if (!best_in[q]) best_in[q] = 1;
      DenseBlock b;
      const int taken = absorb(f, best_in, f.head, &b.gates);
      if (taken == 0) break;  // cannot happen: a seed always heads a gate
      for (int q = 0; q < n; ++q)
        if (best_in[q]) b.qubits.push_back(q);
      remaining -= taken;
      out.push_back(std::move(b));
    }
    if (seg + 1 < bounds.size() && !out.empty()) out.back().ckpt_after = (int)seg;
    lo = hi;
  }
  return out;
}

}  // namespace qs
