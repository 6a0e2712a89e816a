// C ABI entry points: validation, launch-shape choice, plan cache, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <cstring>
#include <mutex>
#include <optional>
#include <unordered_map>

#include "qs_internal.h"

namespace qs {
int sv_max_threads(int dtype, int r, int adjoint);
bool no_alloc_call();

namespace {
thread_local void* t_call_stream = nullptr;
thread_local bool t_in_call = false;
}  // namespace

CallStream::CallStream(void* stream) : prev(t_call_stream), prev_in_call(t_in_call) {
  t_call_stream = stream;
  t_in_call = true;
}
CallStream::~CallStream() {
  t_call_stream = prev;
  t_in_call = prev_in_call;
}

namespace {
thread_local bool t_no_alloc = false;
}  // namespace

NoAllocCall::NoAllocCall() : prev(t_no_alloc) { t_no_alloc = true; }
NoAllocCall::~NoAllocCall() { t_no_alloc = prev; }

int plan_upload_status() {
  if (t_no_alloc) return QS_ERR_NOT_PLANNED;
  return call_stream_capturing() ? QS_ERR_CAPTURE : QS_OK;
}

bool no_alloc_call() { return t_no_alloc; }

bool call_stream_capturing() {
  if (!t_in_call) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(static_cast<hipStream_t>(t_call_stream), &cs) != hipSuccess)
    return false;
  return cs != hipStreamCaptureStatusNone;
}
}  // namespace qs

using namespace qs;

namespace {

constexpr int kVersion = 10000;  // 1.0.0
constexpr int64_t kMaxLds = 160 * 1024;

bool is_rotation(int op) { return op == QS_OP_RX || op == QS_OP_RY || op == QS_OP_RZ; }

int validate(const qs_circuit* c) {
  if (!c || c->n_qubits < 1 || c->n_qubits > 30 || c->n_gates < 0 ||
      c->n_params < 0 || c->n_features < 0)
    return QS_ERR_INVALID;
  if (c->n_gates > 0 && !c->gates) return QS_ERR_INVALID;
  for (int g = 0; g < c->n_gates; ++g) {
    const qs_gate& x = c->gates[g];
    if (x.op < QS_OP_RX || x.op > QS_OP_MEASURE || x.flags != 0) return QS_ERR_INVALID;
    if (x.op == QS_OP_RESET || x.op == QS_OP_MEASURE) {  // uniform = feats[b][feat]
      if (x.q0 < 0 || x.q0 >= c->n_qubits || x.q1 != -1) return QS_ERR_INVALID;
      if (x.feat < 0 || x.feat >= c->n_features) return QS_ERR_INVALID;
      continue;
    }
    if (x.q0 < 0 || x.q0 >= c->n_qubits) return QS_ERR_INVALID;
    if (x.op == QS_OP_CNOT || x.op == QS_OP_CZ) {
      if (x.q1 < 0 || x.q1 >= c->n_qubits || x.q1 == x.q0) return QS_ERR_INVALID;
    } else if (x.q1 != -1) {
      return QS_ERR_INVALID;
    }
    if (is_rotation(x.op)) {
      if (x.p_w < -1 || x.p_w >= c->n_params) return QS_ERR_INVALID;
      if (x.p_b < -1 || x.p_b >= c->n_params) return QS_ERR_INVALID;
      if (x.feat < -1 || x.feat >= c->n_features) return QS_ERR_INVALID;
    }
  }
  return QS_OK;
}

bool is_channel(int op) { return op == QS_OP_RESET || op == QS_OP_MEASURE; }

bool has_channels(const qs_circuit& c) {
  for (int g = 0; g < c.n_gates; ++g)
    if (is_channel(c.gates[g].op)) return true;
  return false;
}

int check_ckpt(const qs_circuit* c, const int32_t* ck, int32_t n_ck,
               const void* buf) {
  if (n_ck < 0) return QS_ERR_INVALID;
  if (n_ck == 0) return QS_OK;
  if (!ck || !buf) return QS_ERR_INVALID;
  for (int i = 0; i < n_ck; ++i) {
    // count 0 (the input state) only in front of a channel at gate 0
    const bool zero_ok = ck[i] == 0 && c->n_gates > 0 && is_channel(c->gates[0].op);
    if ((ck[i] <= 0 && !zero_ok) || ck[i] >= c->n_gates) return QS_ERR_INVALID;
    if (i > 0 && ck[i] <= ck[i - 1]) return QS_ERR_INVALID;
  }
  return QS_OK;
}

// ------------------------------------------------------------- launch shape
int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v && *v ? std::atoi(v) : dflt;
}

// ------------------------------------------------------------- tuning table
// Launch choices found by qs_autotune, keyed by (circuit, dtype, batch size
// class, flags). Overrides set while tuning take precedence.
struct TuneVal {
  int fwd_r = 0, adj_r = 0, m = 0;
  int fwd_s = 0, adj_s = 0;  // samples-per-block caps (0: the LDS-limited default)
  int fwd_h = 0, adj_h = 0;  // 1: stage one state component at a time in LDS
  int large = 0;             // large states: 0 tiled engine, 1 dense blocks on MFMA
};
std::mutex g_tmu;
std::mutex g_tune_run_mu;  // one tuning run at a time (overrides are global)
std::unordered_map<std::string, TuneVal> g_tune;
bool g_tune_loaded = false;
int g_force_fwd_r = 0, g_force_adj_r = 0, g_force_m = 0;
int g_force_fwd_s = 0, g_force_adj_s = 0;
int g_force_fwd_h = -1, g_force_adj_h = -1;  // -1: not forced
int g_force_large = -1;                       // -1: not forced
thread_local bool g_in_tune = false;  // calls made by the tuner itself

int batch_class(int64_t B) {
  int k = 0;
  while ((1ll << k) < B) ++k;
  return k;
}

std::string tune_key(const qs_circuit& c, int dtype, int64_t B, int flags) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
  };
  int32_t hdr[7] = {c.n_qubits, c.n_gates, c.n_params, c.n_features, dtype,
                    batch_class(B), flags};
  mix(hdr, sizeof(hdr));
  if (c.n_gates) mix(c.gates, sizeof(qs_gate) * c.n_gates);
  char buf[32];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return buf;
}

void load_tune_file_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("QS_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  // One line per tuned key: key fwd_r adj_r m [fwd_s adj_s [fwd_h adj_h [large]]].
  char line[256], key[64];
  while (std::fgets(line, sizeof(line), f)) {
    TuneVal v;
    const int k = std::sscanf(line, "%63s %d %d %d %d %d %d %d %d", key, &v.fwd_r, &v.adj_r,
                              &v.m, &v.fwd_s, &v.adj_s, &v.fwd_h, &v.adj_h, &v.large);
    if (k != 4 && k != 6 && k != 8 && k != 9) continue;
    if (k < 6) v.fwd_s = v.adj_s = 0;
    if (k < 8) v.fwd_h = v.adj_h = 0;
    if (k < 9) v.large = 0;
    g_tune[key] = v;
  }
  std::fclose(f);
}

bool tuned_lookup(const qs_circuit& c, int dtype, int64_t B, int flags, TuneVal* out) {
  std::lock_guard<std::mutex> lock(g_tmu);
  load_tune_file_locked();
  if (g_tune.empty()) return false;
  auto it = g_tune.find(tune_key(c, dtype, B, flags));
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

// Bytes of LDS the engine uses for a block of S samples.
// `block` threads hold S samples of T = block / S threads each; gradient sums
// take one slot per wave (shared parameters) and per wave of a sample
// (features); per-sample parameter sets take none.
// Sizes of a plan's LDS tables: fused-matrix slots and generator-frame
// slots. Without them lds_bytes bounds both by the single-qubit gates with
// shared angles, which holds for every plan of the circuit.
struct TableCounts {
  int n_fu = 0, n_gen = 0;
};

int64_t lds_bytes(int dtype, const qs_circuit& c, int S, int n_slots, int block,
                  bool ps, bool adjoint, const TableCounts* tc = nullptr, bool half = false) {
  const int64_t rs = dtype == QS_C64 ? 4 : 8;
  const int64_t waves = (block + 63) / 64;
  const int64_t T = block / (S > 0 ? S : 1);
  const int64_t wps = T > 64 ? T / 64 : 1;
  // Fused-matrix slots: one per block with shared angles, so at most one per
  // single-qubit gate whose angle (if any) is shared.
  int64_t n1q = 0;
  for (int g = 0; g < c.n_gates; ++g) {
    const qs_gate& x = c.gates[g];
    if (x.op > QS_OP_H) continue;
    const bool per_sample = is_rotation(x.op) &&
                            (ps ? (x.p_w >= 0 || x.p_b >= 0 || x.feat >= 0) : x.feat >= 0);
    n1q += per_sample ? 0 : 1;
  }
  int64_t b = (int64_t)S * ((half ? 1 : 2) * rs << c.n_qubits);  // state staging
  b += 2 * rs * c.n_gates;                          // shared angle table
  const int64_t n_fu = tc ? tc->n_fu : n1q, n_gen = tc ? tc->n_gen : n1q;
  b += 8 * rs * (n_fu + 1);                         // fused block matrices, identity
  if (adjoint) b += 3 * rs * n_gen;                 // generator frames
  b += 2 * rs * (int64_t)n_slots * S;               // per-sample angle table
  if (adjoint)                                      // gradient sums, features
    b += rs * (waves * (int64_t)grad_columns(c, ps).size() +
               (int64_t)S * wps * c.n_features + (int64_t)S * c.n_features);
  if (adjoint) b += 8 * (int64_t)S + 8;             // training step: squared residuals
  return (b + 15) & ~15ll;
}

// Choose amplitudes-per-thread 2^r and the block shape for one direction.
// Returns false when the fused engine cannot hold the circuit. Preference
// orders come from the register budgets of the instantiations: the forward
// holds one state per thread group, the adjoint two (psi and lam), so the
// adjoint prefers a narrower register tile.
TableCounts plan_counts(const qs_circuit& c, int r, bool ps, const int32_t* ck, int n_ck);

bool choose_shape(int dtype, const qs_circuit& c, int n_slots, int r_force,
                  bool adjoint, SvShape* out, bool ps = false,
                  const int32_t* ck = nullptr, int n_ck = 0, bool exact = true,
                  int s_cap = 0, bool half = false) {
  if (dtype != QS_C64) half = false;  // half staging exists for complex64 only
  const int n = c.n_qubits;
  if (n > kMaxQubitsFused) return false;
  static const int pref_c64_fwd[] = {5, 4, 3, 2, 1};
  static const int pref_c64_adj[] = {4, 5, 3, 2, 1};
  static const int pref_c128_fwd[] = {3, 4, 2, 1};
  static const int pref_c128_adj[] = {3, 2, 1, 4};
  const int* pref = dtype == QS_C64 ? (adjoint ? pref_c64_adj : pref_c64_fwd)
                                    : (adjoint ? pref_c128_adj : pref_c128_fwd);
  const int np = dtype == QS_C64 ? 5 : 4;
  int cand[6];
  int nc = 0;
  if (r_force > 0) cand[nc++] = r_force;
  for (int i = 0; i < np; ++i) cand[nc++] = pref[i];
  for (int i = 0; i < nc; ++i) {
    const int r = cand[i];
    if (r < 1 || r > n) continue;
    const int maxT = sv_max_threads(dtype, r, adjoint);
    if (maxT == 0) continue;
    const int t = n - r;
    const int T = 1 << t;
    if (T > maxT) continue;
    int block = T > 256 ? T : 256;
    if (block > maxT) block = maxT;
    int S = block / T;
    // LDS tables sized for the plan of this split (exact), or bounded for
    // any plan of the circuit.
    TableCounts counts;
    if (exact) counts = plan_counts(c, r, ps, ck, n_ck);
    const TableCounts* tc = exact ? &counts : nullptr;
    // Shrink the block until the LDS fits.
    while (S > 1 && lds_bytes(dtype, c, S, n_slots, S * T, ps, adjoint, tc, half) > kMaxLds) {
      S >>= 1;
    }
    // A smaller block can fit more workgroups per CU (an autotuner choice).
    while (s_cap > 0 && S > s_cap) S >>= 1;
    block = S * T;
    if (block < 64) {  // keep whole waves
      S = 64 / T;
      block = 64;
    }
    const int64_t lds = lds_bytes(dtype, c, S, n_slots, block, ps, adjoint, tc, half);
    if (lds > kMaxLds) continue;
    out->r = r;
    out->t = t;
    out->block_threads = block;
    out->samples_per_block = S;
    out->lds_bytes = lds;
    out->half = half ? 1 : 0;
    return true;
  }
  return false;
}

// ---------------------------------------------------------------- plan cache
struct Key {
  std::string bytes;
  bool operator==(const Key& o) const { return bytes == o.bytes; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char ch : k.bytes) { h ^= ch; h *= 1099511628211ull; }
    return (size_t)h;
  }
};
struct Entry {
  SvDevPlan dev;
  SvPlan host;
  int device;
};

std::mutex g_mu;
std::unordered_map<Key, Entry*, KeyHash> g_cache;
std::unordered_map<Key, qs_gate*, KeyHash> g_gate_cache;  // plain path

Key make_key(const qs_circuit& c, int r, bool ps, const int32_t* ck, int n_ck,
             int device, bool fixed_fold = false) {
  Key k;
  int32_t hdr[9] = {c.n_qubits, c.n_gates, c.n_params, c.n_features, r, ps, n_ck, device,
                    fixed_fold};
  k.bytes.append(reinterpret_cast<const char*>(hdr), sizeof(hdr));
  if (c.n_gates)
    k.bytes.append(reinterpret_cast<const char*>(c.gates), sizeof(qs_gate) * c.n_gates);
  if (n_ck) k.bytes.append(reinterpret_cast<const char*>(ck), sizeof(int32_t) * n_ck);
  return k;
}

// Table sizes of the host plan for (circuit, r, flags, checkpoints), planned
// once and cached (host only, so plan queries work without a device).
TableCounts plan_counts(const qs_circuit& c, int r, bool ps, const int32_t* ck, int n_ck) {
  static std::mutex mu;
  static std::unordered_map<Key, TableCounts, KeyHash> cache;
  Key key = make_key(c, r, ps, ck, n_ck, -1);
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const SvPlan P = plan_sv(c, r, ps, ck, n_ck);
  TableCounts t;
  t.n_fu = P.n_fu;
  t.n_gen = P.n_gen;
  std::lock_guard<std::mutex> lock(mu);
  cache.emplace(std::move(key), t);
  return t;
}

template <typename T>
bool upload(T** dst, const T* src, size_t n) {
  *dst = nullptr;
  const size_t bytes = sizeof(T) * (n ? n : 1);
  if (hipMalloc(reinterpret_cast<void**>(dst), bytes) != hipSuccess) return false;
  if (n && hipMemcpy(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice) != hipSuccess)
    return false;
  return true;
}

void free_dev(SvDevPlan& d) {
  (void)hipFree(d.seg_map);
  (void)hipFree(d.seg_lay);
  (void)hipFree(d.seg_begin);
  (void)hipFree(d.seg_ckpt);
  (void)hipFree(d.ops);
  (void)hipFree(d.gates);
  (void)hipFree(d.gate_slot);
  (void)hipFree(d.slot_gate);
  (void)hipFree(d.l1q);
  (void)hipFree(d.diag);
  (void)hipFree(d.blk_begin);
  (void)hipFree(d.blk_rec);
  (void)hipFree(d.blk_fu);
  (void)hipFree(d.blk_gen);
  (void)hipFree(d.grad_cols);
}

// GF(2) rank of bit vectors.
int gf2_rank(std::vector<uint32_t> v) {
  int r = 0;
  for (int bit = 15; bit >= 0; --bit) {
    size_t k = r;
    while (k < v.size() && !((v[k] >> bit) & 1)) ++k;
    if (k == v.size()) continue;
    std::swap(v[r], v[k]);
    for (size_t j = 0; j < v.size(); ++j)
      if (j != (size_t)r && ((v[j] >> bit) & 1)) v[j] ^= v[r];
    ++r;
  }
  return r;
}

// The LDS staging swizzle of a plan: slot(L) = L ^ (XOR of fold[b] over the
// set bits b >= 5 of L), each fold[b] a five-bit pattern, so the map is a
// bijection on a sample's slots and linear over GF(2). The LDS serves 128
// bytes per pass: 32 lanes of 4-byte slots, 16 of 8-byte, 8 of 16-byte; a
// pass is free of bank conflicts when the low p bits (p = 5, 4, 3) of its
// lanes' slots differ, i.e. when the swizzled masks of the layout's first p
// thread bits (with the salt vectors of samples sharing the pass) have full
// rank in those bits. The folds are chosen by coordinate descent from the
// fixed fold (bit b onto bit (b - 5) mod 5), maximising that rank summed
// over every layout the kernels stage under, weighted toward 8-byte slots.
struct StageSwizzle {
  uint32_t fold[16] = {};
  uint32_t apply(uint32_t L) const {
    uint32_t x = L;
    for (int b = 5; b < 16; ++b)
      if ((L >> b) & 1) x ^= fold[b];
    return x;
  }
};

// The thread-bit masks of every staged layout: each segment's read and write
// layouts and the HBM order (thread bit i on logical bit i).
std::vector<std::vector<uint32_t>> staged_thread_masks(const SvPlan& P) {
  std::vector<std::vector<uint32_t>> lays;
  std::vector<uint32_t> id;
  for (int i = 0; i < P.t; ++i) id.push_back(1u << i);
  lays.push_back(id);
  for (int s = 0; s < P.nseg(); ++s)
    for (int h = 0; h < 2; ++h) {
      std::vector<uint32_t> v;
      for (int i = 0; i < P.t; ++i)
        v.push_back(P.seg_lay[(size_t)s * kLayWords + h * kMapStride + P.r + i]);
      lays.push_back(v);
    }
  return lays;
}

StageSwizzle stage_swizzle(const SvPlan& P, bool fixed) {
  StageSwizzle sw;
  for (int b = 5; b < 15; ++b) sw.fold[b] = 1u << ((b - 5) % 5);
  if (P.n <= 5 || fixed) return sw;
  const auto lays = staged_thread_masks(P);
  const int t = P.t;
  auto score = [&](const StageSwizzle& z) {
    long sc = 0;
    for (const auto& l : lays)
      for (int p = 3; p <= 5; ++p) {
        const uint32_t mask = (1u << p) - 1;
        std::vector<uint32_t> v;
        for (int i = 0; i < t && i < p; ++i) v.push_back(z.apply(l[i]) & mask);
        for (int j = 0; t + j < p; ++j) v.push_back((1u << (t + j)) & mask);  // default salts
        sc += (p == 4 ? 4 : p == 5 ? 2 : 1) * gf2_rank(v);
      }
    return sc;
  };
  long best = score(sw);
  for (int sweep = 0; sweep < 3; ++sweep) {
    bool moved = false;
    for (int b = 5; b < P.n; ++b) {
      const uint32_t keep = sw.fold[b];
      uint32_t arg = keep;
      for (uint32_t c = 0; c < 32; ++c) {
        sw.fold[b] = c;
        const long sc = score(sw);
        if (sc > best) {
          best = sc;
          arg = c;
        }
      }
      sw.fold[b] = arg;
      moved |= arg != keep;
    }
    if (!moved) break;
  }
  return sw;
}

// Salts of one-component staging (4-byte slots, 32 lanes per LDS pass). The
// salt of the sample at position s within its wave is the XOR of basis
// vectors for the set bits of s. The vectors of the samples sharing a pass
// are picked greedily to maximise the rank of the swizzled thread masks and
// salts in the slots' low five bits, summed over the staged layouts (then
// the six-bit rank of the whole wave breaks ties; ties keep the default
// vector). `lays` holds the swizzled thread masks.
uint64_t half_salt_basis(const SvPlan& P, const std::vector<std::vector<uint32_t>>& lays) {
  const int t = P.t;
  if (t >= 6 || P.n > 16) return 0;
  const uint32_t N = 1u << P.n;
  std::vector<uint32_t> basis;
  uint64_t packed = 0;
  for (int k = 0; k < 6 - t; ++k) {
    const uint32_t dflt = (1u << (t + k)) & 63u & (N - 1);
    uint32_t best = dflt;
    long best_score = -1;
    for (uint32_t c = 0; c < 64 && c < N; ++c) {
      long sc = 0;
      for (const auto& l : lays) {
        std::vector<uint32_t> v5, v6;
        for (int i = 0; i < t; ++i) {
          if (i < 5) v5.push_back(l[i] & 31u);
          v6.push_back(l[i] & 63u);
        }
        for (size_t j = 0; j < basis.size(); ++j) {
          if (t + (int)j < 5) v5.push_back(basis[j] & 31u);
          v6.push_back(basis[j]);
        }
        if (t + k < 5) v5.push_back(c & 31u);
        v6.push_back(c);
        sc += 8 * gf2_rank(v5) + gf2_rank(v6);
      }
      if (sc > best_score || (sc == best_score && c == dflt)) {
        best_score = sc;
        best = c;
      }
    }
    basis.push_back(best);
    packed |= (uint64_t)best << (6 * k);
  }
  return packed;
}

// Plans on the host and uploads once per (circuit, r, flags, device). The
// upload is synchronous, so the first call for a circuit must not be inside
// a stream capture; later calls only look the plan up.
Entry* get_plan(const qs_circuit& c, int r, bool ps, const int32_t* ck, int n_ck,
                int* rc, bool fixed_fold = false) {
  int device = 0;
  (void)hipGetDevice(&device);
  Key key = make_key(c, r, ps, ck, n_ck, device, fixed_fold);
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) return it->second;
  if (const int up = plan_upload_status(); up != QS_OK) {
    *rc = up;
    return nullptr;
  }
  Entry* e = new Entry();
  e->device = device;
  e->host = plan_sv(c, r, ps, ck, n_ck);
  const SvPlan& P = e->host;
  bool in_order = true;  // the kernels read op o's record as record o
  for (size_t o = 0; o < P.ops.size(); ++o) in_order &= P.ops[o].gate == (int32_t)o;
  if (!P.layered || !in_order) {  // the engine runs layer ops only
    delete e;
    *rc = QS_ERR_UNSUPPORTED;
    return nullptr;
  }
  SvDevPlan& d = e->dev;
  d.n = P.n;
  d.r = P.r;
  d.t = P.t;
  d.nseg = P.nseg();
  d.n_gates = P.n_gates;
  d.n_slots = (int)P.slot_gate.size();
  d.n_params = c.n_params;
  d.n_features = c.n_features;
  d.n_remaps = P.n_remaps;
  d.n_ops = (int)P.ops.size();
  d.n_blocks = P.n_blocks();
  d.n_fu = P.n_fu;
  d.n_gen = P.n_gen;
  d.n_acc = (int)P.grad_cols.size();
  // Device layouts: every mask swizzled, plus the HBM-order row.
  const StageSwizzle sw = stage_swizzle(P, fixed_fold);
  std::vector<uint16_t> lay_dev((size_t)(d.nseg + 1) * kLayWords, 0);
  for (size_t i = 0; i < P.seg_lay.size(); ++i) lay_dev[i] = (uint16_t)sw.apply(P.seg_lay[i]);
  uint16_t* hrow = &lay_dev[(size_t)d.nseg * kLayWords];
  for (int j = 0; j < P.r; ++j) hrow[j] = (uint16_t)sw.apply(1u << (P.t + j));
  for (int i = 0; i < P.t; ++i) hrow[P.r + i] = (uint16_t)sw.apply(1u << i);
  {
    auto lays = staged_thread_masks(P);
    for (auto& l : lays)
      for (auto& m : l) m = sw.apply(m);
    d.salt_half = half_salt_basis(P, lays);
  }
  // (the RY-then-RZ pass also reads block b's records at 2 b)
  d.ryrz = d.n_blocks > 0 && P.blk_begin[0] == 0;
  for (int b = 0; b < d.n_blocks && d.ryrz; ++b)
    d.ryrz = P.blk_begin[b + 1] - P.blk_begin[b] == 2 &&
             c.gates[P.blk_gates[P.blk_begin[b]]].op == QS_OP_RY &&
             c.gates[P.blk_gates[P.blk_begin[b] + 1]].op == QS_OP_RZ;
  std::vector<BGate> rec(P.blk_gates.size());
  for (size_t i = 0; i < rec.size(); ++i) {
    const int g = P.blk_gates[i];
    const qs_gate& x = c.gates[g];
    BGate& b = rec[i];
    b.g = g;
    b.kind_slot = x.op | ((P.gate_slot[g] + 1) << 4);
    b.feat = x.feat;
    b.p_w = x.p_w;
    b.p_b = x.p_b;
    b.col_w = P.gate_cols.empty() ? -1 : P.gate_cols[2 * (size_t)g];
    b.col_b = P.gate_cols.empty() ? -1 : P.gate_cols[2 * (size_t)g + 1];
    b.scale = x.scale;
  }
  bool okk = upload(&d.seg_map, P.seg_map.data(), P.seg_map.size()) &&
             upload(&d.seg_lay, lay_dev.data(), lay_dev.size()) &&
             upload(&d.seg_begin, P.seg_begin.data(), P.seg_begin.size()) &&
             upload(&d.seg_ckpt, P.seg_ckpt.data(), P.seg_ckpt.size()) &&
             upload(&d.ops, P.ops.data(), P.ops.size()) &&
             upload(&d.gates, c.gates, (size_t)c.n_gates) &&
             upload(&d.gate_slot, P.gate_slot.data(), P.gate_slot.size()) &&
             upload(&d.slot_gate, P.slot_gate.data(), P.slot_gate.size()) &&
             upload(&d.l1q, P.l1q.data(), P.l1q.size()) &&
             upload(&d.diag, P.diag.data(), P.diag.size()) &&
             upload(&d.blk_begin, P.blk_begin.data(), P.blk_begin.size()) &&
             upload(&d.blk_rec, rec.data(), rec.size()) &&
             upload(&d.blk_fu, P.blk_fu.data(), P.blk_fu.size()) &&
             upload(&d.blk_gen, P.blk_gen.data(), P.blk_gen.size()) &&
             upload(&d.grad_cols, P.grad_cols.data(), P.grad_cols.size());
  if (!okk) {
    free_dev(d);
    delete e;
    *rc = QS_ERR_NOMEM;
    return nullptr;
  }
  g_cache.emplace(std::move(key), e);
  return e;
}

// The plan's LDS tables fit the launch's dynamic LDS (the shape was sized
// from the same plan; this guards the kernel's LDS carve-up).
bool tables_fit(const Entry& e, int dtype, const qs_circuit& c, const SvShape& shape,
                bool ps, bool adjoint) {
  TableCounts tc;
  tc.n_fu = e.host.n_fu;
  tc.n_gen = e.host.n_gen;
  return lds_bytes(dtype, c, shape.samples_per_block, (int)e.host.slot_gate.size(),
                   shape.block_threads, ps, adjoint, &tc, shape.half != 0) <= shape.lds_bytes;
}

qs_gate* get_dev_gates(const qs_circuit& c, int* rc) {
  int device = 0;
  (void)hipGetDevice(&device);
  Key key = make_key(c, -1, false, nullptr, 0, device);
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_gate_cache.find(key);
  if (it != g_gate_cache.end()) return it->second;
  if (const int up = plan_upload_status(); up != QS_OK) {
    *rc = up;
    return nullptr;
  }
  qs_gate* d = nullptr;
  if (!upload(&d, c.gates, (size_t)c.n_gates)) {
    *rc = QS_ERR_NOMEM;
    return nullptr;
  }
  g_gate_cache.emplace(std::move(key), d);
  return d;
}

// ------------------------------------------------------------ tiled plans
// One engine plan per epoch and direction, plus the epoch's qubit maps.
struct TiledEpochDev {
  Entry* fwd = nullptr;
  Entry* adj = nullptr;
  SvShape fshape, ashape;
  uint8_t* tile_q = nullptr;
  uint8_t* outer_q = nullptr;
  int ckpt_after = -1;
  std::vector<qs_gate> gates;  // the epoch's local gate list (kept alive)
};
struct TiledEntry {
  int m = 0;
  std::vector<TiledEpochDev> epochs;
};
std::unordered_map<Key, TiledEntry*, KeyHash> g_tiled;

int tile_qubits(int dtype, int n, int m_pref = 0) {
  // The tuner's trial choice first, then the environment override.
  int m = g_force_m;
  if (m == 0) m = env_int("QS_TILE_QUBITS", 0);
  if (m == 0) m = m_pref;
  if (m == 0) m = dtype == QS_C64 ? 13 : 12;
  if (m > n) m = n;
  if (m > kMaxQubitsFused) m = kMaxQubitsFused;
  if (m < 3) m = n < 3 ? n : 3;
  return m;
}

// Tile size and the register split of the epochs' forward and adjoint
// launches (0: the defaults).
struct TileCfg {
  int m_pref = 0, fwd_r = 0, adj_r = 0;
};
TileCfg tile_cfg(bool tuned, const TuneVal& tv) {
  TileCfg t;
  t.m_pref = tuned ? tv.m : 0;
  t.fwd_r = g_force_fwd_r;
  if (t.fwd_r == 0) t.fwd_r = env_int("QS_TILE_FWD_LOG2_REGS", 0);
  if (t.fwd_r == 0 && tuned) t.fwd_r = tv.fwd_r;
  t.adj_r = g_force_adj_r;
  if (t.adj_r == 0) t.adj_r = env_int("QS_TILE_ADJ_LOG2_REGS", 0);
  if (t.adj_r == 0 && tuned) t.adj_r = tv.adj_r;
  return t;
}

TiledEntry* get_tiled(const qs_circuit& c, int dtype, bool ps, const int32_t* ck,
                      int n_ck, const TileCfg& tc, int* rc) {
  int device = 0;
  (void)hipGetDevice(&device);
  const int m = tile_qubits(dtype, c.n_qubits, tc.m_pref);
  Key key = make_key(c, -100 - m - 32 * dtype - 1024 * tc.fwd_r - 8192 * tc.adj_r, ps, ck,
                     n_ck, device);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_tiled.find(key);
    if (it != g_tiled.end()) return it->second;
  }
  if (const int up = plan_upload_status(); up != QS_OK) {
    *rc = up;
    return nullptr;
  }
  const int low_keep = m >= 6 ? 4 : (m >= 4 ? m - 2 : 0);
  std::vector<TiledEpoch> eps = plan_tiled(c, m, low_keep, ck, n_ck);
  TiledEntry* te = new TiledEntry();
  auto drop = [&te]() -> TiledEntry* {  // a failed plan: release what was uploaded
    for (auto& d : te->epochs) {
      (void)hipFree(d.tile_q);
      (void)hipFree(d.outer_q);
    }
    delete te;
    return nullptr;
  };
  te->m = m;
  te->epochs.resize(eps.size());
  for (size_t i = 0; i < eps.size(); ++i) {
    TiledEpochDev& d = te->epochs[i];
    d.gates = eps[i].gates;
    d.ckpt_after = eps[i].ckpt_after;
    qs_circuit sub{(int32_t)eps[i].L.size(), (int32_t)d.gates.size(), c.n_params,
                   c.n_features, d.gates.empty() ? nullptr : d.gates.data()};
    const int slots = [&] {
      int k = 0;
      for (const qs_gate& x : d.gates)
        if (is_rotation(x.op) && (ps ? (x.p_w >= 0 || x.p_b >= 0 || x.feat >= 0) : x.feat >= 0)) ++k;
      return k;
    }();
    if (!choose_shape(dtype, sub, slots, tc.fwd_r, false, &d.fshape, ps) ||
        !choose_shape(dtype, sub, slots, tc.adj_r, true, &d.ashape, ps)) {
      *rc = QS_ERR_UNSUPPORTED;
      return drop();
    }
    d.fwd = get_plan(sub, d.fshape.r, ps, nullptr, 0, rc);
    d.adj = get_plan(sub, d.ashape.r, ps, nullptr, 0, rc);
    if (!d.fwd || !d.adj) return drop();
    std::vector<uint8_t> tq(eps[i].L.begin(), eps[i].L.end()), oq;
    std::vector<char> in(c.n_qubits, 0);
    for (int q : eps[i].L) in[q] = 1;
    for (int q = 0; q < c.n_qubits; ++q)
      if (!in[q]) oq.push_back((uint8_t)q);
    if (!upload(&d.tile_q, tq.data(), tq.size()) || !upload(&d.outer_q, oq.data(), oq.size())) {
      *rc = QS_ERR_NOMEM;
      return drop();
    }
  }
  std::lock_guard<std::mutex> lock(g_mu);
  auto ins = g_tiled.emplace(std::move(key), te);
  if (!ins.second) {  // planned meanwhile by another thread: keep that one
    for (auto& d : te->epochs) {
      (void)hipFree(d.tile_q);
      (void)hipFree(d.outer_q);
    }
    delete te;
    return ins.first->second;
  }
  return te;
}

// -------------------------------------------------------- dense-block plans
// Large states on MFMA: complex64, angles shared by the whole batch (no
// per-sample parameters, no rotation reading a feature), 2^(n-5) >= 32
// columns per state.
constexpr int kDbK = 5;
constexpr int kDbGrid = 512;  // persistent workgroups (two per CU of 256)

bool db_supported(const qs_circuit& c, int dtype, bool ps) {
  if (dtype != QS_C64 || ps || c.n_qubits < kDbK + 5 || has_channels(c)) return false;
  for (int g = 0; g < c.n_gates; ++g)
    if (is_rotation(c.gates[g].op) && c.gates[g].feat >= 0) return false;
  return true;
}

struct DbEntry {
  std::vector<DenseBlock> blocks;
  std::vector<int32_t> h_blk_q;  // [n_blocks][kDbGeoWords] block geometry
  int32_t* blk_begin = nullptr;
  DbGate* gates = nullptr;
  int32_t* blk_q = nullptr;
  int32_t* p_begin = nullptr;    // [n_params + 1] rotations reading each parameter
  int32_t* p_gate = nullptr;
  float* p_scale = nullptr;
};
std::unordered_map<Key, DbEntry*, KeyHash> g_db;

void free_db(DbEntry* e) {
  (void)hipFree(e->blk_begin);
  (void)hipFree(e->gates);
  (void)hipFree(e->blk_q);
  (void)hipFree(e->p_begin);
  (void)hipFree(e->p_gate);
  (void)hipFree(e->p_scale);
  delete e;
}

// The host side of a dense-block plan (no device memory): blocks, device
// records, per-parameter rotation lists. False when the blocks do not cover
// every gate once.
bool db_host_plan(const qs_circuit& c, const int32_t* ck, int n_ck, DbEntry& e,
                  std::vector<int32_t>& begin, std::vector<DbGate>& recs,
                  std::vector<int32_t>& pb, std::vector<int32_t>& pg,
                  std::vector<float>& psc) {
  e.blocks = plan_blocks(c, kDbK, ck, n_ck);
  std::vector<char> seen(c.n_gates, 0);
  begin.assign(1, 0);
  e.h_blk_q.clear();
  for (const DenseBlock& b : e.blocks) {
    if ((int)b.qubits.size() != kDbK) return false;
    std::vector<int> local(c.n_qubits, -1);
    for (int i = 0; i < kDbK; ++i) local[b.qubits[i]] = i;
    for (int g : b.gates) {
      if (g < 0 || g >= c.n_gates || seen[g]) return false;
      seen[g] = 1;
      const qs_gate& x = c.gates[g];
      DbGate r{};
      r.op = x.op;
      r.q0 = local[x.q0];
      r.q1 = x.q1 >= 0 ? local[x.q1] : -1;
      if (r.q0 < 0 || (x.q1 >= 0 && r.q1 < 0)) return false;
      r.p_w = x.p_w;
      r.p_b = x.p_b;
      r.scale = x.scale;
      r.g = g;
      recs.push_back(r);
    }
    begin.push_back((int32_t)recs.size());
    // Geometry of the block's tiles (see DbGeo): the block qubits, the 10
    // address bits of a 32-column tile (block qubits and the 5 lowest other
    // positions, ascending) and the rank of each block and column bit there.
    int32_t geo[kDbGeoWords] = {};
    std::vector<int> pos(b.qubits.begin(), b.qubits.end()), low;
    for (int q = 0; q < c.n_qubits && (int)low.size() < 5; ++q)
      if (std::find(b.qubits.begin(), b.qubits.end(), q) == b.qubits.end()) low.push_back(q);
    if ((int)low.size() < 5) return false;
    pos.insert(pos.end(), low.begin(), low.end());
    std::sort(pos.begin(), pos.end());
    auto rank = [&](int q) { return (int)(std::find(pos.begin(), pos.end(), q) - pos.begin()); };
    for (int i = 0; i < kDbK; ++i) {
      geo[i] = b.qubits[i];
      geo[15 + i] = rank(b.qubits[i]);
      geo[20 + i] = rank(low[i]);
    }
    for (int i = 0; i < 10; ++i) geo[5 + i] = pos[i];
    e.h_blk_q.insert(e.h_blk_q.end(), geo, geo + kDbGeoWords);
  }
  for (char v : seen)
    if (!v) return false;
  // theta = scale (w + bias): dtheta/dw = dtheta/dbias = scale
  std::vector<std::vector<std::pair<int, float>>> lists(c.n_params);
  for (int g = 0; g < c.n_gates; ++g) {
    const qs_gate& x = c.gates[g];
    if (!is_rotation(x.op)) continue;
    if (x.p_w >= 0) lists[x.p_w].push_back({g, x.scale});
    if (x.p_b >= 0) lists[x.p_b].push_back({g, x.scale});
  }
  pb.assign(1, 0);
  for (int p = 0; p < c.n_params; ++p) {
    for (auto& t : lists[p]) {
      pg.push_back(t.first);
      psc.push_back(t.second);
    }
    pb.push_back((int32_t)pg.size());
  }
  return true;
}

DbEntry* get_db(const qs_circuit& c, const int32_t* ck, int n_ck, int* rc) {
  int device = 0;
  (void)hipGetDevice(&device);
  Key key = make_key(c, -5000 - kDbK, false, ck, n_ck, device);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_db.find(key);
    if (it != g_db.end()) return it->second;
  }
  if (const int up = plan_upload_status(); up != QS_OK) {
    *rc = up;
    return nullptr;
  }
  DbEntry* e = new DbEntry();
  std::vector<int32_t> begin, pb, pg;
  std::vector<DbGate> recs;
  std::vector<float> psc;
  if (!db_host_plan(c, ck, n_ck, *e, begin, recs, pb, pg, psc)) {
    delete e;
    *rc = QS_ERR_UNSUPPORTED;
    return nullptr;
  }
  if (!upload(&e->blk_begin, begin.data(), begin.size()) ||
      !upload(&e->gates, recs.data(), recs.size()) ||
      !upload(&e->blk_q, e->h_blk_q.data(), e->h_blk_q.size()) ||
      !upload(&e->p_begin, pb.data(), pb.size()) || !upload(&e->p_gate, pg.data(), pg.size()) ||
      !upload(&e->p_scale, psc.data(), psc.size())) {
    free_db(e);
    *rc = QS_ERR_NOMEM;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  auto ins = g_db.emplace(std::move(key), e);
  if (!ins.second) {  // planned meanwhile by another thread: keep that one
    free_db(e);
    return ins.first->second;
  }
  return e;
}

// Adjoint workspace of the dense-block path: psi and lam copies, one pass's
// per-workgroup rho partial sums, every block's rho (FP64) and the per-gate
// gradients (FP64), each 256-byte aligned.
struct DbWs {
  size_t psi = 0, lam = 0, part = 0, rho = 0, gth = 0, total = 0;
};
DbWs db_ws_layout(const qs_circuit& c, int64_t B, int n_blocks) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  DbWs w;
  const size_t st = al(((size_t)B << c.n_qubits) * 8);
  w.psi = 0;
  w.lam = st;
  w.part = 2 * st;
  w.rho = w.part + al((size_t)kDbGrid * 2 * 32 * 32 * sizeof(float));
  w.gth = w.rho + al((size_t)n_blocks * 2 * 32 * 32 * sizeof(double));
  w.total = w.gth + al((size_t)std::max(c.n_gates, 1) * sizeof(double));
  return w;
}
// Sized for as many blocks as gates (every block holds a gate), so it covers
// every checkpoint placement.
size_t db_ws_bytes(const qs_circuit& c, int64_t B) {
  return db_ws_layout(c, B, std::max(c.n_gates, 1)).total;
}

// Host-only view of the tiled plan: tile size, epochs, largest adjoint grid
// and a bound on the per-block gradient-sum array (blocks x gradient columns)
// that holds for every checkpoint placement: checkpoints move the epoch
// boundaries, so the bound takes the largest possible grid (one tile-sample
// per workgroup) times the gradient columns of the whole circuit, which no
// epoch can exceed.
// max_part_plan is the largest array of the plan for the given checkpoints.
struct TiledHostInfo {
  int m = 0, n_epochs = 0;
  int64_t max_grid = 1, max_part = 1, max_part_plan = 0;
  bool ok = true;
};
TiledHostInfo tiled_host_info(const qs_circuit& c, int dtype, int64_t B, bool ps,
                              const TileCfg& tc, const int32_t* ck = nullptr,
                              int n_ck = 0) {
  TiledHostInfo h;
  h.m = tile_qubits(dtype, c.n_qubits, tc.m_pref);
  const int low_keep = h.m >= 6 ? 4 : (h.m >= 4 ? h.m - 2 : 0);
  std::vector<TiledEpoch> eps = plan_tiled(c, h.m, low_keep, ck, n_ck);
  h.n_epochs = (int)eps.size();
  const int64_t samples = B << (c.n_qubits - h.m);
  for (const TiledEpoch& e : eps) {
    qs_circuit sub{(int32_t)e.L.size(), (int32_t)e.gates.size(), c.n_params,
                   c.n_features, e.gates.empty() ? nullptr : e.gates.data()};
    int slots = 0;
    for (const qs_gate& x : e.gates)
      if (is_rotation(x.op) && (ps ? (x.p_w >= 0 || x.p_b >= 0 || x.feat >= 0) : x.feat >= 0))
        ++slots;
    SvShape a;
    if (!choose_shape(dtype, sub, slots, tc.adj_r, true, &a, ps)) { h.ok = false; continue; }
    const int64_t g = (samples + a.samples_per_block - 1) / a.samples_per_block;
    if (g > h.max_grid) h.max_grid = g;
    const int64_t cols = (int64_t)grad_columns(sub, ps).size();
    if (g * cols > h.max_part_plan) h.max_part_plan = g * cols;
  }
  h.max_part = std::max<int64_t>(1, samples * (int64_t)grad_columns(c, ps).size());
  return h;
}

size_t tiled_ws_bytes(const qs_circuit& c, int dtype, int64_t B, bool ps,
                      const TileCfg& tc, int* rc) {
  TiledHostInfo h = tiled_host_info(c, dtype, B, ps, tc);
  if (!h.ok) {
    *rc = QS_ERR_UNSUPPORTED;
    return 0;
  }
  const size_t cs = dtype == QS_C64 ? 8 : 16;
  const size_t acc = dtype == QS_C64 ? 4 : 8;
  const size_t st = ((size_t)B << c.n_qubits) * cs;
  size_t part = ps ? 0 : (size_t)h.max_part * acc;
  return 2 * st + ((part + 255) & ~(size_t)255);
}

// Path and launch shape of one direction: the tuner's trial first, then the
// environment overrides, then the tuned choice for this circuit (tv).
int pick_path(const qs_circuit& c, int dtype, int flags, SvShape* shape,
              int n_slots, bool adjoint, const TuneVal* tv = nullptr,
              const int32_t* ck = nullptr, int n_ck = 0) {
  int path = flags & QS_PATH_MASK;
  int rf = adjoint ? g_force_adj_r : g_force_fwd_r;
  if (rf == 0) rf = env_int(adjoint ? "QS_ADJ_LOG2_REGS" : "QS_FWD_LOG2_REGS", 0);
  if (rf == 0 && tv) rf = adjoint ? tv->adj_r : tv->fwd_r;
  int sc = adjoint ? g_force_adj_s : g_force_fwd_s;
  if (sc == 0)
    sc = env_int(adjoint ? "QS_ADJ_SAMPLES_PER_BLOCK" : "QS_FWD_SAMPLES_PER_BLOCK", 0);
  if (sc == 0 && tv) sc = adjoint ? tv->adj_s : tv->fwd_s;
  int hf = adjoint ? g_force_adj_h : g_force_fwd_h;
  if (hf < 0) hf = env_int(adjoint ? "QS_ADJ_HALF_STAGING" : "QS_FWD_HALF_STAGING", -1);
  if (hf < 0) hf = tv ? (adjoint ? tv->adj_h : tv->fwd_h) : 0;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  if (path == QS_PATH_AUTO) {
    if (choose_shape(dtype, c, n_slots, rf, adjoint, shape, ps, ck, n_ck, true, sc, hf > 0))
      path = QS_PATH_FUSED;
    else  // states too large for one workgroup: LDS tiles, else gate by gate
      path = c.n_qubits > kMaxQubitsFused || tile_qubits(dtype, c.n_qubits) < c.n_qubits
                 ? QS_PATH_HBM
                 : QS_PATH_PLAIN;
    if (path == QS_PATH_HBM) {
      // large states: the tiled engine, or dense blocks on MFMA where the
      // tuner found them faster (the tuner's trial, then the environment)
      int large = g_force_large;
      if (large < 0) large = env_int("QS_LARGE_PATH_MFMA", -1);
      if (large < 0) large = tv ? tv->large : 0;
      if (large == 1 && db_supported(c, dtype, ps)) path = QS_PATH_MFMA;
    }
  } else if (path == QS_PATH_FUSED) {
    if (!choose_shape(dtype, c, n_slots, rf, adjoint, shape, ps, ck, n_ck, true, sc, hf > 0))
      return QS_ERR_UNSUPPORTED;
  } else if (path == QS_PATH_MFMA) {
    if (!db_supported(c, dtype, ps)) return QS_ERR_UNSUPPORTED;
  } else if (path != QS_PATH_PLAIN && path != QS_PATH_HBM) {
    return QS_ERR_INVALID;
  }
  return path;
}

int count_slots(const qs_circuit& c, bool ps) {
  int n = 0;
  for (int g = 0; g < c.n_gates; ++g) {
    const qs_gate& x = c.gates[g];
    if (!is_rotation(x.op)) continue;
    if (ps ? (x.p_w >= 0 || x.p_b >= 0 || x.feat >= 0) : x.feat >= 0) ++n;
  }
  return n;
}

int64_t grid_of(const SvShape& s, int64_t B) {
  return (B + s.samples_per_block - 1) / s.samples_per_block;
}

// Partial-sum workspace of the fused adjoint with register split s.r. The
// grid is counted with the LDS tables bounded (fewer samples per block than
// any plan of the circuit gets, with or without checkpoints), so the size
// covers every launch of that split.
// Workgroups of the fused adjoint with register split s.r, bounded over the
// plans of the circuit (see fused_ws_bytes).
int64_t fused_rows_bound(const qs_circuit& c, int dtype, const SvShape& s, int64_t B, bool ps) {
  SvShape wide = s;
  if (!choose_shape(dtype, c, count_slots(c, ps), s.r, true, &wide, ps, nullptr, 0, false) ||
      wide.r != s.r)
    wide = s;
  const int64_t S = std::min(wide.samples_per_block, s.samples_per_block);
  return (B + S - 1) / S;
}

size_t fused_ws_bytes(const qs_circuit& c, int dtype, const SvShape& s, int64_t B,
                      bool ps) {
  if (ps) return 0;
  const size_t acc = dtype == QS_C64 ? sizeof(float) : sizeof(double);
  const size_t cols = std::max<size_t>(grad_columns(c, false).size(), 1);
  return (size_t)fused_rows_bound(c, dtype, s, B, ps) * cols * acc;
}

bool tuned_for_call(const qs_circuit& c, int dtype, int64_t B, int flags, void* stream,
                    TuneVal* out);

// ------------------------------------- circuits with mid-circuit channels
// A circuit with RESET / MEASURE gates runs as unitary runs between them:
// each run through the register/LDS engine, each channel as its own kernel
// (one trajectory per sample). The state in front of every channel must be
// stored as a checkpoint (a checkpoint at the channel's gate index): the
// adjoint cannot un-apply a channel, it restarts from that state.
struct Run {
  int b, e, ch;  // gates [b, e), then channel gate ch (-1 after the last run)
};
std::vector<Run> unitary_runs(const qs_circuit& c) {
  std::vector<Run> runs;
  int b = 0;
  for (int g = 0; g < c.n_gates; ++g)
    if (is_channel(c.gates[g].op)) {
      runs.push_back({b, g, g});
      b = g + 1;
    }
  runs.push_back({b, c.n_gates, -1});
  return runs;
}
int slot_of(const int32_t* ck, int n_ck, int count) {
  for (int i = 0; i < n_ck; ++i)
    if (ck[i] == count) return i;
  return -1;
}
qs_circuit run_circuit_of(const qs_circuit& c, const Run& r) {
  return qs_circuit{c.n_qubits, r.e - r.b, c.n_params, c.n_features,
                    r.e > r.b ? c.gates + r.b : nullptr};
}
// Checkpoints strictly inside run r, as gate counts of the run, and the slot
// of the first of them.
void run_ckpts(const int32_t* ck, int n_ck, const Run& r, std::vector<int32_t>& rel,
               int* first) {
  rel.clear();
  *first = 0;
  for (int i = 0; i < n_ck; ++i)
    if (ck[i] > r.b && ck[i] < r.e) {
      if (rel.empty()) *first = i;
      rel.push_back(ck[i] - r.b);
    }
}
// Register/LDS engine only (the adjoint needs each run's cotangent at its
// start), no inverse, a checkpoint at every channel.
int channels_check(const qs_circuit& c, int flags, const int32_t* ck, int n_ck) {
  const int path = flags & QS_PATH_MASK;
  if (path != QS_PATH_AUTO && path != QS_PATH_FUSED) return QS_ERR_UNSUPPORTED;
  for (const Run& r : unitary_runs(c))
    if (r.ch >= 0 && slot_of(ck, n_ck, r.ch) < 0) return QS_ERR_INVALID;
  return QS_OK;
}
// Adjoint workspace: psi and lam of the whole batch, then the largest run's
// partial-sum area.
size_t channel_ws_bytes(const qs_circuit& c, int dtype, int64_t B, int flags) {
  const int path = flags & QS_PATH_MASK;
  if (path != QS_PATH_AUTO && path != QS_PATH_FUSED) return 0;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  size_t part = 0;
  for (const Run& r : unitary_runs(c)) {
    if (r.e == r.b) continue;
    const qs_circuit sub = run_circuit_of(c, r);
    SvShape sh;
    if (pick_path(sub, dtype, (flags & ~QS_PATH_MASK) | QS_PATH_FUSED, &sh,
                  count_slots(sub, ps), true) != QS_PATH_FUSED)
      return 0;
    part = std::max(part, fused_ws_bytes(sub, dtype, sh, B, ps));
  }
  const size_t st = (((size_t)B << c.n_qubits) * (dtype == QS_C64 ? 8 : 16) + 255) & ~(size_t)255;
  return 2 * st + part;
}

int adjoint_channels(const qs_circuit& c, int dtype, int64_t B, const void* params,
                     const void* feats, const void* state, const double* dexpz,
                     const void* dstate, double* grad_params, double* grad_feats,
                     const int32_t* ck, int n_ck, const void* ckpt, void* ws, int flags,
                     void* stream) {
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  const int sub_flags = (flags & ~QS_PATH_MASK) | QS_PATH_FUSED;
  const int64_t per = B << c.n_qubits;
  const size_t cs = dtype == QS_C64 ? 8 : 16;
  const size_t st = (per * cs + 255) & ~(size_t)255;
  char* psi_w = static_cast<char*>(ws);
  char* lam_w = psi_w + st;
  void* part = lam_w + st;
  const char* cb = static_cast<const char*>(ckpt);
  int rc = launch_copy_state(dtype, state, psi_w, per, stream);
  if (rc != QS_OK) return rc;
  rc = dstate ? launch_copy_state(dtype, dstate, lam_w, per, stream)
              : launch_obs_cot(dtype, c.n_qubits, B, dexpz, psi_w, lam_w, stream);
  if (rc != QS_OK) return rc;
  if (c.n_params && (rc = launch_fill_f64(grad_params, ps ? B * c.n_params : c.n_params,
                                          stream)) != QS_OK)
    return rc;
  if (c.n_features && grad_feats &&
      (rc = launch_fill_f64(grad_feats, B * c.n_features, stream)) != QS_OK)
    return rc;
  const std::vector<Run> runs = unitary_runs(c);
  std::vector<int32_t> rel;
  for (int k = (int)runs.size() - 1; k >= 0; --k) {
    const Run& r = runs[k];
    if (r.e > r.b) {  // the run backwards, psi and lam in place at its start
      const qs_circuit sub = run_circuit_of(c, r);
      int first = 0;
      run_ckpts(ck, n_ck, r, rel, &first);
      const int32_t* rk = rel.empty() ? nullptr : rel.data();
      TuneVal tv;
      const bool tuned = tuned_for_call(sub, dtype, B, sub_flags, stream, &tv);
      SvShape shape;
      if (pick_path(sub, dtype, sub_flags, &shape, count_slots(sub, ps), true,
                    tuned ? &tv : nullptr, rk, (int)rel.size()) != QS_PATH_FUSED)
        return QS_ERR_UNSUPPORTED;
      Entry* e = get_plan(sub, shape.r, ps, rk, (int)rel.size(), &rc);
      if (!e) return rc;
      if (!tables_fit(*e, dtype, sub, shape, ps, true)) return QS_ERR_UNSUPPORTED;
      SvLaunch L{};
      L.p = &e->dev;
      L.shape = shape;
      L.B = B;
      L.per_sample_params = ps;
      L.params = params;
      L.feats = feats;
      L.state = psi_w;
      L.dstate = lam_w;
      L.out_psi = psi_w;
      L.out_lam = lam_w;
      L.ckpt = rel.empty() ? nullptr : const_cast<char*>(cb) + cs * per * first;
      L.ws_partials = part;
      L.grad_params = grad_params;
      L.grad_feats = c.n_features ? grad_feats : nullptr;
      L.accum_feats = 1;
      L.stream = stream;
      if ((rc = launch_sv_adjoint(dtype, L)) != QS_OK) return rc;
      if (!ps && e->dev.n_acc &&
          (rc = launch_reduce_partials(dtype, part, grid_of(shape, B), e->dev.n_acc,
                                       e->dev.grad_cols, grad_params, 1, stream)) != QS_OK)
        return rc;
    }
    if (k == 0) break;
    // the channel in front of this run: restart from the state stored there
    const int ch = runs[k - 1].ch;
    const qs_gate& g = c.gates[ch];
    rc = launch_channel_adjoint(dtype, c.n_qubits, g.q0, g.op == QS_OP_RESET, B, feats,
                                c.n_features, g.feat, cb + cs * per * slot_of(ck, n_ck, ch),
                                lam_w, psi_w, stream);
    if (rc != QS_OK) return rc;
  }
  return QS_OK;
}

}  // namespace

namespace qs {
void free_programs();  // prog_api.cpp
struct ProgEnginePlan {
  SvDevPlan* dev;
};
// Engine plan of one uneven-batch class: every rotation's angle is per circuit.
ProgEnginePlan program_engine_plan(const qs_circuit& c, int r, int* rc) {
  Entry* e = get_plan(c, r, true, nullptr, 0, rc);
  return {e ? &e->dev : nullptr};
}
int64_t engine_lds_bytes(int dtype, const qs_circuit& c, int S, int n_slots, int block,
                         bool ps, bool adjoint, bool half) {
  return lds_bytes(dtype, c, S, n_slots, block, ps, adjoint, nullptr, half);
}
}  // namespace qs

namespace {

// QS_FLAG_INVERSE: the calls run U^dagger of the circuit: its gates in
// reverse order with every rotation angle negated (scale -> -scale); X, Y, Z,
// H, CNOT and CZ are their own inverses. The inverted list is built on the
// host for the duration of the call (plans are cached by gate content).
struct InvCircuit {
  std::vector<qs_gate> g;
  qs_circuit c;
};
const qs_circuit* apply_inverse(const qs_circuit* c, int* flags, InvCircuit& inv) {
  if (!c || !(*flags & QS_FLAG_INVERSE)) return c;
  if (validate(c) != QS_OK) return c;  // the call itself reports it
  // A channel has no inverse: the flag stays set and the call rejects it.
  if (has_channels(*c)) return c;
  *flags &= ~QS_FLAG_INVERSE;
  if (c->n_gates > 0 && c->gates) inv.g.assign(c->gates, c->gates + c->n_gates);
  std::reverse(inv.g.begin(), inv.g.end());
  for (qs_gate& x : inv.g)
    if (x.op == QS_OP_RX || x.op == QS_OP_RY || x.op == QS_OP_RZ) x.scale = -x.scale;
  inv.c = *c;
  inv.c.gates = inv.g.empty() ? c->gates : inv.g.data();
  return &inv.c;
}

float time_ms(hipStream_t st, const std::function<int()>& fn, int reps, int* rc) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    *rc = QS_ERR_LAUNCH;
    return 0.f;
  }
  // The first run warms plans and caches; the result is the best of the
  // following `reps` calls, each synchronised on its own. (Timing a call
  // repeated back to back was tried: it favoured a smaller forward block
  // that then ran slower inside the training step.)
  float best = 1e30f;
  for (int i = 0; i <= reps; ++i) {
    (void)hipEventRecord(a, st);
    int r = fn();
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    if (r != QS_OK) {
      *rc = r;
      best = 1e30f;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (i > 0 && ms < best) best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

struct Scratch {
  std::vector<void*> ptrs;
  void* get(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) return nullptr;
    (void)hipMemset(p, 0, bytes ? bytes : 8);
    ptrs.push_back(p);
    return p;
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

bool tuned_for_call(const qs_circuit& c, int dtype, int64_t B, int flags, void* stream,
                    TuneVal* out) {
  if (g_in_tune) return false;
  if (tuned_lookup(c, dtype, B, flags, out)) return true;
  if (env_int("QS_AUTOTUNE", 0) != 1 || no_alloc_call()) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(static_cast<hipStream_t>(stream), &cs) == hipSuccess &&
      cs != hipStreamCaptureStatusNone)
    return false;
  if (qs_autotune(&c, dtype, B, flags, stream, nullptr) != QS_OK) return false;
  return tuned_lookup(c, dtype, B, flags, out);
}

}  // namespace

extern "C" {

int qs_autotune(const qs_circuit* c, int dtype, int64_t B, int flags, void* stream,
                qs_tune_info* out) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  int rc = validate(c);
  if (rc != QS_OK) return rc;
  if (has_channels(*c)) return QS_ERR_UNSUPPORTED;  // runs of the engine, planned per call
  if ((dtype != QS_C64 && dtype != QS_C128) || B < 1) return QS_ERR_INVALID;
  if (flags & ~(QS_PATH_MASK | QS_FLAG_PER_SAMPLE_PARAMS)) return QS_ERR_INVALID;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SvShape probe;
  const int path = pick_path(*c, dtype, flags, &probe, count_slots(*c, ps), false);
  if (path != QS_PATH_FUSED && path != QS_PATH_HBM) return QS_ERR_UNSUPPORTED;
  const size_t rs = dtype == QS_C64 ? 4 : 8;
  const int64_t per = B << c->n_qubits;
  Scratch sc;
  void* state = sc.get(2 * rs * per);
  void* params = sc.get(rs * (size_t)(ps ? B : 1) * (c->n_params ? c->n_params : 1));
  void* feats = sc.get(rs * (size_t)B * (c->n_features ? c->n_features : 1));
  double* expz = static_cast<double*>(sc.get(sizeof(double) * B * c->n_qubits));
  double* dexpz = static_cast<double*>(sc.get(sizeof(double) * B * c->n_qubits));
  double* gp = static_cast<double*>(
      sc.get(sizeof(double) * (size_t)(ps ? B : 1) * (c->n_params ? c->n_params : 1)));
  double* gf = static_cast<double*>(sc.get(sizeof(double) * B * (c->n_features ? c->n_features : 1)));
  if (!state || !params || !feats || !expz || !dexpz || !gp || !gf) return QS_ERR_NOMEM;
  if ((rc = launch_encode(QS_ENC_ZERO, dtype, c->n_qubits, B, 0, 0, nullptr, 0, state,
                          nullptr, stream)) != QS_OK)
    return rc;
  const void* fe = c->n_features ? feats : nullptr;
  auto fwd = [&]() {
    return qs_forward(c, dtype, B, params, fe, state, expz, nullptr, 0, nullptr, flags, stream);
  };
  auto adj = [&](void* ws, size_t wsb) {
    return qs_adjoint_backward(c, dtype, B, params, fe, state, dexpz, nullptr, gp,
                               c->n_features ? gf : nullptr, nullptr, 0, nullptr, ws, wsb,
                               flags, stream);
  };
  TuneVal best;
  qs_tune_info info;
  std::memset(&info, 0, sizeof(info));
  info.path = path;
  float bf = 1e30f, ba = 1e30f;
  std::lock_guard<std::mutex> tune_lock(g_tune_run_mu);
  struct InTune {
    InTune() { g_in_tune = true; }
    ~InTune() { g_in_tune = false; }
  } in_tune;
  if (path == QS_PATH_FUSED) {
    // Register split r; for each, the LDS staging mode (whole amplitudes,
    // or one component at a time: half the LDS per sample) and the samples
    // per block: the LDS-limited default and two smaller blocks (more
    // workgroups per CU).
    const int slots = count_slots(*c, ps);
    for (int dir = 0; dir < 2; ++dir) {
      const bool adjoint = dir == 1;
      int& force_r = adjoint ? g_force_adj_r : g_force_fwd_r;
      int& force_s = adjoint ? g_force_adj_s : g_force_fwd_s;
      int& force_h = adjoint ? g_force_adj_h : g_force_fwd_h;
      float& bt = adjoint ? ba : bf;
      for (int r = 1; r <= 5; ++r) {
        for (int half = 0; half <= (dtype == QS_C64 ? 1 : 0); ++half) {
          SvShape base;
          if (!choose_shape(dtype, *c, slots, r, adjoint, &base, ps, nullptr, 0, true, 0,
                            half != 0) ||
              base.r != r)
            continue;
          int last_block = 0;
          for (int div = 1; div <= 4; div *= 2) {
            const int cap = div == 1 ? 0 : base.samples_per_block / div;
            if (div > 1 && cap < 1) break;
            SvShape sh;
            if (!choose_shape(dtype, *c, slots, r, adjoint, &sh, ps, nullptr, 0, true, cap,
                              half != 0) ||
                sh.r != r || sh.block_threads == last_block)
              continue;
            last_block = sh.block_threads;
            force_r = r;
            force_s = cap;
            force_h = half;
            float ms;
            if (adjoint) {
              const size_t wsb = fused_ws_bytes(*c, dtype, sh, B, ps);
              void* ws = sc.get(wsb);
              if (!ws) { force_r = force_s = 0; force_h = -1; return QS_ERR_NOMEM; }
              ms = time_ms(st, [&]() { return adj(ws, wsb); }, 5, &rc);
            } else {
              ms = time_ms(st, fwd, 5, &rc);
            }
            force_r = force_s = 0;
            force_h = -1;
            info.n_candidates++;
            if (rc != QS_OK) return rc;
            // A smaller block or half staging must win clearly (by 5 %): within
            // timing noise the LDS-limited default is kept.
            if (ms < ((cap || half) ? 0.95f : 1.0f) * bt) {
              bt = ms;
              (adjoint ? best.adj_r : best.fwd_r) = r;
              (adjoint ? best.adj_s : best.fwd_s) = cap;
              (adjoint ? best.adj_h : best.fwd_h) = half;
            }
          }
        }
      }
    }
  } else {
    // Tile size m, and for each m the register split of the epochs'
    // forward and adjoint launches, timed separately.
    const int hi = std::min(c->n_qubits, dtype == QS_C64 ? kMaxQubitsFused : 13);
    const int rmax = dtype == QS_C64 ? 5 : 4;
    float bt = 1e30f;
    g_force_large = 0;  // the tiled engine first
    for (int m = std::max(6, hi - 3); m <= hi; ++m) {
      g_force_m = m;
      float mf = 1e30f, ma = 1e30f;
      int rf_best = 0, ra_best = 0;
      for (int r = 3; r <= rmax; ++r) {
        g_force_fwd_r = r;
        const float t = time_ms(st, fwd, 1, &rc);
        g_force_fwd_r = 0;
        if (rc != QS_OK) { rc = QS_OK; continue; }  // shape infeasible for this m
        info.n_candidates++;
        if (t < mf) { mf = t; rf_best = r; }
      }
      for (int r = 3; r <= rmax; ++r) {
        g_force_adj_r = r;
        TileCfg tc;
        tc.m_pref = m;
        tc.adj_r = r;
        const size_t wsb = tiled_ws_bytes(*c, dtype, B, ps, tc, &rc);
        void* ws = rc == QS_OK ? sc.get(wsb) : nullptr;
        const float t = ws ? time_ms(st, [&]() { return adj(ws, wsb); }, 1, &rc) : 0.f;
        g_force_adj_r = 0;
        if (!ws || rc != QS_OK) { rc = QS_OK; continue; }
        info.n_candidates++;
        if (t < ma) { ma = t; ra_best = r; }
      }
      g_force_m = 0;
      if (rf_best == 0 || ra_best == 0) continue;
      if (mf + ma < bt) {
        bt = mf + ma;
        bf = mf;
        ba = ma;
        best.m = m;
        best.fwd_r = rf_best;
        best.adj_r = ra_best;
      }
    }
    g_force_large = -1;
    if (best.m == 0) return QS_ERR_UNSUPPORTED;
    // Dense blocks on MFMA against the best tiled configuration (forward +
    // adjoint); the faster becomes the automatic path's choice.
    if ((flags & QS_PATH_MASK) == QS_PATH_AUTO && db_supported(*c, dtype, ps)) {
      g_force_large = 1;
      const float tf = time_ms(st, fwd, 1, &rc);
      float ta = 0.f;
      if (rc == QS_OK) {
        const size_t wsb = db_ws_bytes(*c, B);
        void* ws = sc.get(wsb);
        if (!ws) rc = QS_ERR_NOMEM;
        else ta = time_ms(st, [&]() { return adj(ws, wsb); }, 1, &rc);
      }
      g_force_large = -1;
      if (rc == QS_OK) {
        info.n_candidates += 2;
        if (tf + ta < bf + ba) {
          best.large = 1;
          bf = tf;
          ba = ta;
        }
      }
      rc = QS_OK;
    }
    if (best.large) info.path = QS_PATH_MFMA;
  }
  info.fwd_log2_regs = best.fwd_r;
  info.adj_log2_regs = best.adj_r;
  info.fwd_samples_cap = best.fwd_s;
  info.adj_samples_cap = best.adj_s;
  info.fwd_half_staging = best.fwd_h;
  info.adj_half_staging = best.adj_h;
  info.tile_qubits = best.m;
  info.fwd_ms = bf;
  info.adj_ms = ba;
  {
    std::lock_guard<std::mutex> lock(g_tmu);
    load_tune_file_locked();
    const std::string key = tune_key(*c, dtype, B, flags);
    g_tune[key] = best;
    const char* path_env = std::getenv("QS_AUTOTUNE_CACHE");
    if (path_env && *path_env) {
      if (FILE* f = std::fopen(path_env, "a")) {
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", key.c_str(), best.fwd_r, best.adj_r,
                     best.m, best.fwd_s, best.adj_s, best.fwd_h, best.adj_h, best.large);
        std::fclose(f);
      }
    }
  }
  if (out) *out = info;
  return QS_OK;
}

int qs_version(void) { return kVersion; }

const char* qs_status_string(int s) {
  switch (s) {
    case QS_OK: return "ok";
    case QS_ERR_INVALID: return "invalid descriptor, shape, pointer or flag";
    case QS_ERR_UNSUPPORTED: return "unsupported dtype or path for this shape";
    case QS_ERR_WORKSPACE: return "workspace missing or too small";
    case QS_ERR_ZERO_NORM: return "amplitude input row with zero norm";
    case QS_ERR_LAUNCH: return "HIP runtime or kernel launch failure";
    case QS_ERR_NOMEM: return "device allocation for the plan cache failed";
    case QS_ERR_CAPTURE:
      return "this shape has no plan yet and its upload is not allowed inside a stream "
             "capture: run the call once before capturing";
    case QS_ERR_NOT_PLANNED:
      return "this shape has no plan yet and the call may not allocate one: run the "
             "allocating call once first";
    default: return "unknown status";
  }
}

int qs_validate(const qs_circuit* c) { return validate(c); }

int qs_encode(int enc, int dtype, int n, int64_t B, int64_t D, int x_is_f64,
              const void* x, int64_t x_stride, void* state, int32_t* bad_rows,
              void* stream) {
  if ((dtype != QS_C64 && dtype != QS_C128) || n < 1 || n > 30 || B < 0)
    return QS_ERR_INVALID;
  if (B == 0) return QS_OK;
  if (!state) return QS_ERR_INVALID;
  if (enc == QS_ENC_AMPLITUDE) {
    if (!x || D < 1 || D > (1ll << n) || x_stride < D) return QS_ERR_INVALID;
  } else if (enc != QS_ENC_ZERO) {
    return QS_ERR_INVALID;
  }
  return launch_encode(enc, dtype, n, B, D, x_is_f64, x, x_stride, state,
                       bad_rows, stream);
}

int qs_encode_check(const int32_t* bad_rows, void* stream) {
  if (!bad_rows) return QS_ERR_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return QS_ERR_LAUNCH;
  if (cs != hipStreamCaptureStatusNone) return QS_ERR_CAPTURE;
  if (hipStreamSynchronize(st) != hipSuccess) return QS_ERR_LAUNCH;
  int32_t h = 0;
  if (hipMemcpy(&h, bad_rows, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return QS_ERR_LAUNCH;
  return h != 0 ? QS_ERR_ZERO_NORM : QS_OK;
}

namespace {

// The amplitude-encoded input of qs_forward_amplitude.
struct EncIn {
  const void* x;
  int x_is_f64;
  int64_t D, x_stride;
  int32_t* bad_rows;
};

// Encodes into `state` with its own kernel (every path but the fused engine
// with x in the state's precision, which encodes while it loads).
int encode_first(const EncIn* enc, int dtype, int n, int64_t B, void* state, void* stream) {
  if (!enc) return QS_OK;
  return launch_encode(QS_ENC_AMPLITUDE, dtype, n, B, enc->D, enc->x_is_f64, enc->x,
                       enc->x_stride, state, enc->bad_rows, stream);
}

int forward_impl(const qs_circuit* c, int dtype, int64_t B, const void* params,
                 const void* feats, void* state, double* expz, const int32_t* ckpt_gates,
                 int32_t n_ckpt, void* ckpt, int flags, void* stream, const EncIn* enc);

}  // namespace

int qs_forward(const qs_circuit* c, int dtype, int64_t B, const void* params,
               const void* feats, void* state, double* expz,
               const int32_t* ckpt_gates, int32_t n_ckpt, void* ckpt, int flags,
               void* stream) {
  CallStream call_(stream);
  return forward_impl(c, dtype, B, params, feats, state, expz, ckpt_gates, n_ckpt, ckpt,
                      flags, stream, nullptr);
}

int qs_forward_amplitude(const qs_circuit* c, int dtype, int64_t B, const void* params,
                         const void* feats, const void* x, int x_is_f64, int64_t D,
                         int64_t x_stride, int32_t* bad_rows, void* state, double* expz,
                         const int32_t* ckpt_gates, int32_t n_ckpt, void* ckpt, int flags,
                         void* stream) {
  CallStream call_(stream);
  if (!c || c->n_qubits < 1 || c->n_qubits > 30) return QS_ERR_INVALID;
  if (B > 0 && (!x || D < 1 || D > (1ll << c->n_qubits) || x_stride < D))
    return QS_ERR_INVALID;
  const EncIn enc{x, x_is_f64 ? 1 : 0, D, x_stride, bad_rows};
  return forward_impl(c, dtype, B, params, feats, state, expz, ckpt_gates, n_ckpt, ckpt,
                      flags, stream, &enc);
}

namespace {

int forward_impl(const qs_circuit* c, int dtype, int64_t B, const void* params,
                 const void* feats, void* state, double* expz, const int32_t* ckpt_gates,
                 int32_t n_ckpt, void* ckpt, int flags, void* stream, const EncIn* enc) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  int rc = validate(c);
  if (rc != QS_OK) return rc;
  if ((dtype != QS_C64 && dtype != QS_C128) || B < 0) return QS_ERR_INVALID;
  if (flags & ~(QS_PATH_MASK | QS_FLAG_PER_SAMPLE_PARAMS)) return QS_ERR_INVALID;
  if (B == 0) return QS_OK;  // nothing to read or write; pointers may be NULL
  if (!state) return QS_ERR_INVALID;
  if (c->n_params > 0 && !params) return QS_ERR_INVALID;
  if (c->n_features > 0 && !feats) return QS_ERR_INVALID;
  if ((rc = check_ckpt(c, ckpt_gates, n_ckpt, ckpt)) != QS_OK) return rc;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  if (has_channels(*c)) {  // unitary runs through the engine, channels between them
    if ((rc = channels_check(*c, flags, ckpt_gates, n_ckpt)) != QS_OK) return rc;
    if ((rc = encode_first(enc, dtype, c->n_qubits, B, state, stream)) != QS_OK) return rc;
    const int64_t per = B << c->n_qubits;
    const size_t cs = dtype == QS_C64 ? 8 : 16;
    char* cb = static_cast<char*>(ckpt);
    const std::vector<Run> runs = unitary_runs(*c);
    std::vector<int32_t> rel;
    for (size_t k = 0; k < runs.size(); ++k) {
      const Run& r = runs[k];
      const bool last = k + 1 == runs.size();
      if (r.e > r.b) {
        const qs_circuit sub = run_circuit_of(*c, r);
        int first = 0;
        run_ckpts(ckpt_gates, n_ckpt, r, rel, &first);
        rc = qs_forward(&sub, dtype, B, params, feats, state, last ? expz : nullptr,
                        rel.empty() ? nullptr : rel.data(), (int32_t)rel.size(),
                        rel.empty() ? nullptr : cb + cs * per * first,
                        (flags & ~QS_PATH_MASK) | QS_PATH_FUSED, stream);
      } else if (last && expz) {
        rc = launch_expz(dtype, c->n_qubits, B, state, expz, stream);
      }
      if (rc != QS_OK) return rc;
      if (r.ch < 0) continue;
      const qs_gate& g = c->gates[r.ch];
      rc = launch_copy_state(dtype, state, cb + cs * per * slot_of(ckpt_gates, n_ckpt, r.ch),
                             per, stream);
      if (rc == QS_OK)
        rc = launch_channel(dtype, c->n_qubits, g.q0, g.op == QS_OP_RESET, B, feats,
                            c->n_features, g.feat, state, stream);
      const int after = slot_of(ckpt_gates, n_ckpt, r.ch + 1);  // state just after it
      if (rc == QS_OK && after >= 0)
        rc = launch_copy_state(dtype, state, cb + cs * per * after, per, stream);
      if (rc != QS_OK) return rc;
    }
    return QS_OK;
  }
  TuneVal tv;
  const bool tuned = tuned_for_call(*c, dtype, B, flags, stream, &tv);
  SvShape shape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), false,
                             tuned ? &tv : nullptr, ckpt_gates, n_ckpt);
  if (path < 0) return path;
  // The fused engine encodes while it loads when x is in the state's precision
  // and the launch stages whole amplitudes.
  const bool fuse_enc = enc && path == QS_PATH_FUSED && shape.half == 0 &&
                        (enc->x_is_f64 != 0) == (dtype == QS_C128);
  if (!fuse_enc && (rc = encode_first(enc, dtype, c->n_qubits, B, state, stream)) != QS_OK)
    return rc;
  if (path == QS_PATH_PLAIN) {
    PlainLaunch L{};
    L.c = c;
    L.dtype = dtype;
    L.B = B;
    L.per_sample_params = ps;
    L.params = params;
    L.feats = feats;
    L.state = state;
    L.expz = expz;
    L.ckpt_gates = ckpt_gates;
    L.n_ckpt = n_ckpt;
    L.ckpt = ckpt;
    L.stream = stream;
    return run_plain_forward(L);
  }
  if (path == QS_PATH_MFMA) {
    DbEntry* e = get_db(*c, ckpt_gates, n_ckpt, &rc);
    if (!e) return rc;
    const DbLaunch L{kDbK, c->n_qubits, B, e->blk_begin, e->gates, e->blk_q,
                     e->h_blk_q.data(), params, kDbGrid, stream};
    const int64_t per = B << c->n_qubits;
    for (size_t i = 0; i < e->blocks.size(); ++i) {
      if ((rc = launch_db_forward(L, (int)i, state)) != QS_OK) return rc;
      const int slot = e->blocks[i].ckpt_after;
      if (slot >= 0 &&
          (rc = launch_copy_state(dtype, state, static_cast<char*>(ckpt) + 8 * per * slot, per,
                                  stream)) != QS_OK)
        return rc;
    }
    return expz ? launch_expz(dtype, c->n_qubits, B, state, expz, stream) : QS_OK;
  }
  if (path == QS_PATH_HBM) {
    TiledEntry* te = get_tiled(*c, dtype, ps, ckpt_gates, n_ckpt, tile_cfg(tuned, tv), &rc);
    if (!te) return rc;
    const int64_t per = B << c->n_qubits;  // complex elements per state batch
    const size_t cs = dtype == QS_C64 ? 8 : 16;
    for (const TiledEpochDev& d : te->epochs) {
      SvLaunch L{};
      L.p = &d.fwd->dev;
      L.shape = d.fshape;
      L.B = B;
      L.per_sample_params = ps;
      L.params = params;
      L.feats = feats;
      L.state = state;
      L.n_tot = c->n_qubits;
      L.ob = c->n_qubits - te->m;
      L.tile_q = d.tile_q;
      L.outer_q = d.outer_q;
      L.stream = stream;
      if ((rc = launch_sv_forward(dtype, L)) != QS_OK) return rc;
      if (d.ckpt_after >= 0 && ckpt) {
        rc = launch_copy_state(dtype, state,
                               static_cast<char*>(ckpt) + cs * per * d.ckpt_after, per,
                               stream);
        if (rc != QS_OK) return rc;
      }
    }
    return expz ? launch_expz(dtype, c->n_qubits, B, state, expz, stream) : QS_OK;
  }
  Entry* e = get_plan(*c, shape.r, ps, ckpt_gates, n_ckpt, &rc);
  if (!e) return rc;
  if (!tables_fit(*e, dtype, *c, shape, ps, false)) return QS_ERR_UNSUPPORTED;
  SvLaunch L{};
  L.p = &e->dev;
  L.shape = shape;
  L.B = B;
  L.per_sample_params = ps;
  L.params = params;
  L.feats = feats;
  L.state = state;
  L.expz = expz;
  L.ckpt = ckpt;
  L.stream = stream;
  if (fuse_enc) {
    L.x_in = enc->x;
    L.x_stride = enc->x_stride;
    L.x_D = enc->D;
    L.bad_rows = enc->bad_rows;
  }
  return launch_sv_forward(dtype, L);
}

}  // namespace

size_t qs_workspace_size(const qs_circuit* c, int dtype, int64_t B, int flags) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  if (validate(c) != QS_OK || B < 0) return 0;
  if (has_channels(*c)) return channel_ws_bytes(*c, dtype, B, flags);
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  TuneVal tv;
  const bool tuned = tuned_lookup(*c, dtype, B, flags, &tv);
  SvShape shape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), true,
                             tuned ? &tv : nullptr);
  if (path == QS_PATH_PLAIN) return plain_workspace_bytes(*c, dtype, B);
  if (path == QS_PATH_FUSED) return fused_ws_bytes(*c, dtype, shape, B, ps);
  if (path == QS_PATH_HBM) {
    int rc = QS_OK;
    return tiled_ws_bytes(*c, dtype, B, ps, tile_cfg(tuned, tv), &rc);
  }
  if (path == QS_PATH_MFMA) return db_ws_bytes(*c, B);
  return 0;
}

int qs_adjoint_backward(const qs_circuit* c, int dtype, int64_t B,
                        const void* params, const void* feats, const void* state,
                        const double* dexpz, const void* dstate,
                        double* grad_params, double* grad_feats,
                        const int32_t* ckpt_gates, int32_t n_ckpt,
                        const void* ckpt, void* ws, size_t ws_bytes, int flags,
                        void* stream) {
  return adjoint_backward_impl(c, dtype, B, params, feats, state, dexpz, dstate, grad_params,
                               grad_feats, ckpt_gates, n_ckpt, ckpt, ws, ws_bytes, flags,
                               stream, false);
}

}  // extern "C"

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The one-launch training step runs on the fused engine with the adjoint's
// (tuned) shape when that shape has a training-step kernel: complex64, angles
// shared by the batch, no channels. Returns the shape, or false.
bool train_shape(const qs_circuit& c, int dtype, int64_t B, int flags, void* stream, bool tune,
                 SvShape* shape) {
  if (dtype != QS_C64 || (flags & QS_FLAG_PER_SAMPLE_PARAMS) || has_channels(c)) return false;
  TuneVal tv;
  const bool tuned = tune ? tuned_for_call(c, dtype, B, flags, stream, &tv)
                          : tuned_lookup(c, dtype, B, flags, &tv);
  const int path = pick_path(c, dtype, flags, shape, count_slots(c, false), true,
                             tuned ? &tv : nullptr);
  return path == QS_PATH_FUSED && sv_train_supported(dtype, *shape);
}

}  // namespace

extern "C" {

size_t qs_train_workspace_size(const qs_circuit* c, int dtype, int64_t B, int flags) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  if (validate(c) != QS_OK || B <= 0) return 0;
  if (flags & ~(QS_PATH_MASK | QS_FLAG_PER_SAMPLE_PARAMS)) return 0;
  SvShape shape;
  if (!train_shape(*c, dtype, B, flags, nullptr, false, &shape)) return 0;
  return align256(fused_ws_bytes(*c, dtype, shape, B, false)) +
         (size_t)fused_rows_bound(*c, dtype, shape, B, false) * sizeof(double);
}

int qs_train_step_mse(const qs_circuit* c, int dtype, int64_t B, const void* params,
                      const void* feats, const void* x, int x_is_f64, int64_t D,
                      int64_t x_stride, int32_t* bad_rows, const double* y, int q,
                      double* expz, double* loss, double* grad_params, double* grad_feats,
                      void* ws, size_t ws_bytes, int flags, void* stream) {
  CallStream call_(stream);
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  int rc = validate(c);
  if (rc != QS_OK) return rc;
  if ((dtype != QS_C64 && dtype != QS_C128) || B < 0) return QS_ERR_INVALID;
  if (flags & ~(QS_PATH_MASK | QS_FLAG_PER_SAMPLE_PARAMS)) return QS_ERR_INVALID;
  if (q < 0 || q >= c->n_qubits) return QS_ERR_INVALID;
  if (B == 0) return QS_OK;
  if (!y || !loss) return QS_ERR_INVALID;
  if (c->n_params > 0 && (!params || !grad_params)) return QS_ERR_INVALID;
  if (c->n_features > 0 && !feats) return QS_ERR_INVALID;
  if (x && (D < 1 || D > (1ll << c->n_qubits) || x_stride < D)) return QS_ERR_INVALID;
  if (x && x_is_f64) return QS_ERR_UNSUPPORTED;  // complex64 reads float32 inputs
  SvShape shape;
  if (!train_shape(*c, dtype, B, flags, stream, true, &shape)) return QS_ERR_UNSUPPORTED;
  Entry* e = get_plan(*c, shape.r, false, nullptr, 0, &rc);
  if (!e) return rc;
  if (!tables_fit(*e, dtype, *c, shape, false, true)) return QS_ERR_UNSUPPORTED;
  const int64_t grid = grid_of(shape, B);
  const size_t part = align256(fused_ws_bytes(*c, dtype, shape, B, false));
  if (!ws || ws_bytes < part + (size_t)grid * sizeof(double)) return QS_ERR_WORKSPACE;
  SvLaunch L{};
  L.p = &e->dev;
  L.shape = shape;
  L.B = B;
  L.params = params;
  L.feats = feats;
  L.state = nullptr;  // the state never leaves the registers
  L.x_in = x;
  L.x_stride = x_stride;
  L.x_D = D;
  L.bad_rows = bad_rows;
  L.expz = expz;
  L.ws_partials = ws;
  L.grad_params = grad_params;
  L.grad_feats = c->n_features ? grad_feats : nullptr;
  L.y = y;
  L.loss_q = q;
  L.loss_part = reinterpret_cast<double*>(static_cast<char*>(ws) + part);
  L.stream = stream;
  if ((rc = launch_sv_train(dtype, L)) != QS_OK) return rc;
  const int n_acc = c->n_params ? e->dev.n_acc : 0;
  if (c->n_params && n_acc < c->n_params &&
      (rc = launch_fill_f64(grad_params, c->n_params, stream)) != QS_OK)
    return rc;
  return launch_reduce_partials(dtype, ws, grid, n_acc, e->dev.grad_cols, grad_params,
                                n_acc < c->n_params, stream, L.loss_part, loss,
                                1.0 / (double)B);
}

}  // extern "C"

namespace qs {
int adjoint_backward_impl(const qs_circuit* c, int dtype, int64_t B, const void* params,
                          const void* feats, const void* state, const double* dexpz,
                          const void* dstate, double* grad_params, double* grad_feats,
                          const int32_t* ckpt_gates, int32_t n_ckpt, const void* ckpt,
                          void* ws, size_t ws_bytes, int flags, void* stream,
                          bool no_alloc) {
  CallStream call_(stream);
  std::optional<NoAllocCall> na_;
  if (no_alloc) na_.emplace();
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  int rc = validate(c);
  if (rc != QS_OK) return rc;
  if ((dtype != QS_C64 && dtype != QS_C128) || B < 0) return QS_ERR_INVALID;
  if (flags & ~(QS_PATH_MASK | QS_FLAG_PER_SAMPLE_PARAMS)) return QS_ERR_INVALID;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  if (B == 0) {  // an empty batch: shared gradients are zero, nothing else
    if (c->n_params && !ps && grad_params)
      rc = launch_fill_f64(grad_params, c->n_params, stream);
    return rc;
  }
  if (!state) return QS_ERR_INVALID;
  if ((dexpz == nullptr) == (dstate == nullptr)) return QS_ERR_INVALID;
  if (c->n_params > 0 && (!params || !grad_params)) return QS_ERR_INVALID;
  if (c->n_features > 0 && !feats) return QS_ERR_INVALID;
  if ((rc = check_ckpt(c, ckpt_gates, n_ckpt, ckpt)) != QS_OK) return rc;
  if (has_channels(*c)) {
    if (no_alloc) return QS_ERR_UNSUPPORTED;
    if ((rc = channels_check(*c, flags, ckpt_gates, n_ckpt)) != QS_OK) return rc;
    const size_t need = channel_ws_bytes(*c, dtype, B, flags);
    if (need == 0) return QS_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < need) return QS_ERR_WORKSPACE;
    return adjoint_channels(*c, dtype, B, params, feats, state, dexpz, dstate, grad_params,
                            grad_feats, ckpt_gates, n_ckpt, ckpt, ws, flags, stream);
  }
  TuneVal tv;
  const bool tuned = tuned_for_call(*c, dtype, B, flags, stream, &tv);
  SvShape shape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), true,
                             tuned ? &tv : nullptr, ckpt_gates, n_ckpt);
  if (path < 0) return path;
  if (no_alloc && path != QS_PATH_FUSED) return QS_ERR_UNSUPPORTED;
  const TileCfg tcfg = tile_cfg(tuned, tv);
  const size_t need = path == QS_PATH_PLAIN ? plain_workspace_bytes(*c, dtype, B)
                     : path == QS_PATH_HBM   ? tiled_ws_bytes(*c, dtype, B, ps, tcfg, &rc)
                     : path == QS_PATH_MFMA  ? db_ws_bytes(*c, B)
                                             : fused_ws_bytes(*c, dtype, shape, B, ps);
  if (rc != QS_OK) return rc;
  if (need > 0 && (!ws || ws_bytes < need)) return QS_ERR_WORKSPACE;
  if (path == QS_PATH_MFMA) {
    DbEntry* e = get_db(*c, ckpt_gates, n_ckpt, &rc);
    if (!e) return rc;
    const DbLaunch L{kDbK, c->n_qubits, B, e->blk_begin, e->gates, e->blk_q,
                     e->h_blk_q.data(), params, kDbGrid, stream};
    const int nb = (int)e->blocks.size();
    const DbWs lay = db_ws_layout(*c, B, nb);
    if (lay.total > ws_bytes) return QS_ERR_WORKSPACE;
    const int64_t per = B << c->n_qubits;
    char* w = static_cast<char*>(ws);
    void* psi_w = w + lay.psi;
    void* lam_w = w + lay.lam;
    float* part = reinterpret_cast<float*>(w + lay.part);
    double* rho = reinterpret_cast<double*>(w + lay.rho);
    double* gth = reinterpret_cast<double*>(w + lay.gth);
    if ((rc = launch_copy_state(dtype, state, psi_w, per, stream)) != QS_OK) return rc;
    rc = dstate ? launch_copy_state(dtype, dstate, lam_w, per, stream)
                : launch_obs_cot(dtype, c->n_qubits, B, dexpz, psi_w, lam_w, stream);
    if (rc != QS_OK) return rc;
    for (int i = nb - 1; i >= 0; --i) {
      const int slot = e->blocks[i].ckpt_after;
      if (slot >= 0 && ckpt &&  // psi after this block = the stored checkpoint
          (rc = launch_copy_state(dtype, static_cast<const char*>(ckpt) + 8 * per * slot,
                                  psi_w, per, stream)) != QS_OK)
        return rc;
      if ((rc = launch_db_adjoint(L, i, psi_w, lam_w, part)) != QS_OK) return rc;
      if ((rc = launch_db_reduce(L, part, rho + (size_t)i * 2 * 32 * 32)) != QS_OK) return rc;
    }
    if ((rc = launch_fill_f64(gth, std::max(c->n_gates, 1), stream)) != QS_OK) return rc;
    if ((rc = launch_db_grads(L, nb, rho, gth)) != QS_OK) return rc;
    if ((rc = launch_db_chain(c->n_params, e->p_begin, e->p_gate, e->p_scale, gth,
                              grad_params, stream)) != QS_OK)
      return rc;
    if (c->n_features && grad_feats)  // no rotation reads a feature on this path
      rc = launch_fill_f64(grad_feats, B * c->n_features, stream);
    return rc;
  }
  if (path == QS_PATH_HBM) {
    TiledEntry* te = get_tiled(*c, dtype, ps, ckpt_gates, n_ckpt, tcfg, &rc);
    if (!te) return rc;
    const int64_t per = B << c->n_qubits;
    const size_t cs = dtype == QS_C64 ? 8 : 16;
    const int64_t samples = B << (c->n_qubits - te->m);
    if (!ps) {  // every epoch's partial sums must fit behind the two states
      const size_t acc = dtype == QS_C64 ? 4 : 8;
      for (const TiledEpochDev& d : te->epochs) {
        const int64_t g = (samples + d.ashape.samples_per_block - 1) / d.ashape.samples_per_block;
        if (2 * cs * (size_t)per + (size_t)g * d.adj->dev.n_acc * acc > ws_bytes)
          return QS_ERR_WORKSPACE;
      }
    }
    char* psi_w = static_cast<char*>(ws);
    char* lam_w = psi_w + cs * per;
    void* part = lam_w + cs * per;
    if ((rc = launch_copy_state(dtype, state, psi_w, per, stream)) != QS_OK) return rc;
    rc = dstate ? launch_copy_state(dtype, dstate, lam_w, per, stream)
                : launch_obs_cot(dtype, c->n_qubits, B, dexpz, psi_w, lam_w, stream);
    if (rc != QS_OK) return rc;
    const int64_t gp_n = ps ? B * c->n_params : c->n_params;
    if (c->n_params && (rc = launch_fill_f64(grad_params, gp_n, stream)) != QS_OK) return rc;
    if (c->n_features && grad_feats &&
        (rc = launch_fill_f64(grad_feats, B * c->n_features, stream)) != QS_OK)
      return rc;
    for (int i = (int)te->epochs.size() - 1; i >= 0; --i) {
      const TiledEpochDev& d = te->epochs[i];
      if (d.ckpt_after >= 0 && ckpt) {  // psi after this epoch = the checkpoint
        rc = launch_copy_state(dtype,
                               static_cast<const char*>(ckpt) + cs * per * d.ckpt_after,
                               psi_w, per, stream);
        if (rc != QS_OK) return rc;
      }
      SvLaunch L{};
      L.p = &d.adj->dev;
      L.shape = d.ashape;
      L.B = B;
      L.per_sample_params = ps;
      L.params = params;
      L.feats = feats;
      L.state = psi_w;
      L.dstate = lam_w;
      L.out_psi = psi_w;
      L.out_lam = lam_w;
      L.ws_partials = part;
      L.grad_params = grad_params;
      L.grad_feats = c->n_features ? grad_feats : nullptr;
      L.n_tot = c->n_qubits;
      L.ob = c->n_qubits - te->m;
      L.tile_q = d.tile_q;
      L.outer_q = d.outer_q;
      L.stream = stream;
      if ((rc = launch_sv_adjoint(dtype, L)) != QS_OK) return rc;
      if (!ps && d.adj->dev.n_acc) {
        const int64_t grid = (samples + d.ashape.samples_per_block - 1) / d.ashape.samples_per_block;
        rc = launch_reduce_partials(dtype, part, grid, d.adj->dev.n_acc, d.adj->dev.grad_cols,
                                    grad_params, 1, stream);
        if (rc != QS_OK) return rc;
      }
    }
    return QS_OK;
  }
  if (path == QS_PATH_PLAIN) {
    qs_gate* dg = get_dev_gates(*c, &rc);
    if (!dg && c->n_gates) return rc;
    PlainLaunch L{};
    L.c = c;
    L.d_gates = dg;
    L.dtype = dtype;
    L.B = B;
    L.per_sample_params = ps;
    L.params = params;
    L.feats = feats;
    L.state = const_cast<void*>(state);
    L.ckpt_gates = ckpt_gates;
    L.n_ckpt = n_ckpt;
    L.ckpt = const_cast<void*>(ckpt);
    L.dexpz = dexpz;
    L.dstate = dstate;
    L.grad_params = grad_params;
    L.grad_feats = grad_feats;
    L.ws = ws;
    L.stream = stream;
    return run_plain_adjoint(L);
  }
  Entry* e = get_plan(*c, shape.r, ps, ckpt_gates, n_ckpt, &rc);
  if (!e) return rc;
  if (!tables_fit(*e, dtype, *c, shape, ps, true)) return QS_ERR_UNSUPPORTED;
  if (ps && c->n_params) {
    if ((rc = launch_fill_f64(grad_params, B * c->n_params, stream)) != QS_OK) return rc;
  }
  SvLaunch L{};
  L.p = &e->dev;
  L.shape = shape;
  L.B = B;
  L.per_sample_params = ps;
  L.params = params;
  L.feats = feats;
  L.state = const_cast<void*>(state);
  L.ckpt = const_cast<void*>(ckpt);
  L.dexpz = dexpz;
  L.dstate = dstate;
  L.ws_partials = ws;
  L.grad_params = grad_params;
  L.grad_feats = c->n_features ? grad_feats : nullptr;
  L.stream = stream;
  if ((rc = launch_sv_adjoint(dtype, L)) != QS_OK) return rc;
  if (!ps && c->n_params) {
    // Parameters no rotation reads get a zero gradient.
    const int n_acc = e->dev.n_acc;
    if (n_acc < c->n_params && (rc = launch_fill_f64(grad_params, c->n_params, stream)) != QS_OK)
      return rc;
    rc = launch_reduce_partials(dtype, ws, grid_of(shape, B), n_acc, e->dev.grad_cols,
                                grad_params, n_acc < c->n_params, stream);
  }
  return rc;
}

}  // namespace qs

extern "C" {

int qs_expz(int dtype, int n, int64_t B, const void* state, double* expz,
            void* stream) {
  if ((dtype != QS_C64 && dtype != QS_C128) || n < 1 || n > 30 || B < 0 || !state ||
      !expz)
    return QS_ERR_INVALID;
  return launch_expz(dtype, n, B, state, expz, stream);
}

int qs_loss_mse_z(int n, int64_t B, int q, const double* expz, const double* y,
                  double* dexpz, double* loss, void* stream) {
  if (n < 1 || n > 30 || q < 0 || q >= n || B < 0) return QS_ERR_INVALID;
  if (B > 0 && (!expz || !y)) return QS_ERR_INVALID;
  if (!dexpz && !loss) return QS_OK;
  return launch_loss_mse_z(n, B, q, expz, y, dexpz, loss, stream);
}

int qs_fidelity_reset(int dtype, int n, int n_trash, int64_t B, const void* psi,
                      const void* chi, double* fid, const double* dfid,
                      void* lam_psi, void* lam_chi, void* stream) {
  if ((dtype != QS_C64 && dtype != QS_C128) || n < 1 || n > 30 || B < 0 ||
      B > 0x7fffffff || n_trash < 0 || n_trash > 6 || n_trash >= n)
    return QS_ERR_INVALID;
  if (B == 0) return QS_OK;
  if (!psi || !chi || !fid || (dfid && (!lam_psi || !lam_chi))) return QS_ERR_INVALID;
  return launch_fidelity(dtype, n, n_trash, B, psi, chi, fid, dfid, lam_psi,
                         lam_chi, stream);
}

int qs_fidelity_postselect(int dtype, int n, int n_trash, int64_t B, const void* psi,
                           const void* chi, double* fid, const double* dfid,
                           void* lam_psi, void* lam_chi, void* stream) {
  if ((dtype != QS_C64 && dtype != QS_C128) || n < 1 || n > 30 || B < 0 ||
      B > 0x7fffffff || n_trash < 0 || n_trash >= n)
    return QS_ERR_INVALID;
  if (B == 0) return QS_OK;
  if (!psi || !chi || !fid || (dfid && (!lam_psi || !lam_chi))) return QS_ERR_INVALID;
  return launch_fidelity_postselect(dtype, n, n_trash, B, psi, chi, fid, dfid, lam_psi,
                                    lam_chi, stream);
}

int qs_fidelity_trajectory(int dtype, int n, int n_trash, int64_t B, const void* psi,
                           const void* chi, const double* u, double* fid, int32_t* outcome,
                           const double* dfid, void* lam_psi, void* lam_chi,
                           void* stream) {
  if ((dtype != QS_C64 && dtype != QS_C128) || n < 1 || n > 30 || B < 0 ||
      B > 0x7fffffff || n_trash < 0 || n_trash > 6 || n_trash >= n)
    return QS_ERR_INVALID;
  if (B == 0) return QS_OK;
  if (!psi || !chi || !u || !fid || (dfid && (!lam_psi || !lam_chi))) return QS_ERR_INVALID;
  return launch_fidelity_trajectory(dtype, n, n_trash, B, psi, chi, u, fid, outcome, dfid,
                                    lam_psi, lam_chi, stream);
}

int qs_plan_info_get(const qs_circuit* c, int dtype, int64_t B, int flags,
                     qs_plan_info* out) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  int rc = validate(c);
  if (rc != QS_OK) return rc;
  if (has_channels(*c)) return QS_ERR_UNSUPPORTED;  // runs of the engine, planned per call
  if (!out || (dtype != QS_C64 && dtype != QS_C128)) return QS_ERR_INVALID;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  TuneVal tv;
  const bool tuned = tuned_lookup(*c, dtype, B, flags, &tv);
  SvShape shape, ashape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), false,
                             tuned ? &tv : nullptr);
  if (path < 0) return path;
  std::memset(out, 0, sizeof(*out));
  out->path = path;
  if (path == QS_PATH_HBM) {
    TiledHostInfo h = tiled_host_info(*c, dtype, B, ps, tile_cfg(tuned, tv));
    if (!h.ok) return QS_ERR_UNSUPPORTED;
    out->n_segments = h.n_epochs;  // epochs
    out->log2_threads = h.m;       // tile qubits
    return QS_OK;
  }
  if (path == QS_PATH_MFMA) {
    out->n_segments = (int32_t)plan_blocks(*c, kDbK, nullptr, 0).size();  // blocks
    out->log2_threads = kDbK;                                             // block qubits
    return QS_OK;
  }
  if (path != QS_PATH_FUSED) return QS_OK;
  if (pick_path(*c, dtype, flags, &ashape, count_slots(*c, ps), true,
                tuned ? &tv : nullptr) == QS_PATH_FUSED) {
    out->adj_log2_regs = ashape.r;
    out->adj_samples_per_block = ashape.samples_per_block;
    out->adj_block_threads = ashape.block_threads;
  }
  SvPlan P = plan_sv(*c, shape.r, ps, nullptr, 0);
  out->log2_regs = shape.r;
  out->log2_threads = shape.t;
  out->samples_per_block = shape.samples_per_block;
  out->block_threads = shape.block_threads;
  out->n_segments = P.nseg();
  out->n_remaps = P.n_remaps;
  out->n_ops = (int32_t)(P.exec.size() / 3);
  out->n_engine_ops = (int32_t)P.ops.size();
  out->lds_bytes = shape.lds_bytes;
  (void)B;
  return QS_OK;
}

int qs_hbm_info_get(const qs_circuit* c, int dtype, int64_t B, int flags,
                    const int32_t* ckpt_gates, int32_t n_ckpt, qs_hbm_info* out) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  int rc = validate(c);
  if (rc != QS_OK) return rc;
  if (has_channels(*c)) return QS_ERR_UNSUPPORTED;  // runs of the engine, planned per call
  if (!out || (dtype != QS_C64 && dtype != QS_C128) || B < 0) return QS_ERR_INVALID;
  static const char dummy = 0;  // check_ckpt wants a buffer; none is touched here
  if ((rc = check_ckpt(c, ckpt_gates, n_ckpt, &dummy)) != QS_OK) return rc;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  TuneVal tv;
  const bool tuned = tuned_lookup(*c, dtype, B, flags, &tv);
  SvShape shape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), true,
                             tuned ? &tv : nullptr, ckpt_gates, n_ckpt);
  if (path < 0) return path;
  if (path == QS_PATH_MFMA) {
    std::memset(out, 0, sizeof(*out));
    out->path = path;
    DbEntry e;
    std::vector<int32_t> b0, pb, pg;
    std::vector<DbGate> recs;
    std::vector<float> psc;
    if (!db_host_plan(*c, ckpt_gates, n_ckpt, e, b0, recs, pb, pg, psc))
      return QS_ERR_UNSUPPORTED;
    out->n_passes = (int32_t)e.blocks.size();
    out->tile_qubits = kDbK;
    out->max_partial_bytes = (int64_t)kDbGrid * 2 * 32 * 32 * sizeof(float);
    out->ws_bytes = (int64_t)db_ws_bytes(*c, B);
    return QS_OK;
  }
  if (path != QS_PATH_HBM) return QS_ERR_UNSUPPORTED;
  std::memset(out, 0, sizeof(*out));
  out->path = path;
  const TileCfg tc = tile_cfg(tuned, tv);
  TiledHostInfo h = tiled_host_info(*c, dtype, B, ps, tc, ckpt_gates, n_ckpt);
  if (!h.ok) return QS_ERR_UNSUPPORTED;
  out->n_passes = h.n_epochs;
  out->tile_qubits = h.m;
  out->max_partial_bytes = h.max_part_plan * (dtype == QS_C64 ? 4 : 8);
  out->ws_bytes = (int64_t)tiled_ws_bytes(*c, dtype, B, ps, tc, &rc);
  return rc;
}

int qs_block_plan_export(const qs_circuit* c, int dtype, int flags, const int32_t* ckpt_gates,
                         int32_t n_ckpt, int32_t* n_blocks, int32_t* blk_qubits,
                         int32_t* blk_begin, int32_t* blk_gates, int32_t* blk_ckpt) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  int rc = validate(c);
  if (rc != QS_OK) return rc;
  if (!n_blocks) return QS_ERR_INVALID;
  static const char dummy = 0;  // check_ckpt wants a buffer; none is touched here
  if ((rc = check_ckpt(c, ckpt_gates, n_ckpt, &dummy)) != QS_OK) return rc;
  if (!db_supported(*c, dtype, (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0))
    return QS_ERR_UNSUPPORTED;
  DbEntry e;
  std::vector<int32_t> begin, pb, pg;
  std::vector<DbGate> recs;
  std::vector<float> psc;
  if (!db_host_plan(*c, ckpt_gates, n_ckpt, e, begin, recs, pb, pg, psc))
    return QS_ERR_UNSUPPORTED;
  *n_blocks = (int32_t)e.blocks.size();
  for (size_t b = 0; b < e.blocks.size(); ++b) {
    if (blk_qubits)
      for (int i = 0; i < kDbK; ++i) blk_qubits[b * kDbK + i] = e.blocks[b].qubits[i];
    if (blk_ckpt) blk_ckpt[b] = e.blocks[b].ckpt_after;
  }
  if (blk_begin) std::memcpy(blk_begin, begin.data(), sizeof(int32_t) * begin.size());
  if (blk_gates)
    for (size_t i = 0; i < recs.size(); ++i) blk_gates[i] = recs[i].g;
  return QS_OK;
}

int qs_plan_export(const qs_circuit* c, int dtype, int64_t B, int flags,
                   qs_plan_info* info, int32_t* ops, int32_t* seg_begin,
                   uint8_t* seg_map) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  int rc = qs_plan_info_get(c, dtype, B, flags, info);
  if (rc != QS_OK) return rc;
  if (info->path != QS_PATH_FUSED) return QS_ERR_UNSUPPORTED;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  SvPlan P = plan_sv(*c, info->log2_regs, ps, nullptr, 0);  // the forward plan
  if (ops)
    for (size_t o = 0; o < P.exec.size() / 3; ++o) {
      const int g = P.exec[3 * o];
      ops[4 * o] = c->gates[g].op;
      ops[4 * o + 1] = P.exec[3 * o + 1];
      ops[4 * o + 2] = P.exec[3 * o + 2];
      ops[4 * o + 3] = g;
    }
  if (seg_begin)
    std::memcpy(seg_begin, P.exec_seg.data(), sizeof(int32_t) * P.exec_seg.size());
  if (seg_map) std::memcpy(seg_map, P.seg_map.data(), P.seg_map.size());
  return QS_OK;
}

int qs_plan_dump(const qs_circuit* c, int dtype, int64_t B, int flags, int adjoint,
                 qs_engine_dump* info, int32_t* ops, int32_t* seg_begin, uint16_t* seg_lay,
                 int32_t* l1q, uint32_t* diag, int32_t* blk_begin, int32_t* blk_gates) {
  InvCircuit inv_;
  c = apply_inverse(c, &flags, inv_);
  if (!info) return QS_ERR_INVALID;
  qs_plan_info pi;
  int rc = qs_plan_info_get(c, dtype, B, flags, &pi);
  if (rc != QS_OK) return rc;
  if (pi.path != QS_PATH_FUSED) return QS_ERR_UNSUPPORTED;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  const int r = adjoint ? pi.adj_log2_regs : pi.log2_regs;
  if (r <= 0) return QS_ERR_UNSUPPORTED;
  SvPlan P = plan_sv(*c, r, ps, nullptr, 0);
  info->n_qubits = P.n;
  info->log2_regs = P.r;
  info->n_ops = (int32_t)P.ops.size();
  info->n_segments = P.nseg();
  info->n_l1q = (int32_t)(P.l1q.size() / kL1QWords);
  info->n_diag = (int32_t)(P.diag.size() / kDiagWords);
  info->n_blocks = P.n_blocks();
  info->n_block_gates = (int32_t)P.blk_gates.size();
  if (ops)
    for (size_t o = 0; o < P.ops.size(); ++o) {
      ops[5 * o] = P.ops[o].kind;
      ops[5 * o + 1] = P.ops[o].a;
      ops[5 * o + 2] = P.ops[o].b;
      ops[5 * o + 3] = P.ops[o].aux;
      ops[5 * o + 4] = P.ops[o].gate;
    }
  if (seg_begin)
    std::memcpy(seg_begin, P.seg_begin.data(), sizeof(int32_t) * P.seg_begin.size());
  if (seg_lay) std::memcpy(seg_lay, P.seg_lay.data(), sizeof(uint16_t) * P.seg_lay.size());
  if (l1q) std::memcpy(l1q, P.l1q.data(), sizeof(int32_t) * P.l1q.size());
  if (diag) std::memcpy(diag, P.diag.data(), sizeof(uint32_t) * P.diag.size());
  if (blk_begin)
    std::memcpy(blk_begin, P.blk_begin.data(), sizeof(int32_t) * P.blk_begin.size());
  if (blk_gates)
    std::memcpy(blk_gates, P.blk_gates.data(), sizeof(int32_t) * P.blk_gates.size());
  return QS_OK;
}

void qs_shutdown(void) {
  qs::free_programs();  // they reference the engine plans released below
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& kv : g_cache) {
    free_dev(kv.second->dev);
    delete kv.second;
  }
  g_cache.clear();
  for (auto& kv : g_gate_cache) (void)hipFree(kv.second);
  g_gate_cache.clear();
  for (auto& kv : g_tiled) {
    for (auto& d : kv.second->epochs) {
      (void)hipFree(d.tile_q);
      (void)hipFree(d.outer_q);
    }
    delete kv.second;
  }
  g_tiled.clear();
  for (auto& kv : g_db) free_db(kv.second);
  g_db.clear();
}

}  // extern "C"
