// C ABI entry points: validation, launch-shape choice, plan cache, dispatch.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "qs_internal.h"

namespace qs {
int sv_max_threads(int dtype, int r, int adjoint);
}

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
    if (x.op < QS_OP_RX || x.op > QS_OP_CZ || x.flags != 0) return QS_ERR_INVALID;
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

int check_ckpt(const qs_circuit* c, const int32_t* ck, int32_t n_ck,
               const void* buf) {
  if (n_ck < 0) return QS_ERR_INVALID;
  if (n_ck == 0) return QS_OK;
  if (!ck || !buf) return QS_ERR_INVALID;
  for (int i = 0; i < n_ck; ++i) {
    if (ck[i] <= 0 || ck[i] >= c->n_gates) return QS_ERR_INVALID;
    if (i > 0 && ck[i] <= ck[i - 1]) return QS_ERR_INVALID;
  }
  return QS_OK;
}

// ------------------------------------------------------------- launch shape
int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v && *v ? std::atoi(v) : dflt;
}

// Bytes of LDS the engine uses for a block of S samples.
int64_t lds_bytes(int dtype, int n, int S, int n_gates, int n_slots,
                  int n_params, int n_feats) {
  const int64_t rs = dtype == QS_C64 ? 4 : 8;
  int64_t b = (int64_t)S * (2 * rs << n);      // states
  b += 2 * rs * n_gates;                       // shared angle table
  b += 2 * rs * (int64_t)n_slots * S;          // per-sample angle table
  b += rs * ((int64_t)n_params + (int64_t)S * n_feats);  // gradient accumulators
  return (b + 15) & ~15ll;
}

// Choose amplitudes-per-thread 2^r and the block shape for one direction.
// Returns false when the fused engine cannot hold the circuit. Preference
// orders come from the register budgets of the instantiations: the forward
// holds one state per thread group, the adjoint two (psi and lam), so the
// adjoint prefers a narrower register tile.
bool choose_shape(int dtype, const qs_circuit& c, int n_slots, int r_force,
                  bool adjoint, SvShape* out) {
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
    // Shrink the block until the LDS fits.
    while (S > 1 && lds_bytes(dtype, n, S, c.n_gates, n_slots, c.n_params,
                              c.n_features) > kMaxLds) {
      S >>= 1;
    }
    block = S * T;
    if (block < 64) {  // keep whole waves
      S = 64 / T;
      block = 64;
    }
    const int64_t lds = lds_bytes(dtype, n, S, c.n_gates, n_slots, c.n_params,
                                  c.n_features);
    if (lds > kMaxLds) continue;
    out->r = r;
    out->t = t;
    out->block_threads = block;
    out->samples_per_block = S;
    out->lds_bytes = lds;
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
             int device) {
  Key k;
  int32_t hdr[8] = {c.n_qubits, c.n_gates, c.n_params, c.n_features, r, ps, n_ck, device};
  k.bytes.append(reinterpret_cast<const char*>(hdr), sizeof(hdr));
  if (c.n_gates)
    k.bytes.append(reinterpret_cast<const char*>(c.gates), sizeof(qs_gate) * c.n_gates);
  if (n_ck) k.bytes.append(reinterpret_cast<const char*>(ck), sizeof(int32_t) * n_ck);
  return k;
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
  (void)hipFree(d.seg_begin);
  (void)hipFree(d.seg_ckpt);
  (void)hipFree(d.ops);
  (void)hipFree(d.gates);
  (void)hipFree(d.angle_slot);
  (void)hipFree(d.slot_gate);
}

// Plans on the host and uploads once per (circuit, r, flags, device). The
// upload is synchronous, so the first call for a circuit must not be inside
// a stream capture; later calls only look the plan up.
Entry* get_plan(const qs_circuit& c, int r, bool ps, const int32_t* ck, int n_ck,
                int* rc) {
  int device = 0;
  (void)hipGetDevice(&device);
  Key key = make_key(c, r, ps, ck, n_ck, device);
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) return it->second;
  Entry* e = new Entry();
  e->device = device;
  e->host = plan_sv(c, r, ps, ck, n_ck);
  const SvPlan& P = e->host;
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
  bool okk = upload(&d.seg_map, P.seg_map.data(), P.seg_map.size()) &&
             upload(&d.seg_begin, P.seg_begin.data(), P.seg_begin.size()) &&
             upload(&d.seg_ckpt, P.seg_ckpt.data(), P.seg_ckpt.size()) &&
             upload(&d.ops, P.ops.data(), P.ops.size()) &&
             upload(&d.gates, c.gates, (size_t)c.n_gates) &&
             upload(&d.angle_slot, P.angle_slot.data(), P.angle_slot.size()) &&
             upload(&d.slot_gate, P.slot_gate.data(), P.slot_gate.size());
  if (!okk) {
    free_dev(d);
    delete e;
    *rc = QS_ERR_NOMEM;
    return nullptr;
  }
  g_cache.emplace(std::move(key), e);
  return e;
}

qs_gate* get_dev_gates(const qs_circuit& c, int* rc) {
  int device = 0;
  (void)hipGetDevice(&device);
  Key key = make_key(c, -1, false, nullptr, 0, device);
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_gate_cache.find(key);
  if (it != g_gate_cache.end()) return it->second;
  qs_gate* d = nullptr;
  if (!upload(&d, c.gates, (size_t)c.n_gates)) {
    *rc = QS_ERR_NOMEM;
    return nullptr;
  }
  g_gate_cache.emplace(std::move(key), d);
  return d;
}

int pick_path(const qs_circuit& c, int dtype, int flags, SvShape* shape,
              int n_slots, bool adjoint) {
  int path = flags & QS_PATH_MASK;
  const int rf = env_int(adjoint ? "QS_ADJ_LOG2_REGS" : "QS_FWD_LOG2_REGS", 0);
  if (path == QS_PATH_AUTO) {
    path = choose_shape(dtype, c, n_slots, rf, adjoint, shape) ? QS_PATH_FUSED
                                                                : QS_PATH_PLAIN;
  } else if (path == QS_PATH_FUSED) {
    if (!choose_shape(dtype, c, n_slots, rf, adjoint, shape)) return -QS_ERR_UNSUPPORTED;
  } else if (path == QS_PATH_HBM) {
    return -QS_ERR_UNSUPPORTED;
  } else if (path != QS_PATH_PLAIN) {
    return -QS_ERR_INVALID;
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

size_t fused_ws_bytes(const qs_circuit& c, int dtype, const SvShape& s, int64_t B,
                      bool ps) {
  if (ps) return 0;
  const size_t acc = dtype == QS_C64 ? sizeof(float) : sizeof(double);
  return (size_t)grid_of(s, B) * (size_t)(c.n_params ? c.n_params : 1) * acc;
}

}  // namespace

extern "C" {

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

int qs_forward(const qs_circuit* c, int dtype, int64_t B, const void* params,
               const void* feats, void* state, double* expz,
               const int32_t* ckpt_gates, int32_t n_ckpt, void* ckpt, int flags,
               void* stream) {
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
  SvShape shape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), false);
  if (path < 0) return -path;
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
  Entry* e = get_plan(*c, shape.r, ps, ckpt_gates, n_ckpt, &rc);
  if (!e) return rc;
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
  return launch_sv_forward(dtype, L);
}

size_t qs_workspace_size(const qs_circuit* c, int dtype, int64_t B, int flags) {
  if (validate(c) != QS_OK || B < 0) return 0;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  SvShape shape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), true);
  if (path == QS_PATH_PLAIN) return plain_workspace_bytes(*c, dtype, B);
  if (path == QS_PATH_FUSED) return fused_ws_bytes(*c, dtype, shape, B, ps);
  return 0;
}

int qs_adjoint_backward(const qs_circuit* c, int dtype, int64_t B,
                        const void* params, const void* feats, const void* state,
                        const double* dexpz, const void* dstate,
                        double* grad_params, double* grad_feats,
                        const int32_t* ckpt_gates, int32_t n_ckpt,
                        const void* ckpt, void* ws, size_t ws_bytes, int flags,
                        void* stream) {
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
  SvShape shape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), true);
  if (path < 0) return -path;
  const size_t need = path == QS_PATH_PLAIN ? plain_workspace_bytes(*c, dtype, B)
                                            : fused_ws_bytes(*c, dtype, shape, B, ps);
  if (need > 0 && (!ws || ws_bytes < need)) return QS_ERR_WORKSPACE;
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
  if (!ps && c->n_params)
    rc = launch_reduce_partials(dtype, ws, grid_of(shape, B), c->n_params,
                                grad_params, stream);
  return rc;
}

int qs_expz(int dtype, int n, int64_t B, const void* state, double* expz,
            void* stream) {
  if ((dtype != QS_C64 && dtype != QS_C128) || n < 1 || n > 30 || B < 0 || !state ||
      !expz)
    return QS_ERR_INVALID;
  return launch_expz(dtype, n, B, state, expz, stream);
}

int qs_fidelity_reset(int dtype, int n, int n_trash, int64_t B, const void* psi,
                      const void* chi, double* fid, const double* dfid,
                      void* lam_psi, void* lam_chi, void* stream) {
  if ((dtype != QS_C64 && dtype != QS_C128) || n < 1 || n > 30 || B < 0 ||
      n_trash < 0 || n_trash > 6 || n_trash >= n || !psi || !chi || !fid)
    return QS_ERR_INVALID;
  if (dfid && (!lam_psi || !lam_chi)) return QS_ERR_INVALID;
  return launch_fidelity(dtype, n, n_trash, B, psi, chi, fid, dfid, lam_psi,
                         lam_chi, stream);
}

int qs_plan_info_get(const qs_circuit* c, int dtype, int64_t B, int flags,
                     qs_plan_info* out) {
  int rc = validate(c);
  if (rc != QS_OK) return rc;
  if (!out || (dtype != QS_C64 && dtype != QS_C128)) return QS_ERR_INVALID;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  SvShape shape, ashape;
  const int path = pick_path(*c, dtype, flags, &shape, count_slots(*c, ps), false);
  if (path < 0) return -path;
  std::memset(out, 0, sizeof(*out));
  out->path = path;
  if (path != QS_PATH_FUSED) return QS_OK;
  if (pick_path(*c, dtype, flags, &ashape, count_slots(*c, ps), true) == QS_PATH_FUSED) {
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
  out->n_ops = (int32_t)P.ops.size();
  out->lds_bytes = shape.lds_bytes;
  (void)B;
  return QS_OK;
}

int qs_plan_export(const qs_circuit* c, int dtype, int64_t B, int flags,
                   qs_plan_info* info, int32_t* ops, int32_t* seg_begin,
                   uint8_t* seg_map) {
  int rc = qs_plan_info_get(c, dtype, B, flags, info);
  if (rc != QS_OK) return rc;
  if (info->path != QS_PATH_FUSED) return QS_ERR_UNSUPPORTED;
  const bool ps = (flags & QS_FLAG_PER_SAMPLE_PARAMS) != 0;
  SvPlan P = plan_sv(*c, info->log2_regs, ps, nullptr, 0);
  if (ops)
    for (size_t o = 0; o < P.ops.size(); ++o) {
      ops[4 * o] = P.ops[o].kind;
      ops[4 * o + 1] = P.ops[o].a;
      ops[4 * o + 2] = P.ops[o].b;
      ops[4 * o + 3] = P.ops[o].gate;
    }
  if (seg_begin)
    std::memcpy(seg_begin, P.seg_begin.data(), sizeof(int32_t) * P.seg_begin.size());
  if (seg_map) std::memcpy(seg_map, P.seg_map.data(), P.seg_map.size());
  return QS_OK;
}

void qs_shutdown(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& kv : g_cache) {
    free_dev(kv.second->dev);
    delete kv.second;
  }
  g_cache.clear();
  for (auto& kv : g_gate_cache) (void)hipFree(kv.second);
  g_gate_cache.clear();
}

}  // extern "C"
