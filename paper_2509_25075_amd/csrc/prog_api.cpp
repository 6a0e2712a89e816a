// Uneven batches: the qs_program_* calls. Classes of identically-structured
// circuits are planned once (cached), cut into work items of S circuits
// (S = 512 threads / threads per circuit), ordered longest first (cost
// = circuits x 2^n x gates), and run by one persistent launch that pulls
// items from an atomic queue. A class whose circuit needs more than one
// workgroup (2^n amplitudes over more than 512 threads: complex128 at 14
// qubits) runs through the batched calls on its own slices of the packed
// buffers, with per-circuit parameters; such classes go to a few
// library-owned side streams, forked from and joined back into the caller's
// stream with events, so that they overlap each other and the persistent
// launch (one class alone fills only part of the chip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "qs_internal.h"

namespace qs {
// Engine plans shared with the batched calls (qs_api.cpp).
struct ProgEnginePlan {
  SvDevPlan* dev;
};
ProgEnginePlan program_engine_plan(const qs_circuit& c, int r, int* rc);
int64_t engine_lds_bytes(int dtype, const qs_circuit& c, int S, int n_slots, int block,
                         bool ps, bool adjoint, bool half);
}  // namespace qs

using namespace qs;

namespace {

constexpr int kBlock = 512;
constexpr int64_t kMaxLds = 160 * 1024;
constexpr int64_t kStaticLds = 256;  // the persistent kernel's own __shared__ words

struct ProgPlan {
  ProgClass* d_classes = nullptr;
  ProgItem* d_items = nullptr;
  int n_items = 0;
  int* d_counter = nullptr;
  int grid = 0, r = 0, half = 0;
  int64_t lds = 0;
  int64_t* d_cum = nullptr;
  int32_t* d_nq = nullptr;
  int64_t* d_state_off = nullptr;
  int64_t n_circuits = 0;
  std::vector<int> overflow;  // classes run through the batched calls
  std::vector<int> lane;      // side stream of each overflow class
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_done;
  hipEvent_t fork = nullptr;
  void* d_ws = nullptr;       // adjoint workspace, one slice per side stream
  size_t ws_bytes = 0;        // bytes per slice
};

constexpr int kSideStreams = 3;

std::mutex g_pmu;
std::unordered_map<std::string, ProgPlan*> g_prog;

void destroy_plan(ProgPlan* pp) {
  for (hipStream_t s : pp->side)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : pp->side_done)
    if (e) (void)hipEventDestroy(e);
  if (pp->fork) (void)hipEventDestroy(pp->fork);
  (void)hipFree(pp->d_classes);
  (void)hipFree(pp->d_items);
  (void)hipFree(pp->d_counter);
  (void)hipFree(pp->d_cum);
  (void)hipFree(pp->d_nq);
  (void)hipFree(pp->d_state_off);
  (void)hipFree(pp->d_ws);
  delete pp;
}

int check_program(const qs_program* p, int dtype) {
  if (!p || p->n_classes < 1 || !p->circuits || !p->counts) return QS_ERR_INVALID;
  if (dtype != QS_C64 && dtype != QS_C128) return QS_ERR_INVALID;
  const int nlo = dtype == QS_C64 ? 5 : 4, nhi = kMaxQubitsFused;
  for (int k = 0; k < p->n_classes; ++k) {
    if (p->counts[k] < 0) return QS_ERR_INVALID;
    if (qs_validate(&p->circuits[k]) != QS_OK) return QS_ERR_INVALID;
    if (p->circuits[k].n_features != 0) return QS_ERR_UNSUPPORTED;
    if (p->circuits[k].n_qubits < nlo || p->circuits[k].n_qubits > nhi)
      return QS_ERR_UNSUPPORTED;
  }
  return QS_OK;
}

void layout(const qs_program* p, std::vector<int64_t>& so, std::vector<int64_t>& po,
            std::vector<int64_t>& eo, int64_t tot[3]) {
  so.resize(p->n_classes);
  po.resize(p->n_classes);
  eo.resize(p->n_classes);
  tot[0] = tot[1] = tot[2] = 0;
  for (int k = 0; k < p->n_classes; ++k) {
    const qs_circuit& c = p->circuits[k];
    so[k] = tot[0];
    po[k] = tot[1];
    eo[k] = tot[2];
    tot[0] += p->counts[k] << c.n_qubits;
    tot[1] += p->counts[k] * c.n_params;
    tot[2] += p->counts[k] * c.n_qubits;
  }
}

template <typename T>
bool up(T** d, const std::vector<T>& h) {
  *d = nullptr;
  const size_t bytes = sizeof(T) * (h.empty() ? 1 : h.size());
  if (hipMalloc(reinterpret_cast<void**>(d), bytes) != hipSuccess) return false;
  return h.empty() ||
         hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice) == hipSuccess;
}

ProgPlan* get_prog(const qs_program* p, int dtype, int* rc) {
  int device = 0;
  (void)hipGetDevice(&device);
  std::string key;
  int32_t hdr[3] = {p->n_classes, dtype, device};
  key.append(reinterpret_cast<const char*>(hdr), sizeof(hdr));
  for (int k = 0; k < p->n_classes; ++k) {
    const qs_circuit& c = p->circuits[k];
    int32_t ch[4] = {c.n_qubits, c.n_gates, c.n_params, c.n_features};
    key.append(reinterpret_cast<const char*>(ch), sizeof(ch));
    key.append(reinterpret_cast<const char*>(&p->counts[k]), sizeof(int64_t));
    if (c.n_gates)
      key.append(reinterpret_cast<const char*>(c.gates), sizeof(qs_gate) * c.n_gates);
  }
  {
    std::lock_guard<std::mutex> lock(g_pmu);
    auto it = g_prog.find(key);
    if (it != g_prog.end()) return it->second;
  }
  if (call_stream_capturing()) {
    *rc = QS_ERR_CAPTURE;
    return nullptr;
  }
  const int r = dtype == QS_C64 ? 5 : 4;
  std::vector<int64_t> so, po, eo;
  int64_t tot[3];
  layout(p, so, po, eo, tot);
  std::vector<ProgClass> cls(p->n_classes);
  std::vector<int64_t> cum(p->n_classes + 1, 0);
  std::vector<int32_t> nq(p->n_classes);
  struct Cand { ProgItem it; double cost; };
  std::vector<Cand> items;
  int64_t lds = 0, lds_half = 0;
  std::vector<int64_t> table_lds(p->n_classes, 0), table_lds_half(p->n_classes, 0);
  std::vector<int> overflow;
  size_t ws_bytes = 0;
  for (int k = 0; k < p->n_classes; ++k) {
    const qs_circuit& c = p->circuits[k];
    cum[k + 1] = cum[k] + p->counts[k];
    nq[k] = c.n_qubits;
    if ((kBlock >> (c.n_qubits - r)) < 1) {
      overflow.push_back(k);
      std::memset(&cls[k], 0, sizeof(ProgClass));
      ws_bytes = std::max(ws_bytes, qs_workspace_size(&c, dtype, p->counts[k],
                                                      QS_FLAG_PER_SAMPLE_PARAMS));
      continue;
    }
    ProgEnginePlan ep = program_engine_plan(c, r, rc);
    if (!ep.dev) return nullptr;
    ProgClass& d = cls[k];
    std::memset(&d, 0, sizeof(d));
    d.seg_map = ep.dev->seg_map;
    d.seg_lay = ep.dev->seg_lay;
    d.seg_begin = ep.dev->seg_begin;
    d.seg_ckpt = ep.dev->seg_ckpt;
    d.ops = ep.dev->ops;
    d.gates = ep.dev->gates;
    d.gate_slot = ep.dev->gate_slot;
    d.slot_gate = ep.dev->slot_gate;
    d.l1q = ep.dev->l1q;
    d.diag = ep.dev->diag;
    d.blk_begin = ep.dev->blk_begin;
    d.blk_rec = ep.dev->blk_rec;
    d.blk_fu = ep.dev->blk_fu;
    d.blk_gen = ep.dev->blk_gen;
    d.n_blocks = ep.dev->n_blocks;
    d.n_fu = ep.dev->n_fu;
    d.n_gen = ep.dev->n_gen;
    d.ryrz = dtype == QS_C64 ? ep.dev->ryrz : 0;
    d.n = c.n_qubits;
    d.t = c.n_qubits - r;
    d.nseg = ep.dev->nseg;
    d.n_gates = c.n_gates;
    d.n_slots = ep.dev->n_slots;
    d.n_params = c.n_params;
    d.S = kBlock >> d.t;
    d.count = p->counts[k];
    d.state_off = so[k];
    d.param_off = po[k];
    d.expz_off = eo[k];
    lds = std::max(lds, engine_lds_bytes(dtype, c, d.S, 0, kBlock, true, true, false));
    lds_half = std::max(lds_half, engine_lds_bytes(dtype, c, d.S, 0, kBlock, true, true, true));
    table_lds[k] = engine_lds_bytes(dtype, c, d.S, d.n_slots, kBlock, true, true, false);
    table_lds_half[k] = engine_lds_bytes(dtype, c, d.S, d.n_slots, kBlock, true, true, true);
    for (int64_t f = 0; f < d.count; f += d.S) {
      const int64_t m = std::min<int64_t>(d.S, d.count - f);
      items.push_back({{k, (int32_t)f}, (double)m * (double)(1ll << d.n) *
                                            (double)(c.n_gates > 0 ? c.n_gates : 1)});
    }
  }
  // Whole-amplitude staging when the largest class fits it, else one state
  // component at a time (half the staging LDS).
  int half = 0;
  if (lds > kMaxLds) {
    half = 1;
    lds = lds_half;
  }
  if (lds > kMaxLds) {
    *rc = QS_ERR_UNSUPPORTED;
    return nullptr;
  }
  // Classes whose per-circuit angle table fits next to the staging (within
  // the one workgroup per CU the staging already implies) take the table
  // path; the launch's LDS grows to the largest such class.
  const int64_t per_cu_fly = std::max<int64_t>(1, std::min<int64_t>(4, kMaxLds / std::max<int64_t>(lds, 1)));
  const int64_t budget = kMaxLds / per_cu_fly - kStaticLds;
  if (lds <= budget && dtype == QS_C64) {
    for (int k = 0; k < p->n_classes; ++k) {
      const int64_t need = half ? table_lds_half[k] : table_lds[k];
      if (cls[k].S > 0 && cls[k].n_slots > 0 && need <= budget) {
        cls[k].table = 1;
        lds = std::max(lds, need);
      }
    }
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const Cand& a, const Cand& b) { return a.cost > b.cost; });
  std::vector<ProgItem> its;
  for (const Cand& c : items) its.push_back(c.it);
  ProgPlan* pp = new ProgPlan();
  pp->n_items = (int)its.size();
  pp->r = r;
  pp->half = half;
  pp->lds = lds;
  pp->n_circuits = cum.back();
  pp->overflow = overflow;
  pp->ws_bytes = (ws_bytes + 255) & ~(size_t)255;
  // Overflow classes, longest first, each to the least-loaded side stream.
  const int n_side = std::min<int>(kSideStreams, (int)overflow.size());
  if (n_side > 0) {
    std::vector<double> load(n_side, 0.0);
    std::vector<int> order(overflow.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    auto cost = [&](int i) {
      const qs_circuit& c = p->circuits[overflow[i]];
      return (double)p->counts[overflow[i]] * (double)(1ll << c.n_qubits) * (c.n_gates + 1);
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cost(a) > cost(b); });
    pp->lane.assign(overflow.size(), 0);
    for (int i : order) {
      const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      pp->lane[i] = s;
      load[s] += cost(i);
    }
    pp->side.assign(n_side, nullptr);
    pp->side_done.assign(n_side, nullptr);
    bool okk = hipEventCreateWithFlags(&pp->fork, hipEventDisableTiming) == hipSuccess;
    for (int s = 0; s < n_side && okk; ++s)
      okk = hipStreamCreateWithFlags(&pp->side[s], hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&pp->side_done[s], hipEventDisableTiming) == hipSuccess;
    if (!okk) {
      destroy_plan(pp);
      *rc = QS_ERR_LAUNCH;
      return nullptr;
    }
  }
  hipDeviceProp_t prop;
  int cus = 256;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) cus = prop.multiProcessorCount;
  const int per_cu = std::max<int>(1, std::min<int>(4, (int)(kMaxLds / std::max<int64_t>(lds, 1))));
  pp->grid = std::max(1, std::min(pp->n_items, cus * per_cu));
  std::vector<int32_t> zero(1, 0);
  if (!up(&pp->d_classes, cls) || !up(&pp->d_items, its) || !up(&pp->d_counter, zero) ||
      !up(&pp->d_cum, cum) || !up(&pp->d_nq, nq) || !up(&pp->d_state_off, so) ||
      (pp->ws_bytes && hipMalloc(&pp->d_ws, pp->ws_bytes * pp->side.size()) != hipSuccess)) {
    destroy_plan(pp);
    *rc = QS_ERR_NOMEM;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_pmu);
  auto ins = g_prog.emplace(key, pp);
  if (!ins.second) {  // planned meanwhile by another thread: keep that one
    destroy_plan(pp);
    return ins.first->second;
  }
  return pp;
}

int run_persistent(ProgPlan* pp, int dtype, const void* params, void* states, double* expz,
                   const double* dexpz, double* grad, bool adjoint, void* stream);

int run(const qs_program* p, int dtype, const void* params, void* states,
        double* expz, const double* dexpz, double* grad, bool adjoint, void* stream) {
  int rc = QS_OK;
  ProgPlan* pp = get_prog(p, dtype, &rc);
  if (!pp) return rc;
  int64_t tot[3];
  std::vector<int64_t> so, po, eo;
  layout(p, so, po, eo, tot);
  if (adjoint && tot[1] && (rc = launch_fill_f64(grad, tot[1], stream)) != QS_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool forked = !pp->side.empty();
  if (forked) {
    if (hipEventRecord(pp->fork, st) != hipSuccess) return QS_ERR_LAUNCH;
    for (hipStream_t s : pp->side)
      if (hipStreamWaitEvent(s, pp->fork, 0) != hipSuccess) return QS_ERR_LAUNCH;
  }
  rc = run_persistent(pp, dtype, params, states, expz, dexpz, grad, adjoint, stream);
  // Classes beyond one workgroup, each through the batched path on its slices,
  // on the side streams.
  const size_t rs = dtype == QS_C64 ? sizeof(float) : sizeof(double);
  for (size_t i = 0; i < pp->overflow.size() && rc == QS_OK; ++i) {
    const int k = pp->overflow[i];
    const qs_circuit& c = p->circuits[k];
    const int64_t B = p->counts[k];
    if (B == 0) continue;
    hipStream_t s = pp->side[pp->lane[i]];
    void* ws = static_cast<char*>(pp->d_ws) + pp->ws_bytes * pp->lane[i];
    const void* pk = static_cast<const char*>(params) + rs * po[k];
    void* sk = static_cast<char*>(states) + 2 * rs * so[k];
    if (adjoint)
      rc = qs_adjoint_backward(&c, dtype, B, pk, nullptr, sk, dexpz + eo[k], nullptr,
                               grad + po[k], nullptr, nullptr, 0, nullptr, ws,
                               pp->ws_bytes, QS_FLAG_PER_SAMPLE_PARAMS, s);
    else
      rc = qs_forward(&c, dtype, B, pk, nullptr, sk, expz ? expz + eo[k] : nullptr, nullptr,
                      0, nullptr, QS_FLAG_PER_SAMPLE_PARAMS, s);
  }
  // Join every side stream back into the caller's, also after an error.
  if (forked) {
    for (size_t s = 0; s < pp->side.size(); ++s)
      if (hipEventRecord(pp->side_done[s], pp->side[s]) != hipSuccess ||
          hipStreamWaitEvent(st, pp->side_done[s], 0) != hipSuccess)
        return QS_ERR_LAUNCH;
  }
  return rc;
}

int run_persistent(ProgPlan* pp, int dtype, const void* params, void* states, double* expz,
                   const double* dexpz, double* grad, bool adjoint, void* stream) {
  int rc = QS_OK;
  if (pp->n_items == 0) return QS_OK;
  if ((rc = launch_zero_i32(pp->d_counter, stream)) != QS_OK) return rc;
  ProgLaunch L{};
  L.classes = pp->d_classes;
  L.items = pp->d_items;
  L.n_items = pp->n_items;
  L.counter = pp->d_counter;
  L.grid = pp->grid;
  L.block = kBlock;
  L.r = pp->r;
  L.half = pp->half;
  L.lds_bytes = pp->lds;
  L.params = params;
  L.states = states;
  L.expz = expz;
  L.dexpz = dexpz;
  L.grad_params = grad;
  L.stream = stream;
  return launch_program(dtype, L, adjoint);
}

}  // namespace

namespace qs {
// Releases every program plan (device tables, queue counter, side streams,
// events, workspace). Program plans point into the engine plan cache, so
// they go first when the library releases its caches.
void free_programs() {
  std::lock_guard<std::mutex> lock(g_pmu);
  for (auto& kv : g_prog) destroy_plan(kv.second);
  g_prog.clear();
}
}  // namespace qs

extern "C" {

int qs_program_layout(const qs_program* p, int64_t* state_off, int64_t* param_off,
                      int64_t* expz_off, int64_t* totals) {
  if (!p || p->n_classes < 1 || !p->circuits || !p->counts) return QS_ERR_INVALID;
  std::vector<int64_t> so, po, eo;
  int64_t tot[3];
  layout(p, so, po, eo, tot);
  if (state_off) std::memcpy(state_off, so.data(), sizeof(int64_t) * so.size());
  if (param_off) std::memcpy(param_off, po.data(), sizeof(int64_t) * po.size());
  if (expz_off) std::memcpy(expz_off, eo.data(), sizeof(int64_t) * eo.size());
  if (totals) std::memcpy(totals, tot, sizeof(tot));
  return QS_OK;
}

int qs_program_encode(const qs_program* p, int dtype, const void* x, int x_is_f64,
                      void* states, int32_t* bad_rows, void* stream) {
  CallStream call_(stream);
  int rc = check_program(p, dtype);
  if (rc != QS_OK) return rc;
  if (!x || !states) return QS_ERR_INVALID;
  ProgPlan* pp = get_prog(p, dtype, &rc);
  if (!pp) return rc;
  return launch_program_encode(dtype, p->n_classes, pp->d_cum, pp->d_nq,
                               pp->d_state_off, pp->n_circuits, x, x_is_f64, states,
                               bad_rows, stream);
}

int qs_program_forward(const qs_program* p, int dtype, const void* params,
                       void* states, double* expz, void* stream) {
  CallStream call_(stream);
  int rc = check_program(p, dtype);
  if (rc != QS_OK) return rc;
  if (!states || !params) return QS_ERR_INVALID;
  return run(p, dtype, params, states, expz, nullptr, nullptr, false, stream);
}

int qs_program_adjoint(const qs_program* p, int dtype, const void* params,
                       const void* states, const double* dexpz, double* grad_params,
                       void* stream) {
  CallStream call_(stream);
  int rc = check_program(p, dtype);
  if (rc != QS_OK) return rc;
  if (!states || !params || !dexpz || !grad_params) return QS_ERR_INVALID;
  return run(p, dtype, params, const_cast<void*>(states), nullptr, dexpz, grad_params,
             true, stream);
}

}  // extern "C"
