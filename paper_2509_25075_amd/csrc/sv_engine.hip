// Register-resident batched state-vector engine for gfx950 (forward and
// adjoint).
//
// Layout. A sample's 2^n amplitudes live in the registers of T = 2^t
// threads, R = 2^r amplitudes per thread (n = r + t). Physical index of
// amplitude k of thread tau is k + R * tau, so physical bits 0..r-1 are
// register bits and r..n-1 are thread bits. A segment of the planned gate
// program fixes which logical qubit sits on which physical bit; every
// pair-mixing gate of a segment targets a register bit, so it is applied
// with no communication. Diagonal gates (RZ, Z, CZ) and CNOT controls on
// thread bits use the lane's own bit. Between segments the state is written
// to LDS in logical order and read back under the next placement (a remap).
//
// LDS slots are swizzled, slot(L) = L ^ fold5(L >> 5) ^ (per-sample salt),
// which is linear over GF(2), so the address of amplitude k of a lane is
// (per-lane part) XOR (uniform per-k part): one VALU op per access.
//
// Gates: R_P(t) = exp(-i t P / 2) (Nielsen & Chuang sec. 4.2); the adjoint
// step computes dL/dtheta = Im <lam|P|psi> and un-applies the gate from psi
// and lam (Jones & Gacon, arXiv:2009.02823, sec. 3).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "qs_internal.h"

namespace qs {
namespace {

#define QS_AI __attribute__((always_inline))

template <int V>
using IC = std::integral_constant<int, V>;

// ------------------------------------------------------------------ wave ops
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  long long u = __double_as_longlong(v);
  int lo = (int)(u & 0xffffffffll), hi = (int)(u >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) { return dpp_f32<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ double dpp(double v) { return dpp_f64<CTRL>(v); }

// Sum over aligned groups of G lanes (G a power of two, 1..64, uniform);
// every lane of a group receives the group's sum. Requires a full wave.
template <typename real>
__device__ __forceinline__ real group_sum(real v, int G) {
  if (G >= 2) v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]  (lane ^ 1)
  if (G >= 4) v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]  (lane ^ 2)
  if (G >= 8) v += dpp<0x141>(v);  // row_half_mirror: the other quad of 8
  if (G >= 16) v += dpp<0x140>(v); // row_mirror: the other 8 of a row
  if (G >= 32) v += __shfl_xor(v, 16);
  if (G >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Plan data is read-only for the whole launch: reading it through the
// constant address space lets uniform indices become scalar loads.
#define QS_K __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const QS_K T* kc(const T* p) {
  return (const QS_K T*)p;
}

// Load a plan record (SvOp, qs_gate) word by word through the constant
// address space.
template <typename T>
__device__ __forceinline__ T kload(const T* base, int i) {
  static_assert(sizeof(T) % 4 == 0, "record of 32-bit words");
  T out;
  uint32_t* o = reinterpret_cast<uint32_t*>(&out);
  const QS_K uint32_t* src = reinterpret_cast<const QS_K uint32_t*>(kc(base + i));
#pragma unroll
  for (int w = 0; w < (int)(sizeof(T) / 4); ++w) o[w] = src[w];
  return out;
}

__device__ __forceinline__ int uni(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// Slot swizzle inside a sample's LDS region (in complex elements).
__device__ __forceinline__ uint32_t swz(uint32_t L) {
  return L ^ ((L >> 5) & 31u) ^ ((L >> 10) & 31u);
}

// --------------------------------------------------------------- state ops
// Amplitudes of one thread: R-wide vector values (not arrays), so branches
// that touch different elements can never be merged into a pointer select
// that would push the state out of registers.
template <typename real, int R>
struct St {
  typedef real V __attribute__((ext_vector_type(R)));
  V re;
  V im;
};

// Dispatch a uniform runtime position j in [0, LR) to a compile-time one.
template <int LR, typename F>
__device__ __forceinline__ void for_pos(int j, F&& f) {
  if constexpr (LR > 0) { if (j == 0) { f(IC<0>{}); return; } }
  if constexpr (LR > 1) { if (j == 1) { f(IC<1>{}); return; } }
  if constexpr (LR > 2) { if (j == 2) { f(IC<2>{}); return; } }
  if constexpr (LR > 3) { if (j == 3) { f(IC<3>{}); return; } }
  if constexpr (LR > 4) { if (j == 4) { f(IC<4>{}); return; } }
}

// RX(theta) = [[c, -i s], [-i s, c]] on register bit J (s may carry the sign
// of an inverse).
template <int J, typename real, int R>
__device__ __forceinline__ void g_rx(St<real, R>& x, real c, real s) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    real a0r = x.re[k], a0i = x.im[k], a1r = x.re[k1], a1i = x.im[k1];
    x.re[k] = c * a0r + s * a1i;
    x.im[k] = c * a0i - s * a1r;
    x.re[k1] = c * a1r + s * a0i;
    x.im[k1] = c * a1i - s * a0r;
  }
}
// RY(theta) = [[c, -s], [s, c]].
template <int J, typename real, int R>
__device__ __forceinline__ void g_ry(St<real, R>& x, real c, real s) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    real a0r = x.re[k], a0i = x.im[k], a1r = x.re[k1], a1i = x.im[k1];
    x.re[k] = c * a0r - s * a1r;
    x.im[k] = c * a0i - s * a1i;
    x.re[k1] = s * a0r + c * a1r;
    x.im[k1] = s * a0i + c * a1i;
  }
}
// RZ(theta) = diag(c - i s, c + i s) on register bit J.
template <int J, typename real, int R>
__device__ __forceinline__ void g_rz(St<real, R>& x, real c, real s) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const real sk = (k & (1 << J)) ? s : -s;  // phase c + i sk
    real ar = x.re[k], ai = x.im[k];
    x.re[k] = c * ar - sk * ai;
    x.im[k] = c * ai + sk * ar;
  }
}
// A lane-uniform phase c + i s on every amplitude (RZ on a thread bit).
template <typename real, int R>
__device__ __forceinline__ void g_phase_all(St<real, R>& x, real c, real s) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    real ar = x.re[k], ai = x.im[k];
    x.re[k] = c * ar - s * ai;
    x.im[k] = c * ai + s * ar;
  }
}
template <int J, typename real, int R>
__device__ __forceinline__ void g_x(St<real, R>& x) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    real tr = x.re[k], ti = x.im[k];
    x.re[k] = x.re[k1];
    x.im[k] = x.im[k1];
    x.re[k1] = tr;
    x.im[k1] = ti;
  }
}
// Y = [[0, -i], [i, 0]]: (a0, a1) -> (-i a1, i a0).
template <int J, typename real, int R>
__device__ __forceinline__ void g_y(St<real, R>& x) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    real a0r = x.re[k], a0i = x.im[k], a1r = x.re[k1], a1i = x.im[k1];
    x.re[k] = a1i;
    x.im[k] = -a1r;
    x.re[k1] = -a0i;
    x.im[k1] = a0r;
  }
}
template <int J, typename real, int R>
__device__ __forceinline__ void g_z(St<real, R>& x) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (!(k & (1 << J))) continue;
    x.re[k] = -x.re[k];
    x.im[k] = -x.im[k];
  }
}
template <int J, typename real, int R>
__device__ __forceinline__ void g_h(St<real, R>& x) {
  const real h = (real)0.70710678118654752440;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    real a0r = x.re[k], a0i = x.im[k], a1r = x.re[k1], a1i = x.im[k1];
    x.re[k] = h * (a0r + a1r);
    x.im[k] = h * (a0i + a1i);
    x.re[k1] = h * (a0r - a1r);
    x.im[k1] = h * (a0i - a1i);
  }
}
// Negate every amplitude of lanes where `cond` holds.
template <typename real, int R>
__device__ __forceinline__ void g_neg_if(St<real, R>& x, bool cond) {
  const real sg = cond ? (real)-1 : (real)1;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    x.re[k] *= sg;
    x.im[k] *= sg;
  }
}
// CZ between register bits A < B.
template <int A, int B, typename real, int R>
__device__ __forceinline__ void g_cz_rr(St<real, R>& x) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if ((k & (1 << A)) && (k & (1 << B))) {
      x.re[k] = -x.re[k];
      x.im[k] = -x.im[k];
    }
  }
}
// CZ between register bit A and a thread bit whose value is `tb`.
template <int A, typename real, int R>
__device__ __forceinline__ void g_cz_rt(St<real, R>& x, bool tb) {
  const real sg = tb ? (real)-1 : (real)1;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << A)) {
      x.re[k] *= sg;
      x.im[k] *= sg;
    }
  }
}
// CNOT, control register bit C, target register bit J.
template <int C, int J, typename real, int R>
__device__ __forceinline__ void g_cnot_rr(St<real, R>& x) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if ((k & (1 << J)) || !(k & (1 << C))) continue;
    const int k1 = k | (1 << J);
    real tr = x.re[k], ti = x.im[k];
    x.re[k] = x.re[k1];
    x.im[k] = x.im[k1];
    x.re[k1] = tr;
    x.im[k1] = ti;
  }
}
// CNOT, control on a thread bit (value tb), target register bit J.
template <int J, typename real, int R>
__device__ __forceinline__ void g_cnot_tr(St<real, R>& x, bool tb) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    real a0r = x.re[k], a0i = x.im[k], a1r = x.re[k1], a1i = x.im[k1];
    x.re[k] = tb ? a1r : a0r;
    x.im[k] = tb ? a1i : a0i;
    x.re[k1] = tb ? a0r : a1r;
    x.im[k1] = tb ? a0i : a1i;
  }
}

// Per-thread partial sums of Im <lam|P|psi> for the rotation generators.
template <int J, typename real, int R>
__device__ __forceinline__ real gr_x(const St<real, R>& p, const St<real, R>& l) {
  real acc = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    // Im(conj(l0) p1 + conj(l1) p0)
    acc += l.re[k] * p.im[k1] - l.im[k] * p.re[k1];
    acc += l.re[k1] * p.im[k] - l.im[k1] * p.re[k];
  }
  return acc;
}
template <int J, typename real, int R>
__device__ __forceinline__ real gr_y(const St<real, R>& p, const St<real, R>& l) {
  real acc = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    // Im(conj(l0)(-i p1) + conj(l1)(i p0)) = -Re(conj(l0) p1) + Re(conj(l1) p0)
    acc += l.re[k1] * p.re[k] + l.im[k1] * p.im[k];
    acc -= l.re[k] * p.re[k1] + l.im[k] * p.im[k1];
  }
  return acc;
}
template <int J, typename real, int R>
__device__ __forceinline__ real gr_z(const St<real, R>& p, const St<real, R>& l) {
  real acc = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    real v = l.re[k] * p.im[k] - l.im[k] * p.re[k];  // Im(conj(l) p)
    acc += (k & (1 << J)) ? -v : v;
  }
  return acc;
}
template <typename real, int R>
__device__ __forceinline__ real gr_all(const St<real, R>& p, const St<real, R>& l) {
  real acc = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) acc += l.re[k] * p.im[k] - l.im[k] * p.re[k];
  return acc;
}

// ------------------------------------------------------------- kernel args
template <typename real>
struct Args {
  const uint8_t* seg_map;
  const int32_t* seg_begin;
  const int32_t* seg_ckpt;
  const SvOp* ops;
  const qs_gate* gates;
  const int32_t* angle_slot;
  const int32_t* slot_gate;
  int n, t, nseg, n_gates, n_slots, n_params, n_feats, S;
  int per_sample_params;
  int64_t B;               // samples processed (tiled: batch rows << ob)
  int n_tot, ob;           // tiled: qubits of the whole state, outer bits
  const uint8_t* tile_q;   // tiled: [n] global qubit of each local bit
  const uint8_t* outer_q;  // tiled: [ob] global qubit of each outer bit
  real* out_psi;           // adjoint: store the final psi here (or null)
  real* out_lam;           // adjoint: store the final lam here (or null)
  const real* params;
  const real* feats;
  real* state;
  double* expz;
  real* ckpt;
  const double* dexpz;
  const real* dstate;
  real* ws_partials;
  double* grad_params;
  double* grad_feats;
};

template <typename real>
struct V2;
template <>
struct V2<float> { using T = float2; };
template <>
struct V2<double> { using T = double2; };

__device__ __forceinline__ void fsincos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void fsincos(double x, double* s, double* c) { sincos(x, s, c); }

template <typename real>
__device__ __forceinline__ const real* param_row(const Args<real>& A, int64_t b) {
  return A.per_sample_params ? A.params + (size_t)b * A.n_params : A.params;
}

template <typename real>
__device__ __forceinline__ real theta_of(const Args<real>& A, const qs_gate& g,
                                         int64_t b) {
  const real* P = param_row(A, b);
  real w = g.p_w >= 0 ? P[g.p_w] : (real)1;
  real f = g.feat >= 0 ? A.feats[(size_t)b * A.n_feats + g.feat] : (real)1;
  real bias = g.p_b >= 0 ? P[g.p_b] : (real)0;
  return (real)g.scale * (w * f + bias);
}

// Per-sample sync: a wave barrier when a sample lives in one wave,
// otherwise a workgroup barrier (T is uniform over the workgroup).
__device__ __forceinline__ void sample_sync(int t) {
  if (t > 6) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// The engine's per-thread context.
template <typename real, int LR, bool FLY = false>
struct Ctx {
  static constexpr int R = 1 << LR;
  using v2 = typename V2<real>::T;
  const Args<real>& A;
  int tau, sl;       // thread within sample, sample within block
  int64_t b;         // global sample index
  int64_t row;       // batch row of the sample (for parameters and features)
  int64_t base;      // offset (complex elements) of the sample's amplitude 0
  uint32_t dep_tau;  // tiled: global offset of this thread's low local bits
  bool active;
  v2* lds;           // this sample's state region
  uint32_t salt;     // per-sample slot salt
  real* ang_sh;      // [G][2] shared (cos, sin) of theta/2
  real* ang_ps;      // [n_slots][S][2] per-sample
  real* gacc;        // [waves][n_params] shared-parameter gradient sums
  real* facc;        // [S * wps][n_feats] feature gradient sums
  int wps;           // waves per sample (1 when a wave holds whole samples)

  __device__ Ctx(const Args<real>& a) : A(a) {}

  __device__ __forceinline__ bool tbit(int p) const {
    return (tau >> (p - LR)) & 1;
  }

  // Logical index bits of this thread's thread-bit part under placement s.
  __device__ __forceinline__ uint32_t lane_part(const QS_K uint8_t* map) const {
    uint32_t L = 0;
    for (int i = 0; i < A.t; ++i)
      if ((tau >> i) & 1) L |= 1u << map[LR + i];
    return swz(L) ^ salt;
  }

  __device__ __forceinline__ void write_mapped(const St<real, R>& x,
                                               const QS_K uint8_t* map) {
    const uint32_t base = lane_part(map);
    uint32_t m[LR > 0 ? LR : 1];
#pragma unroll
    for (int j = 0; j < LR; ++j) m[j] = swz(1u << uni(map[j]));
#pragma unroll
    for (int k = 0; k < R; ++k) {
      uint32_t off = 0;
#pragma unroll
      for (int j = 0; j < LR; ++j)
        if (k & (1 << j)) off ^= m[j];
      v2 v;
      v.x = x.re[k];
      v.y = x.im[k];
      lds[base ^ off] = v;
    }
  }
  __device__ __forceinline__ void read_mapped(St<real, R>& x,
                                              const QS_K uint8_t* map) {
    const uint32_t base = lane_part(map);
    uint32_t m[LR > 0 ? LR : 1];
#pragma unroll
    for (int j = 0; j < LR; ++j) m[j] = swz(1u << uni(map[j]));
#pragma unroll
    for (int k = 0; k < R; ++k) {
      uint32_t off = 0;
#pragma unroll
      for (int j = 0; j < LR; ++j)
        if (k & (1 << j)) off ^= m[j];
      v2 v = lds[base ^ off];
      x.re[k] = v.x;
      x.im[k] = v.y;
    }
  }
  __device__ __forceinline__ void remap(St<real, R>& x, const QS_K uint8_t* from,
                                        const QS_K uint8_t* to) {
    sample_sync(A.t);
    write_mapped(x, from);
    sample_sync(A.t);
    read_mapped(x, to);
  }

  // Global offset (complex elements) of local amplitude i = tau + x, x a
  // multiple of T: the sample's base plus the local bits deposited onto the
  // tile's qubits (identity when not tiled).
  __device__ __forceinline__ int64_t addr(int x) const {
    if (A.tile_q == nullptr) return base + tau + x;
    int64_t d = dep_tau;
    for (int j = A.t; j < A.n; ++j)
      if ((x >> j) & 1) d |= 1ll << kc(A.tile_q)[j];
    return base + d;
  }

  // HBM (logical order) -> LDS -> registers under placement `map`.
  __device__ __forceinline__ void load_state(St<real, R>& x, const real* src,
                                             const QS_K uint8_t* map) {
    const int N = 1 << A.n, T = 1 << A.t;
    sample_sync(A.t);
    const v2* s2 = reinterpret_cast<const v2*>(src);
    for (int i = tau; i < N; i += T) {
      v2 v;
      if (active) {
        v = s2[addr(i - tau)];
      } else {
        v.x = 0;
        v.y = 0;
      }
      lds[swz((uint32_t)i) ^ salt] = v;
    }
    sample_sync(A.t);
    read_mapped(x, map);
  }
  // Registers under `map` -> LDS -> HBM (logical order).
  __device__ __forceinline__ void store_state(const St<real, R>& x, real* dst,
                                              const QS_K uint8_t* map) {
    const int N = 1 << A.n, T = 1 << A.t;
    sample_sync(A.t);
    write_mapped(x, map);
    sample_sync(A.t);
    if (active) {
      v2* d2 = reinterpret_cast<v2*>(dst);
      for (int i = tau; i < N; i += T) d2[addr(i - tau)] = lds[swz((uint32_t)i) ^ salt];
    }
  }

  // cos, sin of theta/2 for op number o (op o comes from gate o).
  __device__ __forceinline__ void angle(int o, const SvOp& op, real& c, real& s) const {
    if constexpr (FLY) {
      if (op.aux & 1) {
        // per-sample angle computed in place (no per-sample table in LDS)
        const qs_gate gt = kload(A.gates, op.gate);
        const real th = active ? theta_of(A, gt, row) : (real)0;
        fsincos(th * (real)0.5, &s, &c);
        return;
      }
    }
    if (op.aux & 1) {
      const int slot = kc(A.angle_slot)[o];
      const real* p = ang_ps + 2 * ((size_t)slot * A.S + sl);
      c = p[0];
      s = p[1];
    } else {
      c = ang_sh[2 * o];
      s = ang_sh[2 * o + 1];
    }
  }

  // Apply op (its inverse when `inv`) to x. For rotations (c, s) are
  // cos, sin of theta/2 already signed for the direction.
  __device__ __forceinline__ void apply(St<real, R>& x, int kind, int a, int bq,
                                        real c, real s) const {
    switch (kind) {
      case QS_OP_RX:
        for_pos<LR>(a, [&](auto J) QS_AI { g_rx<decltype(J)::value>(x, c, s); });
        break;
      case QS_OP_RY:
        for_pos<LR>(a, [&](auto J) QS_AI { g_ry<decltype(J)::value>(x, c, s); });
        break;
      case QS_OP_RZ:
        if (a < LR)
          for_pos<LR>(a, [&](auto J) QS_AI { g_rz<decltype(J)::value>(x, c, s); });
        else
          g_phase_all(x, c, tbit(a) ? s : -s);
        break;
      case QS_OP_X:
        for_pos<LR>(a, [&](auto J) QS_AI { g_x<decltype(J)::value>(x); });
        break;
      case QS_OP_Y:
        for_pos<LR>(a, [&](auto J) QS_AI { g_y<decltype(J)::value>(x); });
        break;
      case QS_OP_Z:
        if (a < LR)
          for_pos<LR>(a, [&](auto J) QS_AI { g_z<decltype(J)::value>(x); });
        else
          g_neg_if(x, tbit(a));
        break;
      case QS_OP_H:
        for_pos<LR>(a, [&](auto J) QS_AI { g_h<decltype(J)::value>(x); });
        break;
      case QS_OP_CNOT:  // a = control, bq = target (register)
        if (a < LR) {
          for_pos<LR>(a, [&](auto C) QS_AI {
            for_pos<LR>(bq, [&](auto J) QS_AI {
              if constexpr (decltype(C)::value != decltype(J)::value)
                g_cnot_rr<decltype(C)::value, decltype(J)::value>(x);
            });
          });
        } else {
          const bool tb = tbit(a);
          for_pos<LR>(bq, [&](auto J) QS_AI { g_cnot_tr<decltype(J)::value>(x, tb); });
        }
        break;
      case QS_OP_CZ: {
        int lo = a < bq ? a : bq, hi = a < bq ? bq : a;
        if (hi < LR) {
          for_pos<LR>(lo, [&](auto A0) QS_AI {
            for_pos<LR>(hi, [&](auto B0) QS_AI {
              if constexpr (decltype(A0)::value < decltype(B0)::value)
                g_cz_rr<decltype(A0)::value, decltype(B0)::value>(x);
            });
          });
        } else if (lo < LR) {
          const bool tb = tbit(hi);
          for_pos<LR>(lo, [&](auto A0) QS_AI { g_cz_rt<decltype(A0)::value>(x, tb); });
        } else {
          g_neg_if(x, tbit(lo) && tbit(hi));
        }
        break;
      }
      default:
        break;
    }
  }

  __device__ __forceinline__ real grad_partial(int kind, int a,
                                               const St<real, R>& p,
                                               const St<real, R>& l) const {
    real v = 0;
    switch (kind) {
      case QS_OP_RX:
        for_pos<LR>(a, [&](auto J) QS_AI { v = gr_x<decltype(J)::value>(p, l); });
        break;
      case QS_OP_RY:
        for_pos<LR>(a, [&](auto J) QS_AI { v = gr_y<decltype(J)::value>(p, l); });
        break;
      default:  // RZ
        if (a < LR)
          for_pos<LR>(a, [&](auto J) QS_AI { v = gr_z<decltype(J)::value>(p, l); });
        else
          v = tbit(a) ? -gr_all(p, l) : gr_all(p, l);
        break;
    }
    return v;
  }
};

// Common prologue: LDS carve-up and angle tables.
// `blk` is the global index of the block's first sample. Gradient sums are
// kept in per-wave LDS slots (each written by one lane of one wave) and added
// in a fixed order at the end, so the adjoint is bitwise reproducible.
template <typename real, int LR, bool FLY>
__device__ __forceinline__ void setup(Ctx<real, LR, FLY>& C, const Args<real>& A,
                                      unsigned char* smem, bool adjoint, int64_t blk) {
  const int tid = threadIdx.x;
  const int N = 1 << A.n;
  C.tau = tid & ((1 << A.t) - 1);
  C.sl = tid >> A.t;
  C.b = blk + C.sl;
  C.active = C.b < A.B;
  C.row = C.b >> A.ob;
  if (A.tile_q == nullptr) {
    C.base = C.b * (int64_t)N;
    C.dep_tau = 0;
  } else {
    const int64_t outer = C.b & ((1ll << A.ob) - 1);
    int64_t o = C.row << A.n_tot;
    for (int k = 0; k < A.ob; ++k)
      if ((outer >> k) & 1) o |= 1ll << kc(A.outer_q)[k];
    C.base = o;
    uint32_t d = 0;
    for (int j = 0; j < A.t; ++j)
      if ((C.tau >> j) & 1) d |= 1u << kc(A.tile_q)[j];
    C.dep_tau = d;
  }
  using v2 = typename V2<real>::T;
  v2* st = reinterpret_cast<v2*>(smem);
  C.lds = st + (size_t)C.sl * N;
  C.salt = ((uint32_t)C.sl << A.t) & 31u & (uint32_t)(N - 1);
  real* tail = reinterpret_cast<real*>(st + (size_t)A.S * N);
  C.ang_sh = tail;
  C.ang_ps = C.ang_sh + 2 * (size_t)A.n_gates;
  C.gacc = C.ang_ps + (FLY ? 0 : 2 * (size_t)A.n_slots * A.S);
  C.wps = A.t > 6 ? (1 << (A.t - 6)) : 1;
  const int waves = blockDim.x >> 6;
  C.facc = C.gacc + (A.per_sample_params ? 0 : (size_t)waves * A.n_params);

  // Shared angles in op order (op o applies gate ops[o].gate).
  for (int o = tid; o < A.n_gates; o += blockDim.x) {
    const qs_gate gt = kload(A.gates, kload(A.ops, o).gate);
    real c = 1, s = 0;
    if ((gt.op == QS_OP_RX || gt.op == QS_OP_RY || gt.op == QS_OP_RZ) &&
        kc(A.angle_slot)[o] < 0) {
      real th = theta_of(A, gt, 0);  // shared: no feature, shared params
      fsincos(th * (real)0.5, &s, &c);
    }
    C.ang_sh[2 * o] = c;
    C.ang_sh[2 * o + 1] = s;
  }
  for (int i = tid; i < (FLY ? 0 : A.n_slots * A.S); i += blockDim.x) {
    const int slot = i / A.S, s_l = i % A.S;
    const int64_t bb = blk + s_l;
    real c = 1, s = 0;
    if (bb < A.B) {
      qs_gate gt = kload(A.gates, kc(A.slot_gate)[slot]);
      real th = theta_of(A, gt, bb >> A.ob);
      fsincos(th * (real)0.5, &s, &c);
    }
    C.ang_ps[2 * (size_t)i] = c;
    C.ang_ps[2 * (size_t)i + 1] = s;
  }
  if (adjoint) {
    if (!A.per_sample_params)
      for (int i = tid; i < waves * A.n_params; i += blockDim.x) C.gacc[i] = 0;
    for (int i = tid; i < A.S * C.wps * A.n_feats; i += blockDim.x) C.facc[i] = 0;
  }
  __syncthreads();
}

template <typename real, int LR>
__device__ __forceinline__ const QS_K uint8_t* seg_map(const Args<real>& A, int s) {
  return kc(A.seg_map) + (size_t)s * kMapStride;
}
template <typename real>
__device__ __forceinline__ bool map_changed(const Args<real>& A, int s) {
  const QS_K uint32_t* m = reinterpret_cast<const QS_K uint32_t*>(kc(A.seg_map));
  bool ch = false;
#pragma unroll
  for (int w = 0; w < kMapStride / 4; ++w)
    ch |= m[(size_t)(s - 1) * (kMapStride / 4) + w] != m[(size_t)s * (kMapStride / 4) + w];
  return ch;
}

// ------------------------------------------------------------------ forward
template <typename real, int LR, bool FLY = false>
__device__ __forceinline__ void forward_body(const Args<real>& A, unsigned char* smem,
                                             int64_t blk) {
  constexpr int R = 1 << LR;
  Ctx<real, LR, FLY> C(A);
  setup<real, LR, FLY>(C, A, smem, false, blk);

  St<real, R> x;
  C.load_state(x, A.state, seg_map<real, LR>(A, 0));
  const int nseg = A.nseg;
  const QS_K int32_t* seg_begin = kc(A.seg_begin);
  for (int s = 0; s < nseg; ++s) {
    if (s > 0 && map_changed(A, s))
      C.remap(x, seg_map<real, LR>(A, s - 1), seg_map<real, LR>(A, s));
    const int e = seg_begin[s + 1];
    int o = seg_begin[s];
    if (o < e) {
      // Software pipeline: op o+1's descriptor and op o's angle are in flight
      // while op o is applied.
      SvOp cur = kload(A.ops, o);
      real c, sn;
      C.angle(o, cur, c, sn);
      for (; o < e; ++o) {
        const SvOp nxt = kload(A.ops, o + 1 < e ? o + 1 : o);
        real nc, ns;
        C.angle(o + 1 < e ? o + 1 : o, nxt, nc, ns);
        C.apply(x, uni(cur.kind), uni(cur.a), uni(cur.b), c, sn);
        cur = nxt;
        c = nc;
        sn = ns;
      }
    }
    const int ck = kc(A.seg_ckpt)[s];
    if (ck >= 0 && A.ckpt != nullptr)
      C.store_state(x, A.ckpt + (size_t)ck * A.B * (2ull << A.n),
                    seg_map<real, LR>(A, s));
  }
  const QS_K uint8_t* last = seg_map<real, LR>(A, nseg - 1);
  C.store_state(x, A.state, last);

  if (A.expz != nullptr) {
    // <Z_q> partials in FP64, reduced over the sample's threads.
    const int Tw = (1 << A.t) < 64 ? (1 << A.t) : 64;
    const int nw = (1 << A.t) / Tw;  // waves per sample
    double* red = reinterpret_cast<double*>(C.lds);
    sample_sync(A.t);
    double tot = 0;
#pragma unroll
    for (int k = 0; k < R; ++k)
      tot += (double)x.re[k] * x.re[k] + (double)x.im[k] * x.im[k];
    const int wave_in_sample = C.tau / Tw;
    for (int q = 0; q < A.n; ++q) {
      int p = 0;
      for (int i = 0; i < A.n; ++i)
        if (last[i] == q) p = i;
      p = uni(p);
      double z = 0;
      if (p < LR) {
        for_pos<LR>(p, [&](auto J) QS_AI {
#pragma unroll
          for (int k = 0; k < R; ++k) {
            double pr = (double)x.re[k] * x.re[k] + (double)x.im[k] * x.im[k];
            z += (k & (1 << decltype(J)::value)) ? -pr : pr;
          }
        });
      } else {
        z = C.tbit(p) ? -tot : tot;
      }
      z = group_sum(z, Tw);
      if ((C.tau & (Tw - 1)) == 0) red[(size_t)wave_in_sample * A.n + q] = z;
    }
    sample_sync(A.t);
    if (C.active)
      for (int q = C.tau; q < A.n; q += (1 << A.t)) {
        double z = 0;
        for (int w = 0; w < nw; ++w) z += red[(size_t)w * A.n + q];
        A.expz[(size_t)C.b * A.n + q] = z;
      }
  }
}

// ------------------------------------------------------------------ adjoint
template <typename real, int LR, bool FLY = false>
__device__ __forceinline__ void adjoint_body(const Args<real>& A, unsigned char* smem,
                                             int64_t blk) {
  constexpr int R = 1 << LR;
  Ctx<real, LR, FLY> C(A);
  setup<real, LR, FLY>(C, A, smem, true, blk);
  const int nseg = A.nseg;
  const QS_K uint8_t* last = seg_map<real, LR>(A, nseg - 1);

  St<real, R> psi, lam;
  C.load_state(psi, A.state, last);
  if (A.dstate != nullptr) {
    C.load_state(lam, A.dstate, last);
  } else {
    // lam = sum_q g_q Z_q psi: coefficient of amplitude with logical index L
    // is sum_q g_q - 2 sum_{q : bit q of L = 1} g_q.
    double base = 0;
    double w[LR > 0 ? LR : 1];
#pragma unroll
    for (int j = 0; j < LR; ++j) w[j] = 0;
    if (C.active) {
      const double* g = A.dexpz + (size_t)C.b * A.n;
      for (int p = 0; p < A.n; ++p) {
        const double gq = g[last[p]];
        base += gq;
        if (p >= LR && C.tbit(p)) base -= 2 * gq;
      }
#pragma unroll
      for (int j = 0; j < LR; ++j) w[j] = 2 * g[last[j]];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      double cf = C.active ? base : 0.0;
#pragma unroll
      for (int j = 0; j < LR; ++j)
        if (k & (1 << j)) cf -= w[j];
      lam.re[k] = (real)cf * psi.re[k];
      lam.im[k] = (real)cf * psi.im[k];
    }
  }

  const int Tw = (1 << A.t) < 64 ? (1 << A.t) : 64;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const QS_K int32_t* seg_begin = kc(A.seg_begin);
  for (int s = nseg - 1; s >= 0; --s) {
    const int ck = kc(A.seg_ckpt)[s];
    if (ck >= 0 && A.ckpt != nullptr)  // re-anchor psi to the stored state
      C.load_state(psi, A.ckpt + (size_t)ck * A.B * (2ull << A.n),
                   seg_map<real, LR>(A, s));
    const int beg = seg_begin[s];
    int o = seg_begin[s + 1] - 1;
    if (o >= beg) {
      SvOp cur = kload(A.ops, o);
      real c, sn;
      C.angle(o, cur, c, sn);
      for (; o >= beg; --o) {
        const int on = o - 1 >= beg ? o - 1 : o;
        const SvOp nxt = kload(A.ops, on);
        real nc, ns;
        C.angle(on, nxt, nc, ns);
        const int kind = uni(cur.kind), a = uni(cur.a), bq = uni(cur.b);
        if (kind <= QS_OP_RZ) {
          const real part = C.grad_partial(kind, a, psi, lam);
          const qs_gate gt = kload(A.gates, cur.gate);
          const real scale = (real)gt.scale;
          if (!A.per_sample_params && gt.feat < 0) {
            // shared parameters, no feature: dL/dP += scale sum_b dL/dtheta_b
            const real v = group_sum(part, 64);
            if (lane == 0) {
              real* g = C.gacc + (size_t)wave * A.n_params;
              if (gt.p_w >= 0) g[gt.p_w] += scale * v;
              if (gt.p_b >= 0) g[gt.p_b] += scale * v;
            }
          } else {
            const real gth = group_sum(part, Tw);  // this sample (this wave's share)
            const bool leader = (C.tau & (Tw - 1)) == 0 && C.active;
            const real* P = param_row(A, C.active ? C.row : 0);
            const real f = (gt.feat >= 0 && C.active)
                               ? A.feats[(size_t)C.row * A.n_feats + gt.feat]
                               : (real)1;
            const real w = gt.p_w >= 0 ? P[gt.p_w] : (real)1;
            if (A.per_sample_params) {
              if (leader) {
                double* gp = A.grad_params + (size_t)C.row * A.n_params;
                if (gt.p_w >= 0) atomicAdd(&gp[gt.p_w], (double)(gth * scale * f));
                if (gt.p_b >= 0) atomicAdd(&gp[gt.p_b], (double)(gth * scale));
              }
            } else {
              if (gt.p_w >= 0) {
                const real v = group_sum(leader ? gth * scale * f : (real)0, 64);
                if (lane == 0) C.gacc[(size_t)wave * A.n_params + gt.p_w] += v;
              }
              if (gt.p_b >= 0) {
                const real v = group_sum(leader ? gth * scale : (real)0, 64);
                if (lane == 0) C.gacc[(size_t)wave * A.n_params + gt.p_b] += v;
              }
            }
            if (gt.feat >= 0 && leader)
              C.facc[((size_t)C.sl * C.wps + (C.tau >> 6)) * A.n_feats + gt.feat] +=
                  gth * scale * w;
          }
          sn = -sn;  // inverse rotation
        }
        C.apply(psi, kind, a, bq, c, sn);
        C.apply(lam, kind, a, bq, c, sn);
        cur = nxt;
        c = nc;
        sn = ns;
      }
    }
    if (s > 0 && map_changed(A, s)) {
      C.remap(psi, seg_map<real, LR>(A, s), seg_map<real, LR>(A, s - 1));
      C.remap(lam, seg_map<real, LR>(A, s), seg_map<real, LR>(A, s - 1));
    }
  }
  if (A.out_psi != nullptr) C.store_state(psi, A.out_psi, seg_map<real, LR>(A, 0));
  if (A.out_lam != nullptr) C.store_state(lam, A.out_lam, seg_map<real, LR>(A, 0));
  __syncthreads();
  const int waves = blockDim.x >> 6;
  if (!A.per_sample_params)
    for (int i = threadIdx.x; i < A.n_params; i += blockDim.x) {
      real t = 0;
      for (int w = 0; w < waves; ++w) t += C.gacc[(size_t)w * A.n_params + i];
      A.ws_partials[(size_t)blockIdx.x * A.n_params + i] = t;
    }
  if (A.grad_feats != nullptr)
    for (int i = threadIdx.x; i < A.S * A.n_feats; i += blockDim.x) {
      const int sl = i / A.n_feats, f = i % A.n_feats;
      const int64_t bb = blk + sl;
      if (bb >= A.B) continue;
      real t = 0;
      for (int w = 0; w < C.wps; ++w) t += C.facc[((size_t)sl * C.wps + w) * A.n_feats + f];
      double* dst = &A.grad_feats[(size_t)(bb >> A.ob) * A.n_feats + f];
      if (A.tile_q != nullptr)
        atomicAdd(dst, (double)t);  // several tiles share a batch row
      else
        *dst = t;
    }
}

template <typename real, int LR, int MAXT>
__global__ void __launch_bounds__(MAXT) sv_forward(Args<real> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  forward_body<real, LR>(A, smem, (int64_t)blockIdx.x * A.S);
}

template <typename real, int LR, int MAXT>
__global__ void __launch_bounds__(MAXT) sv_adjoint(Args<real> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  adjoint_body<real, LR>(A, smem, (int64_t)blockIdx.x * A.S);
}

// Uneven batches in one persistent launch: workgroups pull work items (a
// class of identically-structured circuits and a run of S of its circuits)
// from an atomic counter until the queue is empty; items are ordered longest
// first. Every workgroup runs the same engine as the batched kernels, with
// per-circuit angles computed in place (no per-sample LDS table).
template <typename real, int LR, int MAXT, bool ADJ>
__global__ void __launch_bounds__(MAXT)
sv_program(const ProgClass* classes, const ProgItem* items, int n_items,
           int* counter, const real* params, real* states, double* expz,
           const double* dexpz, double* grad_params) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int item_sh;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int it = item_sh;
    __syncthreads();
    if (it >= n_items) break;  // every wave of the workgroup sees the same it
    const ProgItem w = kload(items, it);
    const ProgClass cd = kload(classes, w.cls);
    Args<real> A;
    A.seg_map = cd.seg_map;
    A.seg_begin = cd.seg_begin;
    A.seg_ckpt = cd.seg_ckpt;
    A.ops = cd.ops;
    A.gates = cd.gates;
    A.angle_slot = cd.angle_slot;
    A.slot_gate = cd.slot_gate;
    A.n = cd.n;
    A.t = cd.t;
    A.nseg = cd.nseg;
    A.n_gates = cd.n_gates;
    A.n_slots = cd.n_slots;
    A.n_params = cd.n_params;
    A.n_feats = 0;
    A.S = cd.S;
    A.per_sample_params = 1;
    const int64_t left = cd.count - w.first;
    A.B = left < cd.S ? left : cd.S;
    A.n_tot = 0;
    A.ob = 0;
    A.tile_q = nullptr;
    A.outer_q = nullptr;
    A.out_psi = nullptr;
    A.out_lam = nullptr;
    const int64_t first = w.first;
    A.params = params + cd.param_off + first * cd.n_params;
    A.feats = nullptr;
    A.state = states + 2 * (cd.state_off + (first << cd.n));
    A.expz = expz ? expz + cd.expz_off + first * cd.n : nullptr;
    A.ckpt = nullptr;
    A.dexpz = dexpz ? dexpz + cd.expz_off + first * cd.n : nullptr;
    A.dstate = nullptr;
    A.ws_partials = nullptr;
    A.grad_params = grad_params ? grad_params + cd.param_off + first * cd.n_params : nullptr;
    A.grad_feats = nullptr;
    if (ADJ)
      adjoint_body<real, LR, true>(A, smem, 0);
    else
      forward_body<real, LR, true>(A, smem, 0);
    __syncthreads();  // the next item reuses the LDS
  }
}

__global__ void zero_i32(int* p) { *p = 0; }

template <typename real>
Args<real> make_args(const SvLaunch& L) {
  const SvDevPlan& p = *L.p;
  Args<real> A;
  A.seg_map = p.seg_map;
  A.seg_begin = p.seg_begin;
  A.seg_ckpt = p.seg_ckpt;
  A.ops = p.ops;
  A.gates = p.gates;
  A.angle_slot = p.angle_slot;
  A.slot_gate = p.slot_gate;
  A.n = p.n;
  A.t = p.t;
  A.nseg = p.nseg;
  A.n_gates = p.n_gates;
  A.n_slots = p.n_slots;
  A.n_params = p.n_params;
  A.n_feats = p.n_features;
  A.S = L.shape.samples_per_block;
  A.per_sample_params = L.per_sample_params;
  A.B = L.B << L.ob;
  A.n_tot = L.n_tot;
  A.ob = L.ob;
  A.tile_q = L.tile_q;
  A.outer_q = L.outer_q;
  A.out_psi = static_cast<real*>(L.out_psi);
  A.out_lam = static_cast<real*>(L.out_lam);
  A.params = static_cast<const real*>(L.params);
  A.feats = static_cast<const real*>(L.feats);
  A.state = static_cast<real*>(L.state);
  A.expz = L.expz;
  A.ckpt = static_cast<real*>(L.ckpt);
  A.dexpz = L.dexpz;
  A.dstate = static_cast<const real*>(L.dstate);
  A.ws_partials = static_cast<real*>(L.ws_partials);
  A.grad_params = L.grad_params;
  A.grad_feats = L.grad_feats;
  return A;
}

template <typename real, int LR, int MAXT>
int launch_one(const SvLaunch& L, bool adjoint) {
  Args<real> A = make_args<real>(L);
  const int64_t grid = (A.B + A.S - 1) / A.S;
  if (grid <= 0) return QS_OK;
  dim3 g((unsigned)grid), blk((unsigned)L.shape.block_threads);
  hipStream_t st = static_cast<hipStream_t>(L.stream);
  auto kern = adjoint ? sv_adjoint<real, LR, MAXT> : sv_forward<real, LR, MAXT>;
  if (L.shape.lds_bytes > 65536) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)L.shape.lds_bytes) != hipSuccess)
      return QS_ERR_LAUNCH;
  }
  hipLaunchKernelGGL(kern, g, blk, (size_t)L.shape.lds_bytes, st, A);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_LAUNCH;
}

// (dtype, r, direction) -> the block-size bound of the instantiation. The
// bounds are chosen so that no instantiation spills registers to scratch.
int max_threads(int dtype, int r, bool adjoint) {
  if (dtype == QS_C64) {
    if (r <= 3) return 1024;
    if (r == 4) return adjoint ? 512 : 1024;
    return r == 5 ? 512 : 0;
  }
  if (r <= 2) return 1024;
  if (r == 3) return adjoint ? 1024 : 1024;
  return r == 4 ? 512 : 0;
}

int dispatch(int dtype, const SvLaunch& L, bool adjoint) {
  const int r = L.shape.r;
  if (dtype == QS_C64) {
    switch (r) {
      case 1: return launch_one<float, 1, 1024>(L, adjoint);
      case 2: return launch_one<float, 2, 1024>(L, adjoint);
      case 3: return launch_one<float, 3, 1024>(L, adjoint);
      case 4: return adjoint ? launch_one<float, 4, 512>(L, adjoint)
                             : launch_one<float, 4, 1024>(L, adjoint);
      case 5: return launch_one<float, 5, 512>(L, adjoint);
      default: return QS_ERR_UNSUPPORTED;
    }
  }
  switch (r) {
    case 1: return launch_one<double, 1, 1024>(L, adjoint);
    case 2: return launch_one<double, 2, 1024>(L, adjoint);
    case 3: return launch_one<double, 3, 1024>(L, adjoint);
    case 4: return launch_one<double, 4, 512>(L, adjoint);
    default: return QS_ERR_UNSUPPORTED;
  }
}


template <typename real, int LR, int MAXT>
int launch_prog(const ProgLaunch& L, bool adjoint) {
  hipStream_t st = static_cast<hipStream_t>(L.stream);
  auto kern = adjoint ? sv_program<real, LR, MAXT, true> : sv_program<real, LR, MAXT, false>;
  if (L.lds_bytes > 65536 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)L.lds_bytes) != hipSuccess)
    return QS_ERR_LAUNCH;
  hipLaunchKernelGGL(kern, dim3((unsigned)L.grid), dim3((unsigned)L.block),
                     (size_t)L.lds_bytes, st, L.classes, L.items, L.n_items, L.counter,
                     static_cast<const real*>(L.params), static_cast<real*>(L.states),
                     L.expz, L.dexpz, L.grad_params);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_LAUNCH;
}

}  // namespace

int launch_program(int dtype, const ProgLaunch& L, bool adjoint) {
  if (L.block != 512) return QS_ERR_UNSUPPORTED;
  if (dtype == QS_C64) {
    if (L.r == 5) return launch_prog<float, 5, 512>(L, adjoint);
    if (L.r == 4) return launch_prog<float, 4, 512>(L, adjoint);
    return QS_ERR_UNSUPPORTED;
  }
  if (L.r == 4) return launch_prog<double, 4, 512>(L, adjoint);
  return QS_ERR_UNSUPPORTED;
}

int launch_zero_i32(int* p, void* stream) {
  hipLaunchKernelGGL(zero_i32, dim3(1), dim3(1), 0, static_cast<hipStream_t>(stream), p);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_LAUNCH;
}

int launch_sv_forward(int dtype, const SvLaunch& L) { return dispatch(dtype, L, false); }
int launch_sv_adjoint(int dtype, const SvLaunch& L) { return dispatch(dtype, L, true); }

// Largest block size each (dtype, r, direction) instantiation is compiled for.
int sv_max_threads(int dtype, int r, int adjoint) { return max_threads(dtype, r, adjoint != 0); }

}  // namespace qs
