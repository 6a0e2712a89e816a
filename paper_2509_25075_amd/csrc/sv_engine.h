// Register-resident batched state-vector engine for gfx950 (forward and
// adjoint): device code and launch templates, instantiated by the sv_*.hip
// translation units (one per element type and direction, so that they build
// in parallel).
//
// Layout. A sample's 2^n amplitudes live in the registers of T = 2^t
// threads, R = 2^r amplitudes per thread (n = r + t). Physical index of
// amplitude k of thread tau is k + R * tau, so physical bits 0..r-1 are
// register bits and r..n-1 are thread bits. A segment of the planned gate
// program fixes which logical qubit sits on which physical bit; every
// single-qubit gate of a segment acts on a register bit, so it is applied
// with no communication, and CZs on thread bits use the lane's own bits.
// Between segments the state is written to LDS in logical order and read
// back under the next placement (a remap); CNOTs are folded into the remap
// addresses.
//
// Layer ops. Runs of single-qubit gates on the qubit of each register bit
// are multiplied into one 2x2 matrix per bit ("block"), and one L1Q op
// applies the blocks of all register bits in straight-line code, with a set
// of CZ gates before and after as per-thread sign masks over the register
// index. Every op of a plan is an L1Q op, so the op loop has one path and
// the state stays in the same registers from op to op. The adjoint takes
// every rotation gradient of a block from three Pauli partials
// Im <lam|sigma|psi> (sigma = X, Y, Z on the block's bit) at the block
// output, dotted with the rotation's generator as conjugated by the block's
// later gates.
//
// LDS slots are swizzled, slot(L) = L ^ fold(L >> 5) ^ (per-sample salt),
// with fold a linear map into the low five bits chosen per plan on the host;
// the plan's layout masks arrive already swizzled, so the address of
// amplitude k of a lane is (per-lane part) XOR (uniform per-k part): one VALU
// op per access.
//
// Gates: R_P(t) = exp(-i t P / 2) (Nielsen & Chuang sec. 4.2); the adjoint
// step computes dL/dtheta = Im <lam|P|psi> and un-applies the gate from psi
// and lam (Jones & Gacon, arXiv:2009.02823, sec. 3).
#pragma once

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

// v + (v of lane ^ 16), v + (v of lane ^ 32): gfx950's row-swapping
// permlanes exchange a value between paired rows without LDS; called with
// the same register twice, one result keeps the lane's own value and the
// other receives the partner's, so their sum is the pair sum on every lane.
__device__ __forceinline__ float xor16_sum(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v),
                                                  false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xor32_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v),
                                                  false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// The same for a double: its two 32-bit halves are swapped separately.
__device__ __forceinline__ double xor16_sum(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double x = __longlong_as_double((long long)(((unsigned long long)b[0] << 32) | a[0]));
  const double y = __longlong_as_double((long long)(((unsigned long long)b[1] << 32) | a[1]));
  return x + y;
}
__device__ __forceinline__ double xor32_sum(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double x = __longlong_as_double((long long)(((unsigned long long)b[0] << 32) | a[0]));
  const double y = __longlong_as_double((long long)(((unsigned long long)b[1] << 32) | a[1]));
  return x + y;
}

// Sum over the lanes l, l ^ G, l ^ 2G, ... (G a power of two, uniform): with
// every lane of each aligned group of G lanes holding that group's value,
// each lane receives the sum over all groups of the wave.
template <typename real>
__device__ __forceinline__ real cross_sum(real v, int G) {
  if (G <= 1) v += dpp<0xB1>(v);
  if (G <= 2) v += dpp<0x4E>(v);
  if (G <= 4) v += dpp<0x141>(v);
  if (G <= 8) v += dpp<0x140>(v);
  if (G <= 16) v = xor16_sum(v);
  if (G <= 32) v = xor32_sum(v);
  return v;
}

// Sum over aligned groups of G lanes (G a power of two, 1..64, uniform);
// every lane of a group receives the group's sum. Requires a full wave.
template <typename real>
__device__ __forceinline__ real group_sum(real v, int G) {
  if (G >= 2) v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]  (lane ^ 1)
  if (G >= 4) v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]  (lane ^ 2)
  if (G >= 8) v += dpp<0x141>(v);  // row_half_mirror: the other quad of 8
  if (G >= 16) v += dpp<0x140>(v); // row_mirror: the other 8 of a row
  if (G >= 32) v = xor16_sum(v);
  if (G >= 64) v = xor32_sum(v);
  return v;
}

// Reduce-scatter steps over paired rows: the swap moves the upper 32 lanes of
// its first operand into the lower 32 of its second (and back), so lanes
// 0-31 end with a's sum over the pair l, l ^ 32 and lanes 32-63 with b's;
// the 16-lane form does the same with even rows taking a and odd rows b.
__device__ __forceinline__ float swap32_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b),
                                                  false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b),
                                                  false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double join64(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double swap32_sum(double a, double b) {
  const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
  const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32),
                                                   false, false);
  return join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
}
__device__ __forceinline__ double swap16_sum(double a, double b) {
  const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
  const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32),
                                                   false, false);
  return join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
}

// The wave sums of four per-lane values at once: each swap step halves the
// values a lane carries while the paired lanes sum them, and the in-row
// steps finish one value per row, so every lane of row k (lanes 16k to
// 16k + 15) ends with the sum of v_k. Three swaps and four in-row steps,
// against six steps for each value summed alone.
template <typename real>
__device__ __forceinline__ real rows_sum4(real v0, real v1, real v2, real v3) {
  const real a = swap32_sum(v0, v2);  // lanes 0-31: v0, lanes 32-63: v2
  const real b = swap32_sum(v1, v3);  // lanes 0-31: v1, lanes 32-63: v3
  return group_sum(swap16_sum(a, b), 16);
}

// Lane `l`'s value (l uniform) on every lane.
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  return join64((unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l),
                (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l));
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

// A layer op's record, read in one scalar load.
struct L1QRec {
  int32_t w[kL1QWords];
};

__device__ __forceinline__ int uni(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// A copy of v the compiler cannot see through: per-lane address tables
// derived from it are then recomputed at each use instead of being kept
// live (and spilled) across the whole kernel.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}


// --------------------------------------------------------------- state ops
// Amplitudes of one thread. The engine runs layer ops only, so every index
// into these arrays is a compile-time constant and they live in registers.
template <typename real, int R>
struct St {
  real re[R];
  real im[R];
};

// ------------------------------------------------------ 2x2 complex blocks
// A single-qubit operator [[u00, u01], [u10, u11]] (real, imaginary parts).
template <typename real>
struct U2 {
  real r00, i00, r01, i01, r10, i10, r11, i11;
};

template <typename real>
__device__ __forceinline__ U2<real> u_mul(const U2<real>& a, const U2<real>& b) {
  U2<real> c;
  c.r00 = a.r00 * b.r00 - a.i00 * b.i00 + a.r01 * b.r10 - a.i01 * b.i10;
  c.i00 = a.r00 * b.i00 + a.i00 * b.r00 + a.r01 * b.i10 + a.i01 * b.r10;
  c.r01 = a.r00 * b.r01 - a.i00 * b.i01 + a.r01 * b.r11 - a.i01 * b.i11;
  c.i01 = a.r00 * b.i01 + a.i00 * b.r01 + a.r01 * b.i11 + a.i01 * b.r11;
  c.r10 = a.r10 * b.r00 - a.i10 * b.i00 + a.r11 * b.r10 - a.i11 * b.i10;
  c.i10 = a.r10 * b.i00 + a.i10 * b.r00 + a.r11 * b.i10 + a.i11 * b.r10;
  c.r11 = a.r10 * b.r01 - a.i10 * b.i01 + a.r11 * b.r11 - a.i11 * b.i11;
  c.i11 = a.r10 * b.i01 + a.i10 * b.r01 + a.r11 * b.i11 + a.i11 * b.r11;
  return c;
}
template <typename real>
__device__ __forceinline__ U2<real> u_dag(const U2<real>& a) {
  return U2<real>{a.r00, -a.i00, a.r10, -a.i10, a.r01, -a.i01, a.r11, -a.i11};
}
// The matrix of a single-qubit gate; rotations take (c, s) = cos, sin of
// theta/2, so RX = [[c, -i s], [-i s, c]], RY = [[c, -s], [s, c]],
// RZ = diag(c - i s, c + i s).
template <typename real>
__device__ __forceinline__ U2<real> gate_u(int kind, real c, real s) {
  const real z = 0, o = 1, h = (real)0.70710678118654752440;
  switch (kind) {
    case QS_OP_RX: return U2<real>{c, z, z, -s, z, -s, c, z};
    case QS_OP_RY: return U2<real>{c, z, -s, z, s, z, c, z};
    case QS_OP_RZ: return U2<real>{c, -s, z, z, z, z, c, s};
    case QS_OP_X: return U2<real>{z, z, o, z, o, z, z, z};
    case QS_OP_Y: return U2<real>{z, z, z, -o, z, o, z, z};
    case QS_OP_Z: return U2<real>{o, z, z, z, z, z, -o, z};
    default: return U2<real>{h, z, h, z, h, z, -h, z};  // H
  }
}

// G U for a gate G of `kind` (rotations with (c, s) of theta/2), using the
// gate's structure instead of a full 2x2 complex product.
template <typename real>
__device__ __forceinline__ U2<real> gate_lmul(int kind, real c, real s, const U2<real>& u) {
  U2<real> o;
  switch (kind) {
    case QS_OP_RX:  // [[c, -i s], [-i s, c]]: row0' = c row0 - i s row1, row1' = c row1 - i s row0
      o.r00 = c * u.r00 + s * u.i10; o.i00 = c * u.i00 - s * u.r10;
      o.r01 = c * u.r01 + s * u.i11; o.i01 = c * u.i01 - s * u.r11;
      o.r10 = c * u.r10 + s * u.i00; o.i10 = c * u.i10 - s * u.r00;
      o.r11 = c * u.r11 + s * u.i01; o.i11 = c * u.i11 - s * u.r01;
      return o;
    case QS_OP_RY:  // [[c, -s], [s, c]]
      o.r00 = c * u.r00 - s * u.r10; o.i00 = c * u.i00 - s * u.i10;
      o.r01 = c * u.r01 - s * u.r11; o.i01 = c * u.i01 - s * u.i11;
      o.r10 = s * u.r00 + c * u.r10; o.i10 = s * u.i00 + c * u.i10;
      o.r11 = s * u.r01 + c * u.r11; o.i11 = s * u.i01 + c * u.i11;
      return o;
    case QS_OP_RZ:  // row0 * (c - i s), row1 * (c + i s)
      o.r00 = c * u.r00 + s * u.i00; o.i00 = c * u.i00 - s * u.r00;
      o.r01 = c * u.r01 + s * u.i01; o.i01 = c * u.i01 - s * u.r01;
      o.r10 = c * u.r10 - s * u.i10; o.i10 = c * u.i10 + s * u.r10;
      o.r11 = c * u.r11 - s * u.i11; o.i11 = c * u.i11 + s * u.r11;
      return o;
    default:
      return u_mul(gate_u<real>(kind, c, s), u);
  }
}

// x <- U x on register bit J.
template <int J, typename real, int R>
__device__ __forceinline__ void g_u(St<real, R>& x, const U2<real>& u) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    const real ar = x.re[k], ai = x.im[k], br = x.re[k1], bi = x.im[k1];
    x.re[k] = u.r00 * ar - u.i00 * ai + u.r01 * br - u.i01 * bi;
    x.im[k] = u.r00 * ai + u.i00 * ar + u.r01 * bi + u.i01 * br;
    x.re[k1] = u.r10 * ar - u.i10 * ai + u.r11 * br - u.i11 * bi;
    x.im[k1] = u.r10 * ai + u.i10 * ar + u.r11 * bi + u.i11 * br;
  }
}

// The adjoint's rotation gradients come from three Pauli partials of the
// block output. For a rotation R_P(theta) = exp(-i theta P / 2) of a block
// whose later gates multiply to V, dL/dtheta is a multiple of
// Im <lam|V P V^dagger|psi> at the block output, and V P V^dagger = sum over
// sigma in {X, Y, Z} of e_sigma sigma with real e (the gate's "generator
// frame"), so it is e . (g_X, g_Y, g_Z) with g_sigma = Im <lam|sigma|psi> on
// the block's bit.
template <typename real>
struct G3 {
  real x, y, z;
};

// One pass over the pairs of register bit J: the per-thread parts of the
// Pauli partials g_sigma of the incoming psi and lam (sums over the thread's
// pairs), and psi <- V psi, lam <- V lam. Each pair's old values die as soon
// as its new values exist, so the pass needs no second copy of either state.
template <int J, typename real, int R>
__device__ __forceinline__ G3<real> pauli_and_apply(St<real, R>& p, St<real, R>& l,
                                                    const U2<real>& v) {
  G3<real> g{0, 0, 0};
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    const real p0r = p.re[k], p0i = p.im[k], p1r = p.re[k1], p1i = p.im[k1];
    const real l0r = l.re[k], l0i = l.im[k], l1r = l.re[k1], l1i = l.im[k1];
    // X: Im(p1 conj(l0) + p0 conj(l1))
    g.x = p1i * l0r + g.x;
    g.x = -p1r * l0i + g.x;
    g.x = p0i * l1r + g.x;
    g.x = -p0r * l1i + g.x;
    // Y: Re(p0 conj(l1)) - Re(p1 conj(l0))
    g.y = p0r * l1r + g.y;
    g.y = p0i * l1i + g.y;
    g.y = -p1r * l0r + g.y;
    g.y = -p1i * l0i + g.y;
    // Z: Im(p0 conj(l0)) - Im(p1 conj(l1))
    g.z = p0i * l0r + g.z;
    g.z = -p0r * l0i + g.z;
    g.z = -p1i * l1r + g.z;
    g.z = p1r * l1i + g.z;
    p.re[k] = v.r00 * p0r - v.i00 * p0i + v.r01 * p1r - v.i01 * p1i;
    p.im[k] = v.r00 * p0i + v.i00 * p0r + v.r01 * p1i + v.i01 * p1r;
    p.re[k1] = v.r10 * p0r - v.i10 * p0i + v.r11 * p1r - v.i11 * p1i;
    p.im[k1] = v.r10 * p0i + v.i10 * p0r + v.r11 * p1i + v.i11 * p1r;
    l.re[k] = v.r00 * l0r - v.i00 * l0i + v.r01 * l1r - v.i01 * l1i;
    l.im[k] = v.r00 * l0i + v.i00 * l0r + v.r01 * l1i + v.i01 * l1r;
    l.re[k1] = v.r10 * l0r - v.i10 * l0i + v.r11 * l1r - v.i11 * l1i;
    l.im[k1] = v.r10 * l0i + v.i10 * l0r + v.r11 * l1i + v.i11 * l1r;
  }
  return g;
}

// The same pass for a block RZ(b) RY(a) (c0, s0 of a/2; c1, s1 of b/2),
// one gate at a time: RZ un-applied (a phase per amplitude, the same on psi
// and lam, so the Z partial, RZ's generator at the block output, is
// unchanged by it), the Z and Y partials there (Y is RY's generator between
// the two gates), RY un-applied (a real rotation). 40 FMA-type operations
// per amplitude pair, against 44 for the fused block with three partials;
// returns the Y part in .y and the Z part in .z (.x is zero).
template <int J, typename real, int R>
__device__ __forceinline__ G3<real> ryrz_and_apply(St<real, R>& p, St<real, R>& l, real c0,
                                                   real s0, real c1, real s1) {
  G3<real> g{0, 0, 0};
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    // RZ^dagger = diag(c1 + i s1, c1 - i s1)
    const real p0r = c1 * p.re[k] - s1 * p.im[k], p0i = c1 * p.im[k] + s1 * p.re[k];
    const real p1r = c1 * p.re[k1] + s1 * p.im[k1], p1i = c1 * p.im[k1] - s1 * p.re[k1];
    const real l0r = c1 * l.re[k] - s1 * l.im[k], l0i = c1 * l.im[k] + s1 * l.re[k];
    const real l1r = c1 * l.re[k1] + s1 * l.im[k1], l1i = c1 * l.im[k1] - s1 * l.re[k1];
    // Z: Im(p0 conj(l0)) - Im(p1 conj(l1))
    g.z = p0i * l0r + g.z;
    g.z = -p0r * l0i + g.z;
    g.z = -p1i * l1r + g.z;
    g.z = p1r * l1i + g.z;
    // Y: Re(p0 conj(l1)) - Re(p1 conj(l0))
    g.y = p0r * l1r + g.y;
    g.y = p0i * l1i + g.y;
    g.y = -p1r * l0r + g.y;
    g.y = -p1i * l0i + g.y;
    // RY^dagger = [[c0, s0], [-s0, c0]]
    p.re[k] = c0 * p0r + s0 * p1r;
    p.im[k] = c0 * p0i + s0 * p1i;
    p.re[k1] = c0 * p1r - s0 * p0r;
    p.im[k1] = c0 * p1i - s0 * p0i;
    l.re[k] = c0 * l0r + s0 * l1r;
    l.im[k] = c0 * l0i + s0 * l1i;
    l.re[k1] = c0 * l1r - s0 * l0r;
    l.im[k1] = c0 * l1i - s0 * l0i;
    // Each pair's work stays together: hoisting later pairs' phase steps
    // would hold their values in registers the adjoint does not have.
    __builtin_amdgcn_sched_barrier(0);
  }
  return g;
}

// Generator frames: column a holds the X, Y, Z coefficients of V sigma_a
// V^dagger for the product V of the gates already passed (walking a block
// from its last gate to its first). Passing gate G (V <- V G) maps each
// sigma_a through G sigma_a G^dagger first: a rotation by theta about P
// turns the other two Paulis, R_Z: X -> cos X + sin Y, Y -> -sin X + cos Y
// (and cyclically: R_X turns Y toward Z, R_Y turns Z toward X); a Pauli
// gate negates the other two; H swaps X and Z and negates Y.
template <typename real>
struct P3 {
  real c[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};  // c[column][row]

  __device__ __forceinline__ void turn(int a, int b, real co, real si) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const real x = c[a][r], y = c[b][r];
      c[a][r] = co * x + si * y;
      c[b][r] = co * y - si * x;
    }
  }
  __device__ __forceinline__ void negate(int a, int b) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      c[a][r] = -c[a][r];
      c[b][r] = -c[b][r];
    }
  }
  // (c, s) = cos, sin of theta/2 for a rotation; ignored otherwise.
  __device__ __forceinline__ void conj_by(int kind, real cs, real sn) {
    const real co = cs * cs - sn * sn, si = 2 * cs * sn;  // cos, sin of theta
    switch (kind) {
      case QS_OP_RX: turn(1, 2, co, si); break;
      case QS_OP_RY: turn(2, 0, co, si); break;
      case QS_OP_RZ: turn(0, 1, co, si); break;
      case QS_OP_X: negate(1, 2); break;
      case QS_OP_Y: negate(0, 2); break;
      case QS_OP_Z: negate(0, 1); break;
      default:  // H
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const real t = c[0][r];
          c[0][r] = c[2][r];
          c[2][r] = t;
          c[1][r] = -c[1][r];
        }
        break;
    }
  }
  __device__ __forceinline__ real dot(int a, const G3<real>& g) const {
    return c[a][0] * g.x + c[a][1] * g.y + c[a][2] * g.z;
  }
};

__device__ __forceinline__ float flip_sign(float v, uint32_t bit) {
  return __uint_as_float(__float_as_uint(v) ^ (bit << 31));
}
__device__ __forceinline__ double flip_sign(double v, uint32_t bit) {
  return __longlong_as_double(__double_as_longlong(v) ^
                              (long long)((unsigned long long)bit << 63));
}

template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(IC<I>{});
    static_for<N, I + 1>(f);
  }
}

// ------------------------------------------------------------- kernel args
template <typename real>
struct Args {
  const uint8_t* seg_map;
  const uint16_t* seg_lay;   // [nseg][32] read / write layouts
  const int32_t* seg_begin;
  const int32_t* seg_ckpt;
  const SvOp* ops;
  const qs_gate* gates;
  const int32_t* gate_slot;  // [G] per-sample angle slot or -1
  const int32_t* slot_gate;
  const int32_t* l1q;        // layer-op records
  const uint32_t* diag;
  const int32_t* blk_begin;  // fused single-qubit blocks
  const BGate* blk_rec;      // gate records of the blocks, in block order
  const int32_t* blk_fu;
  const int32_t* blk_gen;    // first generator-frame slot of a shared block
  int n_blocks, n_fu, n_gen;
  int n, t, nseg, n_gates, n_slots, n_params, n_feats, S;
  int n_acc;                 // gradient columns: shared parameters the plan reads
  int per_sample_params;
  int64_t B;               // samples processed (tiled: batch rows << ob)
  int n_tot, ob;           // tiled: qubits of the whole state, outer bits
  const uint8_t* tile_q;   // tiled: [n] global qubit of each local bit
  const uint8_t* outer_q;  // tiled: [ob] global qubit of each outer bit
  real* out_psi;           // adjoint: store the final psi here (or null)
  real* out_lam;           // adjoint: store the final lam here (or null)
  int accum_feats;         // adjoint: add to grad_feats instead of writing
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
  // Forward with amplitude encoding fused into the state load (batched
  // layout only): sample b starts as pad(x[b]) / ||x[b]||, x[b] being the
  // first x_D of the x_stride reals at x_in + b x_stride; the squared norm is
  // summed in FP64 over the sample's threads in a fixed order. A zero row
  // becomes NaN and adds one to *bad_rows (when given). Null: read `state`.
  const real* x_in;
  int64_t x_stride, x_D;
  int32_t* bad_rows;
  // Training step (forward, MSE loss on qubit loss_q against y, adjoint in
  // one launch): y [B] labels; loss_part [grid] per-workgroup sums of the
  // squared residuals. With x_in and state both null the sweep starts from
  // |0...0>.
  const double* y;
  int loss_q;
  double* loss_part;
  // One-component staging: six-bit salt vectors of the samples of a wave
  // (vector i for bit i of the sample's position in its wave), packed six
  // bits each; 0: the default salts.
  uint64_t salt_basis;
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

__device__ __forceinline__ int bg_kind(const BGate& b) { return b.kind_slot & 15; }
__device__ __forceinline__ int bg_slot(const BGate& b) { return (b.kind_slot >> 4) - 1; }

template <typename real>
__device__ __forceinline__ real theta_of(const Args<real>& A, const BGate& g, int64_t b) {
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

// The engine's per-thread context. SHARED: every block of the plan has
// shared angles (its fused matrix and generator frames are in LDS), so the
// per-sample block code is left out. HALF: the LDS staging region of a
// sample holds one component (real or imaginary parts) of its state at a
// time, so remaps and HBM transfers run as two passes; it halves the LDS a
// sample needs, which lets more workgroups share a CU when LDS is what
// limits them (an autotuner choice).
template <typename real, int LR, bool FLY = false, bool SHARED = false, bool HALF = false>
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
  real* ldr;         // this sample's LDS staging region
  v2* lds;           // the same, as complex elements (full staging)
  uint32_t salt;     // per-sample slot salt
  real* ang_sh;      // [G][2] shared (cos, sin) of theta/2, by gate
  real* ang_ps;      // [n_slots][S][2] per-sample
  real* fu_sh;       // [n_fu][8] fused matrices of blocks with shared angles
  real* gen_sh;      // [n_gen][3] generator frames of their gates (adjoint)
  real* gacc;        // [waves][n_acc] shared-parameter gradient sums
  real* facc;        // [S * wps][n_feats] feature gradient sums
  real* fsh;         // [S][n_feats] the block's features (adjoint)
  double* lsq;       // [S] squared residuals of the training step's loss
  int wps;           // waves per sample (1 when a wave holds whole samples)
  // Complex64 adjoint, per-sample blocks with shared parameters and at most
  // four features: the sample's features and this lane's running terms of
  // their gradients, kept in registers (summed per sample once, at the end).
  // (Named scalars, not arrays: an array indexed by a feature number ends up
  // in scratch memory, and the whole context with it.)
  real fx0 = 0, fx1 = 0, fx2 = 0, fx3 = 0;
  real fg0 = 0, fg1 = 0, fg2 = 0, fg3 = 0;
  __device__ __forceinline__ real fx_of(int k) const {
    return k == 0 ? fx0 : k == 1 ? fx1 : k == 2 ? fx2 : fx3;
  }
  __device__ __forceinline__ void fg_add(int k, real d) {
    if (k == 0) fg0 += d;
    else if (k == 1) fg1 += d;
    else if (k == 2) fg2 += d;
    else fg3 += d;
  }

  __device__ Ctx(const Args<real>& a) : A(a) {}
  // The same context over another reference to the launch's arguments.
  __device__ Ctx(const Args<real>& a, const Ctx& o)
      : A(a), tau(o.tau), sl(o.sl), b(o.b), row(o.row), base(o.base), dep_tau(o.dep_tau),
        active(o.active), ldr(o.ldr), lds(o.lds), salt(o.salt), ang_sh(o.ang_sh),
        ang_ps(o.ang_ps), fu_sh(o.fu_sh), gen_sh(o.gen_sh), gacc(o.gacc), facc(o.facc),
        fsh(o.fsh), lsq(o.lsq), wps(o.wps), fx0(o.fx0), fx1(o.fx1), fx2(o.fx2),
        fx3(o.fx3), fg0(o.fg0), fg1(o.fg1), fg2(o.fg2), fg3(o.fg3) {}

  __device__ __forceinline__ bool tbit(int p) const {
    return (tau >> (p - LR)) & 1;
  }

  // A layout `lay` gives, for each physical bit, the logical index mask it
  // contributes (a placement: one bit each; after folded CNOTs: any GF(2)
  // combination). Logical index bits of this thread's thread-bit part:
  // The layout row of HBM transfers (register bit j on logical bit t + j,
  // thread bit i on logical bit i), stored after the plan's segments.
  __device__ __forceinline__ const QS_K uint16_t* hbm_lay() const {
    return kc(A.seg_lay) + (size_t)A.nseg * kLayWords;
  }
  __device__ __forceinline__ uint32_t lane_part(const QS_K uint16_t* lay) const {
    // The row's 16 masks come in one scalar load (a loop over t reading one
    // mask per step waited on a scalar load each time: at 7 to 9 thread bits
    // that cost the adjoint 4-15 % of its time). Thread bit i is entry
    // LR + i, taken where bit i of tau is set; tau < 2^t, so the bits from t
    // up select nothing and need no test (a test per bit would put each load
    // behind its own branch and wait).
    const uint32_t tb = opaque((uint32_t)tau);
    const QS_K uint32_t* w = reinterpret_cast<const QS_K uint32_t*>(lay);
    uint32_t wv[kMapStride / 2];
#pragma unroll
    for (int k = 0; k < kMapStride / 2; ++k) wv[k] = w[k];
    uint32_t L = 0;
#pragma unroll
    for (int i = 0; i < 16 - LR; ++i) {
      const int e = LR + i;
      const uint32_t m = (wv[e >> 1] >> ((e & 1) * 16)) & 0xffffu;
      L ^= m & (0u - ((tb >> i) & 1u));
    }
    return L ^ salt;  // the masks are swizzled slots already
  }


  // Staging writes and reads under a layout: component P of the state
  // (HALF), or whole complex amplitudes (P ignored).
  template <int P>
  __device__ __forceinline__ void write_mapped(const St<real, R>& x,
                                               const QS_K uint16_t* lay) {
    const uint32_t base = lane_part(lay);
    uint32_t m[LR > 0 ? LR : 1];
#pragma unroll
    for (int j = 0; j < LR; ++j) m[j] = uni(lay[j]);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      uint32_t off = 0;
#pragma unroll
      for (int j = 0; j < LR; ++j)
        if (k & (1 << j)) off ^= m[j];
      if constexpr (HALF) {
        ldr[base ^ off] = P ? x.im[k] : x.re[k];
      } else {
        v2 v;
        v.x = x.re[k];
        v.y = x.im[k];
        lds[base ^ off] = v;
      }
    }
  }
  template <int P>
  __device__ __forceinline__ void read_mapped(St<real, R>& x, const QS_K uint16_t* lay) {
    const uint32_t base = lane_part(lay);
    uint32_t m[LR > 0 ? LR : 1];
#pragma unroll
    for (int j = 0; j < LR; ++j) m[j] = uni(lay[j]);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      uint32_t off = 0;
#pragma unroll
      for (int j = 0; j < LR; ++j)
        if (k & (1 << j)) off ^= m[j];
      if constexpr (HALF) {
        (P ? x.im[k] : x.re[k]) = ldr[base ^ off];
      } else {
        const v2 v = lds[base ^ off];
        x.re[k] = v.x;
        x.im[k] = v.y;
      }
    }
  }
  // Staging passes: two with HALF (real parts, then imaginary), else one.
  static constexpr int kPasses = HALF ? 2 : 1;

  __device__ __forceinline__ void remap(St<real, R>& x, const QS_K uint16_t* from,
                                        const QS_K uint16_t* to) {
    // The LDS traffic of a remap issues at raised wave priority, so that it
    // starts while the other waves of the SIMD compute (measured on training
    // steps of 10-, 8- and 12-qubit batches: 3 to 8 % shorter; load_state and
    // store_state do the same).
    __builtin_amdgcn_s_setprio(1);
    static_for<kPasses>([&](auto PC) QS_AI {
      constexpr int P = decltype(PC)::value;
      sample_sync(A.t);
      write_mapped<P>(x, from);
      sample_sync(A.t);
      read_mapped<P>(x, to);
    });
    __builtin_amdgcn_s_setprio(0);
  }

  // HBM offsets of the R amplitudes this thread moves between HBM and LDS:
  // element u (local index tau + u T) sits at a0 + sum of off[j] over the set
  // bits j of u. Batched: off[j] = T << j. Tiled: local bit t + j is the
  // tile's global qubit tile_q[t + j].
  __device__ __forceinline__ int64_t hbm_a0() const {
    return A.tile_q == nullptr ? base + tau : base + dep_tau;
  }
  __device__ __forceinline__ void hbm_offsets(int64_t* off) const {
#pragma unroll
    for (int j = 0; j < LR; ++j)
      off[j] = A.tile_q == nullptr ? ((int64_t)1 << (A.t + j))
                                   : ((int64_t)1 << kc(A.tile_q)[A.t + j]);
  }

  // Amplitude encoding of this thread's R elements (logical index tau + u T,
  // as load_state holds them) from the sample's input row; see Args::x_in.
  // The squared norm is summed in FP64: over the thread's elements, over the
  // sample's lanes of each wave, then over its waves through the staging
  // region (which the staging passes after this overwrite).
  __device__ __forceinline__ void load_encoded(St<real, R>& x) {
    const real* xr = A.x_in + (active ? b : 0) * A.x_stride;
    double ss = 0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = tau + ((int64_t)u << A.t);
      const real v = (active && i < A.x_D) ? xr[i] : (real)0;
      x.re[u] = v;
      ss += (double)v * v;
    }
    const int Tw = (1 << A.t) < 64 ? (1 << A.t) : 64;
    ss = group_sum(ss, Tw);
    if (wps > 1) {
      double* red = reinterpret_cast<double*>(ldr);
      if ((tau & 63) == 0) red[tau >> 6] = ss;
      sample_sync(A.t);
      ss = 0;
      for (int w = 0; w < wps; ++w) ss += red[w];
    }
    // (threads past the batch end hold zeros and stay finite)
    const bool zero = active && !(ss > 0);
    const double inv = zero ? (double)NAN : ss > 0 ? 1.0 / sqrt(ss) : 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = tau + ((int64_t)u << A.t);
      x.re[u] = (real)(i < A.x_D ? (double)x.re[u] * inv : (zero ? (double)NAN : 0.0));
      x.im[u] = zero ? (real)NAN : (real)0;
    }
    if (zero && active && tau == 0 && A.bad_rows != nullptr) atomicAdd(A.bad_rows, 1);
  }

  // HBM (logical order) -> LDS -> registers under placement `map`. All R
  // loads of a thread are issued before the first wait.
  __device__ __forceinline__ void load_state(St<real, R>& x, const real* src,
                                             const QS_K uint16_t* map,
                                             bool encode = false) {
    __builtin_amdgcn_s_setprio(1);  // memory phase: issue ahead of computing waves
    if (encode) {
      load_encoded(x);
    } else if (src == nullptr) {
      // |0...0>: amplitude 0 (tau = 0, u = 0) is 1
#pragma unroll
      for (int u = 0; u < R; ++u) {
        x.re[u] = (active && u == 0 && tau == 0) ? (real)1 : (real)0;
        x.im[u] = 0;
      }
    } else {
      const v2* s2 = reinterpret_cast<const v2*>(src);
      int64_t off[LR > 0 ? LR : 1];
      hbm_offsets(off);
      const int64_t a0 = hbm_a0();
#pragma unroll
      for (int u = 0; u < R; ++u) {
        int64_t o = 0;
#pragma unroll
        for (int j = 0; j < LR; ++j)
          if (u & (1 << j)) o += off[j];
        v2 v;
        v.x = 0;
        v.y = 0;
        if (active) v = s2[a0 + o];
        x.re[u] = v.x;  // staging only: read_mapped below sets the placement
        x.im[u] = v.y;
      }
    }
    // the staging order of HBM transfers: logical index tau + u T
    const QS_K uint16_t* hl = hbm_lay();
    const uint32_t hb = lane_part(hl);
    uint32_t hm[LR > 0 ? LR : 1];
#pragma unroll
    for (int j = 0; j < LR; ++j) hm[j] = uni(hl[j]);
    static_for<kPasses>([&](auto PC) QS_AI {
      constexpr int P = decltype(PC)::value;
      sample_sync(A.t);
#pragma unroll
      for (int u = 0; u < R; ++u) {
        uint32_t a = hb;
#pragma unroll
        for (int j = 0; j < LR; ++j)
          if (u & (1 << j)) a ^= hm[j];
        if constexpr (HALF) {
          ldr[a] = P ? x.im[u] : x.re[u];
        } else {
          v2 v;
          v.x = x.re[u];
          v.y = x.im[u];
          lds[a] = v;
        }
      }
      sample_sync(A.t);
      read_mapped<P>(x, map);  // with HALF, the other component is still staged
    });
    __builtin_amdgcn_s_setprio(0);
  }
  // Registers under `map` -> LDS -> HBM (logical order), in runs of 8.
  // In runs of 8. With HALF each pass stores every other real of a run of
  // amplitudes and the second pass fills the gaps (the lines merge in L2).
  __device__ __forceinline__ void store_state(const St<real, R>& x, real* dst,
                                              const QS_K uint16_t* map) {
    __builtin_amdgcn_s_setprio(1);  // memory phase, as in load_state
    int64_t off[LR > 0 ? LR : 1];
    hbm_offsets(off);
    const int64_t a0 = hbm_a0();
    constexpr int W = R < 8 ? R : 8;
    const QS_K uint16_t* hl = hbm_lay();
    const uint32_t hb = lane_part(hl);
    uint32_t hm[LR > 0 ? LR : 1];
#pragma unroll
    for (int j = 0; j < LR; ++j) hm[j] = uni(hl[j]);
    static_for<kPasses>([&](auto PC) QS_AI {
      constexpr int P = decltype(PC)::value;
      sample_sync(A.t);
      write_mapped<P>(x, map);
      sample_sync(A.t);
      if (active) {
#pragma unroll
        for (int u0 = 0; u0 < R; u0 += W) {
          using E = typename std::conditional<HALF, real, v2>::type;
          E v[W];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            uint32_t a = hb;
#pragma unroll
            for (int j = 0; j < LR; ++j)
              if ((u0 + w) & (1 << j)) a ^= hm[j];
            if constexpr (HALF) v[w] = ldr[a]; else v[w] = lds[a];
          }
#pragma unroll
          for (int w = 0; w < W; ++w) {
            const int u = u0 + w;
            int64_t o = 0;
#pragma unroll
            for (int j = 0; j < LR; ++j)
              if (u & (1 << j)) o += off[j];
            if constexpr (HALF)
              dst[2 * (a0 + o) + P] = v[w];
            else
              reinterpret_cast<v2*>(dst)[a0 + o] = v[w];
          }
        }
      }
    });
    __builtin_amdgcn_s_setprio(0);
  }

  // cos, sin of theta/2 of a block's rotation (uniform record).
  __device__ __forceinline__ void gate_cs(const BGate& b, real& c, real& s) const {
    const int slot = bg_slot(b);
    if (slot >= 0) {
      if constexpr (FLY) {
        // per-sample angle computed in place (no per-sample table in LDS)
        const real th = active ? theta_of(A, b, row) : (real)0;
        fsincos(th * (real)0.5, &s, &c);
      } else {
        const real* p = ang_ps + 2 * ((size_t)slot * A.S + sl);
        c = p[0];
        s = p[1];
      }
    } else {
      c = ang_sh[2 * b.g];
      s = ang_sh[2 * b.g + 1];
    }
  }

  // The product of block `bid`'s gates (first gate rightmost); `fu` is its
  // fused-matrix slot, or -1 when its angles differ per sample.
  __device__ __forceinline__ U2<real> block_u(int bid, int fu) const {
    if (fu >= 0) {
      const real* p = fu_sh + 8 * (size_t)fu;
      return U2<real>{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]};
    }
    const int b0 = kc(A.blk_begin)[bid], b1 = kc(A.blk_begin)[bid + 1];
    if (b1 - b0 == 2) {
      // the common two-gate block: both records and angles fetched together
      const BGate g0 = kload(A.blk_rec, b0), g1 = kload(A.blk_rec, b0 + 1);
      real c0 = 1, s0 = 0, c1 = 1, s1 = 0;
      if (bg_kind(g0) <= QS_OP_RZ) gate_cs(g0, c0, s0);
      if (bg_kind(g1) <= QS_OP_RZ) gate_cs(g1, c1, s1);
      return two_u(bg_kind(g0), c0, s0, bg_kind(g1), c1, s1);
    }
    U2<real> u{1, 0, 0, 0, 0, 0, 1, 0};
    for (int i = b0; i < b1; ++i) {
      const BGate bg = kload(A.blk_rec, i);
      const int kind = bg_kind(bg);
      real c = 1, s = 0;
      if (kind <= QS_OP_RZ) gate_cs(bg, c, s);
      u = i == b0 ? gate_u<real>(kind, c, s) : gate_lmul(kind, c, s, u);
    }
    return u;
  }

  // The matrix of a two-gate block G1 G0. RZ(b) RY(a), the block of
  // hardware-efficient layers, is written out: with (c0, s0) of a/2 and
  // (c1, s1) of b/2 it is [[c0 (c1 - i s1), -s0 (c1 - i s1)],
  // [s0 (c1 + i s1), c0 (c1 + i s1)]].
  __device__ __forceinline__ static U2<real> two_u(int k0, real c0, real s0, int k1, real c1,
                                                   real s1) {
    if (k0 == QS_OP_RY && k1 == QS_OP_RZ) {
      const real a = c0 * c1, b = c0 * s1, d = s0 * c1, e = s0 * s1;
      return U2<real>{a, -b, -d, e, d, e, a, b};
    }
    return gate_lmul(k1, c1, s1, gate_u<real>(k0, c0, s0));
  }

  // The block's matrix, the identity for bid < 0. Register bits without a
  // block still get the (identity) update: a branch around the update would
  // make the compiler copy the whole state at the join.
  // (`fu` is the identity's slot for a register bit without a block.)
  __device__ __forceinline__ U2<real> block_or_id(int bid, int fu) const {
    if constexpr (SHARED) {
      const real* p = fu_sh + 8 * (size_t)fu;
      return U2<real>{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]};
    } else {
      return block_u(bid, fu);
    }
  }

  // L1Q: its first sign pattern, each register bit's block, its second
  // sign pattern. The whole record comes in one scalar load.
  __device__ __forceinline__ void apply_l1q(St<real, R>& x, int rec) const {
    const L1QRec r = kload(reinterpret_cast<const L1QRec*>(A.l1q), rec);
    apply_signs(x, r.w[kL1QPreDiag]);
    static_for<LR>([&](auto J) QS_AI {
      constexpr int j = decltype(J)::value;
      g_u<j>(x, block_or_id(r.w[j], r.w[kL1QFused + j]));
    });
    apply_signs(x, r.w[kL1QPostDiag]);
  }

  // DIAG: the sign (-1)^(sum over the CZ pairs of bit_a bit_b) of every
  // amplitude, built per thread as a mask over its register index k.
  __device__ __forceinline__ uint32_t diag_mask(int rec) const {
    const QS_K uint32_t* d = kc(A.diag) + (size_t)rec * kDiagWords;
    const uint32_t tb = (uint32_t)tau;
    uint32_t par = __builtin_popcount(tb & d[1]);
    for (int i = 0; i < A.t; ++i)
      par += __builtin_popcount(tb & d[7 + i] & (0u - ((tb >> i) & 1u)));
    uint32_t m = d[0] ^ ((par & 1) ? 0xffffffffu : 0u);
    constexpr uint32_t pat[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u,
                                 0xFFFF0000u};
#pragma unroll
    for (int j = 0; j < LR; ++j)
      if (__builtin_popcount(tb & d[2 + j]) & 1) m ^= pat[j];
    return m;
  }
  // The sign pattern of DIAG record `rec` (none for rec < 0) on x; the
  // update is in place, so the branch costs no state copies.
  __device__ __forceinline__ void apply_signs(St<real, R>& x, int rec) const {
    if (rec < 0) return;
    const uint32_t m = diag_mask(rec);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t bit = (m >> k) & 1u;
      x.re[k] = flip_sign(x.re[k], bit);
      x.im[k] = flip_sign(x.im[k], bit);
    }
  }
  __device__ __forceinline__ void apply_signs(St<real, R>& x, St<real, R>& y,
                                              int rec) const {
    if (rec < 0) return;
    const uint32_t m = diag_mask(rec);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t bit = (m >> k) & 1u;
      x.re[k] = flip_sign(x.re[k], bit);
      x.im[k] = flip_sign(x.im[k], bit);
      y.re[k] = flip_sign(y.re[k], bit);
      y.im[k] = flip_sign(y.im[k], bit);
    }
  }
  // Shared parameters: gradient terms gathered per block and summed over the
  // wave together. Slot k holds a per-lane term and up to two LDS columns
  // (the weight's and the bias's when they take the same term) that receive
  // its wave sum.
  struct Terms {
    real v[4] = {0, 0, 0, 0};
    int cw[4] = {-1, -1, -1, -1}, cb[4] = {-1, -1, -1, -1};
  };
  // The per-lane terms of rotation `gt` into slots K (weight, and bias when
  // it has no feature) and, with a feature, K + 1 (bias); its feature
  // gradient, which is per sample, is summed here.
  template <int K>
  __device__ __forceinline__ void shared_terms(Terms& t, const BGate& gt, real part, int Tw) {
    if (bg_kind(gt) > QS_OP_RZ) return;
    const real scale = (real)gt.scale;
    if (gt.feat < 0) {
      t.v[K] = scale * part;
      t.cw[K] = gt.col_w;
      t.cb[K] = gt.col_b;
      return;
    }
    if constexpr (K + 1 < 4) {
      t.v[K + 1] = active ? scale * part : (real)0;
      t.cw[K + 1] = gt.col_b;
      t.cw[K] = gt.col_w;
      const real w = gt.p_w >= 0 ? kc(A.params)[gt.p_w] : (real)1;
      if constexpr (feat_regs) {
        if (A.n_feats <= 4) {
          t.v[K] = t.v[K + 1] * fx_of(gt.feat);
          fg_add(gt.feat, scale * w * part);
          return;
        }
      }
      const real f = active ? fsh[(size_t)sl * A.n_feats + gt.feat] : (real)0;
      t.v[K] = t.v[K + 1] * f;
      const real gth = group_sum(part, Tw);
      if ((tau & (Tw - 1)) == 0 && active)
        atomicAdd(&facc[((size_t)sl * wps + (tau >> 6)) * A.n_feats + gt.feat],
                  gth * scale * w);
    }
  }
  static constexpr bool feat_regs = sizeof(real) == 4 && !SHARED;
  // The register terms of the feature gradients, summed per sample into the
  // LDS sums by each sample's (wave's) leader lane.
  __device__ __forceinline__ void fold_feature_terms(int Tw) {
    if constexpr (feat_regs) {
      if (A.per_sample_params || A.n_feats == 0 || A.n_feats > 4) return;
      const bool leader = (tau & (Tw - 1)) == 0 && active;
      real* fa = facc + ((size_t)sl * wps + (tau >> 6)) * A.n_feats;
      const real g0 = group_sum(fg0, Tw);
      if (leader) fa[0] += g0;
      if (A.n_feats > 1) {
        const real g1 = group_sum(fg1, Tw);
        if (leader) fa[1] += g1;
      }
      if (A.n_feats > 2) {
        const real g2 = group_sum(fg2, Tw);
        if (leader) fa[2] += g2;
      }
      if (A.n_feats > 3) {
        const real g3 = group_sum(fg3, Tw);
        if (leader) fa[3] += g3;
      }
    }
  }
  // The wave sums of the slots (the first two only when N == 2), added to
  // this wave's LDS columns by lane 0, in slot order.
  template <int N>
  __device__ __forceinline__ void add_terms(const Terms& t, int lane, int wave) {
    real s[4];
    if constexpr (N == 2) {
      // lanes 0-31 hold slot 0's sum, lanes 32-63 slot 1's
      const real r = group_sum(swap32_sum(t.v[0], t.v[1]), 32);
      s[0] = lane_value(r, 0);
      s[1] = lane_value(r, 32);
    } else {
      const real r = rows_sum4(t.v[0], t.v[1], t.v[2], t.v[3]);
      s[0] = lane_value(r, 0);
      s[1] = lane_value(r, 16);
      s[2] = lane_value(r, 32);
      s[3] = lane_value(r, 48);
    }
    if (lane == 0) {
      real* ga = gacc + (size_t)wave * A.n_acc;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        if (t.cw[k] >= 0) atomicAdd(&ga[t.cw[k]], s[k]);
        if (t.cb[k] >= 0) atomicAdd(&ga[t.cb[k]], s[k]);
      }
    }
  }
  // The gradient sums of a block's two rotations (shared parameters): one
  // two-slot sum without features, else one four-slot sum.
  __device__ __forceinline__ void accum2(const BGate& ga, real pa, const BGate& gb, real pb,
                                         int lane, int wave, int Tw) {
    Terms t;
    if (ga.feat < 0 && gb.feat < 0) {
      shared_terms<0>(t, ga, pa, Tw);
      shared_terms<1>(t, gb, pb, Tw);
      add_terms<2>(t, lane, wave);
    } else {
      shared_terms<0>(t, ga, pa, Tw);
      shared_terms<2>(t, gb, pb, Tw);
      add_terms<4>(t, lane, wave);
    }
  }

  // Per-sample parameter sets, a sample spanning whole waves, no features:
  // the wave sums of a block's two rotations in one reduce-scatter (lanes
  // 0-31 end with the first, 32-63 with the second), added to the sample's
  // parameter gradients by lane 0 of each wave.
  __device__ __forceinline__ void accum2_rows(const BGate& ga, real pa, const BGate& gb,
                                              real pb, int lane) {
    const bool ra = bg_kind(ga) <= QS_OP_RZ, rb = bg_kind(gb) <= QS_OP_RZ;
    const real r = group_sum(swap32_sum(ra ? (real)ga.scale * pa : (real)0,
                                        rb ? (real)gb.scale * pb : (real)0), 32);
    const real sa = lane_value(r, 0), sb = lane_value(r, 32);
    if (lane == 0 && active) {
      double* gp = A.grad_params + (size_t)row * A.n_params;
      if (ra && ga.p_w >= 0) atomicAdd(&gp[ga.p_w], (double)sa);
      if (ra && ga.p_b >= 0) atomicAdd(&gp[ga.p_b], (double)sa);
      if (rb && gb.p_w >= 0) atomicAdd(&gp[gb.p_w], (double)sb);
      if (rb && gb.p_b >= 0) atomicAdd(&gp[gb.p_b], (double)sb);
    }
  }

  // Adds this thread's partial dL/dtheta of the rotation with record `gt`
  // to the gradient sums: shared parameters through per-wave LDS slots,
  // per-sample parameter sets with FP64 atomics, features per sample. Each
  // LDS slot has a single writer (one lane of one wave), so its LDS atomic
  // adds (which need no wait) happen in program order: the sums stay
  // bitwise reproducible.
  __device__ __forceinline__ void accum(const BGate& gt, real part, int lane, int wave,
                                        int Tw) {
    const real scale = (real)gt.scale;
    if (!A.per_sample_params && gt.feat < 0) {
      // shared parameters, no feature: dL/dP += scale sum_b dL/dtheta_b
      const real v = group_sum(part, 64);
      if (lane == 0) {
        real* ga = gacc + (size_t)wave * A.n_acc;
        if (gt.col_w >= 0) atomicAdd(&ga[gt.col_w], scale * v);
        if (gt.col_b >= 0) atomicAdd(&ga[gt.col_b], scale * v);
      }
      return;
    }
    const real gth = group_sum(part, Tw);  // this sample (this wave's share)
    const bool leader = (tau & (Tw - 1)) == 0 && active;
    const real* P = param_row(A, active ? row : 0);
    const real f = (gt.feat >= 0 && active) ? fsh[(size_t)sl * A.n_feats + gt.feat] : (real)1;
    if (A.per_sample_params) {
      if (leader) {
        double* gp = A.grad_params + (size_t)row * A.n_params;
        if (gt.p_w >= 0) atomicAdd(&gp[gt.p_w], (double)(gth * scale * f));
        if (gt.p_b >= 0) atomicAdd(&gp[gt.p_b], (double)(gth * scale));
      }
    } else {
      // every lane of a sample holds its gth: sum over the wave's samples
      if (gt.p_w >= 0) {
        const real v = cross_sum(active ? gth * scale * f : (real)0, Tw);
        if (lane == 0) atomicAdd(&gacc[(size_t)wave * A.n_acc + gt.col_w], v);
      }
      if (gt.p_b >= 0) {
        const real v = cross_sum(active ? gth * scale : (real)0, Tw);
        if (lane == 0) atomicAdd(&gacc[(size_t)wave * A.n_acc + gt.col_b], v);
      }
    }
    if (gt.feat >= 0 && leader) {
      const real w = gt.p_w >= 0 ? P[gt.p_w] : (real)1;
      atomicAdd(&facc[((size_t)sl * wps + (tau >> 6)) * A.n_feats + gt.feat],
                gth * scale * w);
    }
  }

  // Backward through an L1Q op: its second sign pattern un-applied (a sign
  // pattern is its own inverse); for each register bit, one pass forms the
  // Pauli partials at the block output and un-applies the block from psi
  // and lam, and each rotation of the block takes its gradient as its
  // generator frame dotted with the partials (frames of blocks with shared
  // angles come from LDS; per-sample blocks walk theirs here); then its
  // first sign pattern un-applied.
  template <bool RYRZ = false>
  __device__ __forceinline__ void adjoint_l1q(St<real, R>& psi, St<real, R>& lam, int rec,
                                              int lane, int wave, int Tw) {
    const L1QRec r = kload(reinterpret_cast<const L1QRec*>(A.l1q), rec);
    apply_signs(psi, lam, r.w[kL1QPostDiag]);
    if constexpr (RYRZ) {
      // Every block of the plan is RY then RZ: one gate at a time, with
      // each gate's partial in its own basis (no generator frames); a
      // register bit without a block passes through with angle 0.
      static_for<LR>([&](auto J) QS_AI {
        constexpr int j = decltype(J)::value;
        const int bid = r.w[j];
        BGate g0{}, g1{};
        real c0 = 1, s0 = 0, c1 = 1, s1 = 0;
        if (bid >= 0) {
          // every block holds two gates, so block bid's records start at
          // 2 bid (no scalar load of the block table to wait on)
          g0 = kload(A.blk_rec, 2 * bid);
          g1 = kload(A.blk_rec, 2 * bid + 1);
          gate_cs(g0, c0, s0);
          gate_cs(g1, c1, s1);
        }
        const G3<real> pg = ryrz_and_apply<j>(psi, lam, c0, s0, c1, s1);
        if (bid >= 0) {
          __builtin_amdgcn_s_setprio(1);
          if (!A.per_sample_params) {
            accum2(g0, pg.y, g1, pg.z, lane, wave, Tw);
          } else if (Tw == 64 && g0.feat < 0 && g1.feat < 0) {
            accum2_rows(g0, pg.y, g1, pg.z, lane);
          } else {
            accum(g1, pg.z, lane, wave, Tw);
            accum(g0, pg.y, lane, wave, Tw);
          }
          __builtin_amdgcn_s_setprio(0);
        }
      });
      apply_signs(psi, lam, r.w[kL1QPreDiag]);
      return;
    }
    static_for<LR>([&](auto J) QS_AI {
      constexpr int j = decltype(J)::value;
      const int bid = r.w[j];
      const int fu = r.w[kL1QFused + j];
      // A per-sample block of two gates (RY then RZ, say): its two records
      // and angles are fetched once, together, for the matrix and again
      // for the generator frames.
      bool two = false;
      BGate g0{}, g1{};
      real c0 = 1, s0 = 0, c1 = 1, s1 = 0;
      U2<real> u;
      if constexpr (!SHARED && sizeof(real) == 4) {  // complex128: no registers to spare
        if (bid >= 0 && fu < 0) {
          const int b0 = kc(A.blk_begin)[bid];
          two = kc(A.blk_begin)[bid + 1] - b0 == 2;
          if (two) {
            g0 = kload(A.blk_rec, b0);
            g1 = kload(A.blk_rec, b0 + 1);
            if (bg_kind(g0) <= QS_OP_RZ) gate_cs(g0, c0, s0);
            if (bg_kind(g1) <= QS_OP_RZ) gate_cs(g1, c1, s1);
            u = two_u(bg_kind(g0), c0, s0, bg_kind(g1), c1, s1);
          }
        }
      }
      if (!two) u = block_or_id(bid, fu);
      const G3<real> pg = pauli_and_apply<j>(psi, lam, u_dag(u));
      if (bid >= 0) {  // reads pg only: no state copies at the join
        // The gradient sums (wave reductions, LDS adds) also run at raised
        // priority: they then overlap the other waves' block arithmetic.
        __builtin_amdgcn_s_setprio(1);
        const int b0 = kc(A.blk_begin)[bid], b1 = kc(A.blk_begin)[bid + 1];
        const int gen = kc(A.blk_gen)[bid];
        if (two) {
          // frames of the two gates, last gate first (as in the walk below)
          const int k1 = bg_kind(g1), k0 = bg_kind(g0);
          real p0, p1;
          if (k0 == QS_OP_RY && k1 == QS_OP_RZ) {
            // RZ's frame is Z itself; RY's is Y turned about Z by RZ's angle
            const real co = c1 * c1 - s1 * s1, si = 2 * c1 * s1;
            p1 = pg.z;
            p0 = co * pg.y - si * pg.x;
          } else {
            P3<real> m;
            p1 = k1 == QS_OP_RX ? m.dot(0, pg) : k1 == QS_OP_RY ? m.dot(1, pg) : m.dot(2, pg);
            m.conj_by(k1, c1, s1);
            p0 = k0 == QS_OP_RX ? m.dot(0, pg) : k0 == QS_OP_RY ? m.dot(1, pg) : m.dot(2, pg);
          }
          if (!A.per_sample_params) {
            accum2(g0, p0, g1, p1, lane, wave, Tw);
          } else if (Tw == 64 && g0.feat < 0 && g1.feat < 0) {
            accum2_rows(g0, p0, g1, p1, lane);
          } else {
            if (k1 <= QS_OP_RZ) accum(g1, p1, lane, wave, Tw);
            if (k0 <= QS_OP_RZ) accum(g0, p0, lane, wave, Tw);
          }
        } else if (sizeof(real) == 8 && !A.per_sample_params && (SHARED || gen >= 0)) {
          // Shared angles (so no features): one slot per rotation, four
          // rotations per wave sum. Complex128 only: its FP64 sums take
          // twice the lane moves, and there this measured 2 % faster (on
          // the 10-qubit batch); complex64 ran 1.6 % slower with it.
          for (int i0 = b0; i0 < b1; i0 += 4) {
            Terms t;
            static_for<4>([&](auto KC) QS_AI {
              constexpr int k = decltype(KC)::value;
              if (i0 + k < b1) {
                const BGate gt = kload(A.blk_rec, i0 + k);
                const real* e = gen_sh + 3 * (size_t)(gen + i0 + k - b0);
                shared_terms<k>(t, gt, e[0] * pg.x + e[1] * pg.y + e[2] * pg.z, Tw);
              }
            });
            if (b1 - i0 <= 2)
              add_terms<2>(t, lane, wave);
            else
              add_terms<4>(t, lane, wave);
          }
        } else if (SHARED || gen >= 0) {
          for (int i = b0; i < b1; ++i) {
            const BGate gt = kload(A.blk_rec, i);
            if (bg_kind(gt) > QS_OP_RZ) continue;
            const real* e = gen_sh + 3 * (size_t)(gen + i - b0);
            accum(gt, e[0] * pg.x + e[1] * pg.y + e[2] * pg.z, lane, wave, Tw);
          }
        } else if constexpr (!SHARED) {
          P3<real> m;
          for (int i = b1 - 1; i >= b0; --i) {
            const BGate gt = kload(A.blk_rec, i);
            const int kind = bg_kind(gt);
            real c = 1, sn = 0;
            if (kind <= QS_OP_RZ) {
              gate_cs(gt, c, sn);
              const real part = kind == QS_OP_RX ? m.dot(0, pg)
                                : kind == QS_OP_RY ? m.dot(1, pg) : m.dot(2, pg);
              accum(gt, part, lane, wave, Tw);
            }
            if (i > b0) m.conj_by(kind, c, sn);
          }
        }
        __builtin_amdgcn_s_setprio(0);
      }
    });
    apply_signs(psi, lam, r.w[kL1QPreDiag]);
  }
};

// Common prologue: LDS carve-up and angle tables.
// `blk` is the global index of the block's first sample. Gradient sums are
// kept in per-wave LDS slots (each written by one lane of one wave) and added
// in a fixed order at the end, so the adjoint is bitwise reproducible.
template <typename real, int LR, bool FLY, bool SHARED, bool HALF>
__device__ __forceinline__ void setup(Ctx<real, LR, FLY, SHARED, HALF>& C,
                                      const Args<real>& A, unsigned char* smem, bool adjoint,
                                      int64_t blk) {
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
  constexpr int comps = HALF ? 1 : 2;  // reals per staged amplitude
  real* st = reinterpret_cast<real*>(smem);
  C.ldr = st + (size_t)C.sl * N * comps;
  C.lds = reinterpret_cast<typename V2<real>::T*>(C.ldr);
  // Samples sharing a wave get different salts, so that one LDS access of
  // the wave spreads over all banks: 32 slot values cover the 64 banks when
  // a slot is a complex pair; with one component staged (4-byte slots) the
  // salt takes 64 values.
  C.salt = ((uint32_t)C.sl << A.t) & (HALF ? 63u : 31u) & (uint32_t)(N - 1);
  if (HALF && A.salt_basis != 0 && A.t < 6) {
    // the plan's salts: chosen on the host so that the lanes of a wave hit
    // different banks under as many of the plan's layouts as possible
    uint32_t sv = 0;
    for (int i = 0; i < 6 - A.t; ++i)
      if ((C.sl >> i) & 1) sv ^= (uint32_t)(A.salt_basis >> (6 * i)) & 63u;
    C.salt = sv & (uint32_t)(N - 1);
  }
  real* tail = st + (size_t)A.S * N * comps;
  C.ang_sh = tail;
  C.ang_ps = C.ang_sh + 2 * (size_t)A.n_gates;
  C.fu_sh = C.ang_ps + (FLY ? 0 : 2 * (size_t)A.n_slots * A.S);
  C.gen_sh = C.fu_sh + 8 * ((size_t)A.n_fu + 1);
  C.gacc = C.gen_sh + (adjoint ? 3 * (size_t)A.n_gen : 0);
  C.wps = A.t > 6 ? (1 << (A.t - 6)) : 1;
  const int waves = blockDim.x >> 6;
  C.facc = C.gacc + (A.per_sample_params ? 0 : (size_t)waves * A.n_acc);
  C.fsh = C.facc + (adjoint ? (size_t)A.S * C.wps * A.n_feats : 0);
  {
    // 8-byte aligned, after the features
    const uintptr_t e = reinterpret_cast<uintptr_t>(C.fsh + (adjoint ? (size_t)A.S * A.n_feats : 0));
    C.lsq = reinterpret_cast<double*>((e + 7) & ~(uintptr_t)7);
  }

  // Shared angles, by gate.
  for (int g = tid; g < A.n_gates; g += blockDim.x) {
    const qs_gate gt = A.gates[g];
    real c = 1, s = 0;
    if (gt.op <= QS_OP_RZ && A.gate_slot[g] < 0) {
      real th = theta_of(A, gt, 0);  // shared: no feature, shared params
      fsincos(th * (real)0.5, &s, &c);
    }
    C.ang_sh[2 * g] = c;
    C.ang_sh[2 * g + 1] = s;
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
  if constexpr (sizeof(real) == 4 && !SHARED) {
    if (adjoint && A.n_feats <= 4 && C.active) {
      const real* fr = A.feats + (size_t)C.row * A.n_feats;
      if (A.n_feats > 0) C.fx0 = fr[0];
      if (A.n_feats > 1) C.fx1 = fr[1];
      if (A.n_feats > 2) C.fx2 = fr[2];
      if (A.n_feats > 3) C.fx3 = fr[3];
    }
  }
  if (adjoint) {
    if (!A.per_sample_params)
      for (int i = tid; i < waves * A.n_acc; i += blockDim.x) C.gacc[i] = 0;
    for (int i = tid; i < A.S * C.wps * A.n_feats; i += blockDim.x) C.facc[i] = 0;
    // the features the gradient sums scale by, read from HBM once per sample
    for (int i = tid; i < A.S * A.n_feats; i += blockDim.x) {
      const int64_t bb = blk + i / A.n_feats;
      C.fsh[i] = bb < A.B ? A.feats[(size_t)(bb >> A.ob) * A.n_feats + i % A.n_feats] : (real)0;
    }
  }
  __syncthreads();
  // Fused matrices of the blocks whose angles are shared; slot n_fu holds the
  // identity (register bits without a block).
  if (tid == 0) {
    real* f = C.fu_sh + 8 * (size_t)A.n_fu;
    f[0] = 1; f[1] = 0; f[2] = 0; f[3] = 0; f[4] = 0; f[5] = 0; f[6] = 1; f[7] = 0;
  }
  for (int bid = tid; bid < A.n_blocks; bid += blockDim.x) {
    const int fu = A.blk_fu[bid];
    if (fu < 0) continue;
    U2<real> u{1, 0, 0, 0, 0, 0, 1, 0};
    for (int i = A.blk_begin[bid]; i < A.blk_begin[bid + 1]; ++i) {
      const int g = A.blk_rec[i].g;
      u = gate_lmul(bg_kind(A.blk_rec[i]), C.ang_sh[2 * g], C.ang_sh[2 * g + 1], u);
    }
    real* f = C.fu_sh + 8 * (size_t)fu;
    f[0] = u.r00; f[1] = u.i00; f[2] = u.r01; f[3] = u.i01;
    f[4] = u.r10; f[5] = u.i10; f[6] = u.r11; f[7] = u.i11;
    if (!adjoint) continue;
    // Generator frames, last gate first (see Ctx::adjoint_l1q).
    const int b0 = A.blk_begin[bid], gen = A.blk_gen[bid];
    P3<real> m;
    for (int i = A.blk_begin[bid + 1] - 1; i >= b0; --i) {
      const int g = A.blk_rec[i].g;
      const int kind = bg_kind(A.blk_rec[i]);
      const real c = C.ang_sh[2 * g], sn = C.ang_sh[2 * g + 1];
      real* e = C.gen_sh + 3 * (size_t)(gen + i - b0);
#pragma unroll
      for (int k = 0; k < 3; ++k)  // constant indices keep m in registers
        e[k] = kind == QS_OP_RX ? m.c[0][k] : kind == QS_OP_RY ? m.c[1][k] : m.c[2][k];
      m.conj_by(kind, c, sn);
    }
  }
  __syncthreads();
}

template <typename real, int LR>
__device__ __forceinline__ const QS_K uint8_t* seg_map(const Args<real>& A, int s) {
  return kc(A.seg_map) + (size_t)s * kMapStride;
}
// Layout of segment s when its state is read in (rlay) and written out at its
// end (wlay: includes the CNOTs folded there).
template <typename real>
__device__ __forceinline__ const QS_K uint16_t* rlay(const Args<real>& A, int s) {
  return kc(A.seg_lay) + (size_t)s * kLayWords;
}
template <typename real>
__device__ __forceinline__ const QS_K uint16_t* wlay(const Args<real>& A, int s) {
  return kc(A.seg_lay) + (size_t)s * kLayWords + kMapStride;
}
// A remap is needed between segments s - 1 and s unless the end layout of
// s - 1 is the start layout of s.
template <typename real>
__device__ __forceinline__ bool map_changed(const Args<real>& A, int s) {
  const QS_K uint32_t* a = reinterpret_cast<const QS_K uint32_t*>(wlay(A, s - 1));
  const QS_K uint32_t* b = reinterpret_cast<const QS_K uint32_t*>(rlay(A, s));
  bool ch = false;
#pragma unroll
  for (int w = 0; w < kMapStride / 2; ++w) ch |= a[w] != b[w];
  return ch;
}

// <Z_q> of every qubit in FP64 from the final register state x (arranged by
// the last segment's layout, `last` = its qubit of each physical bit): each
// wave's sums go to the sample's staging region, red[w * n + q], where every
// thread of the sample can read them until the next staging pass; the
// sample's totals go to expz when it is given.
template <typename real, int LR, bool FLY, bool SHARED, bool HALF>
__device__ __forceinline__ void readout(const Ctx<real, LR, FLY, SHARED, HALF>& C,
                                        const Args<real>& A, const St<real, (1 << LR)>& x,
                                        const QS_K uint8_t* last) {
  constexpr int R = 1 << LR;
  // <Z_q> partials in FP64, reduced over the sample's threads.
  const int Tw = (1 << A.t) < 64 ? (1 << A.t) : 64;
  const int nw = (1 << A.t) / Tw;  // waves per sample
  double* red = reinterpret_cast<double*>(C.ldr);
  sample_sync(A.t);
  // tot = sum_k |x_k|^2 and hi[j] = the part with register bit j set, so a
  // register-bit qubit reads tot - 2 hi[j] and a thread-bit one +-tot.
  double tot = 0;
  double hi[LR > 0 ? LR : 1];
#pragma unroll
  for (int j = 0; j < LR; ++j) hi[j] = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const double pk = (double)x.re[k] * x.re[k] + (double)x.im[k] * x.im[k];
    tot += pk;
#pragma unroll
    for (int j = 0; j < LR; ++j)
      if (k & (1 << j)) hi[j] += pk;
  }
  const int wave_in_sample = C.tau / Tw;
  for (int q = 0; q < A.n; ++q) {
    int p = 0;
    for (int i = 0; i < A.n; ++i)
      if (last[i] == q) p = i;
    p = uni(p);
    double z;
    if (p < LR) {
      double h = hi[0];
#pragma unroll
      for (int j = 1; j < LR; ++j)
        if (p == j) h = hi[j];
      z = tot - 2 * h;
    } else {
      z = C.tbit(p) ? -tot : tot;
    }
    z = group_sum(z, Tw);
    if ((C.tau & (Tw - 1)) == 0) red[(size_t)wave_in_sample * A.n + q] = z;
  }
  sample_sync(A.t);
  if (C.active && A.expz != nullptr)
    for (int q = C.tau; q < A.n; q += (1 << A.t)) {
      double z = 0;
      for (int w = 0; w < nw; ++w) z += red[(size_t)w * A.n + q];
      A.expz[(size_t)C.b * A.n + q] = z;
    }
}

// ------------------------------------------------------------------ forward
template <typename real, int LR, bool FLY = false, bool SHARED = false, bool HALF = false>
__device__ __forceinline__ void forward_body(const Args<real>& A, unsigned char* smem,
                                             int64_t blk) {
  constexpr int R = 1 << LR;
  Ctx<real, LR, FLY, SHARED, HALF> C(A);
  setup(C, A, smem, false, blk);

  St<real, R> x;
  // (one-component staging keeps both components live through its passes;
  // an encoding branch there doubles the registers, so such launches get an
  // encoded state instead)
  C.load_state(x, A.state, rlay(A, 0), !FLY && !HALF && A.x_in != nullptr);
  const int nseg = A.nseg;
  const QS_K int32_t* seg_begin = kc(A.seg_begin);
  for (int s = 0; s < nseg; ++s) {
    if (s > 0 && map_changed(A, s))
      C.remap(x, wlay(A, s - 1), rlay(A, s));
    const int e = seg_begin[s + 1];
    for (int o = seg_begin[s]; o < e; ++o) C.apply_l1q(x, o);
    const int ck = kc(A.seg_ckpt)[s];
    if (ck >= 0 && A.ckpt != nullptr)
      C.store_state(x, A.ckpt + (size_t)ck * A.B * (2ull << A.n), wlay(A, s));
  }
  // The last segment ends in a plain placement (no folded CNOTs).
  const QS_K uint8_t* last = seg_map<real, LR>(A, nseg - 1);
  C.store_state(x, A.state, wlay(A, nseg - 1));

  if (A.expz != nullptr) readout(C, A, x, last);
}

// The adjoint's reverse sweep from (psi, lam) at the circuit's end, and the
// flush of its gradient sums.
template <typename real, int LR, bool FLY, bool SHARED, bool HALF, bool RYRZ, bool TRAIN>
__device__ __forceinline__ void adjoint_sweep(const Args<real>& A,
                                              Ctx<real, LR, FLY, SHARED, HALF>& C,
                                              St<real, (1 << LR)>& psi, St<real, (1 << LR)>& lam,
                                              int64_t blk) {
  const int nseg = A.nseg;
  const int Tw = (1 << A.t) < 64 ? (1 << A.t) : 64;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const QS_K int32_t* seg_begin = kc(A.seg_begin);
  for (int s = nseg - 1; s >= 0; --s) {
    const int ck = kc(A.seg_ckpt)[s];
    if (ck >= 0 && A.ckpt != nullptr)  // re-anchor psi to the stored state
      C.load_state(psi, A.ckpt + (size_t)ck * A.B * (2ull << A.n), wlay(A, s));
    const int beg = seg_begin[s];
    for (int o = seg_begin[s + 1] - 1; o >= beg; --o)
      C.template adjoint_l1q<RYRZ>(psi, lam, o, lane, wave, Tw);
    if (s > 0 && map_changed(A, s)) {
      C.remap(psi, rlay(A, s), wlay(A, s - 1));
      C.remap(lam, rlay(A, s), wlay(A, s - 1));
    }
  }
  C.fold_feature_terms(Tw);
  if (A.out_psi != nullptr) C.store_state(psi, A.out_psi, rlay(A, 0));
  if (A.out_lam != nullptr) C.store_state(lam, A.out_lam, rlay(A, 0));
  __syncthreads();
  const int waves = blockDim.x >> 6;
  if (!A.per_sample_params)
    for (int i = threadIdx.x; i < A.n_acc; i += blockDim.x) {
      real t = 0;
      for (int w = 0; w < waves; ++w) t += C.gacc[(size_t)w * A.n_acc + i];
      A.ws_partials[(size_t)blockIdx.x * A.n_acc + i] = t;
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
      else if (A.accum_feats)
        *dst += t;  // one writer per entry; earlier segments' sums are in place
      else
        *dst = t;
    }
  if constexpr (TRAIN) {
    // the workgroup's squared residuals, summed in sample order
    if (threadIdx.x == 0) {
      double t = 0;
      for (int sl = 0; sl < A.S && blk + sl < A.B; ++sl) t += C.lsq[sl];
      A.loss_part[blockIdx.x] = t;
    }
  }
}

// ------------------------------------------------------------------ adjoint
template <typename real, int LR, bool FLY = false, bool SHARED = false, bool HALF = false,
          bool RYRZ = false, bool TRAIN = false,
          bool KERNARG = false>
__device__ __forceinline__ void adjoint_body(const Args<real>& A, unsigned char* smem,
                                             int64_t blk) {
  constexpr int R = 1 << LR;
  Ctx<real, LR, FLY, SHARED, HALF> C(A);
  setup(C, A, smem, true, blk);
  const int nseg = A.nseg;
  const QS_K uint8_t* last = seg_map<real, LR>(A, nseg - 1);

  St<real, R> psi, lam;
  double g_loss = 0;  // training step: dL/d<Z_q> of this sample, q = A.loss_q
  if constexpr (TRAIN) {
    // The forward sweep, its readout and the loss without leaving registers:
    // psi ends in the layout the adjoint starts from.
    C.load_state(psi, A.state, rlay(A, 0), !HALF && A.x_in != nullptr);
    const QS_K int32_t* fseg = kc(A.seg_begin);
    for (int s = 0; s < nseg; ++s) {
      if (s > 0 && map_changed(A, s)) C.remap(psi, wlay(A, s - 1), rlay(A, s));
      const int e = fseg[s + 1];
      for (int o = fseg[s]; o < e; ++o) C.apply_l1q(psi, o);
    }
    readout(C, A, psi, last);
    const int Tw = (1 << A.t) < 64 ? (1 << A.t) : 64;
    const double* red = reinterpret_cast<const double*>(C.ldr);
    double z = 0;
    for (int w = 0; w < (1 << A.t) / Tw; ++w) z += red[(size_t)w * A.n + A.loss_q];
    const double r = C.active ? z - A.y[C.b] : 0.0;
    g_loss = 2.0 * r / (double)A.B;
    if (C.tau == 0) C.lsq[C.sl] = r * r;
  } else {
    C.load_state(psi, A.state, wlay(A, nseg - 1));
  }
  if (!TRAIN && A.dstate != nullptr) {
    C.load_state(lam, A.dstate, wlay(A, nseg - 1));
  } else {
    // lam = sum_q g_q Z_q psi: coefficient of amplitude with logical index L
    // is sum_q g_q - 2 sum_{q : bit q of L = 1} g_q.
    double base = 0;
    double w[LR > 0 ? LR : 1];
#pragma unroll
    for (int j = 0; j < LR; ++j) w[j] = 0;
    if (C.active) {
      const double* g = TRAIN ? nullptr : A.dexpz + (size_t)C.b * A.n;
      auto gq_of = [&](int q) -> double {
        if constexpr (TRAIN)
          return q == A.loss_q ? g_loss : 0.0;
        else
          return g[q];
      };
      for (int p = 0; p < A.n; ++p) {
        const double gq = gq_of(last[p]);
        base += gq;
        if (p >= LR && C.tbit(p)) base -= 2 * gq;
      }
#pragma unroll
      for (int j = 0; j < LR; ++j) w[j] = 2 * gq_of(last[j]);
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

  if constexpr (KERNARG) {
    // The sweep reads the launch's arguments through an address the compiler
    // cannot see through, so their loop invariants are loaded here rather
    // than hoisted to the kernel's entry: the values of the training step's
    // forward sweep then do not compete with them for scalar registers
    // (without this the compiler spills scalars to vector lanes, 200 lane
    // reads per op in the adjoint's loop). The plain adjoint does not take
    // it: there it cut the spills too but ran 2-3 % slower.
    const QS_K Args<real>* pa = (const QS_K Args<real>*)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(pa));
    const Args<real>& A2 = *(const Args<real>*)(pa);
    Ctx<real, LR, FLY, SHARED, HALF> C2(A2, C);
    adjoint_sweep<real, LR, FLY, SHARED, HALF, RYRZ, TRAIN>(A2, C2, psi, lam, blk);
  } else {
    adjoint_sweep<real, LR, FLY, SHARED, HALF, RYRZ, TRAIN>(A, C, psi, lam, blk);
  }
}

template <typename real, int LR, int MAXT, bool SHARED, bool HALF>
__global__ void __launch_bounds__(MAXT) sv_forward(Args<real> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  forward_body<real, LR, false, SHARED, HALF>(A, smem, (int64_t)blockIdx.x * A.S);
}

template <typename real, int LR, int MAXT, bool SHARED, bool HALF, bool RYRZ = false>
__global__ void __launch_bounds__(MAXT) sv_adjoint(Args<real> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  // The sweep re-reads its arguments (see adjoint_body) in the complex64
  // RY-then-RZ kernels, where that measured faster (26-qubit tiled epochs
  // -6 %, 8-qubit re-uploading batch -2 %); the complex64 fused-block
  // adjoint ran 3 % slower with it, and complex128 gained nothing.
  adjoint_body<real, LR, false, SHARED, HALF, RYRZ, false, RYRZ && sizeof(real) == 4>(
      A, smem, (int64_t)blockIdx.x * A.S);
}

// A training step in one launch: forward sweep (from the amplitude encoding
// of x, or from |0...0>), readout, MSE loss on one qubit, adjoint.
template <typename real, int LR, int MAXT, bool SHARED, bool HALF, bool RYRZ = false>
__global__ void __launch_bounds__(MAXT) sv_train(Args<real> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  adjoint_body<real, LR, false, SHARED, HALF, RYRZ, true, true>(A, smem,
                                                               (int64_t)blockIdx.x * A.S);
}

// Uneven batches in one persistent launch: workgroups pull work items (a
// class of identically-structured circuits and a run of S of its circuits)
// from an atomic counter until the queue is empty; items are ordered longest
// first. Every workgroup runs the same engine as the batched kernels, with
// per-circuit angles computed in place (no per-sample LDS table).
template <typename real, int LR, int MAXT, bool ADJ, bool HALF>
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
    A.seg_lay = cd.seg_lay;
    A.seg_begin = cd.seg_begin;
    A.seg_ckpt = cd.seg_ckpt;
    A.ops = cd.ops;
    A.gates = cd.gates;
    A.gate_slot = cd.gate_slot;
    A.slot_gate = cd.slot_gate;
    A.l1q = cd.l1q;
    A.diag = cd.diag;
    A.blk_begin = cd.blk_begin;
    A.blk_rec = cd.blk_rec;
    A.blk_fu = cd.blk_fu;
    A.blk_gen = cd.blk_gen;
    A.n_gen = cd.n_gen;
    A.n_blocks = cd.n_blocks;
    A.n_fu = cd.n_fu;
    A.n = cd.n;
    A.t = cd.t;
    A.nseg = cd.nseg;
    A.n_gates = cd.n_gates;
    A.n_slots = cd.n_slots;
    A.n_params = cd.n_params;
    A.n_acc = 0;
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
    A.accum_feats = 0;
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
    A.x_in = nullptr;
    A.x_stride = 0;
    A.x_D = 0;
    A.bad_rows = nullptr;
    A.y = nullptr;
    A.loss_q = 0;
    A.loss_part = nullptr;
    A.salt_basis = 0;
    // Complex64 classes whose per-circuit angle table fits the LDS budget
    // next to the staging take the table path (sines and cosines once per
    // gate and circuit, in the prologue); the others compute angles where
    // they use them. (Complex128 keeps one path: its adjoint has no
    // registers to spare for a second.)
    bool table = false;
    if constexpr (sizeof(real) == 4) table = cd.table != 0;  // complex64 only
    // Complex64 classes whose blocks are all RY then RZ take the adjoint's
    // gate-at-a-time pass.
    bool ryrz = false;
    if constexpr (sizeof(real) == 4 && ADJ) ryrz = cd.ryrz != 0;
    if (table) {
      if constexpr (ADJ) {
        if (ryrz)
          adjoint_body<real, LR, false, false, HALF, true>(A, smem, 0);
        else
          adjoint_body<real, LR, false, false, HALF>(A, smem, 0);
      } else {
        forward_body<real, LR, false, false, HALF>(A, smem, 0);
      }
    } else {
      if constexpr (ADJ) {
        if (ryrz)
          adjoint_body<real, LR, true, false, HALF, true>(A, smem, 0);
        else
          adjoint_body<real, LR, true, false, HALF>(A, smem, 0);
      } else {
        forward_body<real, LR, true, false, HALF>(A, smem, 0);
      }
    }
    __syncthreads();  // the next item reuses the LDS
  }
}


template <typename real>
Args<real> make_args(const SvLaunch& L) {
  const SvDevPlan& p = *L.p;
  Args<real> A;
  A.seg_map = p.seg_map;
  A.seg_lay = p.seg_lay;
  A.seg_begin = p.seg_begin;
  A.seg_ckpt = p.seg_ckpt;
  A.ops = p.ops;
  A.gates = p.gates;
  A.gate_slot = p.gate_slot;
  A.slot_gate = p.slot_gate;
  A.l1q = p.l1q;
  A.diag = p.diag;
  A.blk_begin = p.blk_begin;
  A.blk_rec = p.blk_rec;
  A.blk_fu = p.blk_fu;
  A.blk_gen = p.blk_gen;
  A.n_gen = p.n_gen;
  A.n_blocks = p.n_blocks;
  A.n_fu = p.n_fu;
  A.n = p.n;
  A.t = p.t;
  A.nseg = p.nseg;
  A.n_gates = p.n_gates;
  A.n_slots = p.n_slots;
  A.n_params = p.n_params;
  A.n_acc = p.n_acc;
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
  A.accum_feats = L.accum_feats;
  A.x_in = static_cast<const real*>(L.x_in);
  A.x_stride = L.x_stride;
  A.x_D = L.x_D;
  A.bad_rows = L.bad_rows;
  A.y = L.y;
  A.loss_q = L.loss_q;
  A.loss_part = L.loss_part;
  A.salt_basis = L.shape.half ? p.salt_half : 0;
  return A;
}

template <typename real, int LR, int MAXT, bool ADJ, bool SHARED = false, bool HALF = false,
          bool RYRZ = false, bool TRAIN = false>
int launch_one(const SvLaunch& L) {
  Args<real> A = make_args<real>(L);
  const int64_t grid = (A.B + A.S - 1) / A.S;
  if (grid <= 0) return QS_OK;
  dim3 g((unsigned)grid), blk((unsigned)L.shape.block_threads);
  hipStream_t st = static_cast<hipStream_t>(L.stream);
  // Only the kernel of this direction is instantiated.
  auto kern = [] {
    if constexpr (TRAIN)
      return sv_train<real, LR, MAXT, SHARED, HALF, RYRZ>;
    else if constexpr (ADJ)
      return sv_adjoint<real, LR, MAXT, SHARED, HALF, RYRZ>;
    else
      return sv_forward<real, LR, MAXT, SHARED, HALF>;
  }();
  if (L.shape.lds_bytes > 65536) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)L.shape.lds_bytes) != hipSuccess)
      return QS_ERR_LAUNCH;
  }
  hipLaunchKernelGGL(kern, g, blk, (size_t)L.shape.lds_bytes, st, A);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_LAUNCH;
}

template <typename real, int LR, int MAXT, bool HALF>
int launch_prog(const ProgLaunch& L, bool adjoint) {
  hipStream_t st = static_cast<hipStream_t>(L.stream);
  auto kern = adjoint ? sv_program<real, LR, MAXT, true, HALF>
                      : sv_program<real, LR, MAXT, false, HALF>;
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

// Per-(element type, direction) dispatchers over the register exponent r.
int sv_c64_forward(const SvLaunch& L);
int sv_c64_adjoint(const SvLaunch& L);
int sv_c128_forward(const SvLaunch& L);
int sv_c128_adjoint(const SvLaunch& L);

}  // namespace qs
