// Dense-block path for large states: each block of gates on K = 5 qubits is
// one 32 x 32 complex unitary M, applied to the whole state as a matrix
// product on MFMA (v_mfma_f32_32x32x2_f32) in its real embedding
//   [[Re M, -Im M], [Im M, Re M]]   (interleaved: row 2i + ci, column 2j + cj),
// with the state viewed as 2^(n-5) columns of 32 amplitudes (the block's
// qubits index the rows, all other qubits the column).
//
// MFMA operand layouts (32x32x2, fp32): lane l supplies A[l % 32][l / 32]
// and B[l / 32][l % 32]; accumulator a of lane l holds D[8 (a / 4) +
// 4 (l / 32) + a % 4][l % 32]. Each wave works on tiles of 32 columns (1024
// amplitudes): a tile moves between HBM and LDS in 16-byte pieces covering
// runs of contiguous amplitudes (whichever qubits the block holds), the next
// tile's loads are in flight while the current one is multiplied, and the
// MFMA operands are read from the tile in LDS.
//
// Adjoint (Jones & Gacon, arXiv:2009.02823, sec. 3, applied to a block): with
// psi and lam at the block's output, the gradient of a rotation g of the
// block is Im tr(P_g rho_g), rho_g the block-local matrix
// sum_columns psi_g lam_g^dagger taken just after g; rho at the block output
// is one more matrix product over the columns (K = the column index, again on
// MFMA), and rho_{g-1} = U_g^dagger rho_g U_g is a 32 x 32 walk done once per
// block. The pass un-applies M from psi and lam (M^dagger on MFMA).
#include <hip/hip_runtime.h>

#include "qs_internal.h"

namespace qs {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kD = 32;        // amplitudes per column (2^K, K = 5)
constexpr int kWaves = 4;     // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kRhoWords = 2 * kD * kD;

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// The 2x2 matrix of a one-qubit gate, u[2 * row + col], in FP64:
// R_P(t) = cos(t/2) I - i sin(t/2) P (Nielsen & Chuang sec. 4.2).
__device__ void gate2(int op, double th, double2 u[4]) {
  double s = 0.0, c = 1.0;
  if (op <= QS_OP_RZ) sincos(0.5 * th, &s, &c);
  const double h = 0.70710678118654752440;
  switch (op) {
    case QS_OP_RX:
      u[0] = make_double2(c, 0); u[1] = make_double2(0, -s);
      u[2] = make_double2(0, -s); u[3] = make_double2(c, 0);
      break;
    case QS_OP_RY:
      u[0] = make_double2(c, 0); u[1] = make_double2(-s, 0);
      u[2] = make_double2(s, 0); u[3] = make_double2(c, 0);
      break;
    case QS_OP_RZ:
      u[0] = make_double2(c, -s); u[1] = make_double2(0, 0);
      u[2] = make_double2(0, 0); u[3] = make_double2(c, s);
      break;
    case QS_OP_X:
      u[0] = make_double2(0, 0); u[1] = make_double2(1, 0);
      u[2] = make_double2(1, 0); u[3] = make_double2(0, 0);
      break;
    case QS_OP_Y:
      u[0] = make_double2(0, 0); u[1] = make_double2(0, -1);
      u[2] = make_double2(0, 1); u[3] = make_double2(0, 0);
      break;
    case QS_OP_Z:
      u[0] = make_double2(1, 0); u[1] = make_double2(0, 0);
      u[2] = make_double2(0, 0); u[3] = make_double2(-1, 0);
      break;
    default:  // QS_OP_H
      u[0] = make_double2(h, 0); u[1] = make_double2(h, 0);
      u[2] = make_double2(h, 0); u[3] = make_double2(-h, 0);
      break;
  }
}

// theta = scale * (w + bias): the descriptor's rule with no features.
__device__ inline double angle(const DbGate& g, const float* P) {
  const double w = g.p_w >= 0 ? (double)P[g.p_w] : 1.0;
  const double b = g.p_b >= 0 ? (double)P[g.p_b] : 0.0;
  return (double)g.scale * (w + b);
}

// M <- U_g ... U_1 (the block's gates in order) in FP64 in LDS, row-major
// [32][32]; the kThreads threads of the workgroup take kPer entries each.
constexpr int kPer = kD * kD / kThreads;
__device__ void build_block(double2* M, const DbGate* gates, int g0, int g1, const float* P) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int e = threadIdx.x + k * kThreads;
    M[e] = make_double2((e >> 5) == (e & 31) ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int j = g0; j < g1; ++j) {
    const DbGate g = gates[j];
    double2 u[4];
    const bool one = g.op <= QS_OP_H;
    if (one) gate2(g.op, g.op <= QS_OP_RZ ? angle(g, P) : 0.0, u);
    double2 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = threadIdx.x + k * kThreads;
      const int r = e >> 5, c = e & 31;
      if (one) {  // left-multiply by U on local bit q0
        const int m = 1 << g.q0, rb = (r >> g.q0) & 1;
        const double2 ua = rb ? u[2] : u[0], ub = rb ? u[3] : u[1];
        v[k] = cadd(cmul(ua, M[((r & ~m) << 5) | c]), cmul(ub, M[((r | m) << 5) | c]));
      } else if (g.op == QS_OP_CNOT) {
        const int src = ((r >> g.q0) & 1) ? r ^ (1 << g.q1) : r;
        v[k] = M[(src << 5) | c];
      } else {  // CZ
        const double2 x = M[e];
        v[k] = (((r >> g.q0) & (r >> g.q1)) & 1) ? make_double2(-x.x, -x.y) : x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) M[threadIdx.x + k * kThreads] = v[k];
    __syncthreads();
  }
}

// A-operand fragments of the real embedding of M (adjoint: of M^dagger):
// a[rt][s] = E[32 rt + l % 32][2 s + l / 32].
template <bool DAGGER>
__device__ void load_frags(const double2* M, float (&a)[2][kD]) {
  const int l = threadIdx.x & 63;
  const int h = l >> 5, ci = l & 1;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int i = rt * 16 + ((l & 31) >> 1);
#pragma unroll
    for (int s = 0; s < kD; ++s) {
      double2 m = DAGGER ? conjd(M[(s << 5) | i]) : M[(i << 5) | s];
      // (ci, cj): (0,0) Re, (0,1) -Im, (1,0) Im, (1,1) Re
      const double v = ci == h ? m.x : (ci ? m.y : -m.y);
      a[rt][s] = (float)v;
    }
  }
}

// A tile: the 32 x 32 amplitudes of 32 consecutive columns, whose addresses
// are base + off(t) for t < 1024, off spreading t's 10 bits over the tile's
// address positions (the first 5 are 0..4, so t's low 5 bits are a run of 32
// contiguous amplitudes). Each of t's bits is a bit of the column index j or
// of the block-local amplitude index s. In LDS a tile is two planes of 1024
// floats (real parts, then imaginary parts), amplitude (j, s) at slot
// 32 j + (j ^ s) of each: reading amplitude s of 32 columns, or the 32
// amplitudes of one column, from one plane touches 32 different banks
// whichever qubits the block holds. The slot is linear over GF(2) in t (and
// in (j, s)), so every LDS address is a per-lane base XOR a uniform term.
constexpr int kTileSlots = kD * kD;

struct Geo {
  int n, nk;          // qubits, column bits per state
  uint32_t qb[5];     // block qubit positions, ascending
  uint32_t pos[10];   // tile address positions, ascending
  uint32_t sv[10];    // slot of t = 1 << k: 1 << i for block bit i, 33 << j for column bit j
};

__device__ inline Geo make_geo(int n, const int32_t* q) {
  Geo G;
  G.n = n;
  G.nk = n - 5;
#pragma unroll
  for (int i = 0; i < 5; ++i) G.qb[i] = (uint32_t)q[i];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    G.pos[k] = (uint32_t)q[5 + k];
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      if (q[15 + i] == k) v = 1u << i;
      if (q[20 + i] == k) v = 33u << i;
    }
    G.sv[k] = v;
  }
  return G;
}

// Global amplitude index of tile g's t = 0: the column index 32 g spread over
// the positions outside the block (zeros inserted at the block's).
__device__ inline int64_t tile_base(const Geo& G, int64_t g) {
  const int64_t c = g << 5;
  const int64_t b = c >> G.nk;
  uint32_t x = (uint32_t)(c & ((int64_t(1) << G.nk) - 1));
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const uint32_t p = G.qb[i];
    x = ((x >> p) << (p + 1)) | (x & ((1u << p) - 1u));
  }
  return (b << G.n) + (int64_t)x;
}

// Lane l moves t = 2 l + 128 i and t + 1 (i < 8): two amplitudes, 16 bytes,
// so a load or store instruction covers 1 KiB of runs of 32 contiguous
// amplitudes. t's low 5 bits are positions 0..4; bits 5, 6 come from the
// lane (l >> 4), bits 7, 8, 9 from i.
__device__ inline uint32_t lane_off(const Geo& G, int lane) {
  const uint32_t t = 2u * lane;
  return (t & 31u) + (((t >> 5) & 1u) << G.pos[5]) + (((t >> 6) & 1u) << G.pos[6]);
}
__device__ inline uint32_t step_off(const Geo& G, int i) {
  return ((uint32_t)(i & 1) << G.pos[7]) + ((uint32_t)((i >> 1) & 1) << G.pos[8]) +
         ((uint32_t)((i >> 2) & 1) << G.pos[9]);
}
__device__ inline uint32_t lane_slot(const Geo& G, int lane) {
  uint32_t v = 0;
#pragma unroll
  for (int k = 1; k <= 6; ++k)
    if (((2u * lane) >> k) & 1u) v ^= G.sv[k];
  return v;
}
__device__ inline uint32_t step_slot(const Geo& G, int i) {
  return ((i & 1) ? G.sv[7] : 0u) ^ ((i & 2) ? G.sv[8] : 0u) ^ ((i & 4) ? G.sv[9] : 0u);
}

// Keeps a per-lane value opaque to the compiler inside a loop, so the
// addresses derived from it are formed where they are used (one XOR each)
// instead of being hoisted out of the loop into dozens of live registers.
__device__ inline uint32_t opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ inline void tile_load(const float* S, const Geo& G, int64_t base, uint32_t loff,
                                 f32x4 (&v)[8]) {
  const f32x4* p = reinterpret_cast<const f32x4*>(S + 2 * (base + loff));
#pragma unroll
  for (int i = 0; i < 8; ++i)
    v[i] = __builtin_nontemporal_load(p + step_off(G, i) / 2);
}
// T: the real plane, T + kTileSlots the imaginary plane.
__device__ inline void tile_to_lds(float* T, const Geo& G, uint32_t lslot, const f32x4 (&v)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t sl = lslot ^ step_slot(G, i), sm = sl ^ G.sv[0];
    T[sl] = v[i][0];
    T[kTileSlots + sl] = v[i][1];
    T[sm] = v[i][2];
    T[kTileSlots + sm] = v[i][3];
  }
}
__device__ inline void tile_store(float* S, const Geo& G, int64_t base, uint32_t loff,
                                  const float* T, uint32_t lslot) {
  f32x4* p = reinterpret_cast<f32x4*>(S + 2 * (base + loff));
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t sl = lslot ^ step_slot(G, i), sm = sl ^ G.sv[0];
    __builtin_nontemporal_store(f32x4{T[sl], T[kTileSlots + sl], T[sm], T[kTileSlots + sm]},
                                p + step_off(G, i) / 2);
  }
}

// D = E X for the tile in T (B operand: lane l takes component h = l / 32 of
// amplitude s of column j = l % 32, slot 33 j ^ s of plane h), written back
// into T (accumulator pair (a, a + 1), a even, of row tile rt holds amplitude
// 16 rt + 4 (a / 4) + (a % 4) / 2 + 2 h of column j).
__device__ inline void tile_apply(const float (&a)[2][kD], float* T, int lane) {
  const int h = lane >> 5, j = lane & 31;
  const uint32_t rd = opaque((h ? kTileSlots : 0u) + 33u * j);
  f32x16 d0{}, d1{};
#pragma unroll
  for (int s = 0; s < kD; ++s) {
    const float x = T[rd ^ (uint32_t)s];
    d0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][s], x, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1][s], x, d1, 0, 0, 0);
  }
  const uint32_t wr = opaque((33u * j) ^ (2u * h));
#pragma unroll
  for (int e = 0; e < 16; e += 2) {
    const uint32_t x0 = 4 * (e / 4) + (e % 4) / 2;
    T[wr ^ x0] = d0[e];
    T[kTileSlots + (wr ^ x0)] = d0[e + 1];
    T[wr ^ (16u + x0)] = d1[e];
    T[kTileSlots + (wr ^ (16u + x0))] = d1[e + 1];
  }
}

__device__ inline void lds_fence() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS accesses are done
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void db_forward(
    const int32_t* __restrict__ blk_begin, const DbGate* __restrict__ gates,
    const int32_t* __restrict__ blk_q, const float* __restrict__ P, int blk, int n,
    int64_t n_groups, float* S) {
  extern __shared__ float lds[];  // max(M build, one tile per wave)
  double2* M = reinterpret_cast<double2*>(lds);
  build_block(M, gates, blk_begin[blk], blk_begin[blk + 1], P);
  float a[2][kD];
  load_frags<false>(M, a);
  __syncthreads();  // M's LDS is reused below
  const Geo G = make_geo(n, blk_q + kDbGeoWords * blk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* T = lds + wave * (2 * kTileSlots);
  const uint32_t loff = lane_off(G, lane);
  const uint32_t lslot = lane_slot(G, lane);
  const int64_t W = (int64_t)gridDim.x * kWaves;
  int64_t g = (int64_t)blockIdx.x * kWaves + wave;
  f32x4 v[8];
  if (g < n_groups) tile_load(S, G, tile_base(G, g), loff, v);
  for (; g < n_groups; g += W) {
    const int64_t base = tile_base(G, g);
    tile_to_lds(T, G, opaque(lslot), v);
    if (g + W < n_groups) tile_load(S, G, tile_base(G, g + W), loff, v);  // next tile in flight
    lds_fence();
    tile_apply(a, T, lane);
    lds_fence();
    tile_store(S, G, base, loff, T, opaque(lslot));
    lds_fence();
  }
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void db_adjoint(
    const int32_t* __restrict__ blk_begin, const DbGate* __restrict__ gates,
    const int32_t* __restrict__ blk_q, const float* __restrict__ P, int blk, int n,
    int64_t n_groups, float* psi, float* lam, float* __restrict__ partials) {
  extern __shared__ float lds[];  // max(M build, psi and lam tiles per wave)
  double2* M = reinterpret_cast<double2*>(lds);
  build_block(M, gates, blk_begin[blk], blk_begin[blk + 1], P);
  float a[2][kD];
  load_frags<true>(M, a);
  __syncthreads();  // M's LDS is reused below
  const Geo G = make_geo(n, blk_q + kDbGeoWords * blk);
  const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
  const int wave = threadIdx.x >> 6;
  float* Tp = lds + wave * (4 * kTileSlots);
  float* Tl = Tp + 2 * kTileSlots;
  const uint32_t loff = lane_off(G, lane);
  const uint32_t lslot = lane_slot(G, lane);
  f32x16 rre{}, rim{};
  const int64_t W = (int64_t)gridDim.x * kWaves;
  int64_t g = (int64_t)blockIdx.x * kWaves + wave;
  f32x4 vp[8], vl[8];
  if (g < n_groups) {
    const int64_t b0 = tile_base(G, g);
    tile_load(psi, G, b0, loff, vp);
    tile_load(lam, G, b0, loff, vl);
  }
  for (; g < n_groups; g += W) {
    const int64_t base = tile_base(G, g);
    tile_to_lds(Tp, G, opaque(lslot), vp);
    tile_to_lds(Tl, G, opaque(lslot), vl);
    if (g + W < n_groups) {  // next tiles in flight during this tile's MFMAs
      const int64_t b1 = tile_base(G, g + W);
      tile_load(psi, G, b1, loff, vp);
      tile_load(lam, G, b1, loff, vl);
    }
    lds_fence();
    // rho[i][j] += sum_c psi[i][c] conj(lam[j][c]) over the tile's columns:
    // k-step = column c, k = (re, im); lane l holds row / column index l % 32.
    {
      // lane l: amplitude index col of column c at slot 33 c ^ col of plane h
      const uint32_t r0 = opaque((h ? kTileSlots : 0u) + col);
      const uint32_t r1 = opaque((h ? 0u : kTileSlots) + col);
      const float sg = h ? 1.f : -1.f;
#pragma unroll
      for (int c = 0; c < 32; ++c) {
        const uint32_t o = 33u * c;
        const float ap = Tp[r0 ^ o];
        const float bq = Tl[r0 ^ o];
        const float bo = Tl[r1 ^ o];
        rre = __builtin_amdgcn_mfma_f32_32x32x2f32(ap, bq, rre, 0, 0, 0);
        rim = __builtin_amdgcn_mfma_f32_32x32x2f32(ap, sg * bo, rim, 0, 0, 0);
      }
    }
    tile_apply(a, Tp, lane);
    lds_fence();
    tile_store(psi, G, base, loff, Tp, opaque(lslot));
    tile_apply(a, Tl, lane);
    lds_fence();
    tile_store(lam, G, base, loff, Tl, opaque(lslot));
    lds_fence();
  }
  // workgroup sum of the waves' rho (real part, then imaginary part)
  __syncthreads();
  float* red = lds;  // [waves][2][32][32]
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int i = 8 * (e / 4) + 4 * h + (e % 4);
    red[((wave * 2 + 0) * kD + i) * kD + col] = rre[e];
    red[((wave * 2 + 1) * kD + i) * kD + col] = rim[e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kRhoWords; e += blockDim.x) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += red[w * kRhoWords + e];
    partials[(int64_t)blockIdx.x * kRhoWords + e] = t;
  }
}

// rho = sum over workgroups of the partial sums, in FP64: 256 workgroups of
// 8 entries each, 32 row-strided partial sums per entry combined in LDS (a
// fixed order, so the result is reproducible bit for bit).
constexpr int kRedEntries = 8;
__global__ __launch_bounds__(256) void db_reduce(const float* __restrict__ partials, int rows,
                                                 double* __restrict__ rho) {
  __shared__ double part[32][kRedEntries];
  const int k = threadIdx.x & (kRedEntries - 1), split = threadIdx.x >> 3;
  const int e = blockIdx.x * kRedEntries + k;
  double t = 0.0;
  for (int r = split; r < rows; r += 32) t += (double)partials[(int64_t)r * kRhoWords + e];
  part[split][k] = t;
  __syncthreads();
  if (threadIdx.x < kRedEntries) {
    double u = 0.0;
#pragma unroll
    for (int j = 0; j < 32; ++j) u += part[j][threadIdx.x];
    rho[blockIdx.x * kRedEntries + threadIdx.x] = u;
  }
}

// One workgroup per block: walks the block's gates backwards on its rho,
// taking each rotation's gradient Im tr(P rho) before un-applying the gate
// (rho <- U^dagger rho U).
__global__ __launch_bounds__(1024) void db_grads(const int32_t* __restrict__ blk_begin,
                                                  const DbGate* __restrict__ gates,
                                                  const float* __restrict__ P,
                                                  const double* __restrict__ rho_all,
                                                  double* __restrict__ gtheta) {
  __shared__ double2 R[kD * kD];
  const int blk = blockIdx.x;
  const double* rho = rho_all + (int64_t)blk * kRhoWords;
  const int e = threadIdx.x, r = e >> 5, c = e & 31;
  R[e] = make_double2(rho[e], rho[kD * kD + e]);
  __syncthreads();
  for (int j = blk_begin[blk + 1] - 1; j >= blk_begin[blk]; --j) {
    const DbGate g = gates[j];
    if (g.op <= QS_OP_RZ && threadIdx.x < 64) {
      const int m = 1 << g.q0, x = threadIdx.x & 31;
      double t = 0.0;
      if (threadIdx.x < 32) {
        const int bit = (x >> g.q0) & 1;
        if (g.op == QS_OP_RX) t = R[((x ^ m) << 5) | x].y;
        else if (g.op == QS_OP_RY) t = (bit ? 1.0 : -1.0) * R[((x ^ m) << 5) | x].x;
        else t = (bit ? -1.0 : 1.0) * R[(x << 5) | x].y;
      }
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) t += __shfl_xor(t, o);
      if (threadIdx.x == 0) gtheta[g.g] = t;
    }
    double2 v;
    if (g.op <= QS_OP_H) {
      double2 u[4];
      gate2(g.op, g.op <= QS_OP_RZ ? angle(g, P) : 0.0, u);
      const int m = 1 << g.q0, rb = (r >> g.q0) & 1, cb = (c >> g.q0) & 1;
      const int r0 = r & ~m, r1 = r | m, c0 = c & ~m, c1 = c | m;
      // (U^dagger R U)[r][c] = sum_{x, y} conj(U[x][r]) R[x][y] U[y][c]
      const double2 uc0 = cb ? u[1] : u[0], uc1 = cb ? u[3] : u[2];
      const double2 ur0 = rb ? u[1] : u[0], ur1 = rb ? u[3] : u[2];
      const double2 t0 = cadd(cmul(R[(r0 << 5) | c0], uc0), cmul(R[(r0 << 5) | c1], uc1));
      const double2 t1 = cadd(cmul(R[(r1 << 5) | c0], uc0), cmul(R[(r1 << 5) | c1], uc1));
      v = cadd(cmul(conjd(ur0), t0), cmul(conjd(ur1), t1));
    } else if (g.op == QS_OP_CNOT) {
      const int pr = ((r >> g.q0) & 1) ? r ^ (1 << g.q1) : r;
      const int pc = ((c >> g.q0) & 1) ? c ^ (1 << g.q1) : c;
      v = R[(pr << 5) | pc];
    } else {
      const int s = (((r >> g.q0) & (r >> g.q1)) ^ ((c >> g.q0) & (c >> g.q1))) & 1;
      v = s ? make_double2(-R[e].x, -R[e].y) : R[e];
    }
    __syncthreads();
    R[e] = v;
    __syncthreads();
  }
}

__global__ void db_chain(int n_params, const int32_t* __restrict__ p_begin,
                         const int32_t* __restrict__ p_gate, const float* __restrict__ p_scale,
                         const double* __restrict__ gtheta, double* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_params) return;
  double t = 0.0;
  for (int k = p_begin[p]; k < p_begin[p + 1]; ++k) t += (double)p_scale[k] * gtheta[p_gate[k]];
  grad[p] = t;
}

constexpr size_t kFwdLds = size_t(kWaves) * 2 * kTileSlots * sizeof(float);
constexpr size_t kAdjLds = 2 * kFwdLds;
static_assert(kFwdLds >= kD * kD * sizeof(double2), "M build fits the forward's LDS");
static_assert(kAdjLds >= size_t(kWaves) * kRhoWords * sizeof(float), "rho sums fit");

int status(hipError_t e) { return e == hipSuccess ? QS_OK : QS_ERR_LAUNCH; }

}  // namespace

int db_adjoint_lds_bytes() { return (int)kAdjLds; }
int db_threads() { return kThreads; }

int launch_db_forward(const DbLaunch& L, int i, void* state) {
  if (L.K != 5 || L.n < 10) return QS_ERR_UNSUPPORTED;
  const int64_t groups = (L.B << (L.n - 5)) >> 5;
  // three workgroups per CU (the forward holds three waves per SIMD)
  hipLaunchKernelGGL(db_forward, dim3(3 * L.grid / 2), dim3(kThreads), kFwdLds,
                     static_cast<hipStream_t>(L.stream), L.blk_begin, L.gates, L.blk_q,
                     static_cast<const float*>(L.params), i, L.n, groups,
                     static_cast<float*>(state));
  return status(hipGetLastError());
}

int launch_db_adjoint(const DbLaunch& L, int i, void* psi, void* lam, float* partials) {
  if (L.K != 5 || L.n < 10) return QS_ERR_UNSUPPORTED;
  const int64_t groups = (L.B << (L.n - 5)) >> 5;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(db_adjoint), hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)kAdjLds);
  if (attr != hipSuccess) return QS_ERR_LAUNCH;
  hipLaunchKernelGGL(db_adjoint, dim3(L.grid), dim3(kThreads), kAdjLds,
                     static_cast<hipStream_t>(L.stream), L.blk_begin, L.gates, L.blk_q,
                     static_cast<const float*>(L.params), i, L.n, groups,
                     static_cast<float*>(psi), static_cast<float*>(lam), partials);
  return status(hipGetLastError());
}

int launch_db_reduce(const DbLaunch& L, const float* partials, double* rho) {
  hipLaunchKernelGGL(db_reduce, dim3(kRhoWords / kRedEntries), dim3(256), 0,
                     static_cast<hipStream_t>(L.stream), partials, L.grid, rho);
  return status(hipGetLastError());
}

int launch_db_grads(const DbLaunch& L, int n_blocks, const double* rho, double* gtheta) {
  if (n_blocks <= 0) return QS_OK;
  hipLaunchKernelGGL(db_grads, dim3(n_blocks), dim3(kD * kD), 0,
                     static_cast<hipStream_t>(L.stream), L.blk_begin, L.gates,
                     static_cast<const float*>(L.params), rho, gtheta);
  return status(hipGetLastError());
}

int launch_db_chain(int n_params, const int32_t* p_begin, const int32_t* p_gate,
                    const float* p_scale, const double* gtheta, double* grad, void* stream) {
  if (n_params <= 0) return QS_OK;
  hipLaunchKernelGGL(db_chain, dim3((n_params + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), n_params, p_begin, p_gate, p_scale,
                     gtheta, grad);
  return status(hipGetLastError());
}

}  // namespace qs
