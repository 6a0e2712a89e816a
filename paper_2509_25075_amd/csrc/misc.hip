// Encoding, readout, fidelity and reduction kernels.
//
// Amplitude encoding |x> = x / ||x||_2 zero-padded to 2^n with the squared
// norm summed in FP64 (Schuld & Petruccione 2018, sec. 5.2); Pauli-Z readout
// <Z_q> = sum_i |psi_i|^2 (1 - 2 bit_q(i)) summed in FP64; autoencoder
// fidelity with reset trash qubits F = sum_m |<chi_0|psi_m>|^2 (Romero, Olson
// & Aspuru-Guzik 2017), the post-selected variant F' = |<chi_0|psi_0>|^2 /
// ||psi_0||^2 (trash qubits measured, only the all-zero outcome kept and
// renormalised), one trajectory of the reset channel (outcome m drawn from
// the Born probabilities by a given uniform, F = |<chi_0|psi_m>|^2 /
// ||psi_m||^2), and their state cotangents.
#include <hip/hip_runtime.h>

#include <cmath>

#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // sh: kBlock / 64 doubles
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

template <typename real, typename xin>
__global__ void __launch_bounds__(kBlock)
encode_amplitude(int n, int64_t B, int64_t D, const xin* x, int64_t xs,
                 real* state, int32_t* bad_rows) {
  __shared__ double sh[kBlock / 64];
  const int64_t b = blockIdx.x;
  const int64_t N = 1ll << n;
  const xin* row = x + b * xs;
  double s = 0;
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) {
    double v = (double)row[i];
    s += v * v;
  }
  s = block_sum(s, sh);
  const bool zero = !(s > 0);
  const double inv = zero ? NAN : 1.0 / sqrt(s);
  real* out = state + 2 * b * N;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    double v = i < D ? (double)row[i] * inv : (zero ? NAN : 0.0);
    out[2 * i] = (real)v;
    out[2 * i + 1] = (real)(zero ? NAN : 0.0);
  }
  if (zero && threadIdx.x == 0 && bad_rows != nullptr) atomicAdd(bad_rows, 1);
}

// Amplitude encoding of an uneven batch: one block per circuit; the class of
// circuit `c` is found by binary search over the cumulative class counts.
template <typename real, typename xin>
__global__ void __launch_bounds__(kBlock)
encode_program(int n_classes, const int64_t* cum, const int32_t* nq,
               const int64_t* state_off, const xin* x, real* states,
               int32_t* bad_rows) {
  __shared__ double sh[kBlock / 64];
  const int64_t c = blockIdx.x;
  int lo = 0, hi = n_classes - 1;
  while (lo < hi) {  // last class k with cum[k] <= c
    const int mid = (lo + hi + 1) >> 1;
    if (cum[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int n = nq[lo];
  const int64_t N = 1ll << n;
  const int64_t off = state_off[lo] + (c - cum[lo]) * N;
  const xin* row = x + off;
  double s = 0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const double v = (double)row[i];
    s += v * v;
  }
  s = block_sum(s, sh);
  const bool zero = !(s > 0);
  const double inv = zero ? NAN : 1.0 / sqrt(s);
  real* out = states + 2 * off;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    out[2 * i] = (real)((double)row[i] * inv);
    out[2 * i + 1] = (real)(zero ? NAN : 0.0);
  }
  if (zero && threadIdx.x == 0 && bad_rows != nullptr) atomicAdd(bad_rows, 1);
}

template <typename real>
__global__ void __launch_bounds__(kBlock)
encode_zero(int n, int64_t total, real* state) {
  const int64_t N = 1ll << n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    state[2 * i] = (i & (N - 1)) == 0 ? (real)1 : (real)0;
    state[2 * i + 1] = 0;
  }
}

// Mid-circuit measurement of qubit q in the Z basis, one trajectory per
// sample (projective-measurement postulate, Nielsen & Chuang sec. 2.2.3):
// p_m = sum of |psi_i|^2 over the amplitudes whose bit q is m (FP64), the
// outcome m drawn from the uniform u by inverse CDF (the smallest m with
// u (p_0 + p_1) < p_0 + ... + p_m, else the last m with p_m > 0), the state
// projected on bit q = m and divided by sqrt(p_m); a reset then moves it to
// bit q = 0. One workgroup per sample; amplitude pairs (i0, i0 | 1 << q).
struct ChanDraw {
  int m;
  double inv;  // 1 / sqrt(p_m)
};

template <typename real>
__device__ ChanDraw channel_draw(int n, int q, const real* s, double u, double* sh) {
  const int64_t half = 1ll << (n - 1);
  const int64_t lo = (1ll << q) - 1;
  double p0 = 0, p1 = 0;
  for (int64_t k = threadIdx.x; k < half; k += blockDim.x) {
    const int64_t i0 = ((k & ~lo) << 1) | (k & lo), i1 = i0 | (1ll << q);
    const double a = s[2 * i0], b = s[2 * i0 + 1], c = s[2 * i1], d = s[2 * i1 + 1];
    p0 += a * a + b * b;
    p1 += c * c + d * d;
  }
  p0 = block_sum(p0, sh);
  p1 = block_sum(p1, sh);
  const double x = u * (p0 + p1);
  int m = x < p0 ? 0 : (x < p0 + p1 ? 1 : (p1 > 0 ? 1 : 0));
  const double pm = m ? p1 : p0;
  return ChanDraw{m, 1.0 / sqrt(pm)};  // p_m = 0 only for a zero row: NaN
}

template <typename real>
__global__ void __launch_bounds__(kBlock)
channel_forward(int n, int q, int reset, const real* feats, int n_feats, int feat,
                real* state) {
  __shared__ double sh[kBlock / 64];
  const int64_t b = blockIdx.x;
  real* s = state + 2 * b * (1ll << n);
  const ChanDraw d = channel_draw(n, q, s, (double)feats[b * n_feats + feat], sh);
  const int64_t half = 1ll << (n - 1), lo = (1ll << q) - 1;
  for (int64_t k = threadIdx.x; k < half; k += blockDim.x) {
    const int64_t i0 = ((k & ~lo) << 1) | (k & lo), i1 = i0 | (1ll << q);
    const int64_t src = d.m ? i1 : i0;
    const double re = (double)s[2 * src] * d.inv, im = (double)s[2 * src + 1] * d.inv;
    const int64_t dst = reset ? i0 : src, other = dst == i0 ? i1 : i0;
    s[2 * dst] = (real)re;
    s[2 * dst + 1] = (real)im;
    s[2 * other] = 0;
    s[2 * other + 1] = 0;
  }
}

// Backward through the channel with its outcome held fixed (pathwise; state
// cotangents with dL = 2 Re<lam|d psi>): from the stored state in front of
// the channel, psi' = K psi / r (K = |0><m| or the projector on m, r =
// sqrt(p_m)); the cotangent in front is K^dagger (lam' - Re<lam'|psi'> psi')
// / r. lam is updated in place, psi_out receives the state in front.
template <typename real>
__global__ void __launch_bounds__(kBlock)
channel_adjoint(int n, int q, int reset, const real* feats, int n_feats, int feat,
                const real* psi_pre, real* lam, real* psi_out) {
  __shared__ double sh[kBlock / 64];
  const int64_t b = blockIdx.x, N = 1ll << n;
  const real* s = psi_pre + 2 * b * N;
  real* l = lam + 2 * b * N;
  const ChanDraw d = channel_draw(n, q, s, (double)feats[b * n_feats + feat], sh);
  const int64_t half = 1ll << (n - 1), lo = (1ll << q) - 1;
  // psi' is nonzero only at dst = (reset ? i0 : the outcome's index)
  double c = 0;
  for (int64_t k = threadIdx.x; k < half; k += blockDim.x) {
    const int64_t i0 = ((k & ~lo) << 1) | (k & lo), i1 = i0 | (1ll << q);
    const int64_t src = d.m ? i1 : i0, dst = reset ? i0 : src;
    const double pr = (double)s[2 * src] * d.inv, pi = (double)s[2 * src + 1] * d.inv;
    c += (double)l[2 * dst] * pr + (double)l[2 * dst + 1] * pi;
  }
  c = block_sum(c, sh);
  for (int64_t k = threadIdx.x; k < half; k += blockDim.x) {
    const int64_t i0 = ((k & ~lo) << 1) | (k & lo), i1 = i0 | (1ll << q);
    const int64_t src = d.m ? i1 : i0, dst = reset ? i0 : src;
    const double pr = (double)s[2 * src] * d.inv, pi = (double)s[2 * src + 1] * d.inv;
    const double gr = ((double)l[2 * dst] - c * pr) * d.inv;
    const double gi = ((double)l[2 * dst + 1] - c * pi) * d.inv;
    const int64_t other = src == i0 ? i1 : i0;  // K^dagger: slice dst -> slice src
    l[2 * src] = (real)gr;
    l[2 * src + 1] = (real)gi;
    l[2 * other] = 0;
    l[2 * other + 1] = 0;
    real* o = psi_out + 2 * b * N;
    o[2 * i0] = s[2 * i0];
    o[2 * i0 + 1] = s[2 * i0 + 1];
    o[2 * i1] = s[2 * i1];
    o[2 * i1 + 1] = s[2 * i1 + 1];
  }
}

// <Z_q> for q < 32: grid (blocks_per_sample, B); partial sums in registers
// (compile-time indexed), block sums, FP64 atomics into a zeroed expz.
template <typename real>
__global__ void __launch_bounds__(kBlock)
expz_kernel(int n, int64_t B, const real* state, double* expz) {
  __shared__ double sh[kBlock / 64];
  const int64_t N = 1ll << n;
  for (int64_t b = blockIdx.y; b < B; b += gridDim.y) {
  const real* s = state + 2 * b * N;
  double z[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) z[q] = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double re = s[2 * i], im = s[2 * i + 1];
    const double p = re * re + im * im;
#pragma unroll
    for (int q = 0; q < 32; ++q)
      if (q < n) z[q] += ((i >> q) & 1) ? -p : p;
  }
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    if (q < n) {
      double t = block_sum(z[q], sh);
      if (threadIdx.x == 0) atomicAdd(&expz[b * n + q], t);
    }
  }
  }
}

template <typename real>
__global__ void __launch_bounds__(kBlock)
fidelity_kernel(int n, int nt, const real* psi, const real* chi, double* fid,
                const double* dfid, real* lam_psi, real* lam_chi) {
  __shared__ double cre[64], cim[64];
  const int64_t b = blockIdx.x;
  const int k = n - nt;
  const int64_t K = 1ll << k, M = 1ll << nt, N = 1ll << n;
  const real* p = psi + 2 * b * N;
  const real* c = chi + 2 * b * N;  // chi_0 = first K amplitudes
  // c_m = <chi_0|psi_m>: one wave per trash outcome m at a time (the sum
  // over j within the wave, no workgroup barrier per m)
  const int lane = threadIdx.x & 63, waves = blockDim.x >> 6;
  for (int64_t m = threadIdx.x >> 6; m < M; m += waves) {
    double ar = 0, ai = 0;
    for (int64_t j = lane; j < K; j += 64) {
      const double xr = c[2 * j], xi = c[2 * j + 1];
      const double yr = p[2 * (m * K + j)], yi = p[2 * (m * K + j) + 1];
      ar += xr * yr + xi * yi;  // conj(x) y
      ai += xr * yi - xi * yr;
    }
    for (int o = 32; o >= 1; o >>= 1) {
      ar += __shfl_xor(ar, o);
      ai += __shfl_xor(ai, o);
    }
    if (lane == 0) {
      cre[m] = ar;
      cim[m] = ai;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double F = 0;
    for (int64_t m = 0; m < M; ++m) F += cre[m] * cre[m] + cim[m] * cim[m];
    fid[b] = F;
  }
  if (dfid == nullptr) return;
  const double d = dfid[b];
  real* lp = lam_psi + 2 * b * N;
  real* lc = lam_chi + 2 * b * N;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const int64_t m = i / K, j = i % K;
    const double xr = c[2 * j], xi = c[2 * j + 1];
    // lam_psi = d c_m chi0_j
    lp[2 * i] = (real)(d * (cre[m] * xr - cim[m] * xi));
    lp[2 * i + 1] = (real)(d * (cre[m] * xi + cim[m] * xr));
    if (m == 0) {
      // lam_chi_j = d sum_m conj(c_m) psi_{m j}
      double sr = 0, si = 0;
      for (int64_t mm = 0; mm < M; ++mm) {
        const double yr = p[2 * (mm * K + j)], yi = p[2 * (mm * K + j) + 1];
        sr += cre[mm] * yr + cim[mm] * yi;
        si += cre[mm] * yi - cim[mm] * yr;
      }
      lc[2 * i] = (real)(d * sr);
      lc[2 * i + 1] = (real)(d * si);
    } else {
      lc[2 * i] = 0;
      lc[2 * i + 1] = 0;
    }
  }
}

// Post-selected fidelity, one block per sample. In FP64: c = <chi_0|psi_0>
// and p = ||psi_0||^2 over the trash-0 slice (the first K = 2^(n-nt)
// amplitudes), F' = |c|^2 / p (NaN when p = 0). Cotangents (dL = 2 Re<lam|d psi>)
// scaled by d = dL/dF': lam_psi = d ((c/p) chi_0 - (F'/p) psi_0) and
// lam_chi = d (conj(c)/p) psi_0 on that slice, zero on the others.
template <typename real>
__global__ void __launch_bounds__(kBlock)
fidelity_postselect_kernel(int n, int nt, const real* psi, const real* chi, double* fid,
                           const double* dfid, real* lam_psi, real* lam_chi) {
  __shared__ double sh[kBlock / 64];
  const int64_t b = blockIdx.x;
  const int64_t K = 1ll << (n - nt), N = 1ll << n;
  const real* p = psi + 2 * b * N;
  const real* c = chi + 2 * b * N;
  double ar = 0, ai = 0, pp = 0;
  for (int64_t j = threadIdx.x; j < K; j += blockDim.x) {
    const double xr = c[2 * j], xi = c[2 * j + 1];
    const double yr = p[2 * j], yi = p[2 * j + 1];
    ar += xr * yr + xi * yi;  // conj(x) y
    ai += xr * yi - xi * yr;
    pp += yr * yr + yi * yi;
  }
  ar = block_sum(ar, sh);
  ai = block_sum(ai, sh);
  pp = block_sum(pp, sh);
  const double F = (ar * ar + ai * ai) / pp;
  if (threadIdx.x == 0) fid[b] = F;
  if (dfid == nullptr) return;
  const double d = dfid[b];
  const double gr = d * ar / pp, gi = d * ai / pp, gf = d * F / pp;
  real* lp = lam_psi + 2 * b * N;
  real* lc = lam_chi + 2 * b * N;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    if (i < K) {
      const double xr = c[2 * i], xi = c[2 * i + 1];
      const double yr = p[2 * i], yi = p[2 * i + 1];
      lp[2 * i] = (real)(gr * xr - gi * xi - gf * yr);
      lp[2 * i + 1] = (real)(gr * xi + gi * xr - gf * yi);
      lc[2 * i] = (real)(gr * yr + gi * yi);
      lc[2 * i + 1] = (real)(gr * yi - gi * yr);
    } else {
      lp[2 * i] = 0;
      lp[2 * i + 1] = 0;
      lc[2 * i] = 0;
      lc[2 * i + 1] = 0;
    }
  }
}

// One trajectory of the reset channel, one block per sample (nt <= 6). In
// FP64: p_m = ||psi_m||^2 for every outcome m (slice m = amplitudes
// [m K, (m+1) K)), the outcome = the smallest m with u * sum p < p_0 + ... +
// p_m (summed in m order; the last m with p_m > 0 if rounding leaves none),
// c = <chi_0|psi_m>, F = |c|^2 / p_m. Cotangents scaled by d = dL/dF for that
// outcome: lam_psi = d ((c/p) chi_0 - (F/p) psi_m) on slice m, lam_chi =
// d (conj(c)/p) psi_m on slice 0, zero elsewhere.
template <typename real>
__global__ void __launch_bounds__(kBlock)
fidelity_trajectory_kernel(int n, int nt, const real* psi, const real* chi, const double* u,
                           double* fid, int32_t* outcome, const double* dfid,
                           real* lam_psi, real* lam_chi) {
  __shared__ double sh[kBlock / 64];
  __shared__ double pm[64];
  __shared__ int pick_sh;
  const int64_t b = blockIdx.x;
  const int64_t K = 1ll << (n - nt), M = 1ll << nt, N = 1ll << n;
  const real* p = psi + 2 * b * N;
  const real* c = chi + 2 * b * N;
  for (int64_t m = 0; m < M; ++m) {
    double s = 0;
    for (int64_t j = threadIdx.x; j < K; j += blockDim.x) {
      const double yr = p[2 * (m * K + j)], yi = p[2 * (m * K + j) + 1];
      s += yr * yr + yi * yi;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) pm[m] = s;
  }
  if (threadIdx.x == 0) {
    double tot = 0;
    for (int64_t m = 0; m < M; ++m) tot += pm[m];
    const double target = u[b] * tot;
    double acc = 0;
    int pick = -1, last = 0;
    for (int64_t m = 0; m < M; ++m) {
      acc += pm[m];
      if (pm[m] > 0) last = (int)m;
      if (pick < 0 && target < acc) pick = (int)m;
    }
    pick_sh = pick < 0 ? last : pick;
  }
  __syncthreads();
  const int64_t m = pick_sh;
  double ar = 0, ai = 0;
  for (int64_t j = threadIdx.x; j < K; j += blockDim.x) {
    const double xr = c[2 * j], xi = c[2 * j + 1];
    const double yr = p[2 * (m * K + j)], yi = p[2 * (m * K + j) + 1];
    ar += xr * yr + xi * yi;  // conj(x) y
    ai += xr * yi - xi * yr;
  }
  ar = block_sum(ar, sh);
  ai = block_sum(ai, sh);
  const double pp = pm[m];
  const double F = (ar * ar + ai * ai) / pp;
  if (threadIdx.x == 0) {
    fid[b] = F;
    if (outcome != nullptr) outcome[b] = (int32_t)m;
  }
  if (dfid == nullptr) return;
  const double d = dfid[b];
  const double gr = d * ar / pp, gi = d * ai / pp, gf = d * F / pp;
  real* lp = lam_psi + 2 * b * N;
  real* lc = lam_chi + 2 * b * N;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const int64_t s = i / K, j = i - s * K;
    double pr = 0, pi = 0, cr = 0, ci = 0;
    if (s == m) {
      const double xr = c[2 * j], xi = c[2 * j + 1];
      const double yr = p[2 * i], yi = p[2 * i + 1];
      pr = gr * xr - gi * xi - gf * yr;
      pi = gr * xi + gi * xr - gf * yi;
    }
    if (s == 0) {
      const double yr = p[2 * (m * K + j)], yi = p[2 * (m * K + j) + 1];
      cr = gr * yr + gi * yi;
      ci = gr * yi - gi * yr;
    }
    lp[2 * i] = (real)pr;
    lp[2 * i + 1] = (real)pi;
    lc[2 * i] = (real)cr;
    lc[2 * i + 1] = (real)ci;
  }
}

// out[col_param[c]] (+)= sum_r partials[r][c] in FP64: one block per column,
// threads stride over rows with four independent sums each, then a block
// reduction. The order of the additions is fixed, so the result is
// reproducible bit for bit.
template <typename acc_t>
__global__ void __launch_bounds__(kBlock)
reduce_partials(const acc_t* partials, int64_t rows, int cols, const int32_t* col_param,
                double* out, int accumulate, const double* loss_part, double* loss,
                double loss_scale) {
  __shared__ double sh[kBlock / 64];
  const int c = blockIdx.x;
  if (c == cols) {
    // the training step's loss: per-workgroup sums added in a fixed order
    double s = 0;
    for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) s += loss_part[r];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) loss[0] = s * loss_scale;
    return;
  }
  const int64_t step = blockDim.x;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int64_t r = threadIdx.x;
  for (; r + 3 * step < rows; r += 4 * step) {
    s0 += (double)partials[r * cols + c];
    s1 += (double)partials[(r + step) * cols + c];
    s2 += (double)partials[(r + 2 * step) * cols + c];
    s3 += (double)partials[(r + 3 * step) * cols + c];
  }
  for (; r < rows; r += step) s0 += (double)partials[r * cols + c];
  double s = block_sum((s0 + s1) + (s2 + s3), sh);
  const int o = col_param != nullptr ? col_param[c] : c;
  if (threadIdx.x == 0) out[o] = accumulate ? out[o] + s : s;
}

__global__ void __launch_bounds__(kBlock) fill_f64(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

template <typename v2>
__global__ void __launch_bounds__(kBlock)
copy_state(const v2* src, v2* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

unsigned grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

int ok() { return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_LAUNCH; }

// Mean-squared error on qubit q's readout. Workgroup 0 sums the squared
// residuals, each thread over a fixed stride of rows (their loads in flight
// together) and then the workgroup in a fixed order, so the loss is bitwise
// reproducible; the other workgroups write the upstream gradient rows
// (2/B)(z_b - y_b) e_q, one element per thread.
constexpr int kLossBlock = 1024;
__global__ void __launch_bounds__(kLossBlock)
loss_mse_z(int n, int64_t B, int q, const double* expz, const double* y, double* dexpz,
           double* loss) {
  __shared__ double sh[kLossBlock / 64];
  const double inv_b = B > 0 ? 1.0 / (double)B : 0.0;
  if (blockIdx.x > 0) {
    if (dexpz == nullptr) return;
    // row-major [B][n]: element i is row i / n, column i % n (32-bit
    // division while the index fits, which it does for any batch in HBM)
    const int64_t total = B * n;
    const bool small = total < (1ll << 31);
    for (int64_t i = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)(gridDim.x - 1) * blockDim.x) {
      const int64_t b = small ? (int64_t)((uint32_t)i / (uint32_t)n) : i / n;
      const int k = (int)(i - b * n);
      dexpz[i] = k == q ? 2.0 * inv_b * (expz[b * n + q] - y[b]) : 0.0;
    }
    return;
  }
  if (loss == nullptr) return;
  double s = 0;
  const int64_t T = blockDim.x;
  constexpr int kRows = 32;  // rows of a thread whose loads are in flight together
  for (int64_t b0 = threadIdx.x; b0 < B; b0 += kRows * T) {
    double r[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      const int64_t b = b0 + u * T;
      r[u] = b < B ? expz[b * n + q] - y[b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kRows; ++u) s += r[u] * r[u];
  }
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    loss[0] = t * inv_b;
  }
}


}  // namespace

int launch_encode(int enc, int dtype, int n, int64_t B, int64_t D, int x_is_f64,
                  const void* x, int64_t x_stride, void* state,
                  int32_t* bad_rows, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (B == 0) return QS_OK;
  if (enc == QS_ENC_ZERO) {
    const int64_t total = B << n;
    if (dtype == QS_C64)
      hipLaunchKernelGGL(encode_zero<float>, grid_for(total), kBlock, 0, st, n,
                         total, (float*)state);
    else
      hipLaunchKernelGGL(encode_zero<double>, grid_for(total), kBlock, 0, st,
                         n, total, (double*)state);
    return ok();
  }
  dim3 g((unsigned)B);
  if (dtype == QS_C64) {
    if (x_is_f64)
      hipLaunchKernelGGL((encode_amplitude<float, double>), g, kBlock, 0, st, n,
                         B, D, (const double*)x, x_stride, (float*)state, bad_rows);
    else
      hipLaunchKernelGGL((encode_amplitude<float, float>), g, kBlock, 0, st, n,
                         B, D, (const float*)x, x_stride, (float*)state, bad_rows);
  } else {
    if (x_is_f64)
      hipLaunchKernelGGL((encode_amplitude<double, double>), g, kBlock, 0, st,
                         n, B, D, (const double*)x, x_stride, (double*)state,
                         bad_rows);
    else
      hipLaunchKernelGGL((encode_amplitude<double, float>), g, kBlock, 0, st, n,
                         B, D, (const float*)x, x_stride, (double*)state,
                         bad_rows);
  }
  return ok();
}

int launch_program_encode(int dtype, int n_classes, const int64_t* cum,
                          const int32_t* nq, const int64_t* state_off,
                          int64_t n_circuits, const void* x, int x_is_f64,
                          void* states, int32_t* bad_rows, void* stream) {
  if (n_circuits <= 0) return QS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  dim3 g((unsigned)n_circuits);
  if (dtype == QS_C64) {
    if (x_is_f64)
      hipLaunchKernelGGL((encode_program<float, double>), g, kBlock, 0, st, n_classes,
                         cum, nq, state_off, (const double*)x, (float*)states, bad_rows);
    else
      hipLaunchKernelGGL((encode_program<float, float>), g, kBlock, 0, st, n_classes,
                         cum, nq, state_off, (const float*)x, (float*)states, bad_rows);
  } else {
    if (x_is_f64)
      hipLaunchKernelGGL((encode_program<double, double>), g, kBlock, 0, st, n_classes,
                         cum, nq, state_off, (const double*)x, (double*)states, bad_rows);
    else
      hipLaunchKernelGGL((encode_program<double, float>), g, kBlock, 0, st, n_classes,
                         cum, nq, state_off, (const float*)x, (double*)states, bad_rows);
  }
  return ok();
}

int launch_channel(int dtype, int n, int q, int reset, int64_t B, const void* feats,
                   int n_feats, int feat, void* state, void* stream) {
  if (B == 0) return QS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(channel_forward<float>, dim3((unsigned)B), kBlock, 0, st, n, q, reset,
                       (const float*)feats, n_feats, feat, (float*)state);
  else
    hipLaunchKernelGGL(channel_forward<double>, dim3((unsigned)B), kBlock, 0, st, n, q, reset,
                       (const double*)feats, n_feats, feat, (double*)state);
  return ok();
}

int launch_channel_adjoint(int dtype, int n, int q, int reset, int64_t B, const void* feats,
                           int n_feats, int feat, const void* psi_pre, void* lam,
                           void* psi_out, void* stream) {
  if (B == 0) return QS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(channel_adjoint<float>, dim3((unsigned)B), kBlock, 0, st, n, q, reset,
                       (const float*)feats, n_feats, feat, (const float*)psi_pre,
                       (float*)lam, (float*)psi_out);
  else
    hipLaunchKernelGGL(channel_adjoint<double>, dim3((unsigned)B), kBlock, 0, st, n, q, reset,
                       (const double*)feats, n_feats, feat, (const double*)psi_pre,
                       (double*)lam, (double*)psi_out);
  return ok();
}

int launch_fill_f64(double* p, int64_t n, void* stream) {
  if (n <= 0) return QS_OK;
  hipLaunchKernelGGL(fill_f64, grid_for(n), kBlock, 0,
                     static_cast<hipStream_t>(stream), p, n);
  return ok();
}

int launch_loss_mse_z(int n, int64_t B, int q, const double* expz, const double* y,
                      double* dexpz, double* loss, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  // workgroup 0: the loss; the others: one gradient element per thread
  int64_t g = (B * n + kLossBlock - 1) / kLossBlock;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(loss_mse_z, dim3((unsigned)(g + 1)), kLossBlock, 0, st, n, B, q, expz,
                     y, dexpz, loss);
  return ok();
}

int launch_expz(int dtype, int n, int64_t B, const void* state, double* expz,
                void* stream) {
  if (B == 0) return QS_OK;
  int rc = launch_fill_f64(expz, B * n, stream);
  if (rc != QS_OK) return rc;
  const int64_t N = 1ll << n;
  int64_t bx = (N + kBlock * 16 - 1) / (kBlock * 16);
  if (bx > 4096) bx = 4096;
  dim3 g((unsigned)bx, (unsigned)(B < 65535 ? B : 65535));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(expz_kernel<float>, g, kBlock, 0, st, n, B,
                       (const float*)state, expz);
  else
    hipLaunchKernelGGL(expz_kernel<double>, g, kBlock, 0, st, n, B,
                       (const double*)state, expz);
  return ok();
}

int launch_fidelity(int dtype, int n, int n_trash, int64_t B, const void* psi,
                    const void* chi, double* fid, const double* dfid,
                    void* lam_psi, void* lam_chi, void* stream) {
  if (B == 0) return QS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(fidelity_kernel<float>, dim3((unsigned)B), kBlock, 0, st,
                       n, n_trash, (const float*)psi, (const float*)chi, fid,
                       dfid, (float*)lam_psi, (float*)lam_chi);
  else
    hipLaunchKernelGGL(fidelity_kernel<double>, dim3((unsigned)B), kBlock, 0,
                       st, n, n_trash, (const double*)psi, (const double*)chi,
                       fid, dfid, (double*)lam_psi, (double*)lam_chi);
  return ok();
}

int launch_fidelity_postselect(int dtype, int n, int n_trash, int64_t B, const void* psi,
                               const void* chi, double* fid, const double* dfid,
                               void* lam_psi, void* lam_chi, void* stream) {
  if (B == 0) return QS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(fidelity_postselect_kernel<float>, dim3((unsigned)B), kBlock, 0, st,
                       n, n_trash, (const float*)psi, (const float*)chi, fid, dfid,
                       (float*)lam_psi, (float*)lam_chi);
  else
    hipLaunchKernelGGL(fidelity_postselect_kernel<double>, dim3((unsigned)B), kBlock, 0, st,
                       n, n_trash, (const double*)psi, (const double*)chi, fid, dfid,
                       (double*)lam_psi, (double*)lam_chi);
  return ok();
}

int launch_fidelity_trajectory(int dtype, int n, int n_trash, int64_t B, const void* psi,
                               const void* chi, const double* u, double* fid,
                               int32_t* outcome, const double* dfid, void* lam_psi,
                               void* lam_chi, void* stream) {
  if (B == 0) return QS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(fidelity_trajectory_kernel<float>, dim3((unsigned)B), kBlock, 0, st,
                       n, n_trash, (const float*)psi, (const float*)chi, u, fid, outcome,
                       dfid, (float*)lam_psi, (float*)lam_chi);
  else
    hipLaunchKernelGGL(fidelity_trajectory_kernel<double>, dim3((unsigned)B), kBlock, 0, st,
                       n, n_trash, (const double*)psi, (const double*)chi, u, fid, outcome,
                       dfid, (double*)lam_psi, (double*)lam_chi);
  return ok();
}

int launch_reduce_partials(int dtype, const void* partials, int64_t rows,
                           int cols, const int32_t* col_param, double* out,
                           int accumulate, void* stream, const double* loss_part,
                           double* loss, double loss_scale) {
  const int blocks = cols + (loss != nullptr ? 1 : 0);
  if (blocks <= 0) return QS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(reduce_partials<float>, dim3((unsigned)blocks), kBlock, 0, st,
                       (const float*)partials, rows, cols, col_param, out, accumulate,
                       loss_part, loss, loss_scale);
  else
    hipLaunchKernelGGL(reduce_partials<double>, dim3((unsigned)blocks), kBlock, 0, st,
                       (const double*)partials, rows, cols, col_param, out, accumulate,
                       loss_part, loss, loss_scale);
  return ok();
}

int launch_copy_state(int dtype, const void* src, void* dst, int64_t n_amp,
                      void* stream) {
  if (n_amp <= 0) return QS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(copy_state<float2>, grid_for(n_amp), kBlock, 0, st,
                       (const float2*)src, (float2*)dst, n_amp);
  else
    hipLaunchKernelGGL(copy_state<double2>, grid_for(n_amp), kBlock, 0, st,
                       (const double2*)src, (double2*)dst, n_amp);
  return ok();
}

}  // namespace qs
