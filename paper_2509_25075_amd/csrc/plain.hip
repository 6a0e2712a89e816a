// Plain path: one kernel launch per gate over the whole batch, states in
// HBM. Same mathematics as the fused engine (R_P(t) = exp(-i t P / 2), adjoint
// dL/dtheta = Im <lam|P|psi>), with no fusion, no register residency and no
// LDS staging: the baseline the fused engine is measured against, and the
// path for states too large for the fused engine.
#include <hip/hip_runtime.h>

#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBlock = 256;

template <typename real>
struct PArgs {
  int n;
  int64_t B;
  int per_sample;
  int n_params, n_feats;
  const real* params;
  const real* feats;
};

template <typename real>
__device__ __forceinline__ real p_theta(const PArgs<real>& A, const qs_gate& g,
                                        int64_t b) {
  const real* P = A.per_sample ? A.params + b * A.n_params : A.params;
  real w = g.p_w >= 0 ? P[g.p_w] : (real)1;
  real f = g.feat >= 0 ? A.feats[b * A.n_feats + g.feat] : (real)1;
  real bias = g.p_b >= 0 ? P[g.p_b] : (real)0;
  return (real)g.scale * (w * f + bias);
}

__device__ __forceinline__ void p_sincos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void p_sincos(double x, double* s, double* c) { sincos(x, s, c); }

// Apply gate (inverse when inv) to up to two states (x, and y if non-null).
// One thread per amplitude pair (1-qubit gates, CNOT) or per amplitude (CZ).
template <typename real>
__global__ void __launch_bounds__(kBlock)
plain_gate(PArgs<real> A, qs_gate g, int inv, real* x, real* y) {
  const int n = A.n;
  const int64_t half = 1ll << (n - 1);
  const int64_t total = (g.op == QS_OP_CZ) ? (A.B << n) : (A.B * half);
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= total) return;
  if (g.op == QS_OP_CZ) {
    const int64_t i = idx & ((1ll << n) - 1);
    if (((i >> g.q0) & 1) && ((i >> g.q1) & 1)) {
      x[2 * idx] = -x[2 * idx];
      x[2 * idx + 1] = -x[2 * idx + 1];
      if (y) {
        y[2 * idx] = -y[2 * idx];
        y[2 * idx + 1] = -y[2 * idx + 1];
      }
    }
    return;
  }
  const int64_t b = idx >> (n - 1), pr = idx & (half - 1);
  const int q = g.op == QS_OP_CNOT ? g.q1 : g.q0;
  const int64_t lo = pr & ((1ll << q) - 1);
  const int64_t i0 = (b << n) + (((pr >> q) << (q + 1)) | lo);
  const int64_t i1 = i0 + (1ll << q);
  if (g.op == QS_OP_CNOT && !(((i0 - (b << n)) >> g.q0) & 1)) return;
  real c = 1, s = 0;
  if (g.op <= QS_OP_RZ) {
    real th = p_theta(A, g, b);
    p_sincos(th * (real)0.5, &s, &c);
    if (inv) s = -s;
  }
  real* st[2] = {x, y};
  for (int w = 0; w < 2; ++w) {
    real* v = st[w];
    if (!v) continue;
    real a0r = v[2 * i0], a0i = v[2 * i0 + 1], a1r = v[2 * i1], a1i = v[2 * i1 + 1];
    real o0r, o0i, o1r, o1i;
    switch (g.op) {
      case QS_OP_RX:
        o0r = c * a0r + s * a1i; o0i = c * a0i - s * a1r;
        o1r = c * a1r + s * a0i; o1i = c * a1i - s * a0r;
        break;
      case QS_OP_RY:
        o0r = c * a0r - s * a1r; o0i = c * a0i - s * a1i;
        o1r = s * a0r + c * a1r; o1i = s * a0i + c * a1i;
        break;
      case QS_OP_RZ:  // diag(c - i s, c + i s)
        o0r = c * a0r + s * a0i; o0i = c * a0i - s * a0r;
        o1r = c * a1r - s * a1i; o1i = c * a1i + s * a1r;
        break;
      case QS_OP_X:
      case QS_OP_CNOT:
        o0r = a1r; o0i = a1i; o1r = a0r; o1i = a0i;
        break;
      case QS_OP_Y:
        o0r = a1i; o0i = -a1r; o1r = -a0i; o1i = a0r;
        break;
      case QS_OP_Z:
        o0r = a0r; o0i = a0i; o1r = -a1r; o1i = -a1i;
        break;
      default: {  // H
        const real h = (real)0.70710678118654752440;
        o0r = h * (a0r + a1r); o0i = h * (a0i + a1i);
        o1r = h * (a0r - a1r); o1i = h * (a0i - a1i);
      }
    }
    v[2 * i0] = o0r; v[2 * i0 + 1] = o0i; v[2 * i1] = o1r; v[2 * i1 + 1] = o1i;
  }
}

// dL/dtheta_g(b) = Im <lam|P|psi> for one rotation gate, reduced per sample
// with FP64 atomics into gth[b * G + g] (zeroed beforehand).
template <typename real>
__global__ void __launch_bounds__(kBlock)
plain_grad(int n, int64_t B, qs_gate g, int gidx, int G, const real* psi,
           const real* lam, double* gth) {
  __shared__ double sh[kBlock / 64];
  const int64_t half = 1ll << (n - 1);
  for (int64_t b = blockIdx.y; b < B; b += gridDim.y) {
  double acc = 0;
  for (int64_t pr = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pr < half;
       pr += (int64_t)gridDim.x * blockDim.x) {
    const int q = g.q0;
    const int64_t lo = pr & ((1ll << q) - 1);
    const int64_t i0 = (b << n) + (((pr >> q) << (q + 1)) | lo);
    const int64_t i1 = i0 + (1ll << q);
    const double p0r = psi[2 * i0], p0i = psi[2 * i0 + 1];
    const double p1r = psi[2 * i1], p1i = psi[2 * i1 + 1];
    const double l0r = lam[2 * i0], l0i = lam[2 * i0 + 1];
    const double l1r = lam[2 * i1], l1i = lam[2 * i1 + 1];
    if (g.op == QS_OP_RX)
      acc += l0r * p1i - l0i * p1r + l1r * p0i - l1i * p0r;
    else if (g.op == QS_OP_RY)
      acc += l1r * p0r + l1i * p0i - l0r * p1r - l0i * p1i;
    else
      acc += (l0r * p0i - l0i * p0r) - (l1r * p1i - l1i * p1r);
  }
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    atomicAdd(&gth[b * G + gidx], t);
  }
  __syncthreads();
  }
}

// Chain rule theta = scale (w f + bias) -> parameter and feature gradients.
// One block per gate; threads stride over samples.
template <typename real>
__global__ void __launch_bounds__(kBlock)
plain_chain(PArgs<real> A, const qs_gate* gates, int G, const double* gth,
            double* gp, double* gf) {
  __shared__ double sh[2][kBlock / 64];
  const int g = blockIdx.x;
  const qs_gate gt = gates[g];
  if (gt.op > QS_OP_RZ) return;
  double sw = 0, sb = 0;
  for (int64_t b = threadIdx.x; b < A.B; b += blockDim.x) {
    const double v = gth[b * G + g] * (double)gt.scale;
    const real* P = A.per_sample ? A.params + b * A.n_params : A.params;
    const double f = gt.feat >= 0 ? (double)A.feats[b * A.n_feats + gt.feat] : 1.0;
    const double w = gt.p_w >= 0 ? (double)P[gt.p_w] : 1.0;
    if (A.per_sample) {
      if (gt.p_w >= 0) atomicAdd(&gp[b * A.n_params + gt.p_w], v * f);
      if (gt.p_b >= 0) atomicAdd(&gp[b * A.n_params + gt.p_b], v);
    } else {
      sw += v * f;
      sb += v;
    }
    if (gt.feat >= 0 && gf) atomicAdd(&gf[b * A.n_feats + gt.feat], v * w);
  }
  if (A.per_sample) return;
  for (int o = 32; o >= 1; o >>= 1) {
    sw += __shfl_xor(sw, o);
    sb += __shfl_xor(sb, o);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = sw;
    sh[1][threadIdx.x >> 6] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tw = 0, tb = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      tw += sh[0][i];
      tb += sh[1][i];
    }
    if (gt.p_w >= 0) atomicAdd(&gp[gt.p_w], tw);
    if (gt.p_b >= 0) atomicAdd(&gp[gt.p_b], tb);
  }
}

// lam = sum_q dexpz[b][q] Z_q psi
template <typename real>
__global__ void __launch_bounds__(kBlock)
plain_obs_cot(int n, int64_t B, const double* dexpz, const real* psi, real* lam) {
  const int64_t total = B << n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx >> n, i = idx & ((1ll << n) - 1);
    double cf = 0;
    for (int q = 0; q < n; ++q) cf += ((i >> q) & 1) ? -dexpz[b * n + q] : dexpz[b * n + q];
    lam[2 * idx] = (real)(cf * psi[2 * idx]);
    lam[2 * idx + 1] = (real)(cf * psi[2 * idx + 1]);
  }
}

unsigned grid1(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > (1ll << 31) - 1) g = (1ll << 31) - 1;
  return (unsigned)(g < 1 ? 1 : g);
}

int ok() { return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_LAUNCH; }

template <typename real>
PArgs<real> pargs(const PlainLaunch& L) {
  PArgs<real> A;
  A.n = L.c->n_qubits;
  A.B = L.B;
  A.per_sample = L.per_sample_params;
  A.n_params = L.c->n_params;
  A.n_feats = L.c->n_features;
  A.params = static_cast<const real*>(L.params);
  A.feats = static_cast<const real*>(L.feats);
  return A;
}

template <typename real>
int launch_gate(const PArgs<real>& A, const qs_gate& g, int inv, real* x,
                real* y, hipStream_t st) {
  const int64_t total = (g.op == QS_OP_CZ) ? (A.B << A.n) : (A.B << (A.n - 1));
  hipLaunchKernelGGL(plain_gate<real>, grid1(total), kBlock, 0, st, A, g, inv,
                     x, y);
  return ok();
}

template <typename real>
int forward_t(const PlainLaunch& L) {
  PArgs<real> A = pargs<real>(L);
  hipStream_t st = static_cast<hipStream_t>(L.stream);
  real* x = static_cast<real*>(L.state);
  const int64_t per = L.B << A.n;  // complex elements per state batch
  int ck = 0;
  for (int g = 0; g < L.c->n_gates; ++g) {
    if (ck < L.n_ckpt && L.ckpt_gates[ck] == g) {
      int rc = launch_copy_state(L.dtype, x, static_cast<real*>(L.ckpt) + 2 * per * ck,
                                 per, L.stream);
      if (rc != QS_OK) return rc;
      ++ck;
    }
    int rc = launch_gate<real>(A, L.c->gates[g], 0, x, nullptr, st);
    if (rc != QS_OK) return rc;
  }
  if (L.expz) return launch_expz(L.dtype, A.n, L.B, x, L.expz, L.stream);
  return QS_OK;
}

template <typename real>
int adjoint_t(const PlainLaunch& L) {
  PArgs<real> A = pargs<real>(L);
  hipStream_t st = static_cast<hipStream_t>(L.stream);
  const int n = A.n, G = L.c->n_gates;
  const int64_t per = L.B << n;
  real* lam = static_cast<real*>(L.ws);
  real* psi = lam + 2 * per;
  double* gth = reinterpret_cast<double*>(psi + 2 * per);
  int rc = launch_copy_state(L.dtype, L.state, psi, per, L.stream);
  if (rc != QS_OK) return rc;
  if (L.dstate) {
    rc = launch_copy_state(L.dtype, L.dstate, lam, per, L.stream);
  } else {
    hipLaunchKernelGGL(plain_obs_cot<real>, grid1(per), kBlock, 0, st, n, L.B,
                       L.dexpz, psi, lam);
    rc = ok();
  }
  if (rc != QS_OK) return rc;
  rc = launch_fill_f64(gth, L.B * G, L.stream);
  if (rc != QS_OK) return rc;
  int ck = L.n_ckpt - 1;
  const int64_t half = 1ll << (n - 1);
  int64_t bx = (half + kBlock * 8 - 1) / (kBlock * 8);
  if (bx > 1024) bx = 1024;
  for (int g = G - 1; g >= 0; --g) {
    // psi after the first g+1 gates is psi_g; re-anchor at a checkpoint that
    // holds the state after exactly g+1 gates.
    if (L.ckpt && ck >= 0 && L.ckpt_gates[ck] == g + 1) {
      rc = launch_copy_state(L.dtype, static_cast<const real*>(L.ckpt) + 2 * per * ck,
                             psi, per, L.stream);
      if (rc != QS_OK) return rc;
      --ck;
    }
    const qs_gate& gt = L.c->gates[g];
    if (gt.op <= QS_OP_RZ) {
      hipLaunchKernelGGL(plain_grad<real>, dim3((unsigned)bx, (unsigned)(L.B < 65535 ? L.B : 65535)),
                         kBlock, 0, st, n, L.B, gt, g, G, psi, lam, gth);
      if ((rc = ok()) != QS_OK) return rc;
    }
    rc = launch_gate<real>(A, gt, 1, psi, lam, st);
    if (rc != QS_OK) return rc;
  }
  const int64_t gp_n = L.per_sample_params ? L.B * L.c->n_params : L.c->n_params;
  rc = launch_fill_f64(L.grad_params, gp_n, L.stream);
  if (rc != QS_OK) return rc;
  if (L.grad_feats) {
    rc = launch_fill_f64(L.grad_feats, L.B * L.c->n_features, L.stream);
    if (rc != QS_OK) return rc;
  }
  if (G > 0) {
    hipLaunchKernelGGL(plain_chain<real>, dim3((unsigned)G), kBlock, 0, st, A,
                       L.d_gates, G, gth, L.grad_params, L.grad_feats);
    rc = ok();
  }
  return rc;
}

}  // namespace

int launch_obs_cot(int dtype, int n, int64_t B, const double* dexpz,
                   const void* psi, void* lam, void* stream) {
  const int64_t per = B << n;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QS_C64)
    hipLaunchKernelGGL(plain_obs_cot<float>, grid1(per), kBlock, 0, st, n, B, dexpz,
                       (const float*)psi, (float*)lam);
  else
    hipLaunchKernelGGL(plain_obs_cot<double>, grid1(per), kBlock, 0, st, n, B, dexpz,
                       (const double*)psi, (double*)lam);
  return ok();
}

size_t plain_workspace_bytes(const qs_circuit& c, int dtype, int64_t B) {
  const size_t real_sz = dtype == QS_C64 ? 4 : 8;
  const size_t per = (size_t)B << c.n_qubits;
  return 2 * (2 * per * real_sz) + (size_t)B * c.n_gates * sizeof(double);
}

int run_plain_forward(const PlainLaunch& L) {
  return L.dtype == QS_C64 ? forward_t<float>(L) : forward_t<double>(L);
}
int run_plain_adjoint(const PlainLaunch& L) {
  return L.dtype == QS_C64 ? adjoint_t<float>(L) : adjoint_t<double>(L);
}

}  // namespace qs
