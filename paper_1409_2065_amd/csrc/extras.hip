// Principal components of the data and the projection of the cluster path
// onto them, on the device (Evaluation of Clusters: the path is viewed on
// principal components of the original data; Discussion: projecting on the
// GPU before any transfer saves moving U off the device for every gamma).
//
// cc_pca: X~ = X with missing entries replaced by their observed column
// means, centred by those means (C = X~ - 1 mean^T, FP64 throughout).  The
// top r right singular vectors of C come from subspace iteration on C^T C
// with s = min(r + 8, p) columns: Q <- orth(C^T (C Q)), orthonormalised by
// modified Gram-Schmidt in two passes, from counter-based start vectors;
// then a Rayleigh-Ritz step: the eigenpairs of (C Q)^T (C Q) by cyclic
// Jacobi rotations give V = Q W and the singular values sqrt(lambda).
// Each column of V is signed so that its entry of largest magnitude (the
// first such on ties) is positive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "ccmi_internal.h"

namespace ccmi {
namespace {

constexpr int kMaxR = 16;   // principal components returned
constexpr int kMaxS = 24;   // subspace columns
constexpr int kOrthThreads = 1024;

inline int64_t cdivx(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block sum in a fixed order, returned to every thread.  red: one double per
// wave.  Two barriers, so red may be reused right after.
__device__ inline double bsum(double v, double *red) {
  v = wsum(v);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x / kWave); ++q) t += red[q];
  __syncthreads();
  return t;
}

// Observed column means (0 for a column with no observed entry), one thread
// per column, rows in order.
template <typename TI>
__global__ void k_pca_mean(int n, int p, const TI *X, int64_t ldx, const uint8_t *M, int64_t ldm,
                           double *mean) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= p) return;
  double s = 0.0;
  int64_t c = 0;
  for (int i = 0; i < n; ++i) {
    if (M && !M[(size_t)i * ldm + f]) continue;
    s += (double)X[(size_t)i * ldx + f];
    ++c;
  }
  mean[f] = c ? s / (double)c : 0.0;
}

// C = X~ - mean (a missing entry becomes 0), n x p dense.
template <typename TI>
__global__ void k_pca_center(int n, int p, const TI *X, int64_t ldx, const uint8_t *M, int64_t ldm,
                             const double *mean, double *C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * p) return;
  const int i = (int)(e / p), f = (int)(e - (int64_t)i * p);
  const bool obs = !M || M[(size_t)i * ldm + f];
  C[e] = obs ? (double)X[(size_t)i * ldx + f] - mean[f] : 0.0;
}

// Start vectors: SplitMix64 of the element index, mapped to [-1, 1).
__global__ void k_pca_start(int64_t m, double *Q) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  uint64_t z = (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  Q[e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// B = C Q (n x s): one wave per row, S accumulators per lane.
template <int S>
__global__ __launch_bounds__(256) void k_pca_cq(int n, int p, int s, const double *C,
                                               const double *Q, double *B) {
  const int i = blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (i >= n) return;
  double acc[S];
#pragma unroll
  for (int c = 0; c < S; ++c) acc[c] = 0.0;
  for (int f = lane; f < p; f += kWave) {
    const double x = C[(size_t)i * p + f];
    const double *q = Q + (size_t)f * s;
#pragma unroll
    for (int c = 0; c < S; ++c)
      if (c < s) acc[c] = fma(x, q[c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < S; ++c) acc[c] = wsum(acc[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < S; ++c)
      if (c < s) B[(size_t)i * s + c] = acc[c];
  }
}

// Q = C^T B (p x s): one thread per feature, rows in order.
template <int S>
__global__ __launch_bounds__(256) void k_pca_ctb(int n, int p, int s, const double *C,
                                                const double *B, double *Q) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= p) return;
  double acc[S];
#pragma unroll
  for (int c = 0; c < S; ++c) acc[c] = 0.0;
  for (int i = 0; i < n; ++i) {
    const double x = C[(size_t)i * p + f];
    const double *b = B + (size_t)i * s;
#pragma unroll
    for (int c = 0; c < S; ++c)
      if (c < s) acc[c] = fma(x, b[c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < S; ++c)
    if (c < s) Q[(size_t)f * s + c] = acc[c];
}

// Orthonormal columns of Q (p x s) by modified Gram-Schmidt, two passes; a
// column that vanishes stays zero.  One block; every thread owns the same
// rows f = tid + k * blockDim in every step.
__global__ __launch_bounds__(kOrthThreads) void k_pca_orth(int p, int s, double *Q) {
  __shared__ double red[kOrthThreads / kWave];
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < s; ++j) {
      for (int k = 0; k < j; ++k) {
        double d = 0.0;
        for (int f = threadIdx.x; f < p; f += blockDim.x) d = fma(Q[(size_t)f * s + k], Q[(size_t)f * s + j], d);
        d = bsum(d, red);
        for (int f = threadIdx.x; f < p; f += blockDim.x) Q[(size_t)f * s + j] -= d * Q[(size_t)f * s + k];
      }
      double nn = 0.0;
      for (int f = threadIdx.x; f < p; f += blockDim.x) {
        const double q = Q[(size_t)f * s + j];
        nn = fma(q, q, nn);
      }
      nn = bsum(nn, red);
      const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int f = threadIdx.x; f < p; f += blockDim.x) Q[(size_t)f * s + j] *= inv;
    }
  }
}

// H = B^T B (s x s); entries (a, b) and (b, a) sum the same products in the
// same order, so H is exactly symmetric.
__global__ __launch_bounds__(256) void k_pca_gram(int n, int s, const double *B, double *H) {
  for (int t = threadIdx.x; t < s * s; t += blockDim.x) {
    const int a = t / s, b = t - a * s;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc = fma(B[(size_t)i * s + a], B[(size_t)i * s + b], acc);
    H[t] = acc;
  }
}

// Eigenpairs of the symmetric s x s matrix H by cyclic Jacobi rotations in
// LDS (one wave; thread t updates row or column entry t), sorted by
// decreasing eigenvalue: lam (s), W (s x s, eigenvectors in columns).
__global__ __launch_bounds__(kWave) void k_pca_eig(int s, const double *Hg, double *Wg, double *lam) {
  __shared__ double H[kMaxS][kMaxS], W[kMaxS][kMaxS];
  __shared__ int order[kMaxS];
  const int t = threadIdx.x;
  for (int e = t; e < s * s; e += kWave) {
    const int a = e / s, b = e - a * s;
    H[a][b] = Hg[e];
    W[a][b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int a = 0; a < s; ++a) {
      dia = fma(H[a][a], H[a][a], dia);
      for (int b = a + 1; b < s; ++b) off = fma(H[a][b], H[a][b], off);
    }
    if (!(off > 1e-32 * dia)) break;  // the same decision in every thread
    for (int a = 0; a < s - 1; ++a) {
      for (int b = a + 1; b < s; ++b) {
        const double hab = H[a][b];
        if (hab == 0.0) continue;
        const double tau = (H[b][b] - H[a][a]) / (2.0 * hab);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(fma(tau, tau, 1.0)));
        const double c = 1.0 / sqrt(fma(tt, tt, 1.0)), sn = tt * c;
        __syncthreads();
        if (t < s) {
          const double ha = H[a][t], hb = H[b][t];
          H[a][t] = c * ha - sn * hb;
          H[b][t] = sn * ha + c * hb;
        }
        __syncthreads();
        if (t < s) {
          const double ha = H[t][a], hb = H[t][b];
          H[t][a] = c * ha - sn * hb;
          H[t][b] = sn * ha + c * hb;
          const double wa = W[t][a], wb = W[t][b];
          W[t][a] = c * wa - sn * wb;
          W[t][b] = sn * wa + c * wb;
        }
        __syncthreads();
      }
    }
  }
  if (t == 0) {
    // insertion sort by decreasing eigenvalue; equal values keep their order
    for (int a = 0; a < s; ++a) order[a] = a;
    for (int a = 1; a < s; ++a) {
      const int v = order[a];
      const double key = H[v][v];
      int b = a - 1;
      while (b >= 0 && H[order[b]][order[b]] < key) {
        order[b + 1] = order[b];
        --b;
      }
      order[b + 1] = v;
    }
  }
  __syncthreads();
  for (int e = t; e < s * s; e += kWave) {
    const int a = e / s, c = e - a * s;
    Wg[e] = W[a][order[c]];
  }
  if (t < s) lam[t] = H[order[t]][order[t]];
}

// V = Q W[:, :r] (p x r).
__global__ void k_pca_rotate(int p, int s, int r, const double *Q, const double *W, double *V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)p * r) return;
  const int f = (int)(e / r), c = (int)(e - (int64_t)f * r);
  double acc = 0.0;
  for (int u = 0; u < s; ++u) acc = fma(Q[(size_t)f * s + u], W[(size_t)u * s + c], acc);
  V[e] = acc;
}

// Sign of each column: its entry of largest magnitude (first on ties) > 0.
__global__ __launch_bounds__(kOrthThreads) void k_pca_sign(int p, int r, double *V) {
  __shared__ double bv[kOrthThreads / kWave];
  __shared__ int bi[kOrthThreads / kWave];
  __shared__ double flip;
  for (int c = 0; c < r; ++c) {
    double best = -1.0;
    int idx = p;
    for (int f = threadIdx.x; f < p; f += blockDim.x) {
      const double a = fabs(V[(size_t)f * r + c]);
      if (a > best) { best = a; idx = f; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, kWave);
      const int oi = __shfl_xor(idx, off, kWave);
      if (ob > best || (ob == best && oi < idx)) { best = ob; idx = oi; }
    }
    if (threadIdx.x % kWave == 0) { bv[threadIdx.x / kWave] = best; bi[threadIdx.x / kWave] = idx; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = -1.0;
      int k = p;
      for (int w = 0; w < (int)(blockDim.x / kWave); ++w)
        if (bv[w] > b || (bv[w] == b && bi[w] < k)) { b = bv[w]; k = bi[w]; }
      flip = (k < p && V[(size_t)k * r + c] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    const double sg = flip;
    for (int f = threadIdx.x; f < p; f += blockDim.x) V[(size_t)f * r + c] *= sg;
    __syncthreads();
  }
}

// out (n x r) = (U - center) V: one wave per row of U (row stride ld).
template <typename TS>
__global__ __launch_bounds__(256) void k_project(int n, int p, int ld, const TS *U, int r,
                                                const double *V, const double *center, double *out) {
  const int i = blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (i >= n) return;
  double acc[kMaxR];
#pragma unroll
  for (int c = 0; c < kMaxR; ++c) acc[c] = 0.0;
  for (int f = lane; f < p; f += kWave) {
    const double u = (double)U[(size_t)i * ld + f] - (center ? center[f] : 0.0);
    const double *v = V + (size_t)f * r;
#pragma unroll
    for (int c = 0; c < kMaxR; ++c)
      if (c < r) acc[c] = fma(u, v[c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < kMaxR; ++c) acc[c] = wsum(acc[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < kMaxR; ++c)
      if (c < r) out[(size_t)i * r + c] = acc[c];
  }
}

struct Buf {
  void *p = nullptr;
  ~Buf() { if (p) (void)hipFree(p); }
  cc_status alloc(size_t bytes) {
    if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) {
      p = nullptr;
      set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
      return CC_ERR_OUT_OF_MEMORY;
    }
    return CC_OK;
  }
  double *d() const { return reinterpret_cast<double *>(p); }
};

#define PC_TRY(x)               \
  do {                          \
    cc_status _s = (x);         \
    if (_s != CC_OK) return _s; \
  } while (0)

template <int S>
void power_step(int n, int p, int s, const double *C, double *Q, double *B, hipStream_t st) {
  hipLaunchKernelGGL((k_pca_cq<S>), dim3((int)cdivx(n, 4)), dim3(256), 0, st, n, p, s, C, Q, B);
  hipLaunchKernelGGL((k_pca_ctb<S>), dim3((int)cdivx(p, 256)), dim3(256), 0, st, n, p, s, C, B, Q);
  hipLaunchKernelGGL(k_pca_orth, dim3(1), dim3(kOrthThreads), 0, st, p, s, Q);
}

template <int S>
void ritz_product(int n, int p, int s, const double *C, const double *Q, double *B, hipStream_t st) {
  hipLaunchKernelGGL((k_pca_cq<S>), dim3((int)cdivx(n, 4)), dim3(256), 0, st, n, p, s, C, Q, B);
}

template <typename TI>
cc_status pca_impl(int n, int p, const TI *X, int64_t ldx, const uint8_t *M, int64_t ldm, int r,
                   int iters, double *V, double *sval, double *center, hipStream_t st) {
  const int s = std::min(std::min(r + 8, p), kMaxS);
  Buf mean, C, Q, B, H, W, lam;
  PC_TRY(mean.alloc((size_t)p * 8));
  PC_TRY(C.alloc((size_t)n * p * 8));
  PC_TRY(Q.alloc((size_t)p * s * 8));
  PC_TRY(B.alloc((size_t)n * s * 8));
  PC_TRY(H.alloc((size_t)s * s * 8));
  PC_TRY(W.alloc((size_t)s * s * 8));
  PC_TRY(lam.alloc((size_t)s * 8));
  hipLaunchKernelGGL((k_pca_mean<TI>), dim3((int)cdivx(p, 256)), dim3(256), 0, st, n, p, X, ldx, M,
                     ldm, mean.d());
  hipLaunchKernelGGL((k_pca_center<TI>), dim3((int)cdivx((int64_t)n * p, 256)), dim3(256), 0, st, n,
                     p, X, ldx, M, ldm, mean.d(), C.d());
  hipLaunchKernelGGL(k_pca_start, dim3((int)cdivx((int64_t)p * s, 256)), dim3(256), 0, st,
                     (int64_t)p * s, Q.d());
  hipLaunchKernelGGL(k_pca_orth, dim3(1), dim3(kOrthThreads), 0, st, p, s, Q.d());
  CC_HIP(hipGetLastError());
  for (int it = 0; it < iters; ++it) {
    if (s <= 8) power_step<8>(n, p, s, C.d(), Q.d(), B.d(), st);
    else if (s <= 16) power_step<16>(n, p, s, C.d(), Q.d(), B.d(), st);
    else power_step<24>(n, p, s, C.d(), Q.d(), B.d(), st);
  }
  if (s <= 8) ritz_product<8>(n, p, s, C.d(), Q.d(), B.d(), st);
  else if (s <= 16) ritz_product<16>(n, p, s, C.d(), Q.d(), B.d(), st);
  else ritz_product<24>(n, p, s, C.d(), Q.d(), B.d(), st);
  hipLaunchKernelGGL(k_pca_gram, dim3(1), dim3(256), 0, st, n, s, B.d(), H.d());
  hipLaunchKernelGGL(k_pca_eig, dim3(1), dim3(kWave), 0, st, s, H.d(), W.d(), lam.d());
  hipLaunchKernelGGL(k_pca_rotate, dim3((int)cdivx((int64_t)p * r, 256)), dim3(256), 0, st, p, s, r,
                     Q.d(), W.d(), V);
  hipLaunchKernelGGL(k_pca_sign, dim3(1), dim3(kOrthThreads), 0, st, p, r, V);
  CC_HIP(hipGetLastError());
  if (center) CC_HIP(hipMemcpyAsync(center, mean.p, (size_t)p * 8, hipMemcpyDeviceToDevice, st));
  double hl[kMaxS];
  CC_HIP(hipMemcpyAsync(hl, lam.p, (size_t)s * 8, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  for (int c = 0; c < r; ++c) sval[c] = std::sqrt(std::max(hl[c], 0.0));
  return CC_OK;
}

}  // namespace

cc_status pca(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
              const uint8_t *mask, int64_t ldm, int32_t r, int32_t iters, double *V,
              double *sval, double *center, hipStream_t stream) {
  if (n < 2 || p < 1) { set_error("need n >= 2 and p >= 1"); return CC_ERR_INVALID_ARG; }
  if (n * p > ((int64_t)1 << 31) - 1) { set_error("n * p too large"); return CC_ERR_INVALID_ARG; }
  if (r < 1 || r > kMaxR || r > p || r > n) { set_error("need 1 <= r <= min(16, n, p)"); return CC_ERR_INVALID_ARG; }
  if (iters < 0 || iters > 100000) { set_error("need 0 <= iters <= 100000"); return CC_ERR_INVALID_ARG; }
  if (!X || !V || !sval) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  if (x_dtype != CC_DTYPE_F32 && x_dtype != CC_DTYPE_F64) { set_error("bad x_dtype"); return CC_ERR_INVALID_ARG; }
  if (ldx < p || (mask && ldm < p)) { set_error("leading dimension < p"); return CC_ERR_INVALID_ARG; }
  const int it = iters > 0 ? iters : 100;
  if (x_dtype == CC_DTYPE_F32)
    return pca_impl<float>((int)n, (int)p, (const float *)X, ldx, mask, ldm, r, it, V, sval, center, stream);
  return pca_impl<double>((int)n, (int)p, (const double *)X, ldx, mask, ldm, r, it, V, sval, center, stream);
}

cc_status project_U(Problem *P, int32_t r, const double *V, const double *center, double *out) {
  if (r < 1 || r > kMaxR) { set_error("need 1 <= r <= 16"); return CC_ERR_INVALID_ARG; }
  if (!V || !out) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  const dim3 grid((unsigned)cdivx(P->n, 4));
  if (P->precision == kF32)
    hipLaunchKernelGGL((k_project<float>), grid, dim3(256), 0, P->stream, (int)P->n, (int)P->p,
                       (int)P->ld, (const float *)P->U, r, V, center, out);
  else
    hipLaunchKernelGGL((k_project<double>), grid, dim3(256), 0, P->stream, (int)P->n, (int)P->p,
                       (int)P->ld, (const double *)P->U, r, V, center, out);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

}  // namespace ccmi
