// k-nearest-neighbour Gaussian-kernel weights (Methods, "Calibration of
// Weights", eq_weighting) and column standardisation on gfx950.
//
// Pipeline of cc_build_knn_weights:
//   1. observed column means; X-tilde = X with missing entries replaced by
//      them, kept in FP32 (for ranking) and FP64 (for exact distances);
//   2. Gram matrix G = X~ X~^T on the matrix cores (v_mfma_f32_16x16x4_f32),
//      d2_ij = |x_i|^2 + |x_j|^2 - 2 G_ij in FP32 for every pair;
//   3. per row, a bitonic sort in LDS of (d2, j) keys, self excluded, ties to
//      the lower index, keeps the K = k + margin best candidates;
//   4. exact FP64 distances of the candidates, re-sorted by (d2, j), keep k;
//   5. the relation i ~_k j (either direction) as a bitmap, counted and
//      prefix-summed per row, written out as sorted edges (i < j);
//   6. exact FP64 d2 per edge, phi (literal or |phi| / lower median d2),
//      w = exp(-phi d2), optional normalisation to sum 1.
//
// Also here: the smallest k whose kNN graph is connected (Results, "Impact
// of the Constants k and phi": bisection over k with a graph search), and
// weights from the composite distance of genotypes and coordinates
// (composite_distance).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "ccmi_internal.h"

namespace ccmi {

static inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------- column stats
template <typename TI>
__global__ void k_col_moments(int n, int p, const TI *X, int64_t ldx, const uint8_t *M,
                              int64_t ldm, double *mean, double *sd, int *nonfinite) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= p) return;
  double sum = 0.0;
  int cnt = 0, bad = 0;
  for (int i = 0; i < n; ++i) {
    if (M && M[(size_t)i * ldm + f] == 0) continue;
    const double x = (double)X[(size_t)i * ldx + f];
    if (!isfinite(x)) { ++bad; continue; }
    sum += x; ++cnt;
  }
  const double mu = cnt > 0 ? sum / cnt : 0.0;
  double ss = 0.0;
  for (int i = 0; i < n; ++i) {
    if (M && M[(size_t)i * ldm + f] == 0) continue;
    const double x = (double)X[(size_t)i * ldx + f];
    if (!isfinite(x)) continue;
    ss += (x - mu) * (x - mu);
  }
  mean[f] = mu;
  if (sd) sd[f] = cnt > 0 ? sqrt(ss / cnt) : 0.0;
  if (bad) atomicAdd(nonfinite, bad);
}

template <typename TI>
__global__ void k_standardize(int n, int p, TI *X, int64_t ldx, const uint8_t *M, int64_t ldm,
                              const double *mean, const double *sd) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * p) return;
  const int i = (int)(idx / p), f = (int)(idx % p);
  if (M && M[(size_t)i * ldm + f] == 0) return;
  const double s = sd[f];
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  const double x = (double)X[(size_t)i * ldx + f];
  X[(size_t)i * ldx + f] = (TI)((x - mean[f]) * inv);
}

// X-tilde in FP32 (n_pad x ldk, zero padded) and FP64 (n x p), and the FP32
// squared row norms of the FP32 copy.
template <typename TI>
__global__ void k_impute(int n, int p, int n_pad, int ldk, const TI *X, int64_t ldx,
                         const uint8_t *M, int64_t ldm, const double *mean, float *Xf,
                         double *Xd) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n_pad * ldk) return;
  const int i = (int)(idx / ldk), f = (int)(idx % ldk);
  double v = 0.0;
  if (i < n && f < p) {
    const bool obs = M ? (M[(size_t)i * ldm + f] != 0) : true;
    v = obs ? (double)X[(size_t)i * ldx + f] : mean[f];
    Xd[(size_t)i * p + f] = v;
  }
  Xf[idx] = (float)v;
}

__global__ void k_rownorm(int n_pad, int ldk, const float *Xf, float *nrm) {
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int f = threadIdx.x; f < ldk; f += blockDim.x) {
    const double v = Xf[(size_t)i * ldk + f];
    acc = fma(v, v, acc);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  __shared__ double s[16];
  if (threadIdx.x % kWave == 0) s[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += s[w];
    nrm[i] = (float)t;
  }
}

// ------------------------------------------------------------ MFMA Gram
// Output tile 64 x 64 per block of 4 waves; wave w owns rows 16w..16w+15 and
// all 64 columns as four 16 x 16 accumulators.  K is staged through LDS in
// chunks of 32 features; the next chunk's global loads are in flight while
// the current chunk's MFMAs run.  v_mfma_f32_16x16x4_f32 operand layout
// (wave64): A element (row l%16, k l/16), B element (k l/16, col l%16), and
// result register r of lane l holds (row 4*(l/16)+r, col l%16).
// When the output tiles alone cannot fill the chip, blockIdx.z splits K:
// each split writes its partial tile to part, and k_gram_combine adds the
// splits in a fixed order.
constexpr int kGT = 64, kKC = 32;

typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gram_d2(int n, int n_pad, int ldk, int nsplit,
                                                 const float *Xf, const float *nrm, float *D2,
                                                 int64_t ldd, float *part) {
  __shared__ float As[kGT][kKC + 1];
  __shared__ float Bs[kGT][kKC + 1];
  const int bi = blockIdx.y * kGT, bj = blockIdx.x * kGT;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int nch = ldk / kKC;
  const int per = (nch + nsplit - 1) / nsplit;
  const int c0 = blockIdx.z * per, c1 = min(nch, c0 + per);
  // 64 rows x 32 floats per operand: thread tid loads rows r and r + 32,
  // 4 consecutive floats each
  const int r = tid / 8, c4 = (tid % 8) * 4;
  float4 pa[2], pb[2];
  auto gload = [&](int ch) {
    const int k0 = ch * kKC + c4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      pa[h] = *reinterpret_cast<const float4 *>(Xf + (size_t)(bi + r + 32 * h) * ldk + k0);
      pb[h] = *reinterpret_cast<const float4 *>(Xf + (size_t)(bj + r + 32 * h) * ldk + k0);
    }
  };
  floatx4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  if (c0 < c1) gload(c0);
  for (int ch = c0; ch < c1; ++ch) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float *ar = &As[r + 32 * h][c4], *br = &Bs[r + 32 * h][c4];
      ar[0] = pa[h].x; ar[1] = pa[h].y; ar[2] = pa[h].z; ar[3] = pa[h].w;
      br[0] = pb[h].x; br[1] = pb[h].y; br[2] = pb[h].z; br[3] = pb[h].w;
    }
    __syncthreads();
    if (ch + 1 < c1) gload(ch + 1);
#pragma unroll
    for (int kk = 0; kk < kKC; kk += 4) {
      const float a = As[wave * 16 + lane % 16][kk + lane / 16];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float b = Bs[c * 16 + lane % 16][kk + lane / 16];
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = bi + wave * 16 + 4 * (lane / 16) + q;
      const int j = bj + c * 16 + lane % 16;
      if (nsplit > 1)
        part[((size_t)blockIdx.z * n_pad + i) * n_pad + j] = acc[c][q];
      else if (i < n && j < n)
        D2[(size_t)i * ldd + j] = nrm[i] + nrm[j] - 2.0f * acc[c][q];
    }
  }
}

// d2 from the K-split partial Gram tiles, splits added in order.
__global__ void k_gram_combine(int n, int n_pad, int nsplit, const float *part, const float *nrm,
                               float *D2, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
  float g = 0.f;
  for (int z = 0; z < nsplit; ++z) g += part[((size_t)z * n_pad + i) * n_pad + j];
  D2[(size_t)i * ldd + j] = nrm[i] + nrm[j] - 2.0f * g;
}

// Monotone map of a float to an unsigned key (handles negative values).
__device__ inline uint32_t float_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Most candidates k_recheck takes per row (12 bytes of LDS each), and the
// largest n of the kNN builders (a row's sort keys fill 8 * n bytes of LDS).
constexpr int64_t kRecheckMaxK = 12288;
constexpr int64_t kKnnMaxN = 16384;

// Inverse of float_key.
__device__ inline float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Per row: bitonic sort of (key(d2) << 32 | j) in LDS; keep the first K, and
// in dnext the FP32 d2 of the first row left out (infinity when none is).
// todo (may be NULL): only rows with todo[i] != 0.
__global__ __launch_bounds__(1024) void k_row_candidates(int n, const float *D2, int64_t ldd,
                                                         int npow2, int K, int32_t *cand,
                                                         const int *todo, float *dnext) {
  extern __shared__ unsigned long long keys[];
  const int i = blockIdx.x;
  if (todo && !todo[i]) return;
  for (int j = threadIdx.x; j < npow2; j += blockDim.x) {
    unsigned long long key = ~0ull;
    if (j < n && j != i) key = ((unsigned long long)float_key(D2[(size_t)i * ldd + j]) << 32) | (unsigned)j;
    keys[j] = key;
  }
  __syncthreads();
  for (int size = 2; size <= npow2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < npow2 / 2; t += blockDim.x) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const unsigned long long a = keys[lo], b = keys[hi];
        if ((a > b) == up) { keys[lo] = b; keys[hi] = a; }
      }
      __syncthreads();
    }
  }
  for (int r = threadIdx.x; r < K; r += blockDim.x) cand[(size_t)i * K + r] = (int32_t)(keys[r] & 0xffffffffu);
  if (threadIdx.x == 0) dnext[i] = K < n - 1 ? key_float((uint32_t)(keys[K] >> 32)) : INFINITY;
}

// Largest FP32 row norm of the n rows.
__global__ __launch_bounds__(1024) void k_max_norm(int n, const float *nrm, float *nmax) {
  __shared__ float s[1024];
  float m = 0.f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, nrm[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *nmax = s[0];
}

// Exact FP64 squared distances of the candidates, then the k best by (d2, j).
// Certificate: every row left out has an FP32 distance of at least dnext[i],
// so an exact one of at least dnext[i] - bound, with bound = bscale *
// (|x_i|^2 + max_j |x_j|^2) covering the rounding of the FP32 Gram product,
// the norms, their combination and the FP32 copy of X~.  The k best
// candidates are then the k nearest of all rows when the k-th exact distance
// lies below that; otherwise uncert[i] = 1 and the row is counted in *n_uncert.
// todo (may be NULL): only rows with todo[i] != 0.
__global__ __launch_bounds__(256) void k_recheck(int n, int p, const double *Xd, int K, int k,
                                                 const int32_t *cand, int32_t *knn, const int *todo,
                                                 const float *dnext, const float *nrm,
                                                 const float *nmax, double bscale, int *uncert,
                                                 int *n_uncert) {
  extern __shared__ double sd[];  // K doubles + K ints
  int *sj = reinterpret_cast<int *>(sd + K);
  const int i = blockIdx.x;
  if (todo && !todo[i]) return;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int c = wave; c < K; c += nw) {
    const int j = cand[(size_t)i * K + c];
    double acc = 0.0;
    for (int f = lane; f < p; f += kWave) {
      const double d = Xd[(size_t)j * p + f] - Xd[(size_t)i * p + f];
      acc = fma(d, d, acc);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) { sd[c] = acc; sj[c] = j; }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // selection of the k smallest (d2, j); K is small
    for (int r = 0; r < k; ++r) {
      int best = r;
      for (int c = r + 1; c < K; ++c)
        if (sd[c] < sd[best] || (sd[c] == sd[best] && sj[c] < sj[best])) best = c;
      const double td = sd[r]; sd[r] = sd[best]; sd[best] = td;
      const int tj = sj[r]; sj[r] = sj[best]; sj[best] = tj;
      knn[(size_t)i * k + r] = sj[r];
    }
    const double bound = bscale * ((double)nrm[i] + (double)*nmax);
    const bool ok = sd[k - 1] < (double)dnext[i] - bound;
    uncert[i] = ok ? 0 : 1;
    if (!ok) atomicAdd(n_uncert, 1);
  }
}

__global__ void k_mark_pairs(int n, int k, int words, const int32_t *knn, uint32_t *bm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * k) return;
  const int i = (int)(idx / k);
  const int j = knn[idx];
  const int a = min(i, j), b = max(i, j);
  atomicOr(&bm[(size_t)a * words + b / 32], 1u << (b % 32));
}

__global__ void k_row_counts(int n, int words, const uint32_t *bm, int32_t *cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  for (int w = 0; w < words; ++w) c += __popc(bm[(size_t)i * words + w]);
  cnt[i] = c;
}

// Exclusive scan of n counts in one block (sequential chunks, fixed order).
__global__ __launch_bounds__(1024) void k_scan(int n, const int32_t *cnt, int32_t *off, int64_t *total) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int s0 = t * per, s1 = min(n, s0 + per);
  int64_t acc = 0;
  for (int i = s0; i < s1; ++i) acc += cnt[i];
  part[t] = acc;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int q = 0; q < nt; ++q) { const int64_t v = part[q]; part[q] = run; run += v; }
    *total = run;
  }
  __syncthreads();
  int64_t run = part[t];
  for (int i = s0; i < s1; ++i) { off[i] = (int32_t)run; run += cnt[i]; }
}

__global__ void k_emit_edges(int n, int words, const uint32_t *bm, const int32_t *off,
                             int32_t *ei, int32_t *ej) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int pos = off[i];
  for (int w = 0; w < words; ++w) {
    uint32_t bits = bm[(size_t)i * words + w];
    while (bits) {
      const int b = __ffs(bits) - 1;
      bits &= bits - 1;
      ei[pos] = i;
      ej[pos] = w * 32 + b;
      ++pos;
    }
  }
}

__global__ void k_edge_d2(int E, int p, const double *Xd, const int32_t *ei, const int32_t *ej,
                          double *d2) {
  const int e = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (e >= E) return;
  const int i = ei[e], j = ej[e];
  double acc = 0.0;
  for (int f = lane; f < p; f += kWave) {
    const double d = Xd[(size_t)j * p + f] - Xd[(size_t)i * p + f];
    acc = fma(d, d, acc);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  if (lane == 0) d2[e] = acc;
}

// Lower median of E non-negative doubles by an 8-pass radix select on the
// bit patterns (order-preserving for non-negative doubles).  One block.
__global__ __launch_bounds__(1024) void k_lower_median(int E, const double *v, double *out) {
  __shared__ unsigned int hist[256];
  __shared__ unsigned long long prefix_s;
  __shared__ long long rank_s;
  if (threadIdx.x == 0) { prefix_s = 0ull; rank_s = (E - 1) / 2; }
  __syncthreads();
  for (int pass = 7; pass >= 0; --pass) {
    for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[b] = 0u;
    __syncthreads();
    const unsigned long long prefix = prefix_s;
    const int shift = pass * 8;
    const unsigned long long himask = (pass == 7) ? 0ull : (~0ull << (shift + 8));
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
      const unsigned long long k = (unsigned long long)__double_as_longlong(v[e]);
      if ((k & himask) == (prefix & himask)) atomicAdd(&hist[(k >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      long long r = rank_s;
      int digit = 0;
      for (; digit < 256; ++digit) {
        if (r < (long long)hist[digit]) break;
        r -= hist[digit];
      }
      rank_s = r;
      prefix_s = prefix | ((unsigned long long)digit << shift);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = __longlong_as_double((long long)prefix_s);
}

__global__ void k_weights(int E, const double *d2, const double *phi, double *w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) w[e] = exp(-(*phi) * d2[e]);
}

__global__ __launch_bounds__(1024) void k_normalize(int E, double *w) {
  __shared__ double s[1024];
  double acc = 0.0;
  const int per = (E + blockDim.x - 1) / blockDim.x;
  const int e0 = threadIdx.x * per, e1 = min(E, e0 + per);
  for (int e = e0; e < e1; ++e) acc += w[e];
  s[threadIdx.x] = acc;
  __syncthreads();
  __shared__ double tot;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < (int)blockDim.x; ++q) t += s[q];
    tot = t;
  }
  __syncthreads();
  const double inv = 1.0 / tot;
  for (int e = e0; e < e1; ++e) w[e] *= inv;
}

__global__ void k_phi_from_median(const double *med, double c, double *phi) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *phi = (*med > 0.0) ? c / *med : 0.0;
}

// ------------------------------------------------ connectivity over k
// Directed pairs (i, q-th neighbour of i) of the k_max lists.
__global__ void k_knn_pairs(int n, int kmax, const int32_t *knn, int32_t *ei, int32_t *ej) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)n * kmax) {
    ei[e] = (int32_t)(e / kmax);
    ej[e] = knn[e];
  }
}

// Keep the pairs of the first k neighbours: the union graph of i ~_k j.
__global__ void k_keep_prefix(int64_t m, int kmax, int k, uint8_t *keep) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) keep[e] = (e % kmax) < k ? 1 : 0;
}

// ------------------------------------------------ composite distance
// Mean-imputed X in FP64 (n x p dense): missing entries take their
// observed column mean, as the kNN weights do.
template <typename TI>
__global__ void k_impute_d(int n, int p, const TI *X, int64_t ldx, const uint8_t *M, int64_t ldm,
                           const double *mean, double *Xd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * p) return;
  const int i = (int)(e / p), f = (int)(e - (int64_t)i * p);
  Xd[e] = M[(size_t)i * ldm + f] ? (double)X[(size_t)i * ldx + f] : mean[f];
}

constexpr int kMaxCoords = 8;
struct CoordSpec {
  int q, geodesic;
  double radius, alpha;
  double period[kMaxCoords];
};

// One wave per edge: d = alpha ||x_i - x_j|| + (1 - alpha) dist_y(i, j),
// written as d^2.  dist_y is Euclidean over the coordinates, each
// difference taken modulo its period when that is positive, or with
// geodesic != 0 the great-circle distance of (latitude, longitude) in
// degrees (haversine form) times the radius.
template <typename TI>
__global__ void k_edge_composite(int E, int p, const TI *X, int64_t ldx, const double *Y,
                                 int64_t ldy, CoordSpec c, const int32_t *ei, const int32_t *ej,
                                 double *d2) {
  const int e = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (e >= E) return;
  const int i = ei[e], j = ej[e];
  double acc = 0.0;
  for (int f = lane; f < p; f += kWave) {
    const double d = (double)X[(size_t)j * ldx + f] - (double)X[(size_t)i * ldx + f];
    acc = fma(d, d, acc);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  if (lane != 0) return;
  const double *yi = Y + (size_t)i * ldy, *yj = Y + (size_t)j * ldy;
  double dy = 0.0;
  if (c.geodesic) {
    const double r = 3.14159265358979323846 / 180.0;
    const double la1 = yi[0] * r, la2 = yj[0] * r, dla = la2 - la1, dlo = (yj[1] - yi[1]) * r;
    const double sa = sin(0.5 * dla), so = sin(0.5 * dlo);
    const double h = fmin(fmax(sa * sa + cos(la1) * cos(la2) * so * so, 0.0), 1.0);
    dy = c.radius * 2.0 * atan2(sqrt(h), sqrt(1.0 - h));
  } else {
    double s2 = 0.0;
    for (int t = 0; t < c.q; ++t) {
      double d = fabs(yj[t] - yi[t]);
      if (c.period[t] > 0.0) {
        d = fmod(d, c.period[t]);
        d = fmin(d, c.period[t] - d);
      }
      s2 = fma(d, d, s2);
    }
    dy = sqrt(s2);
  }
  const double d = c.alpha * sqrt(acc) + (1.0 - c.alpha) * dy;
  d2[e] = d * d;
}

// ====================================================================== host
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
  cc_status alloc(size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
      set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
      return CC_ERR_OUT_OF_MEMORY;
    }
    return CC_OK;
  }
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

#define KN_TRY(x)               \
  do {                          \
    cc_status _s = (x);         \
    if (_s != CC_OK) return _s; \
  } while (0)

// Steps 1-4: the mean-imputed X~ in FP64 (Xd, n x p) and the k nearest
// neighbours of every row by (exact d2, index) (knn, n x k).
template <typename TI>
static cc_status knn_lists(int64_t n, int64_t p, const TI *X, int64_t ldx, const uint8_t *mask,
                           int64_t ldm, int32_t k, hipStream_t st, DevBuf &Xd, DevBuf &knn) {
  const int64_t n_pad = cdiv64(n, kGT) * kGT;
  const int64_t ldk = cdiv64(p, kKC) * kKC;
  const int K = (int)std::min<int64_t>(n - 1, (int64_t)k + std::max(16, (int)k));
  int npow2 = 1;
  while (npow2 < n) npow2 <<= 1;

  DevBuf mean, bad, Xf, nrm, D2, cand;
  KN_TRY(mean.alloc(p * 8));
  KN_TRY(bad.alloc(4));
  KN_TRY(Xf.alloc((size_t)n_pad * ldk * 4));
  KN_TRY(Xd.alloc((size_t)n * p * 8));
  KN_TRY(nrm.alloc(n_pad * 4));
  KN_TRY(D2.alloc((size_t)n * n * 4));
  KN_TRY(cand.alloc((size_t)n * K * 4));
  KN_TRY(knn.alloc((size_t)n * k * 4));

  CC_HIP(hipMemsetAsync(bad.p, 0, 4, st));
  hipLaunchKernelGGL((k_col_moments<TI>), dim3((int)cdiv64(p, 256)), dim3(256), 0, st, (int)n,
                     (int)p, X, ldx, mask, ldm, mean.as<double>(), (double *)nullptr, bad.as<int>());
  int hbad = 0;
  CC_HIP(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (hbad) { set_error("observed X has non-finite entries"); return CC_ERR_INVALID_ARG; }
  hipLaunchKernelGGL((k_impute<TI>), dim3((int)cdiv64(n_pad * ldk, 256)), dim3(256), 0, st,
                     (int)n, (int)p, (int)n_pad, (int)ldk, X, ldx, mask, ldm, mean.as<double>(),
                     Xf.as<float>(), Xd.as<double>());
  hipLaunchKernelGGL(k_rownorm, dim3((int)n_pad), dim3(256), 0, st, (int)n_pad, (int)ldk,
                     Xf.as<float>(), nrm.as<float>());
  // split K until the launch has about 4 blocks per CU (at most 8 splits)
  const int gb = (int)(n_pad / kGT);
  const int nch = (int)(ldk / kKC);
  int nsplit = (int)std::min<int64_t>(std::min<int64_t>(cdiv64(1024, (int64_t)gb * gb), 8), nch);
  if (nsplit < 1) nsplit = 1;
  DevBuf part;
  if (nsplit > 1) KN_TRY(part.alloc((size_t)nsplit * n_pad * n_pad * 4));
  hipLaunchKernelGGL(k_gram_d2, dim3(gb, gb, nsplit), dim3(256), 0, st, (int)n, (int)n_pad, (int)ldk,
                     nsplit, Xf.as<float>(), nrm.as<float>(), D2.as<float>(), (int64_t)n,
                     part.as<float>());
  if (nsplit > 1)
    hipLaunchKernelGGL(k_gram_combine, dim3((int)cdiv64(n * n, 256)), dim3(256), 0, st, (int)n,
                       (int)n_pad, nsplit, part.as<float>(), nrm.as<float>(), D2.as<float>(),
                       (int64_t)n);
  CC_HIP(hipGetLastError());
  // rounding bound of the FP32 distances (see k_recheck): (2 m + 24) u with
  // m the longest FP32 accumulation (ldk products and the split combine)
  const double bscale = (2.0 * (double)(ldk + nsplit) + 24.0) * std::ldexp(1.0, -24) * 1.001;
  DevBuf dnext, nmax, uncert, nun;
  KN_TRY(dnext.alloc(n * 4));
  KN_TRY(nmax.alloc(4));
  KN_TRY(uncert.alloc(n * 4));
  KN_TRY(nun.alloc(4));
  hipLaunchKernelGGL(k_max_norm, dim3(1), dim3(1024), 0, st, (int)n, nrm.as<float>(), nmax.as<float>());
  // the dynamic LDS limits are set to the largest sizes these kernels take
  // (the same values on every call, so that concurrent builds agree)
  const size_t lds = (size_t)npow2 * 8;
  CC_HIP(hipFuncSetAttribute((const void *)k_row_candidates,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kKnnMaxN * 8)));
  CC_HIP(hipFuncSetAttribute((const void *)k_recheck, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(kRecheckMaxK * 12)));
  // wider passes for the rows a pass could not certify: 8 K (at least 512)
  // candidates, then all rows up to kRecheckMaxK (every row for n up to
  // kRecheckMaxK + 1, which certifies by construction)
  const int64_t widths[3] = {K, std::min<int64_t>({n - 1, std::max<int64_t>(8 * (int64_t)K, 512), kRecheckMaxK}),
                             std::min<int64_t>(n - 1, kRecheckMaxK)};
  const int *todo = nullptr;
  DevBuf cand2;
  int Kp = K;
  int32_t *cp = cand.as<int32_t>();
  for (int pass = 0; pass < 3; ++pass) {
    if (pass > 0) {
      if (widths[pass] <= Kp) continue;
      Kp = (int)widths[pass];
      if (cand2.p) { (void)hipFree(cand2.p); cand2.p = nullptr; }
      KN_TRY(cand2.alloc((size_t)n * Kp * 4));
      cp = cand2.as<int32_t>();
      todo = uncert.as<int>();
    }
    CC_HIP(hipMemsetAsync(nun.p, 0, 4, st));
    hipLaunchKernelGGL(k_row_candidates, dim3((int)n), dim3(1024), lds, st, (int)n,
                       D2.as<float>(), (int64_t)n, npow2, Kp, cp, todo, dnext.as<float>());
    CC_HIP(hipGetLastError());
    const size_t lds2 = (size_t)Kp * 12;
    hipLaunchKernelGGL(k_recheck, dim3((int)n), dim3(256), lds2, st, (int)n, (int)p,
                       Xd.as<double>(), Kp, (int)k, cp, knn.as<int32_t>(), todo,
                       dnext.as<float>(), nrm.as<float>(), nmax.as<float>(), bscale,
                       uncert.as<int>(), nun.as<int>());
    CC_HIP(hipGetLastError());
    int hn = 0;
    CC_HIP(hipMemcpyAsync(&hn, nun.p, 4, hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    if (hn == 0) return CC_OK;
  }
  set_error("kNN: the nearest neighbours of some rows could not be certified exact "
            "(FP32 distances too close to separate them)");
  return CC_ERR_NUMERIC;
}

// Step 6 over E edges with squared distances d2 (device): phi (literal, or
// |phi| / lower median of d2 when phi < 0), w = exp(-phi d2), optional
// normalisation to sum 1; phi_used (host, may be NULL) gets phi.
static cc_status finish_weights(int64_t E, const double *d2, double phi, int32_t normalize,
                                double *w, double *phi_used, hipStream_t st) {
  DevBuf med, phid;
  KN_TRY(med.alloc(8));
  KN_TRY(phid.alloc(8));
  double hphi = phi;
  if (phi < 0.0 && E > 0) {
    hipLaunchKernelGGL(k_lower_median, dim3(1), dim3(1024), 0, st, (int)E, d2, med.as<double>());
    hipLaunchKernelGGL(k_phi_from_median, dim3(1), dim3(1), 0, st, med.as<double>(), -phi,
                       phid.as<double>());
  } else {
    if (phi < 0.0) hphi = 0.0;
    CC_HIP(hipMemcpyAsync(phid.p, &hphi, 8, hipMemcpyHostToDevice, st));
  }
  if (E > 0) {
    hipLaunchKernelGGL(k_weights, dim3((int)cdiv64(E, 256)), dim3(256), 0, st, (int)E, d2,
                       phid.as<double>(), w);
    if (normalize) hipLaunchKernelGGL(k_normalize, dim3(1), dim3(1024), 0, st, (int)E, w);
  }
  CC_HIP(hipGetLastError());
  CC_HIP(hipMemcpyAsync(&hphi, phid.p, 8, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (phi_used) *phi_used = hphi;
  return CC_OK;
}

template <typename TI>
static cc_status knn_impl(int64_t n, int64_t p, const TI *X, int64_t ldx, const uint8_t *mask,
                          int64_t ldm, int32_t k, double phi, int32_t normalize, int32_t *ei,
                          int32_t *ej, double *w, int64_t capacity, int64_t *n_edges,
                          double *phi_used, hipStream_t st) {
  const int words = (int)cdiv64(n, 32);
  DevBuf Xd, knn, bm, cnt, off, total, d2;
  KN_TRY(knn_lists(n, p, X, ldx, mask, ldm, k, st, Xd, knn));
  KN_TRY(bm.alloc((size_t)n * words * 4));
  KN_TRY(cnt.alloc(n * 4));
  KN_TRY(off.alloc(n * 4));
  KN_TRY(total.alloc(8));
  CC_HIP(hipMemsetAsync(bm.p, 0, (size_t)n * words * 4, st));
  hipLaunchKernelGGL(k_mark_pairs, dim3((int)cdiv64(n * k, 256)), dim3(256), 0, st, (int)n,
                     (int)k, words, knn.as<int32_t>(), bm.as<uint32_t>());
  hipLaunchKernelGGL(k_row_counts, dim3((int)cdiv64(n, 256)), dim3(256), 0, st, (int)n, words,
                     bm.as<uint32_t>(), cnt.as<int32_t>());
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, (int)n, cnt.as<int32_t>(),
                     off.as<int32_t>(), total.as<int64_t>());
  int64_t E = 0;
  CC_HIP(hipMemcpyAsync(&E, total.p, 8, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (E > capacity) {
    set_error("edge capacity " + std::to_string(capacity) + " < " + std::to_string(E));
    *n_edges = E;
    return CC_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_emit_edges, dim3((int)cdiv64(n, 256)), dim3(256), 0, st, (int)n, words,
                     bm.as<uint32_t>(), off.as<int32_t>(), ei, ej);
  KN_TRY(d2.alloc(E * 8));
  if (E > 0) {
    hipLaunchKernelGGL(k_edge_d2, dim3((int)cdiv64(E, 4)), dim3(256), 0, st, (int)E, (int)p,
                       Xd.as<double>(), ei, ej, d2.as<double>());
  }
  *n_edges = E;
  return finish_weights(E, d2.as<double>(), phi, normalize, w, phi_used, st);
}

template <typename TI>
static cc_status min_k_impl(int64_t n, int64_t p, const TI *X, int64_t ldx, const uint8_t *mask,
                            int64_t ldm, int32_t kmax, int32_t *k_min, int32_t *n_comp,
                            hipStream_t st) {
  DevBuf Xd, knn, ei, ej, keep, lab, ncl;
  KN_TRY(knn_lists(n, p, X, ldx, mask, ldm, kmax, st, Xd, knn));
  const int64_t m = n * kmax;
  KN_TRY(ei.alloc(m * 4));
  KN_TRY(ej.alloc(m * 4));
  KN_TRY(keep.alloc(m));
  KN_TRY(lab.alloc(n * 4));
  KN_TRY(ncl.alloc(4));
  hipLaunchKernelGGL(k_knn_pairs, dim3((int)cdiv64(m, 256)), dim3(256), 0, st, (int)n, (int)kmax,
                     knn.as<int32_t>(), ei.as<int32_t>(), ej.as<int32_t>());
  CC_HIP(hipGetLastError());
  // components of the union graph of the first k neighbours
  auto count = [&](int k, int32_t *out) -> cc_status {
    hipLaunchKernelGGL(k_keep_prefix, dim3((int)cdiv64(m, 256)), dim3(256), 0, st, m, (int)kmax, k,
                       keep.as<uint8_t>());
    CC_HIP(hipGetLastError());
    KN_TRY(components(n, m, ei.as<int32_t>(), ej.as<int32_t>(), keep.as<uint8_t>(), nullptr,
                      lab.as<int32_t>(), ncl.as<int32_t>(), st));
    CC_HIP(hipMemcpyAsync(out, ncl.p, 4, hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    return CC_OK;
  };
  int32_t c = 0;
  KN_TRY(count(kmax, &c));
  *n_comp = c;
  if (c != 1) {
    *k_min = -1;
    return CC_OK;
  }
  // the graph for k is a subgraph of the one for k + 1: connectivity is
  // monotone in k, so bisection finds the smallest connected k
  int lo = 1, hi = kmax;
  while (lo < hi) {
    const int mid = lo + (hi - lo) / 2;
    KN_TRY(count(mid, &c));
    if (c == 1) hi = mid;
    else lo = mid + 1;
  }
  *k_min = hi;
  return CC_OK;
}

cc_status min_connected_k(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                          const uint8_t *mask, int64_t ldm, int32_t k_max, int32_t *k_min,
                          int32_t *n_components, hipStream_t stream) {
  if (n < 2 || p < 1) { set_error("need n >= 2 and p >= 1"); return CC_ERR_INVALID_ARG; }
  if (n > kKnnMaxN) { set_error("cc_min_connected_k supports n <= 16384"); return CC_ERR_INVALID_ARG; }
  if ((int64_t)n * p > ((int64_t)1 << 31) - 1) { set_error("n * p too large"); return CC_ERR_INVALID_ARG; }
  if (k_max < 1 || k_max >= n || k_max > 1024) { set_error("need 1 <= k_max < n and k_max <= 1024"); return CC_ERR_INVALID_ARG; }
  if ((int64_t)n * k_max > ((int64_t)1 << 31) - 1) { set_error("n * k_max too large"); return CC_ERR_INVALID_ARG; }
  if (!X || !k_min || !n_components) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  if (x_dtype != CC_DTYPE_F32 && x_dtype != CC_DTYPE_F64) { set_error("bad x_dtype"); return CC_ERR_INVALID_ARG; }
  if (ldx < p || (mask && ldm < p)) { set_error("leading dimension < p"); return CC_ERR_INVALID_ARG; }
  if (x_dtype == CC_DTYPE_F32)
    return min_k_impl<float>(n, p, (const float *)X, ldx, mask, ldm, k_max, k_min, n_components, stream);
  return min_k_impl<double>(n, p, (const double *)X, ldx, mask, ldm, k_max, k_min, n_components, stream);
}

cc_status composite_weights(int64_t n, int64_t n_edges, const int32_t *ei, const int32_t *ej,
                            int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                            const uint8_t *mask, int64_t ldm, int32_t q,
                            const double *Y, int64_t ldy, const double *period, int32_t geodesic,
                            double radius, double alpha, double phi, int32_t normalize, double *w,
                            double *phi_used, hipStream_t st) {
  if (n < 1 || p < 0 || n_edges < 0) { set_error("need n >= 1, p >= 0, n_edges >= 0"); return CC_ERR_INVALID_ARG; }
  if (n_edges > ((int64_t)1 << 31) - 1 || n > ((int64_t)1 << 31) - 1) { set_error("n or n_edges too large"); return CC_ERR_INVALID_ARG; }
  if (n_edges > 0 && (!ei || !ej || !w)) { set_error("NULL edge or weight array"); return CC_ERR_INVALID_ARG; }
  if (p > 0 && (!X || ldx < p)) { set_error("X is NULL or ldx < p"); return CC_ERR_INVALID_ARG; }
  if (mask && p > 0 && ldm < p) { set_error("ldm < p"); return CC_ERR_INVALID_ARG; }
  if (n * p > ((int64_t)1 << 31) - 1) { set_error("n * p too large"); return CC_ERR_INVALID_ARG; }
  if (x_dtype != CC_DTYPE_F32 && x_dtype != CC_DTYPE_F64) { set_error("bad x_dtype"); return CC_ERR_INVALID_ARG; }
  if (q < 0 || q > kMaxCoords) { set_error("need 0 <= q <= 8 coordinates"); return CC_ERR_INVALID_ARG; }
  if (q > 0 && (!Y || ldy < q)) { set_error("Y is NULL or ldy < q"); return CC_ERR_INVALID_ARG; }
  if (geodesic && q != 2) { set_error("geodesic distances need q = 2 (latitude, longitude in degrees)"); return CC_ERR_INVALID_ARG; }
  if (!(alpha >= 0.0 && alpha <= 1.0)) { set_error("need 0 <= alpha <= 1"); return CC_ERR_INVALID_ARG; }
  if (!std::isfinite(phi) || !std::isfinite(radius)) { set_error("phi and radius must be finite"); return CC_ERR_INVALID_ARG; }
  CoordSpec c{};
  c.q = q;
  c.geodesic = geodesic ? 1 : 0;
  c.radius = radius > 0.0 ? radius : 1.0;
  c.alpha = alpha;
  for (int t = 0; t < q; ++t) {
    c.period[t] = period ? period[t] : 0.0;
    if (!std::isfinite(c.period[t]) || c.period[t] < 0.0) { set_error("periods must be finite and >= 0"); return CC_ERR_INVALID_ARG; }
  }
  if (n_edges > 0) {  // every endpoint in range before any launch reads rows
    std::vector<int32_t> hi(n_edges), hj(n_edges);
    CC_HIP(hipMemcpyAsync(hi.data(), ei, n_edges * 4, hipMemcpyDeviceToHost, st));
    CC_HIP(hipMemcpyAsync(hj.data(), ej, n_edges * 4, hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    for (int64_t e = 0; e < n_edges; ++e)
      if (hi[e] < 0 || hi[e] >= n || hj[e] < 0 || hj[e] >= n) {
        set_error("edge endpoint out of range");
        return CC_ERR_INVALID_ARG;
      }
  }
  // with a mask: distances on the mean-imputed matrix (FP64)
  DevBuf mean, bad, Xd;
  const void *Xuse = X;
  int64_t ldu = ldx;
  int32_t tuse = x_dtype;
  if (mask && p > 0 && n_edges > 0) {
    KN_TRY(mean.alloc(p * 8));
    KN_TRY(bad.alloc(4));
    KN_TRY(Xd.alloc((size_t)n * p * 8));
    CC_HIP(hipMemsetAsync(bad.p, 0, 4, st));
    const int cb = (int)cdiv64(p, 256), eb = (int)cdiv64(n * p, 256);
    if (x_dtype == CC_DTYPE_F32) {
      hipLaunchKernelGGL((k_col_moments<float>), dim3(cb), dim3(256), 0, st, (int)n, (int)p, (const float *)X,
                         ldx, mask, ldm, mean.as<double>(), (double *)nullptr, bad.as<int>());
      hipLaunchKernelGGL((k_impute_d<float>), dim3(eb), dim3(256), 0, st, (int)n, (int)p, (const float *)X, ldx,
                         mask, ldm, mean.as<double>(), Xd.as<double>());
    } else {
      hipLaunchKernelGGL((k_col_moments<double>), dim3(cb), dim3(256), 0, st, (int)n, (int)p, (const double *)X,
                         ldx, mask, ldm, mean.as<double>(), (double *)nullptr, bad.as<int>());
      hipLaunchKernelGGL((k_impute_d<double>), dim3(eb), dim3(256), 0, st, (int)n, (int)p, (const double *)X, ldx,
                         mask, ldm, mean.as<double>(), Xd.as<double>());
    }
    CC_HIP(hipGetLastError());
    int hbad = 0;
    CC_HIP(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    if (hbad) { set_error("observed X has non-finite entries"); return CC_ERR_INVALID_ARG; }
    Xuse = Xd.p;
    ldu = p;
    tuse = CC_DTYPE_F64;
  }
  DevBuf d2;
  KN_TRY(d2.alloc(n_edges * 8));
  if (n_edges > 0) {
    const int blocks = (int)cdiv64(n_edges, 4);
    if (tuse == CC_DTYPE_F32)
      hipLaunchKernelGGL((k_edge_composite<float>), dim3(blocks), dim3(256), 0, st, (int)n_edges,
                         (int)p, (const float *)Xuse, ldu, Y, ldy, c, ei, ej, d2.as<double>());
    else
      hipLaunchKernelGGL((k_edge_composite<double>), dim3(blocks), dim3(256), 0, st, (int)n_edges,
                         (int)p, (const double *)Xuse, ldu, Y, ldy, c, ei, ej, d2.as<double>());
    CC_HIP(hipGetLastError());
  }
  return finish_weights(n_edges, d2.as<double>(), phi, normalize, w, phi_used, st);
}

cc_status build_knn_weights(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                            const uint8_t *mask, int64_t ldm, int32_t k, double phi,
                            int32_t normalize, int32_t *ei, int32_t *ej, double *w,
                            int64_t capacity, int64_t *n_edges, double *phi_used,
                            hipStream_t stream) {
  if (n < 2 || p < 1) { set_error("need n >= 2 and p >= 1"); return CC_ERR_INVALID_ARG; }
  if (n > kKnnMaxN) { set_error("cc_build_knn_weights supports n <= 16384"); return CC_ERR_INVALID_ARG; }
  if ((int64_t)n * p > ((int64_t)1 << 31) - 1) { set_error("n * p too large"); return CC_ERR_INVALID_ARG; }
  if (k < 1 || k >= n) { set_error("need 1 <= k < n"); return CC_ERR_INVALID_ARG; }
  if (!X || !ei || !ej || !w || !n_edges) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  if (x_dtype != CC_DTYPE_F32 && x_dtype != CC_DTYPE_F64) { set_error("bad x_dtype"); return CC_ERR_INVALID_ARG; }
  if (ldx < p || (mask && ldm < p)) { set_error("leading dimension < p"); return CC_ERR_INVALID_ARG; }
  if (!std::isfinite(phi)) { set_error("phi must be finite"); return CC_ERR_INVALID_ARG; }
  if (capacity < 0) { set_error("capacity < 0"); return CC_ERR_INVALID_ARG; }
  if (x_dtype == CC_DTYPE_F32)
    return knn_impl<float>(n, p, (const float *)X, ldx, mask, ldm, k, phi, normalize, ei, ej, w,
                           capacity, n_edges, phi_used, stream);
  return knn_impl<double>(n, p, (const double *)X, ldx, mask, ldm, k, phi, normalize, ei, ej, w,
                          capacity, n_edges, phi_used, stream);
}

cc_status standardize_columns(int64_t n, int64_t p, int32_t x_dtype, void *X, int64_t ldx,
                              const uint8_t *mask, int64_t ldm, hipStream_t st) {
  if (n < 1 || p < 1) { set_error("need n, p >= 1"); return CC_ERR_INVALID_ARG; }
  if (!X) { set_error("X is NULL"); return CC_ERR_INVALID_ARG; }
  if (ldx < p || (mask && ldm < p)) { set_error("leading dimension < p"); return CC_ERR_INVALID_ARG; }
  if (x_dtype != CC_DTYPE_F32 && x_dtype != CC_DTYPE_F64) { set_error("bad x_dtype"); return CC_ERR_INVALID_ARG; }
  if ((int64_t)n * p > ((int64_t)1 << 31) - 1) { set_error("n * p too large"); return CC_ERR_INVALID_ARG; }
  DevBuf mean, sd, bad;
  KN_TRY(mean.alloc(p * 8));
  KN_TRY(sd.alloc(p * 8));
  KN_TRY(bad.alloc(4));
  CC_HIP(hipMemsetAsync(bad.p, 0, 4, st));
  const int cb = (int)cdiv64(p, 256), eb = (int)cdiv64(n * p, 256);
  if (x_dtype == CC_DTYPE_F32) {
    hipLaunchKernelGGL((k_col_moments<float>), dim3(cb), dim3(256), 0, st, (int)n, (int)p,
                       (const float *)X, ldx, mask, ldm, mean.as<double>(), sd.as<double>(), bad.as<int>());
  } else {
    hipLaunchKernelGGL((k_col_moments<double>), dim3(cb), dim3(256), 0, st, (int)n, (int)p,
                       (const double *)X, ldx, mask, ldm, mean.as<double>(), sd.as<double>(), bad.as<int>());
  }
  int hbad = 0;
  CC_HIP(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (hbad) { set_error("observed X has non-finite entries"); return CC_ERR_INVALID_ARG; }
  if (x_dtype == CC_DTYPE_F32)
    hipLaunchKernelGGL((k_standardize<float>), dim3(eb), dim3(256), 0, st, (int)n, (int)p,
                       (float *)X, ldx, mask, ldm, mean.as<double>(), sd.as<double>());
  else
    hipLaunchKernelGGL((k_standardize<double>), dim3(eb), dim3(256), 0, st, (int)n, (int)p,
                       (double *)X, ldx, mask, ldm, mean.as<double>(), sd.as<double>());
  CC_HIP(hipGetLastError());
  CC_HIP(hipStreamSynchronize(st));
  return CC_OK;
}

// ------------------------------------------- standardisation without allocation
// cc_standardize_columns_noalloc keeps the column statistics in this fixed
// device array instead of memory allocated per call: the means, then the
// standard deviations (kStdMaxCols doubles each), then the count of
// non-finite observed entries.  Each GPU holds its own copy; host code uses
// the device address hipGetSymbolAddress gives on that GPU, never the
// array's name.
constexpr int64_t kStdMaxCols = 65536;
static __device__ __align__(256) double scratch[2 * kStdMaxCols + 32];

constexpr int kMaxScratchDevices = 256;
static std::mutex g_scratch_mutex;
static void *g_scratch_addr[kMaxScratchDevices];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static cc_status scratch_address(void **out) {
  int dev = 0;
  CC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) {
    set_error("device index beyond the library's scratch table");
    return CC_ERR_STATE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) {
      set_error("hipGetSymbolAddress(scratch) gave no address");
      return CC_ERR_HIP;
    }
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return CC_OK;
}

__global__ void k_zero_count(int *count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0;
}

cc_status standardize_columns_noalloc(int64_t n, int64_t p, int32_t x_dtype, void *X, int64_t ldx,
                                      const uint8_t *mask, int64_t ldm, hipStream_t st) {
  if (n < 1 || p < 1) { set_error("need n, p >= 1"); return CC_ERR_INVALID_ARG; }
  if (!X) { set_error("X is NULL"); return CC_ERR_INVALID_ARG; }
  if (ldx < p || (mask && ldm < p)) { set_error("leading dimension < p"); return CC_ERR_INVALID_ARG; }
  if (x_dtype != CC_DTYPE_F32 && x_dtype != CC_DTYPE_F64) { set_error("bad x_dtype"); return CC_ERR_INVALID_ARG; }
  if ((int64_t)n * p > ((int64_t)1 << 31) - 1) { set_error("n * p too large"); return CC_ERR_INVALID_ARG; }
  if (p > kStdMaxCols) {
    set_error("cc_standardize_columns_noalloc takes p <= " + std::to_string(kStdMaxCols) +
              " (the size of its fixed device scratch)");
    return CC_ERR_INVALID_ARG;
  }
  void *base = nullptr;
  KN_TRY(scratch_address(&base));
  double *mean = reinterpret_cast<double *>(base);
  double *sd = mean + kStdMaxCols;
  int *bad = reinterpret_cast<int *>(sd + kStdMaxCols);
  // the array keeps the last call's contents: the count starts at zero
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, st, bad);
  const int cb = (int)cdiv64(p, 256), eb = (int)cdiv64(n * p, 256);
  if (x_dtype == CC_DTYPE_F32)
    hipLaunchKernelGGL((k_col_moments<float>), dim3(cb), dim3(256), 0, st, (int)n, (int)p,
                       (const float *)X, ldx, mask, ldm, mean, sd, bad);
  else
    hipLaunchKernelGGL((k_col_moments<double>), dim3(cb), dim3(256), 0, st, (int)n, (int)p,
                       (const double *)X, ldx, mask, ldm, mean, sd, bad);
  CC_HIP(hipGetLastError());
  int hbad = 0;
  CC_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (hbad) { set_error("observed X has non-finite entries"); return CC_ERR_INVALID_ARG; }
  if (x_dtype == CC_DTYPE_F32)
    hipLaunchKernelGGL((k_standardize<float>), dim3(eb), dim3(256), 0, st, (int)n, (int)p,
                       (float *)X, ldx, mask, ldm, mean, sd);
  else
    hipLaunchKernelGGL((k_standardize<double>), dim3(eb), dim3(256), 0, st, (int)n, (int)p,
                       (double *)X, ldx, mask, ldm, mean, sd);
  CC_HIP(hipGetLastError());
  CC_HIP(hipStreamSynchronize(st));
  return CC_OK;
}

}  // namespace ccmi
