// Proximal-distance MM solver for convex clustering on gfx950 (CDNA4).
//
// One MM iteration m (Section "The Proximal Distance Algorithm", the block-
// descent projection for sparse weights, and Section "Missing Data") runs as
// two kernels over device-resident state:
//
//   k_point   every block first finishes iteration m-1 from the partial rows
//             the edge stage left: the same fixed-order sums in every block
//             give d, the objective, the stopping test and the advanced
//             scalars (block 0 stores them).  Then for every point i and
//             feature tile: the U update
//             u_i = a'_i + theta (y_i - a'_i) with
//             theta = d/(d+rho) and y = x on observed entries, u elsewhere
//             (the same as (d y + rho a)/(d + rho)); then one Jacobi sweep of
//             the paper's block update
//               a_i = (u_i + sum_R v_ij - sum_L v_ji + sum_N a'_j)/(1+|N_i|)
//             with the factored V = diag(s) D A', written in pull form
//               a_i = a'_i + (u_i - a'_i + sum_j c_ij (a'_j - a'_i))/(1+|N_i|),
//             c_ij = 1 - s_ij.  The shrink factors s_ij of the V update
//             (group soft-threshold) are recomputed on the fly from the edge
//             norms and d of iteration m-1.  Per-block FP64 partial sums feed
//             d, the objective and the stopping test.
//   k_edge_items (rows up to 1024 wide: work items of edges sharing a lower
//             end) or k_edge_slab_items / k_edge_slab / k_edge_tiles and
//             k_edge_reduce (wider rows): per edge ||b_e|| of the new A, the
//             terms of ||V - D A||^2 and of the penalty, and the q factors of
//             the next sweep; each block also gathers a fixed subset of the
//             point sweep's block partials into its partial row.
//
// Storage: the mixed precision keeps A as its FP32 gather copy plus an FP32
// low half; single solves with one projection sweep do not store U during
// the solve where nothing reads it (k_u_finish rebuilds it at the end).
//
// ||V - D A||^2 is assembled as sum_e s_e^2 ||b'_e||^2
//   - 2 sum_i <h_i, a_i> + sum_e ||b_e||^2, with h_i = sum_j s_ij (a'_i - a'_j)
// accumulated by k_point in FP64, so the edge pass gathers one row per edge.
//
// Pair arithmetic is FP64 on values read from the gather copy of A (FP32 in
// the F32 and MIXED precisions); every reduction is FP64, atomic-free and in
// a fixed order, so runs are bitwise repeatable.  Blocks are mapped to feature tiles
// tile-major per XCD so that each XCD's L2 holds the rows of the tiles it
// sweeps.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <type_traits>

#include "ccmi_internal.h"

namespace ccmi {

// ------------------------------------------------------------------ traits
template <int PREC> struct Traits;
// TS: U and the stop-test snapshots; TG: the rows the pair sweeps gather;
// TA: the stored A array.  The mixed precision stores A as hi + lo: hi is
// the FP32 gather copy itself and lo (TA) the FP32 rounding of a - hi, 48
// significant bits in all, so the sweeps move 8 bytes of A per entry.
template <> struct Traits<kF32> {
  using TS = float; using TG = float; using TX = float; using TA = float;
  static constexpr bool mirror = false, hilo = false;
};
template <> struct Traits<kMixed> {
  using TS = double; using TG = float; using TX = float; using TA = float;
  static constexpr bool mirror = true, hilo = true;
};
template <> struct Traits<kF64> {
  using TS = double; using TG = double; using TX = double; using TA = double;
  static constexpr bool mirror = false, hilo = false;
};

// ------------------------------------------------------ vector load/store
// Streaming rows of the point sweep (read or written once per iteration):
// non-temporal accesses, so that they do not push the gathered neighbour
// rows out of L2.  Used by the sweep with several items per wave (wide
// rows, whose data do not stay cached); where the whole working set stays
// in the caches (narrow rows, one item per wave) they measured slower.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
template <typename T, int VEC> struct NtIO {
  __device__ static void store(T *p, const double (&v)[VEC]) {
#pragma unroll
    for (int k = 0; k < VEC; ++k) __builtin_nontemporal_store((T)v[k], p + k);
  }
};
template <> struct NtIO<double, 4> {
  __device__ static void store(double *p, const double (&v)[4]) {
    nt_d2 a = {v[0], v[1]}, b = {v[2], v[3]};
    __builtin_nontemporal_store(a, reinterpret_cast<nt_d2 *>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<nt_d2 *>(p + 2));
  }
  __device__ static void load(const double *p, double (&o)[4]) {
    const nt_d2 a = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p));
    const nt_d2 b = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p + 2));
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
};
template <> struct NtIO<float, 4> {
  __device__ static void store(float *p, const double (&v)[4]) {
    nt_f4 a = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    __builtin_nontemporal_store(a, reinterpret_cast<nt_f4 *>(p));
  }
  __device__ static void load(const float *p, float (&o)[4]) {
    const nt_f4 a = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
  }
};

template <int VEC> struct VecIO;
template <> struct VecIO<4> {
  __device__ static void load(const float *p, double (&o)[4]) {
    float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  __device__ static void load(const double *p, double (&o)[4]) {
    double2 a = *reinterpret_cast<const double2 *>(p);
    double2 b = *reinterpret_cast<const double2 *>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
  __device__ static void store(float *p, const double (&v)[4]) {
    *reinterpret_cast<float4 *>(p) =
        make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  }
  __device__ static void store(double *p, const double (&v)[4]) {
    *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2 *>(p + 2) = make_double2(v[2], v[3]);
  }
  __device__ static void load_mask(const uint8_t *p, bool (&o)[4]) {
    uint32_t v = *reinterpret_cast<const uint32_t *>(p);
    o[0] = (v & 0xffu) != 0; o[1] = (v & 0xff00u) != 0;
    o[2] = (v & 0xff0000u) != 0; o[3] = (v & 0xff000000u) != 0;
  }
};
template <> struct VecIO<2> {
  __device__ static void load(const float *p, double (&o)[2]) {
    float2 v = *reinterpret_cast<const float2 *>(p);
    o[0] = v.x; o[1] = v.y;
  }
  __device__ static void load(const double *p, double (&o)[2]) {
    double2 a = *reinterpret_cast<const double2 *>(p);
    o[0] = a.x; o[1] = a.y;
  }
  __device__ static void store(float *p, const double (&v)[2]) {
    *reinterpret_cast<float2 *>(p) = make_float2((float)v[0], (float)v[1]);
  }
  __device__ static void store(double *p, const double (&v)[2]) {
    *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
  }
  __device__ static void load_mask(const uint8_t *p, bool (&o)[2]) {
    uint16_t v = *reinterpret_cast<const uint16_t *>(p);
    o[0] = (v & 0xffu) != 0; o[1] = (v & 0xff00u) != 0;
  }
};
template <> struct VecIO<1> {
  __device__ static void load(const float *p, double (&o)[1]) { o[0] = *p; }
  __device__ static void load(const double *p, double (&o)[1]) { o[0] = *p; }
  __device__ static void store(float *p, const double (&v)[1]) { *p = (float)v[0]; }
  __device__ static void store(double *p, const double (&v)[1]) { *p = v[0]; }
  __device__ static void load_mask(const uint8_t *p, bool (&o)[1]) { o[0] = *p != 0; }
};

// Raw mask bytes of VEC consecutive entries (byte v in bits 8v..8v+7).
template <int VEC> struct RawMask;
template <> struct RawMask<4> {
  __device__ static uint32_t load(const uint8_t *p) { return *reinterpret_cast<const uint32_t *>(p); }
};
template <> struct RawMask<2> {
  __device__ static uint32_t load(const uint8_t *p) { return *reinterpret_cast<const uint16_t *>(p); }
};
template <> struct RawMask<1> {
  __device__ static uint32_t load(const uint8_t *p) { return *p; }
};

// Raw vector loads (no conversion) for the software-pipelined gathers.
template <typename T, int VEC> struct RawIO;
template <> struct RawIO<float, 4> {
  __device__ static void load(const float *p, float (&o)[4]) {
    float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <> struct RawIO<float, 2> {
  __device__ static void load(const float *p, float (&o)[2]) {
    float2 v = *reinterpret_cast<const float2 *>(p);
    o[0] = v.x; o[1] = v.y;
  }
};
template <> struct RawIO<float, 1> {
  __device__ static void load(const float *p, float (&o)[1]) { o[0] = *p; }
};
template <> struct RawIO<double, 4> {
  __device__ static void load(const double *p, double (&o)[4]) {
    double2 a = *reinterpret_cast<const double2 *>(p);
    double2 b = *reinterpret_cast<const double2 *>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
};
template <> struct RawIO<double, 2> {
  __device__ static void load(const double *p, double (&o)[2]) {
    double2 a = *reinterpret_cast<const double2 *>(p);
    o[0] = a.x; o[1] = a.y;
  }
};
template <> struct RawIO<double, 1> {
  __device__ static void load(const double *p, double (&o)[1]) { o[0] = *p; }
};

template <typename T> __device__ inline double round_to(double v) { return (double)(T)v; }

// A new entry of A as the state stores it: returns the stored value, with g
// the gather copy's value and lo the stored low half (mixed precision; the
// state is exactly g + lo and g is the nearest FP32 value to it).
template <int PREC>
__device__ __forceinline__ double state_round(double a, double &g, double &lo) {
  if constexpr (Traits<PREC>::hilo) {
    g = (double)(float)a;
    lo = (double)(float)(a - g);
    return g + lo;
  } else {
    const double r = round_to<typename Traits<PREC>::TS>(a);
    g = round_to<typename Traits<PREC>::TG>(r);
    lo = 0.0;
    return r;
  }
}
// A stored entry: g the gather copy's value, r the stored TA value.
template <int PREC>
__device__ __forceinline__ double state_value(double g, double r) {
  if constexpr (Traits<PREC>::hilo) return g + r;
  else return r;
}

__device__ inline double readlane_d(double v, int k) {
  long long bits = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), k);
  int hi = __builtin_amdgcn_readlane((int)(bits >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sums over the wave of 8 values per lane, value q's total returned to lane
// q (lanes 8..63 get some total).  Transpose steps halve the values held per
// lane (pairs of lanes 32, 16, 8 apart swap halves), leaving value
// 4 b5 + 2 b4 + b3 (b = lane bits) summed over 8 lanes; the 8-lane groups
// then reduce, and lane q reads the total of value q from lane 8q.  A fixed
// order: every run gives the same bits.
__device__ inline double wave_sum8(double (&v)[8]) {
  const int lane = threadIdx.x % kWave;
  {
    const bool hi = (lane & 32) != 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double send = hi ? v[j] : v[4 + j];
      const double keep = hi ? v[4 + j] : v[j];
      v[j] = keep + __shfl_xor(send, 32, kWave);
    }
  }
  {
    const bool hi = (lane & 16) != 0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double send = hi ? v[j] : v[2 + j];
      const double keep = hi ? v[2 + j] : v[j];
      v[j] = keep + __shfl_xor(send, 16, kWave);
    }
  }
  double t;
  {
    const bool hi = (lane & 8) != 0;
    const double send = hi ? v[0] : v[1];
    const double keep = hi ? v[1] : v[0];
    t = keep + __shfl_xor(send, 8, kWave);
  }
  t += __shfl_xor(t, 4, kWave);
  t += __shfl_xor(t, 2, kWave);
  t += __shfl_xor(t, 1, kWave);
  return __shfl(t, (8 * lane) % kWave, kWave);
}

// Fixed-order block reduction of NV doubles per thread; result valid in
// thread 0.  Uses a shared scratch of (waves per block) * NV doubles.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *scratch) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) scratch[wave * NV + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double acc = 0.0;
      for (int w = 0; w < (int)(blockDim.x / kWave); ++w) acc += scratch[w * NV + q];
      v[q] = acc;
    }
  }
  __syncthreads();
}

// Fixed-order block reduction whose result every thread receives: wave
// trees, then thread q sums value q over the NW waves in order and the
// totals are broadcast through LDS.  scratch: (NW + 1) * NV doubles, not
// reused by the caller before its next barrier.
template <int NV, int NW>
__device__ inline void block_sum_all(double (&v)[NV], double *scratch) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) scratch[wave * NV + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) acc += scratch[w * NV + threadIdx.x];
    scratch[NW * NV + threadIdx.x] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = scratch[NW * NV + q];
}

// Block coordinates within one problem's launch: b = block index, nb =
// blocks of the launch, lb = logical index.  Physical block b runs on XCD
// b % 8 (round-robin dispatch); XCD x is given the x-th contiguous eighth of
// the logical range, so each XCD sweeps a contiguous run of feature tiles.
// A single-problem launch takes them from the hardware indices, a batched
// launch from its block table (same mapping, so the same partial sums).
struct Blk {
  int b, nb, lb;
};
__device__ inline int xcd_remap(int b, int nb) {
  return nb % kXcds == 0 ? (b % kXcds) * (nb / kXcds) + b / kXcds : b;  // small grids: identity
}
__device__ inline Blk hw_blk() {
  const int b = blockIdx.x, nb = gridDim.x;
  return Blk{b, nb, xcd_remap(b, nb)};
}

// ---------------------------------------------------------------- params
struct PointArgs {
  int n, ld, ntile, nitems, chunk;
  const void *X;
  const uint8_t *M;
  void *U;
  void *A0, *A1, *G0, *G1;
  void *Usnap, *Asnap;
  int ell_s;            // ELL stride of the neighbour lists
  const int32_t *degE, *colE, *eidE;
  const double *qE;     // mu w / (rho ||b||) of the previous A, per ELL entry
  const double *s;      // state shrink factors (first iteration of a solve)
  int K;                // stop-test window
  int nblk;             // blocks of this problem's launch
  double *psum;         // this sweep's block partials
  const double *esum;   // partial rows of the previous edge stage
  int nrows;            // how many
  double *trace;
  const DevScalars *sin;  // scalars of the previous iteration
  DevScalars *sout;       // advanced scalars (block 0 writes)
  const BatchInst *bi;    // batched solves only (else null)
  // several projection sweeps per MM iteration (k_point_rhs only)
  double *H;              // h_i = sum_j s_ij (a'_i - a'_j), FP64
  void *T0;               // gather copy of the first sweep's increment A - A'
  // U stored lazily (k_point only): U is written only at missing entries,
  // into Umiss at offsets moff[item] + the entry's rank within its item
  int lazy;
  void *Umiss;
  const int32_t *moff;
};

// Per-edge bookkeeping shared by the fused edge kernel and the reduction
// kernel: norms, shrink factors, and the q factors of the next iteration.
struct EdgeState {
  int E;
  const double *w;
  double *s;            // s_m written here (the state's V factors)
  double *nb0, *nb1;    // ||b|| per edge, double-buffered with A
  double *qe;           // q per edge
  double *qE;           // q per ELL entry (both directions)
  const int32_t *epos;  // ELL positions of (i->j) and (j->i) per edge
};

struct EdgeArgs {
  int n, ld, ntile, nitems, chunk, init, nbp;
  int nblk;             // blocks of this problem's launch
  const void *G0, *G1;
  const int32_t *ei, *ej;
  const int32_t *itemI, *itemJ, *itemE;  // edge work items (item sweep)
  const int32_t *rowptr, *uptr, *col, *eid;  // CSR (wide-row tiles)
  double *part;         // E x ntile partial ||b||^2 (ntile > 1)
  EdgeState es;
  double *esum;         // partial rows (fused kernel)
  const double *psum;   // point-sweep block partials, nbp rows
  const DevScalars *sc; // scalars of the iteration in progress
};

// Batched launches read their argument blocks from global memory, so the
// compiler cannot tell that the pointers in them address global memory and
// would use flat loads, which also count against the LDS wait counter and so
// serialise with the wave shuffles.  Rebuilding each pointer from its bits
// in the global address space restores global loads and stores.
template <typename T>
__device__ inline void to_global(T *&p) {
  using G = __attribute__((address_space(1))) T;
  p = (T *)(G *)(uintptr_t)p;
}

__device__ inline void globalize(PointArgs &a) {
  to_global(a.X); to_global(a.M); to_global(a.U); to_global(a.A0); to_global(a.A1);
  to_global(a.G0); to_global(a.G1); to_global(a.Usnap); to_global(a.Asnap);
  to_global(a.degE); to_global(a.colE); to_global(a.eidE); to_global(a.qE); to_global(a.s);
  to_global(a.psum); to_global(a.esum); to_global(a.trace); to_global(a.sin); to_global(a.sout);
  to_global(a.bi);
}

__device__ inline void globalize(EdgeArgs &a) {
  to_global(a.G0); to_global(a.G1); to_global(a.ei); to_global(a.ej);
  to_global(a.itemI); to_global(a.itemJ); to_global(a.itemE);
  to_global(a.rowptr); to_global(a.uptr); to_global(a.col); to_global(a.eid); to_global(a.part);
  to_global(a.es.w); to_global(a.es.s); to_global(a.es.nb0); to_global(a.es.nb1);
  to_global(a.es.qe); to_global(a.es.qE); to_global(a.es.epos);
  to_global(a.esum); to_global(a.psum); to_global(a.sc);
}

struct ReduceArgs {
  int ntile, nbp, init;
  const double *part;
  EdgeState es;
  double *esum;
  const double *psum;
  const DevScalars *sc;
};

// ------------------------------------------------------- iteration finish
// End of MM iteration h.m from the full sums v (point sums, then edge sums):
// d, the objective, the windowed stop test and the advance of the scalars.
__device__ inline void finish_scalars(DevScalars &h, const double (&v)[kIterSums], double *trace,
                                      bool writer) {
  const double uA2 = v[0], dAw = v[1], dUw = v[2], loss2 = v[3], u2 = v[4], cross = v[5];
  const double Cs = v[6], As = v[7], pen = v[8];
  const double viol = fmax(As - 2.0 * cross + Cs, 0.0);
  const double d = sqrt(uA2 + viol + h.eps);
  const double F = 0.5 * loss2 + h.mu * pen + h.rho * d;
  const int m = h.m;
  if (writer && h.record && trace) trace[m] = F;
  if (!isfinite(d) || !isfinite(F)) {
    h.status = CC_ERR_NUMERIC; h.done = 1; h.iters = m;
    return;
  }
  const int K = h.K;
  if (m >= 1) {
    // iteration m-1 of the MM loop has now finished
    h.F_last = h.F_cur;
    h.d_last = h.d_prev;
    if (m % K == 0) {
      const double r = sqrt(dUw + h.dA_prev) / (double)K;
      const double unorm = fmax(1.0, sqrt(u2));
      h.rel_last = r / unorm;
      if (h.thr > 0.0 && m - 1 >= 2 && r <= h.thr * unorm) {
        h.done = 1; h.converged = 1; h.iters = m;
        return;
      }
    }
    if (m >= h.max_iter) {
      h.done = 1; h.converged = 0; h.iters = m;
      return;
    }
  }
  h.F_cur = F;
  h.d_prev = d;
  if (m % K == K - 1) h.dA_prev = dAw;
  h.pa ^= 1;
  h.m = m + 1;
}

// Batched solves: the gamma in progress has ended (stop rule, iteration cap
// or a numeric error).  Block 0 records its fusion flags and info; every
// block then moves to the next gamma with a warm start (the state stays), as
// a single solve along a path does, or marks the path finished.
__device__ inline void next_gamma(DevScalars &h, const BatchInst &bi, const Blk blk) {
  const int k = h.path_k;
  if (blk.b == 0) {
    for (int e = threadIdx.x; e < bi.E; e += blockDim.x)
      bi.fused[(size_t)k * bi.E + e] = bi.s[e] == 0.0 ? 1 : 0;
    if (threadIdx.x == 0) {
      double *inf = bi.info + (size_t)k * kInfoVals;
      inf[0] = h.iters; inf[1] = h.converged; inf[2] = h.status;
      inf[3] = h.F_last; inf[4] = h.d_last; inf[5] = h.rel_last; inf[6] = h.mu;
      inf[7] = (double)wall_clock64();
    }
  }
  if (k + 1 < bi.n_gamma && h.status == 0) {
    h.mu = bi.mu[k + 1]; h.rho = bi.rho[k + 1]; h.eps = bi.eps[k + 1]; h.thr = bi.thr[k + 1];
    h.m = 0; h.done = 0; h.converged = 0; h.status = 0; h.iters = 0;
    h.d_prev = 0.0; h.dA_prev = 0.0; h.F_cur = 0.0;
    h.F_last = 0.0; h.d_last = 0.0; h.rel_last = 0.0;
    h.path_k = k + 1;
  } else {
    h.finished = 1;
    if (blk.b == 0 && threadIdx.x == 0) {
      *bi.t_done = wall_clock64();
      atomicAdd(bi.n_finished, 1);
    }
  }
}

// Start of a point sweep: when a sweep is pending, sum the edge stage's
// partial rows (column-major, the same order in every block) and finish its
// iteration; block 0 stores the scalars of the iteration about to run (or
// the final ones) in the other slot.  Blocks of NW waves; red:
// (NW + 1) * kIterSums.
// The U update of an MM iteration (Missing Data: y is x on observed entries
// and the previous u elsewhere): one fused multiply-add, so that every
// kernel that forms or rebuilds u rounds it the same way.
__device__ __forceinline__ double mm_u(double ap, double theta, double y) {
  return fma(theta, y - ap, ap);
}

// Rank of each missing entry of a work item in the side array of a lazily
// stored U: entries are numbered by feature slot v, then by lane.  mb[v]
// holds the ballot of lanes whose slot v is missing.
template <int VEC>
__device__ __forceinline__ void miss_ballots(uint32_t mr, bool active, uint64_t (&mb)[VEC]) {
#pragma unroll
  for (int v = 0; v < VEC; ++v) mb[v] = __ballot(active && ((mr >> (8 * v)) & 0xffu) == 0u);
}
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// The edge stage's partial rows that a point sweep's block sums first: at
// most two per thread (blocks of at least 256 threads, at most kEsumRows
// rows), each 5 aligned 16-byte loads.  They are issued before the sweep's
// other loads, so that the finish of the previous iteration waits for them
// alone (loads retire in order); loads are unconditional (row 0 stands in
// for a missing row and is not added) so that the wait counts stay exact.
struct EsumLoad {
  double2 t[2][kEsumStride / 2];
};

template <int NW>
__device__ inline void esum_issue(const PointArgs &a, EsumLoad &L) {
  static_assert(NW * kWave * 2 >= kEsumRows, "at most two partial rows per thread");
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int b = threadIdx.x + r * NW * kWave;
    const double2 *row = reinterpret_cast<const double2 *>(a.esum + (size_t)(b < a.nrows ? b : 0) * kEsumStride);
#pragma unroll
    for (int k = 0; k < kEsumStride / 2; ++k) L.t[r][k] = row[k];
  }
}

template <int NW, bool BATCH = false>
__device__ inline DevScalars begin_iteration(const PointArgs &a, double *red, const Blk blk,
                                             const EsumLoad &L) {
  double v[kIterSums];
#pragma unroll
  for (int q = 0; q < kIterSums; ++q) v[q] = 0.0;
  // unused when nothing is pending
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    if (threadIdx.x + r * NW * kWave < a.nrows) {
#pragma unroll
      for (int k = 0; k < kEsumStride / 2; ++k) {
        v[2 * k] += L.t[r][k].x;
        if (2 * k + 1 < kIterSums) v[2 * k + 1] += L.t[r][k].y;
      }
    }
  }
  DevScalars h = *a.sin;
  const bool writer = blk.b == 0 && threadIdx.x == 0;
  if (h.pending && !h.done) {  // uniform
    block_sum_all<kIterSums, NW>(v, red);
    finish_scalars(h, v, a.trace, writer);
    if constexpr (BATCH) {
      if (h.done) next_gamma(h, *a.bi, blk);
    }
  }
  h.pending = h.done ? 0 : 1;
  if (!h.done) {
    h.m_run = h.m;
    h.pa_run = h.pa;
    h.theta_run = (h.m > 0) ? h.d_prev / (h.d_prev + h.rho) : 0.0;
  }
  if (writer) *a.sout = h;
  return h;
}

// ------------------------------------------------------------- k_point
// JAC: the first of several Jacobi sweeps of the projection.  It stores the
// first sweep's A (the state type), a gather copy of its increment A - A'
// (T0) and h_i (FP64, H); k_jacobi runs the other sweeps and the terms of d
// that involve the final A (||U - A||^2, the A window and sum_i <h_i, a_i>).
template <int PREC, int VEC, bool PF, bool BATCH, bool JAC = false, int NW = kPointWaves>
__device__ __forceinline__ void point_sweep(const PointArgs &a, const Blk blk) {
  using TS = typename Traits<PREC>::TS;
  using TG = typename Traits<PREC>::TG;
  using TX = typename Traits<PREC>::TX;
  using TA = typename Traits<PREC>::TA;
  __shared__ double scratch[NW * kPointSums];
  __shared__ double red[(NW + 1) * kIterSums];
  const TX *X = reinterpret_cast<const TX *>(a.X);
  TS *U = reinterpret_cast<TS *>(a.U);
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lb = blk.lb;
  const int it0 = lb * a.chunk, it1 = min(it0 + a.chunk, a.nitems);
  const int W = kWave * VEC;

  // The first item's loads that do not depend on the scalars (mask, the
  // neighbour slots and their q, the U and X rows) are issued before the
  // previous iteration is finished, so they overlap that reduction.
  // With PF, every item's such loads are issued while the previous item
  // gathers (a wave with several items then waits on one chain per item).
  // Without a mask the U row is read only in the first iteration of a solve
  // (afterwards U_m depends on X and A_{m-1} alone).
  const int first = it0 + wave;
  // Lazily stored U: the sweep reads and writes U only at missing entries
  // (Umiss), except in a solve's first iteration, which reads the U rows
  bool lazy = false;
  if constexpr (!BATCH && !JAC) lazy = a.lazy != 0;
  const bool lzm = lazy && a.M != nullptr;
  TS *Umiss = reinterpret_cast<TS *>(a.Umiss);
  int mo0 = 0;  // the item's first rank in Umiss
  uint32_t mr0 = 0xffffffffu;
  int jl0 = -1;
  double ql0 = 0.0;
  TS up0[VEC];
  TX x0[VEC];
  auto u_row = [&](int item, TS (&u)[VEC]) {
    const int t = item / a.n, i = item - t * a.n;
    const int f0 = t * W + lane * VEC;
    RawIO<TS, VEC>::load(U + (size_t)i * a.ld + (f0 < a.ld ? f0 : 0), u);
  };
  // exact: every load is issued whatever the case (no mask: 4 bytes of the
  // slot list stand in; U not needed: row 0, the same lines for every wave;
  // a lane past the list: slot 0) and the values are selected afterwards.
  // Without branches the compiler counts the loads in flight exactly, so
  // the partial rows issued before the first item's loads are waited for
  // alone.  The prefetches of later items keep their conditions, which
  // skip loads that are not needed.
  auto preload = [&](int item, bool needU, bool exact) {
    const int t = item / a.n, i = item - t * a.n;
    const int f0 = t * W + lane * VEC;
    const int f0c = f0 < a.ld ? f0 : 0;
    const size_t rowc = (size_t)i * a.ld + f0c;
    if (lzm) mo0 = a.moff[item];
    if (exact) {
      const uint8_t *Mp = a.M ? a.M + rowc : reinterpret_cast<const uint8_t *>(a.colE);
      const uint32_t mr = RawMask<VEC>::load(Mp);
      mr0 = a.M ? mr : 0xffffffffu;
      const bool has_slot = lane < a.ell_s;
      const int slot = i * a.ell_s + (has_slot ? lane : 0);
      const int jl = a.colE[slot];
      const double ql = a.qE[slot];  // unused in the first iteration of a solve
      jl0 = has_slot ? jl : -1;
      ql0 = has_slot ? ql : 0.0;
      TS ur[VEC];
      RawIO<TS, VEC>::load(U + (needU ? rowc : (size_t)f0c), ur);
#pragma unroll
      for (int v = 0; v < VEC; ++v) up0[v] = needU ? ur[v] : (TS)0;
    } else {
      mr0 = 0xffffffffu;
      if (a.M) mr0 = RawMask<VEC>::load(a.M + rowc);
      jl0 = -1;
      ql0 = 0.0;
      if (lane < a.ell_s) {
        jl0 = a.colE[i * a.ell_s + lane];
        ql0 = a.qE[i * a.ell_s + lane];
      }
      if (needU) {
        RawIO<TS, VEC>::load(U + rowc, up0);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) up0[v] = (TS)0;
      }
    }
    if constexpr (PF && VEC == 4) NtIO<TX, 4>::load(X + rowc, x0);
    else RawIO<TX, VEC>::load(X + rowc, x0);
  };
  EsumLoad el;
  esum_issue<NW>(a, el);
  // waves without an item preload item 0 and never use it
  preload(first < it1 ? first : 0, a.M != nullptr && !lazy, true);

  const DevScalars hs = begin_iteration<NW, BATCH>(a, red, blk, el);
  if (hs.done) return;
  const int m = hs.m, pa = hs.pa;
  const bool needU = (a.M != nullptr && !lazy) || m == 0;
  if ((!a.M || lazy) && m == 0 && first < it1) u_row(first, up0);
  const double rho = hs.rho, dprev = hs.d_prev;
  const double theta = hs.theta_run;
  // stop-test window: U snapshots at m = 0, K, 2K, ...; A snapshots at
  // m = K-1, 2K-1, ... (the start-of-solve A' seeds the first A window)
  const int K = a.K;
  const bool snapU0 = (m == 0), winU = (m > 0) && (m % K == 0);
  const bool initA = (m == 0) && (K > 1), winA = (m % K) == (K - 1);
  TS *Us = reinterpret_cast<TS *>(a.Usnap);
  TS *As = reinterpret_cast<TS *>(a.Asnap);
  const TA *Ap = reinterpret_cast<const TA *>(pa == 0 ? a.A0 : a.A1);
  TA *An = reinterpret_cast<TA *>(pa == 0 ? a.A1 : a.A0);
  const TG *Gp = reinterpret_cast<const TG *>(pa == 0 ? a.G0 : a.G1);
  TG *Gn = reinterpret_cast<TG *>(pa == 0 ? a.G1 : a.G0);
  double ps[kPointSums] = {0, 0, 0, 0, 0, 0};

  for (int item = first; item < it1; item += NW) {
    const int t = item / a.n, i = item - t * a.n;
    const int f0 = t * W + lane * VEC;
    const bool active = f0 < a.ld;
    // Lanes past the row end load (and ignore) feature 0 of the same rows:
    // the loads are unconditional, so the compiler's wait counts stay exact.
    const int f0c = active ? f0 : 0;
    const size_t row = (size_t)i * a.ld + f0;
    const size_t rowc = (size_t)i * a.ld + f0c;
    const int rs = i * a.ell_s;
    // Mask (if any), neighbour slots (unused slots hold -1 and follow the
    // used ones), then the point's own rows kept raw until the epilogue: the
    // gathers wait only on the slot loads.
    uint32_t mr = mr0;
    int jl = jl0;
    double ql = ql0;
    TS upr[VEC];
    TX xr[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) { upr[v] = up0[v]; xr[v] = x0[v]; }
    if (!PF && item != first) {
      if (a.M) mr = RawMask<VEC>::load(a.M + rowc);
      jl = -1;
      ql = 0.0;
      if (lane < a.ell_s) {
        jl = a.colE[rs + lane];
        if (m > 0) ql = a.qE[rs + lane];
      }
      if (needU) u_row(item, upr);
      RawIO<TX, VEC>::load(X + rowc, xr);
    }
    // missing entries of a lazily stored U: u_{m-1} from the side array
    // (the ballots are formed again for the stores: fewer live registers)
    int mbase = mo0;
    if (lzm) {
      if (!PF && item != first) mbase = a.moff[item];
      if (m > 0) {
        uint64_t mb[VEC];
        miss_ballots<VEC>(mr, active, mb);
        // unconditional loads, so that the wait counts stay exact: observed
        // entries read entry 0 into a u they do not use after the first
        // iteration
        int off = mbase;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const bool miss = (mb[v] >> lane) & 1ull;
          upr[v] = Umiss[miss ? off + lanes_below(mb[v]) : 0];
          off += __popcll(mb[v]);
        }
      }
    }
    TG gr[VEC];
    TA apr[VEC];
    RawIO<TG, VEC>::load(Gp + rowc, gr);
    if constexpr (PF && VEC == 4) NtIO<TA, 4>::load(Ap + rowc, apr);
    else RawIO<TA, VEC>::load(Ap + rowc, apr);
    if (PF && item + NW < it1) preload(item + NW, needU, false);
    double sumg[VEC], sumcg[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) sumg[v] = sumcg[v] = 0.0;
    double C = 0.0;
    // One chunk of up to 64 neighbour slots (jl, ql per lane): count the
    // used slots, form c, gather and accumulate; returns the count.
    auto chunk = [&](int base, int jl, double ql) -> int {
      const int cnt = __popcll(__ballot(jl >= 0));
      double cl = 0.0;
      if (lane < cnt) {
        // c = 1 - s with s the V-update shrink factor; from the state at the
        // first iteration of a solve, else min(d q, 1) = min(tau/||b||, 1)
        cl = (m > 0) ? fmin(dprev * ql, 1.0) : 1.0 - a.s[a.eidE[base + lane]];
      }
      // Gathers in batches of 8 rows, two batches in flight: batch b+1 is
      // issued before batch b is accumulated.  Slots past cnt in the last
      // batch read the point's own row with weight 0 and c = 0 (fma(1, x, s)
      // rounds as s + x, so used slots sum exactly as plain additions).
      auto issue = [&](int k0, TG (&r)[8][VEC], double (&c)[8], double (&wt)[8]) {
        int j[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool ok = k0 + q < cnt;
          j[q] = ok ? __builtin_amdgcn_readlane(jl, k0 + q) : i;
          c[q] = ok ? readlane_d(cl, k0 + q) : 0.0;
          wt[q] = ok ? 1.0 : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) RawIO<TG, VEC>::load(Gp + (size_t)j[q] * a.ld + f0c, r[q]);
      };
      auto consume = [&](const TG (&r)[8][VEC], const double (&c)[8], const double (&wt)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) C += c[q];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const double xv = (double)r[q][v];
            sumg[v] = fma(wt[q], xv, sumg[v]);
            sumcg[v] = fma(c[q], xv, sumcg[v]);
          }
        }
      };
      // Every issue is unconditional (a batch past the end is all weight 0),
      // so the wait before each accumulation counts only the batch it needs.
      const int nbat = (cnt + 7) >> 3;
      TG ra[8][VEC], rb[8][VEC];
      double ca[8], cb[8], wa[8], wb[8];
      if (nbat > 0) {
        issue(0, ra, ca, wa);
        for (int b = 0;; b += 2) {
          issue(8 * (b + 1), rb, cb, wb);
          consume(ra, ca, wa);
          if (b + 1 >= nbat) break;
          issue(8 * (b + 2), ra, ca, wa);
          consume(rb, cb, wb);
          if (b + 2 >= nbat) break;
        }
      }
      return cnt;
    };
    // the first chunk is straight-line code after the loads above, so its
    // gathers wait only on the slot loads
    // a point with more than 64 neighbours (waves with one item): the next
    // 64 slots load now, while the first 64 gather, not after them
    int jn = -1;
    double qn = 0.0;
    if (!PF && __popcll(__ballot(jl >= 0)) == kWave && lane < a.ell_s - kWave) {
      jn = a.colE[rs + kWave + lane];
      if (m > 0) qn = a.qE[rs + kWave + lane];
    }
    int deg = chunk(rs, jl, ql);
    if (deg == kWave) {
      for (int k64 = kWave; k64 < a.ell_s; k64 += kWave) {
        int jk = jn;
        double qk = qn;
        if (PF || k64 > kWave) {
          jk = -1;
          qk = 0.0;
          if (lane < a.ell_s - k64) {
            jk = a.colE[rs + k64 + lane];
            if (m > 0) qk = a.qE[rs + k64 + lane];
          }
        }
        const int cnt = chunk(rs + k64, jk, qk);
        deg += cnt;
        if (cnt < kWave) break;
      }
    }
    if (active) {
      double gi[VEC], ap[VEC], up[VEC], x[VEC];
      bool mk[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        gi[v] = (double)gr[v];
        ap[v] = state_value<PREC>(gi[v], (double)apr[v]);
        up[v] = (double)upr[v]; x[v] = (double)xr[v];
        mk[v] = ((mr >> (8 * v)) & 0xffu) != 0u;
      }
      const double inv1d = 1.0 / (1.0 + (double)deg);
      const double S = (double)deg - C;
      double u[VEC], an[VEC], al[VEC], gn[VEC], rr[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        double uu;
        if (m > 0) {
          const double y = mk[v] ? x[v] : up[v];
          uu = mm_u(ap[v], theta, y);
        } else {
          uu = up[v];
        }
        uu = round_to<TS>(uu);
        const double jac = sumcg[v] - C * gi[v];                 // sum_j c (a'_j - a'_i)
        const double h = S * gi[v] - (sumg[v] - sumcg[v]);       // sum_j s (a'_i - a'_j)
        double g, lo;
        const double anew = state_round<PREC>(ap[v] + (uu - ap[v] + jac) * inv1d, g, lo);
        u[v] = uu; an[v] = anew; al[v] = lo; gn[v] = g;
        if constexpr (JAC) {
          rr[v] = h;
          gn[v] = round_to<TG>(anew - ap[v]);
        } else {
          const double dua = uu - anew;
          ps[0] = fma(dua, dua, ps[0]);
          ps[5] = fma(h, g, ps[5]);
        }
        if (mk[v]) { const double r = x[v] - uu; ps[3] = fma(r, r, ps[3]); }
        ps[4] = fma(uu, uu, ps[4]);
      }
      if constexpr (JAC) {
        VecIO<VEC>::store(U + row, u);
        if constexpr (Traits<PREC>::hilo) {
          // the first sweep's A as hi + lo: hi into the gather copy, which
          // the later sweeps update in place (they gather increments)
          double hi[VEC];
#pragma unroll
          for (int v = 0; v < VEC; ++v) hi[v] = an[v] - al[v];
          VecIO<VEC>::store(An + row, al);
          VecIO<VEC>::store(Gn + row, hi);
        } else {
          VecIO<VEC>::store(An + row, an);
        }
        VecIO<VEC>::store(a.H + row, rr);
        VecIO<VEC>::store(reinterpret_cast<TG *>(a.T0) + row, gn);
      } else if constexpr (PF && VEC == 4) {
        // U and, with an FP32 gather copy, A are streaming rows; where A is
        // itself what the next sweep gathers (no copy) it keeps ordinary
        // stores, so that it stays cached for those gathers
        if (!lazy) NtIO<TS, 4>::store(U + row, u);
        if constexpr (Traits<PREC>::hilo) NtIO<TA, 4>::store(An + row, al);
        else if constexpr (Traits<PREC>::mirror) NtIO<TA, 4>::store(An + row, an);
        else VecIO<VEC>::store(An + row, an);
      } else {
        if (!lazy) VecIO<VEC>::store(U + row, u);
        if constexpr (Traits<PREC>::hilo) VecIO<VEC>::store(An + row, al);
        else VecIO<VEC>::store(An + row, an);
      }
      if (lzm) {
        // inside the active lanes: the ballots see exactly the lanes whose
        // entries can be missing
        uint64_t mb[VEC];
        miss_ballots<VEC>(mr, true, mb);
        int off = mbase;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          if ((mb[v] >> lane) & 1ull) Umiss[off + lanes_below(mb[v])] = (TS)u[v];
          off += __popcll(mb[v]);
        }
      }
      if constexpr (!JAC && Traits<PREC>::mirror) VecIO<VEC>::store(Gn + row, gn);
      if (winU) {
        double us[VEC];
        VecIO<VEC>::load(Us + row, us);
#pragma unroll
        for (int v = 0; v < VEC; ++v) { const double du = u[v] - us[v]; ps[2] = fma(du, du, ps[2]); }
      }
      if (snapU0 || winU) VecIO<VEC>::store(Us + row, u);
      if (initA) VecIO<VEC>::store(As + row, ap);
      if (!JAC && winA) {
        double prev[VEC];
        if (m == 0) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) prev[v] = ap[v];
        } else {
          VecIO<VEC>::load(As + row, prev);
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v) { const double da = an[v] - prev[v]; ps[1] = fma(da, da, ps[1]); }
        VecIO<VEC>::store(As + row, an);
      }
    }
  }
  block_sum<kPointSums>(ps, scratch);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kPointSums; ++q) a.psum[(size_t)lb * 8 + q] = ps[q];
  }
}

// PF: prefetch each next item (for waves with several items).  NW waves
// per block.  The FP32 and mixed sweeps are held to 128 VGPRs (4 waves per
// SIMD); the FP64 one needs more and runs at 2.
template <int PREC, int VEC, bool PF, int NW = kPointWaves>
__global__ __launch_bounds__(kWave * NW) __attribute__((amdgpu_waves_per_eu(PREC == kF64 ? 1 : 4))) void k_point(PointArgs a) {
  point_sweep<PREC, VEC, PF, false, false, NW>(a, hw_blk());
}

// First sweep of several (proj_sweeps > 1): the same launch as k_point.
template <int PREC, int VEC, bool PF>
__global__ __launch_bounds__(kPointBlock) void k_point_rhs(PointArgs a) {
  point_sweep<PREC, VEC, PF, false, true>(a, hw_blk());
}

// End of a solve whose point sweeps stored U lazily: rebuild U as the last
// sweep that ran formed it.  Observed entries (all, without a mask) are
// formed again from that sweep's A' and theta with the same arithmetic;
// missing ones come from the side array.  A wave per (point, tile) item.
template <int PREC, int VEC>
__global__ __launch_bounds__(kPointBlock) void k_u_finish(PointArgs a) {
  using TS = typename Traits<PREC>::TS;
  using TX = typename Traits<PREC>::TX;
  using TA = typename Traits<PREC>::TA;
  using TG = typename Traits<PREC>::TG;
  const DevScalars h = *a.sin;
  if (h.m_run == 0) return;  // a first iteration leaves U as it was
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int W = kWave * VEC;
  const TA *Ap = reinterpret_cast<const TA *>(h.pa_run == 0 ? a.A0 : a.A1);
  const TG *Gp = reinterpret_cast<const TG *>(h.pa_run == 0 ? a.G0 : a.G1);
  const TX *X = reinterpret_cast<const TX *>(a.X);
  TS *U = reinterpret_cast<TS *>(a.U);
  const TS *Umiss = reinterpret_cast<const TS *>(a.Umiss);
  const double theta = h.theta_run;
  for (int item = blockIdx.x * kPointWaves + wave; item < a.nitems; item += gridDim.x * kPointWaves) {
    const int t = item / a.n, i = item - t * a.n;
    const int f0 = t * W + lane * VEC;
    const bool active = f0 < a.ld;
    const size_t rowc = (size_t)i * a.ld + (active ? f0 : 0);
    uint32_t mr = 0xffffffffu;
    if (a.M) mr = RawMask<VEC>::load(a.M + rowc);
    TA apr[VEC];
    TG gr[VEC];
    TX xr[VEC];
    RawIO<TA, VEC>::load(Ap + rowc, apr);
    if constexpr (Traits<PREC>::hilo) RawIO<TG, VEC>::load(Gp + rowc, gr);
    RawIO<TX, VEC>::load(X + rowc, xr);
    uint64_t mb[VEC];
    int off = 0;
    if (a.M) {
      off = a.moff[item];
      miss_ballots<VEC>(mr, active, mb);
    } else {
#pragma unroll
      for (int v = 0; v < VEC; ++v) mb[v] = 0ull;
    }
    double u[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      if ((mb[v] >> lane) & 1ull) u[v] = (double)Umiss[off + lanes_below(mb[v])];
      else {
        const double ap = Traits<PREC>::hilo ? state_value<PREC>((double)gr[v], (double)apr[v]) : (double)apr[v];
        u[v] = round_to<TS>(mm_u(ap, theta, (double)xr[v]));
      }
      off += __popcll(mb[v]);
    }
    if (active) VecIO<VEC>::store(U + (size_t)i * a.ld + f0, u);
  }
}

// Batched: block q works for instance tab[q].x as its local block tab[q].y.
template <int PREC, int VEC, bool PF>
__global__ __launch_bounds__(kPointBlock) void k_point_batch(const PointArgs *__restrict__ args,
                                                              const int2 *__restrict__ tab) {
  const int2 t = tab[blockIdx.x];
  PointArgs a = args[t.x];
  globalize(a);
  point_sweep<PREC, VEC, PF, true>(a, Blk{t.y, a.nblk, xcd_remap(t.y, a.nblk)});
}

// ------------------------------------------------------- k_point_slab
// Narrow problems, where an n x F tile of the gather copy fits in LDS: one
// block per (F-feature tile, 256 points).  The block stages the tile of A'
// for all n points in LDS once; each lane owns one point, walks its
// neighbour list (column-major ELL: entry k of point i at k*n + i, so the
// lanes of a wave read consecutive entries) and gathers neighbour rows from
// LDS instead of L2.  Same arithmetic as k_point.
template <int PREC, int F>
__global__ __launch_bounds__(kBlock) void k_point_slab(PointArgs a) {
  using TS = typename Traits<PREC>::TS;
  using TG = typename Traits<PREC>::TG;
  using TX = typename Traits<PREC>::TX;
  constexpr int C4 = F / 4;
  extern __shared__ __align__(16) unsigned char smem[];
  TG *slab = reinterpret_cast<TG *>(smem);
  __shared__ double scratch[kWavesPerBlock * kPointSums];
  __shared__ double red[(kWavesPerBlock + 1) * kIterSums];
  const Blk blk = hw_blk();
  EsumLoad el;
  esum_issue<kWavesPerBlock>(a, el);
  const DevScalars hs = begin_iteration<kWavesPerBlock>(a, red, blk, el);
  if (hs.done) return;
  const int m = hs.m, pa = hs.pa;
  const double rho = hs.rho, dprev = hs.d_prev;
  const double theta = hs.theta_run;
  const int K = a.K;
  const bool snapU0 = (m == 0), winU = (m > 0) && (m % K == 0);
  const bool initA = (m == 0) && (K > 1), winA = (m % K) == (K - 1);
  TS *Us = reinterpret_cast<TS *>(a.Usnap);
  TS *As = reinterpret_cast<TS *>(a.Asnap);
  using TA = typename Traits<PREC>::TA;
  const TA *Ap = reinterpret_cast<const TA *>(pa == 0 ? a.A0 : a.A1);
  TA *An = reinterpret_cast<TA *>(pa == 0 ? a.A1 : a.A0);
  const TG *Gp = reinterpret_cast<const TG *>(pa == 0 ? a.G0 : a.G1);
  TG *Gn = reinterpret_cast<TG *>(pa == 0 ? a.G1 : a.G0);
  const TX *X = reinterpret_cast<const TX *>(a.X);
  TS *U = reinterpret_cast<TS *>(a.U);

  const int lb = blk.lb;
  const int npg = (a.n + kBlock - 1) / kBlock;
  const int t = lb / npg, g = lb - t * npg;
  double ps[kPointSums] = {0, 0, 0, 0, 0, 0};
  if (t < a.ntile) {
    const int fbase = t * F;
    // stage the tile of A' (gather copy) for every point
    for (int idx = threadIdx.x; idx < a.n * C4; idx += blockDim.x) {
      const int row = idx / C4, c = idx - row * C4;
      const int f = fbase + 4 * c;
      TG v[4] = {(TG)0, (TG)0, (TG)0, (TG)0};
      if (f < a.ld) RawIO<TG, 4>::load(Gp + (size_t)row * a.ld + f, v);
      TG *dst = slab + (size_t)row * F + 4 * c;
      dst[0] = v[0]; dst[1] = v[1]; dst[2] = v[2]; dst[3] = v[3];
    }
    __syncthreads();
    const int i = g * kBlock + threadIdx.x;
    if (i < a.n) {
      const int deg = a.degE[i];
      double sumg[F], sumcg[F];
#pragma unroll
      for (int f = 0; f < F; ++f) sumg[f] = sumcg[f] = 0.0;
      double C = 0.0;
      // neighbours in chunks of 8: the list entries of a chunk are loaded
      // together, then its rows are read from LDS
      for (int k0 = 0; k0 < deg; k0 += 8) {
        int jj[8];
        double cc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          jj[u] = i;
          cc[u] = 0.0;
          if (k0 + u < deg) {
            const size_t slot = (size_t)(k0 + u) * a.n + i;
            jj[u] = a.colE[slot];
            cc[u] = (m > 0) ? fmin(dprev * a.qE[slot], 1.0) : 1.0 - a.s[a.eidE[slot]];
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (k0 + u < deg) {
            C += cc[u];
            const TG *rowj = slab + (size_t)jj[u] * F;
#pragma unroll
            for (int f = 0; f < F; ++f) {
              const double xv = (double)rowj[f];
              sumg[f] += xv;
              sumcg[f] = fma(cc[u], xv, sumcg[f]);
            }
          }
        }
      }
      const double inv1d = 1.0 / (1.0 + (double)deg);
      const double S = (double)deg - C;
#pragma unroll
      for (int c4 = 0; c4 < C4; ++c4) {
        const int f0 = fbase + 4 * c4;
        if (f0 < a.ld) {
          const size_t row = (size_t)i * a.ld + f0;
          double ap[4], up[4], x[4], gi[4];
          bool mk[4] = {true, true, true, true};
          VecIO<4>::load(Ap + row, ap);
          VecIO<4>::load(U + row, up);
          VecIO<4>::load(X + row, x);
          if (a.M) VecIO<4>::load_mask(a.M + row, mk);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            gi[v] = (double)slab[(size_t)i * F + 4 * c4 + v];
            ap[v] = state_value<PREC>(gi[v], ap[v]);
          }
          double u[4], an[4], al[4], gn[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int f = 4 * c4 + v;
            double uu;
            if (m > 0) {
              const double y = mk[v] ? x[v] : up[v];
              uu = mm_u(ap[v], theta, y);
            } else {
              uu = up[v];
            }
            uu = round_to<TS>(uu);
            const double jac = sumcg[f] - C * gi[v];
            const double h = S * gi[v] - (sumg[f] - sumcg[f]);
            double gq, lo;
            const double anew = state_round<PREC>(ap[v] + (uu - ap[v] + jac) * inv1d, gq, lo);
            u[v] = uu; an[v] = anew; al[v] = lo; gn[v] = gq;
            const double dua = uu - anew;
            ps[0] = fma(dua, dua, ps[0]);
            if (mk[v]) { const double r = x[v] - uu; ps[3] = fma(r, r, ps[3]); }
            ps[4] = fma(uu, uu, ps[4]);
            ps[5] = fma(h, gq, ps[5]);
          }
          VecIO<4>::store(U + row, u);
          if constexpr (Traits<PREC>::hilo) VecIO<4>::store(An + row, al);
          else VecIO<4>::store(An + row, an);
          if (Traits<PREC>::mirror) VecIO<4>::store(Gn + row, gn);
          if (winU) {
            double us[4];
            VecIO<4>::load(Us + row, us);
#pragma unroll
            for (int v = 0; v < 4; ++v) { const double du = u[v] - us[v]; ps[2] = fma(du, du, ps[2]); }
          }
          if (snapU0 || winU) VecIO<4>::store(Us + row, u);
          if (initA) VecIO<4>::store(As + row, ap);
          if (winA) {
            double prev[4];
            if (m == 0) {
#pragma unroll
              for (int v = 0; v < 4; ++v) prev[v] = ap[v];
            } else {
              VecIO<4>::load(As + row, prev);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) { const double da = an[v] - prev[v]; ps[1] = fma(da, da, ps[1]); }
            VecIO<4>::store(As + row, an);
          }
        }
      }
    }
  }
  block_sum<kPointSums>(ps, scratch);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kPointSums; ++q) a.psum[(size_t)lb * 8 + q] = ps[q];
  }
}

// ------------------------------------------------------------- k_jacobi
// Projection sweeps 2..K of an MM iteration (proj_sweeps = K > 1).  The
// block update of the projection, with V fixed for the iteration, reads
//   a_i <- (u_i + h_i + sum_{j in N_i} a_j) / (1 + |N_i|),
// h_i = sum_j s_ij (a'_i - a'_j) from the projection A' the current V was
// shrunk from.  Between two sweeps only the neighbour sum changes, so sweep
// k+1 adds to a_i the mean increment of its neighbours,
//   a_i^{k+1} = a_i^k + sum_j delta_j^k / (1 + |N_i|),  delta^k = a^k - a^{k-1},
// which equals the block update exactly; gathering the increments (small
// near the fixed point) instead of the values keeps the rounding of an FP32
// gather copy at the scale of the increment.  k_point_rhs stored the first
// sweep's A, its increment over A' and h.  One wave per (point, feature
// tile) item, on the grid and item split of the point sweep, so that block
// lb of the last sweep completes row lb of the point-sweep partials:
// ||U - A||^2 (entry 0), the A window (entry 1) and sum_i <h_i, a_i>
// (entry 5) of the final A.  Each sweep updates A in place (a point reads
// only its own row of A; neighbours are read through the increments); the
// last one also writes the gather copy of A that the edge stage and the
// next iteration read.
struct JacArgs {
  int n, ld, nitems, chunk, ell_s, K;
  const int32_t *colE;
  const double *H;    // h per point-feature, FP64
  const void *Din;    // gather copy of the previous sweep's increment
  void *Dout;         // intermediate sweeps: this sweep's increment
  const void *U;      // last sweep: U_m
  void *A0, *A1, *G0, *G1, *Asnap;
  double *psum;
  const DevScalars *sc;  // scalars of the iteration in progress
};

template <int PREC, int VEC, bool LAST>
__global__ __launch_bounds__(kPointBlock) void k_jacobi(JacArgs a) {
  using TS = typename Traits<PREC>::TS;
  using TG = typename Traits<PREC>::TG;
  __shared__ double scratch[kPointWaves * 3];
  const DevScalars *sc = a.sc;
  if (sc->done) return;
  const int m = sc->m, pa = sc->pa;
  const bool winA = (m % a.K) == (a.K - 1);
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const Blk blk = hw_blk();
  const int lb = blk.lb;
  const int it0 = lb * a.chunk, it1 = min(it0 + a.chunk, a.nitems);
  const int W = kWave * VEC;
  const TG *Di = reinterpret_cast<const TG *>(a.Din);
  TG *Do = reinterpret_cast<TG *>(a.Dout);
  using TA = typename Traits<PREC>::TA;
  constexpr bool hilo = Traits<PREC>::hilo;
  TG *Gn = reinterpret_cast<TG *>(pa == 0 ? a.G1 : a.G0);
  const TG *Gp = reinterpret_cast<const TG *>(pa == 0 ? a.G0 : a.G1);
  TA *An = reinterpret_cast<TA *>(pa == 0 ? a.A1 : a.A0);
  const TA *Ap = reinterpret_cast<const TA *>(pa == 0 ? a.A0 : a.A1);
  const TS *U = reinterpret_cast<const TS *>(a.U);
  TS *As = reinterpret_cast<TS *>(a.Asnap);
  double ps[3] = {0.0, 0.0, 0.0};
  for (int item = it0 + wave; item < it1; item += kPointWaves) {
    const int t = item / a.n, i = item - t * a.n;
    const int f0 = t * W + lane * VEC;
    const bool active = f0 < a.ld;
    // lanes past the row end load feature 0 of the same rows and drop it
    const int f0c = active ? f0 : 0;
    const size_t row = (size_t)i * a.ld + f0;
    const size_t rowc = (size_t)i * a.ld + f0c;
    const size_t rs = (size_t)i * a.ell_s;
    // the state being swept: A (FP32 and FP64), or its low half with the
    // high half in the gather copy (mixed)
    TA akr[VEC];
    TG akh[VEC];
    RawIO<TA, VEC>::load(An + rowc, akr);
    if constexpr (hilo) RawIO<TG, VEC>::load(Gn + rowc, akh);
    double hr[VEC];
    TS ur[VEC];
    if constexpr (LAST) {
      RawIO<double, VEC>::load(a.H + rowc, hr);
      RawIO<TS, VEC>::load(U + rowc, ur);
    }
    double sum[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) sum[v] = 0.0;
    int deg = 0;
    // neighbour slots in chunks of 64 (unused slots hold -1 after the used
    // ones); rows gathered in batches of 8, the next batch issued before the
    // current one is added; a slot past the count reads row i with weight 0
    for (int k64 = 0; k64 < a.ell_s; k64 += kWave) {
      int jl = -1;
      if (lane < a.ell_s - k64) jl = a.colE[rs + k64 + lane];
      const int cnt = __popcll(__ballot(jl >= 0));
      auto issue = [&](int k0, TG (&r)[8][VEC], double (&wt)[8]) {
        int j[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool ok = k0 + q < cnt;
          j[q] = ok ? __builtin_amdgcn_readlane(jl, k0 + q) : i;
          wt[q] = ok ? 1.0 : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) RawIO<TG, VEC>::load(Di + (size_t)j[q] * a.ld + f0c, r[q]);
      };
      auto consume = [&](const TG (&r)[8][VEC], const double (&wt)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) sum[v] = fma(wt[q], (double)r[q][v], sum[v]);
        }
      };
      const int nbat = (cnt + 7) >> 3;
      TG ra[8][VEC], rb[8][VEC];
      double wa[8], wb[8];
      if (nbat > 0) {
        issue(0, ra, wa);
        for (int b = 0;; b += 2) {
          issue(8 * (b + 1), rb, wb);
          consume(ra, wa);
          if (b + 1 >= nbat) break;
          issue(8 * (b + 2), ra, wa);
          consume(rb, wb);
          if (b + 2 >= nbat) break;
        }
      }
      deg += cnt;
      if (cnt < kWave) break;
    }
    if (active) {
      const double inv1d = 1.0 / (1.0 + (double)deg);
      double an[VEC], al[VEC], ah[VEC], dn[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const double inc = sum[v] * inv1d;
        const double ak = hilo ? state_value<PREC>((double)akh[v], (double)akr[v]) : (double)akr[v];
        an[v] = state_round<PREC>(ak + inc, ah[v], al[v]);
        dn[v] = LAST ? ah[v] : round_to<TG>(inc);
      }
      if constexpr (hilo) {
        VecIO<VEC>::store(An + row, al);
        if constexpr (!LAST) VecIO<VEC>::store(Gn + row, ah);
      } else {
        VecIO<VEC>::store(An + row, an);
      }
      if constexpr (LAST) {
        if (Traits<PREC>::mirror) VecIO<VEC>::store(Gn + row, dn);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const double dua = (double)ur[v] - an[v];
          ps[0] = fma(dua, dua, ps[0]);
          ps[2] = fma(hr[v], dn[v], ps[2]);
        }
        if (winA) {
          double prev[VEC];
          if (m == 0) {
            VecIO<VEC>::load(Ap + row, prev);
            if constexpr (hilo) {
              double gp[VEC];
              VecIO<VEC>::load(Gp + row, gp);
#pragma unroll
              for (int v = 0; v < VEC; ++v) prev[v] = state_value<PREC>(gp[v], prev[v]);
            }
          } else {
            VecIO<VEC>::load(As + row, prev);
          }
#pragma unroll
          for (int v = 0; v < VEC; ++v) { const double da = an[v] - prev[v]; ps[1] = fma(da, da, ps[1]); }
          VecIO<VEC>::store(As + row, an);
        }
      } else {
        VecIO<VEC>::store(Do + row, dn);
      }
    }
  }
  if constexpr (LAST) {
    block_sum<3>(ps, scratch);
    if (threadIdx.x == 0) {
      a.psum[(size_t)lb * 8 + 0] = ps[0];
      a.psum[(size_t)lb * 8 + 1] = ps[1];
      a.psum[(size_t)lb * 8 + 5] = ps[2];
    }
  }
}

// --------------------------------------------------- per-edge bookkeeping
// Per-edge inputs of the bookkeeping.  Both norm buffers are loaded and
// the one of A' is picked where it is used, so nothing waits on the loads
// before the row gathers are issued.
struct EdgeIn {
  double qprev, n0, n1, w, s;
  int p0, p1;  // ELL positions of the two directions
};

__device__ inline EdgeIn edge_prefetch(const EdgeState &es, int e) {
  return EdgeIn{es.qe[e], es.nb0[e], es.nb1[e], es.w[e], es.s[e], es.epos[2 * e], es.epos[2 * e + 1]};
}

// Given ||b_e||^2 of the new A_m: store ||b_e||; in an iteration also take
// s_m (the shrink factor the point sweep used), accumulate the edge terms of
// ||V - D A||^2 and of the penalty, and prepare q_e = mu w_e / (rho ||b_e||)
// for the next point sweep (c = min(d q, 1) there, +inf when b_e = 0).
__device__ inline void edge_update(const EdgeState &es, int e, double nb2, const EdgeIn &in, int init,
                                   int pa, const DevScalars *sc, double (&t3)[kEdgeSums]) {
  double *nbout = init ? (pa == 0 ? es.nb0 : es.nb1) : (pa == 0 ? es.nb1 : es.nb0);
  const double nbn = sqrt(nb2);
  nbout[e] = nbn;
  if (init) return;
  const int m = sc->m;
  const double sv = (m > 0) ? 1.0 - fmin(sc->d_prev * in.qprev, 1.0) : in.s;
  es.s[e] = sv;
  const double np = pa == 0 ? in.n0 : in.n1;
  t3[0] += nb2;
  t3[1] += (sv * np) * (sv * np);
  t3[2] += in.w * sv * np;
  const double q = (nbn > 0.0) ? (sc->mu * in.w) / (sc->rho * nbn) : __builtin_inf();
  es.qe[e] = q;
  es.qE[in.p0] = q;
  es.qE[in.p1] = q;
}

// Partial row of edge-stage block b of nb: the point-sweep partials of rows
// b, b + nb, ... summed in that order (pt, held by
// threads 0..5) and the block's edge sums, stored as one padded row for the
// next point sweep.  The point partials of the first kGatherRows rows are
// loaded at the start of the kernel, one value per thread, and summed at
// the end through LDS.
static_assert(kEsumStride % 2 == 0 && kEsumStride > kIterSums, "partial row layout");
constexpr int kGatherRows = 8;

__device__ inline double point_partial_load(const double *psum, int nbp, const Blk blk) {
  const int k = threadIdx.x / kPointSums, q = threadIdx.x - k * kPointSums;
  const int r = blk.b + k * blk.nb;
  return (k < kGatherRows && r < nbp) ? psum[(size_t)r * 8 + q] : 0.0;
}

// Needs blocks of at least kGatherRows * kPointSums threads; a barrier.
__device__ inline double point_partial_sum(double mine, const double *psum, int nbp, const Blk blk) {
  __shared__ double rows[kGatherRows * kPointSums];
  if (threadIdx.x < kGatherRows * kPointSums) rows[threadIdx.x] = mine;
  __syncthreads();
  double pt = 0.0;
  if (threadIdx.x < kPointSums) {
#pragma unroll
    for (int k = 0; k < kGatherRows; ++k) pt += rows[k * kPointSums + threadIdx.x];
    for (int r = blk.b + kGatherRows * blk.nb; r < nbp; r += blk.nb)
      pt += psum[(size_t)r * 8 + threadIdx.x];
  }
  return pt;
}

__device__ inline void edge_block_partials(double (&t3)[kEdgeSums], double pt, double *esum,
                                           const Blk blk) {
  __shared__ double red[kEdgeWaves * kEdgeSums];
  double *row = esum + (size_t)blk.b * kEsumStride;
  if (threadIdx.x < kPointSums) row[threadIdx.x] = pt;
  block_sum<kEdgeSums>(t3, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kEdgeSums; ++q) row[kPointSums + q] = t3[q];
    row[kIterSums] = 0.0;  // padding
  }
}

// -------------------------------------------------------------- k_edge
// Rows up to 1024 wide: edge-parallel.  A work item is a group of 4
// consecutive edges (one per quarter-wave); each quarter sums (a_i - a_j)^2
// over the row, 4 features per lane per 64-feature pass, reduces over its 16
// lanes, and the quarter leader finishes the edge.
template <int PREC, int NPASS>
__global__ __launch_bounds__(kEdgeBlock) void k_edge_fused(EdgeArgs a) {
  using TG = typename Traits<PREC>::TG;
  const DevScalars *sc = a.sc;
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int q = lane / 16, l16 = lane % 16;
  const Blk blk = hw_blk();
  const int lb = blk.lb;
  const int it0 = lb * a.chunk, it1 = min(it0 + a.chunk, a.nitems);
  // An invalid quarter (past the last edge) works on the last edge and
  // stores nothing; item < nitems guarantees E >= 1.  The first item's edge
  // ends are loaded before the scalars, so both arrive together.
  const int first = it0 + wave;
  int i0 = 0, j0 = 0;
  if (first < it1) {
    const int e = 4 * first + q;
    const int ec = e < a.es.E ? e : a.es.E - 1;
    i0 = a.ei[ec];
    j0 = a.ej[ec];
  }
  if (!a.init && sc->done) return;
  const double pmine = a.init ? 0.0 : point_partial_load(a.psum, a.nbp, blk);
  const int pa = sc->pa;
  // iteration: the new A_m sits in buffer pa^1; init: norms of buffer pa
  const int buf = a.init ? pa : (pa ^ 1);
  const TG *Gc = reinterpret_cast<const TG *>(buf == 0 ? a.G0 : a.G1);
  double t3[kEdgeSums] = {0.0, 0.0, 0.0};
  for (int item = first; item < it1; item += kEdgeWaves) {
    const int e = 4 * item + q;
    const bool valid = e < a.es.E;
    const int ec = valid ? e : a.es.E - 1;
    int i = i0, j = j0;
    if (item != first) {
      i = a.ei[ec];
      j = a.ej[ec];
    }
    // Groups of up to 8 passes (4 for FP64 rows and 1024-wide rows), one
    // group at a time.
    // Loads are unconditional: lanes past the row end read feature 0 and
    // their differences are dropped.  The bookkeeping loads follow the
    // first group's row loads.
    double acc = 0.0;
    EdgeIn in{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0};
    {
      constexpr int PGMAX = (sizeof(TG) == 8 || NPASS > 8) ? 4 : 8;
      constexpr int PG = NPASS < PGMAX ? NPASS : PGMAX;
      const TG *pi = Gc + (size_t)i * a.ld;
      const TG *pj = Gc + (size_t)j * a.ld;
#pragma unroll 1
      for (int pg = 0; pg < NPASS; pg += PG) {
        TG ri[PG][4], rj[PG][4];
#pragma unroll
        for (int ps = 0; ps < PG; ++ps) {
          const int fo = (pg + ps) * 64 + l16 * 4;
          const int fc = fo < a.ld ? fo : 0;
          RawIO<TG, 4>::load(pi + fc, ri[ps]);
          RawIO<TG, 4>::load(pj + fc, rj[ps]);
        }
        if (pg == 0 && !a.init) in = edge_prefetch(a.es, ec);
#pragma unroll
        for (int ps = 0; ps < PG; ++ps) {
          const bool ok = (pg + ps) * 64 + l16 * 4 < a.ld;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double d = ok ? (double)ri[ps][v] - (double)rj[ps][v] : 0.0;
            acc = fma(d, d, acc);
          }
        }
      }
    }
    acc += __shfl_xor(acc, 8, kWave);
    acc += __shfl_xor(acc, 4, kWave);
    acc += __shfl_xor(acc, 2, kWave);
    acc += __shfl_xor(acc, 1, kWave);
    if (valid && l16 == 0) edge_update(a.es, e, acc, in, a.init, pa, sc, t3);
  }
  if (a.init) return;
  edge_block_partials(t3, point_partial_sum(pmine, a.psum, a.nbp, blk), a.esum, blk);
}

// Rows up to 1024 wide: one wave per work item of up to kItemEdges edges
// (i, j_q) sharing the lower end i (lists built on the host).  Row i of the
// new A is loaded once, NV features per lane (the whole row across the
// wave), and the rows j_q in the same passes; each ||a_i - a_j||^2 is a
// wave sum and lane q finishes edge q.  Per edge one row is gathered
// instead of two.
template <int PREC, int NV>
__device__ __forceinline__ void edge_items_sweep(const EdgeArgs &a, const Blk blk) {
  using TG = typename Traits<PREC>::TG;
  constexpr int CH = NV < 4 ? NV : 4;  // features per load
  constexpr int NCH = NV / CH;
  constexpr int MAXCH = sizeof(TG) == 8 ? 1 : 2;
  constexpr int PCH = NCH < MAXCH ? NCH : MAXCH;
  const DevScalars *sc = a.sc;
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lb = blk.lb;
  const int it0 = lb * a.chunk, it1 = min(it0 + a.chunk, a.nitems);
  // the first item's lists are loaded before the scalars: both arrive together
  const int first = it0 + wave;
  int jl0 = -1, el0 = -1, i0 = 0;
  if (first < it1) {
    if (lane < kItemEdges) {
      jl0 = a.itemJ[(size_t)first * kItemEdges + lane];
      el0 = a.itemE[(size_t)first * kItemEdges + lane];
    }
    i0 = a.itemI[first];
  }
  if (!a.init && sc->done) return;
  const double pmine = a.init ? 0.0 : point_partial_load(a.psum, a.nbp, blk);
  const int pa = sc->pa;
  // iteration: the new A_m sits in buffer pa^1; init: norms of buffer pa
  const int buf = a.init ? pa : (pa ^ 1);
  const TG *Gc = reinterpret_cast<const TG *>(buf == 0 ? a.G0 : a.G1);
  double t3[kEdgeSums] = {0.0, 0.0, 0.0};
  for (int item = first; item < it1; item += kEdgeWaves) {
    int jl = jl0, el = el0;
    const int i = __builtin_amdgcn_readfirstlane(i0);
    // the next item's lists load while this one gathers
    const int nxt = item + kEdgeWaves;
    if (nxt < it1) {
      jl0 = -1;
      el0 = -1;
      if (lane < kItemEdges) {
        jl0 = a.itemJ[(size_t)nxt * kItemEdges + lane];
        el0 = a.itemE[(size_t)nxt * kItemEdges + lane];
      }
      i0 = a.itemI[nxt];
    }
    // Loads are unconditional: a chunk past the row end reads feature 0 and
    // is dropped, an unused slot reads row i and is not stored.  Chunks go in
    // passes of PCH (8 FP32 or 4 FP64 features per lane in flight).
    int jq[kItemEdges];
#pragma unroll
    for (int q = 0; q < kItemEdges; ++q) {
      const int j = __builtin_amdgcn_readlane(jl, q);
      jq[q] = j >= 0 ? j : i;
    }
    static_assert(kItemEdges == 8, "wave_sum8 reduces 8 values");
    double acc[kItemEdges];
#pragma unroll
    for (int q = 0; q < kItemEdges; ++q) acc[q] = 0.0;
    EdgeIn in{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0};
#pragma unroll 1
    for (int c0 = 0; c0 < NCH; c0 += PCH) {
      TG gi[PCH][CH], rj[kItemEdges][PCH][CH];
#pragma unroll
      for (int c = 0; c < PCH; ++c) {
        const int fo = lane * NV + (c0 + c) * CH;
        RawIO<TG, CH>::load(Gc + (size_t)i * a.ld + (fo < a.ld ? fo : 0), gi[c]);
      }
#pragma unroll
      for (int q = 0; q < kItemEdges; ++q) {
        const size_t rowq = (size_t)jq[q] * a.ld;
#pragma unroll
        for (int c = 0; c < PCH; ++c) {
          const int fo = lane * NV + (c0 + c) * CH;
          RawIO<TG, CH>::load(Gc + rowq + (fo < a.ld ? fo : 0), rj[q][c]);
        }
      }
      if (c0 == 0 && !a.init && el >= 0) in = edge_prefetch(a.es, el);
#pragma unroll
      for (int q = 0; q < kItemEdges; ++q) {
#pragma unroll
        for (int c = 0; c < PCH; ++c) {
          const bool ok = lane * NV + (c0 + c) * CH < a.ld;
#pragma unroll
          for (int v = 0; v < CH; ++v) {
            const double d = ok ? (double)gi[c][v] - (double)rj[q][c][v] : 0.0;
            acc[q] = fma(d, d, acc[q]);
          }
        }
      }
    }
    const double mine = wave_sum8(acc);
    if (el >= 0) edge_update(a.es, el, mine, in, a.init, pa, sc, t3);
  }
  if (a.init) return;
  edge_block_partials(t3, point_partial_sum(pmine, a.psum, a.nbp, blk), a.esum, blk);
}

template <int PREC, int NV>
__global__ __launch_bounds__(kEdgeBlock) void k_edge_items(EdgeArgs a) {
  edge_items_sweep<PREC, NV>(a, hw_blk());
}

// Batched: block q works for instance tab[q].x as its local block tab[q].y.
template <int PREC, int NV>
__global__ __launch_bounds__(kEdgeBlock) void k_edge_items_batch(const EdgeArgs *__restrict__ args,
                                                                  const int2 *__restrict__ tab) {
  const int2 t = tab[blockIdx.x];
  EdgeArgs a = args[t.x];
  globalize(a);
  edge_items_sweep<PREC, NV>(a, Blk{t.y, a.nblk, xcd_remap(t.y, a.nblk)});
}

// Wide rows: one wave per (point i, 256-feature tile); each quarter-wave
// takes one upper neighbour j > i (so a_i is read once per point and tile)
// and writes the tile's partial (a_i - a_j)^2 for k_edge_reduce.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_edge_tiles(EdgeArgs a) {
  using TG = typename Traits<PREC>::TG;
  constexpr int NPASS = 4;
  const DevScalars *sc = a.sc;
  if (!a.init && sc->done) return;
  const int pa = sc->pa;
  const int buf = a.init ? pa : (pa ^ 1);
  const TG *Gc = reinterpret_cast<const TG *>(buf == 0 ? a.G0 : a.G1);
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int q = lane / 16, l16 = lane % 16;
  const Blk blk = hw_blk();
  const int lb = blk.lb;
  const int it0 = lb * a.chunk, it1 = min(it0 + a.chunk, a.nitems);
  const int W = 64 * NPASS;
  for (int item = it0 + wave; item < it1; item += kWavesPerBlock) {
    const int t = item / a.n, i = item - t * a.n;
    double gi[NPASS][4];
#pragma unroll
    for (int ps = 0; ps < NPASS; ++ps) {
      const int fo = t * W + ps * 64 + l16 * 4;
      if (fo < a.ld) VecIO<4>::load(Gc + (size_t)i * a.ld + fo, gi[ps]);
      else { gi[ps][0] = gi[ps][1] = gi[ps][2] = gi[ps][3] = 0.0; }
    }
    const int us = a.uptr[i], re = a.rowptr[i + 1];
    for (int k = us; k < re; k += 4) {
      const int kk = k + q;
      const bool valid = kk < re;
      int j = i, e = 0;
      if (valid) { j = a.col[kk]; e = a.eid[kk]; }
      double acc = 0.0;
      if (valid) {
        TG rj[NPASS][4];
#pragma unroll
        for (int ps = 0; ps < NPASS; ++ps) {
          const int fo = t * W + ps * 64 + l16 * 4;
          if (fo < a.ld) RawIO<TG, 4>::load(Gc + (size_t)j * a.ld + fo, rj[ps]);
          else {
#pragma unroll
            for (int v = 0; v < 4; ++v) rj[ps][v] = (TG)0;
          }
        }
#pragma unroll
        for (int ps = 0; ps < NPASS; ++ps) {
#pragma unroll
          for (int v = 0; v < 4; ++v) { const double d = gi[ps][v] - (double)rj[ps][v]; acc = fma(d, d, acc); }
        }
      }
      acc += __shfl_xor(acc, 8, kWave);
      acc += __shfl_xor(acc, 4, kWave);
      acc += __shfl_xor(acc, 2, kWave);
      acc += __shfl_xor(acc, 1, kWave);
      if (valid && l16 == 0) a.part[(size_t)e * a.ntile + t] = acc;
    }
  }
}

// Wide rows with small n: one 1024-thread block per group of consecutive
// F-feature tiles.  For each tile the block stages the new A (gather copy)
// of all n points in LDS; each thread keeps FP64 accumulators of
// (a_i - a_j)^2 for up to kEdgesPerThread edges across the group's tiles and
// writes one partial per (edge, group) for k_edge_reduce.
constexpr int kEdgesPerThread = 16;
constexpr int kSlabChunks = 4;  // staged four-feature chunks per thread and tile
// LDS row stride of the slab edge sweeps: F + 4 elements.  The sweeps read
// rows at random; a stride of 16 floats would start every row in one of two
// bank groups, the padded stride spreads rows over all of them and keeps the
// 16-byte alignment of four-element reads.
constexpr int kSlabPad = 4;

template <int PREC, int F>
__global__ __launch_bounds__(1024) void k_edge_slab(EdgeArgs a, int tiles_per_group, int ntiles_f) {
  using TG = typename Traits<PREC>::TG;
  constexpr int C4 = F / 4;
  constexpr int RS = F + kSlabPad;
  extern __shared__ __align__(16) unsigned char smem[];
  TG *slab = reinterpret_cast<TG *>(smem);
  const DevScalars *sc = a.sc;
  if (!a.init && sc->done) return;
  const int pa = sc->pa;
  const int buf = a.init ? pa : (pa ^ 1);
  const TG *Gc = reinterpret_cast<const TG *>(buf == 0 ? a.G0 : a.G1);
  const int g = hw_blk().lb;
  const int t0 = g * tiles_per_group, t1 = min(t0 + tiles_per_group, ntiles_f);
  const int E = a.es.E;
  // both ends of an edge in one word (the slab holds n < 2^16 rows)
  uint32_t eij[kEdgesPerThread];
  double acc[kEdgesPerThread];
#pragma unroll
  for (int u = 0; u < kEdgesPerThread; ++u) {
    const int e = threadIdx.x + u * blockDim.x;
    eij[u] = 0u; acc[u] = 0.0;
    if (e < E) eij[u] = ((uint32_t)a.ei[e] << 16) | (uint32_t)a.ej[e];
  }
  // A tile holds n * F / 4 four-feature chunks, at most kSlabChunks per
  // thread (the host sizes F so that the tile takes at most half the LDS
  // budget).  A thread issues all its chunk loads before it stores any, so
  // the staging waits on one HBM latency per tile.  (Carrying the next
  // tile's chunks through the summation instead spills registers.)
  const int nch = a.n * C4;
  TG nv[kSlabChunks][4];
  auto fetch = [&](int t) {
#pragma unroll
    for (int q = 0; q < kSlabChunks; ++q) {
      const int idx = threadIdx.x + q * 1024;
      const int row = idx / C4, c = idx - row * C4;
      const int f = t * F + 4 * c;
      nv[q][0] = nv[q][1] = nv[q][2] = nv[q][3] = (TG)0;
      if (idx < nch && f < a.ld) RawIO<TG, 4>::load(Gc + (size_t)row * a.ld + f, nv[q]);
    }
  };
  for (int t = t0; t < t1; ++t) {
    fetch(t);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSlabChunks; ++q) {
      const int idx = threadIdx.x + q * 1024;
      if (idx < nch) {
        const int row = idx / C4, c = idx - row * C4;
        TG *dst = slab + (size_t)row * RS + 4 * c;
        dst[0] = nv[q][0]; dst[1] = nv[q][1]; dst[2] = nv[q][2]; dst[3] = nv[q][3];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kEdgesPerThread; ++u) {
      const int e = threadIdx.x + u * blockDim.x;
      if (e < E) {
        const TG *ri = slab + (size_t)(eij[u] >> 16) * RS;
        const TG *rj = slab + (size_t)(eij[u] & 0xffffu) * RS;
#pragma unroll
        for (int f = 0; f < F; ++f) {
          const double d = (double)ri[f] - (double)rj[f];
          acc[u] = fma(d, d, acc[u]);
        }
      }
    }
  }
  if (g * tiles_per_group >= ntiles_f) {
    // a padding block (grid rounded up to the XCD count) owns no tiles
#pragma unroll
    for (int u = 0; u < kEdgesPerThread; ++u) acc[u] = 0.0;
  }
#pragma unroll
  for (int u = 0; u < kEdgesPerThread; ++u) {
    const int e = threadIdx.x + u * blockDim.x;
    if (e < E) a.part[(size_t)e * a.ntile + g] = acc[u];
  }
}

// Wide rows with small n, edges grouped into work items (edges sharing their
// lower end i, as for the item edge sweep): as k_edge_slab, but each thread
// takes up to kSlabItemSlots items, reads and converts the tile of row i from
// LDS once per item and then only the rows j of its edges: per edge-feature
// one LDS read and three operations instead of two and four.  Each edge's
// partial is the same sum in the same order as in k_edge_slab.
constexpr int kSlabItemSlots = 3;

template <int PREC, int F>
__global__ __launch_bounds__(1024) void k_edge_slab_items(EdgeArgs a, int tiles_per_group, int ntiles_f) {
  using TG = typename Traits<PREC>::TG;
  constexpr int C4 = F / 4;
  constexpr int RS = F + kSlabPad;
  extern __shared__ __align__(16) unsigned char smem[];
  TG *slab = reinterpret_cast<TG *>(smem);
  const DevScalars *sc = a.sc;
  if (!a.init && sc->done) return;
  const int pa = sc->pa;
  const int buf = a.init ? pa : (pa ^ 1);
  const TG *Gc = reinterpret_cast<const TG *>(buf == 0 ? a.G0 : a.G1);
  const int g = hw_blk().lb;
  const int t0 = g * tiles_per_group, t1 = min(t0 + tiles_per_group, ntiles_f);
  // the items of this thread: lower end (-1: none) and the upper ends in
  // 16-bit halves (0xffff: unused slot; the slab holds n < 2^16 rows)
  int ii[kSlabItemSlots];
  uint32_t jj[kSlabItemSlots][kItemEdges / 2];
  double acc[kSlabItemSlots][kItemEdges];
#pragma unroll
  for (int u = 0; u < kSlabItemSlots; ++u) {
    const int it = threadIdx.x + u * 1024;
    ii[u] = -1;
#pragma unroll
    for (int h = 0; h < kItemEdges / 2; ++h) jj[u][h] = 0xffffffffu;
#pragma unroll
    for (int q = 0; q < kItemEdges; ++q) acc[u][q] = 0.0;
    if (it < a.nitems) {
      ii[u] = a.itemI[it];
#pragma unroll
      for (int h = 0; h < kItemEdges / 2; ++h) {
        const int j0 = a.itemJ[(size_t)it * kItemEdges + 2 * h];
        const int j1 = a.itemJ[(size_t)it * kItemEdges + 2 * h + 1];
        jj[u][h] = (j0 >= 0 ? (uint32_t)j0 : 0xffffu) | ((j1 >= 0 ? (uint32_t)j1 : 0xffffu) << 16);
      }
    }
  }
  const int nch = a.n * C4;
  TG nv[kSlabChunks][4];
  auto fetch = [&](int t) {
#pragma unroll
    for (int q = 0; q < kSlabChunks; ++q) {
      const int idx = threadIdx.x + q * 1024;
      const int row = idx / C4, c = idx - row * C4;
      const int f = t * F + 4 * c;
      nv[q][0] = nv[q][1] = nv[q][2] = nv[q][3] = (TG)0;
      if (idx < nch && f < a.ld) RawIO<TG, 4>::load(Gc + (size_t)row * a.ld + f, nv[q]);
    }
  };
  for (int t = t0; t < t1; ++t) {
    fetch(t);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSlabChunks; ++q) {
      const int idx = threadIdx.x + q * 1024;
      if (idx < nch) {
        const int row = idx / C4, c = idx - row * C4;
        TG *dst = slab + (size_t)row * RS + 4 * c;
        dst[0] = nv[q][0]; dst[1] = nv[q][1]; dst[2] = nv[q][2]; dst[3] = nv[q][3];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kSlabItemSlots; ++u) {
      if (ii[u] >= 0) {
        const TG *ri = slab + (size_t)ii[u] * RS;
        // four features of row i at a time; each edge still adds its
        // features in ascending order
#pragma unroll
        for (int f0 = 0; f0 < F; f0 += 4) {
          const double x0 = (double)ri[f0], x1 = (double)ri[f0 + 1];
          const double x2 = (double)ri[f0 + 2], x3 = (double)ri[f0 + 3];
#pragma unroll
          for (int q = 0; q < kItemEdges; ++q) {
            const uint32_t j = (jj[u][q / 2] >> (16 * (q % 2))) & 0xffffu;
            if (j != 0xffffu) {
              const TG *rj = slab + (size_t)j * RS + f0;
              double d = x0 - (double)rj[0];
              acc[u][q] = fma(d, d, acc[u][q]);
              d = x1 - (double)rj[1];
              acc[u][q] = fma(d, d, acc[u][q]);
              d = x2 - (double)rj[2];
              acc[u][q] = fma(d, d, acc[u][q]);
              d = x3 - (double)rj[3];
              acc[u][q] = fma(d, d, acc[u][q]);
            }
          }
        }
      }
    }
  }
  const bool pad = g * tiles_per_group >= ntiles_f;  // a padding block owns no tiles
#pragma unroll
  for (int u = 0; u < kSlabItemSlots; ++u) {
    const int it = threadIdx.x + u * 1024;
    if (it < a.nitems) {
#pragma unroll
      for (int q = 0; q < kItemEdges; ++q) {
        const int e = a.itemE[(size_t)it * kItemEdges + q];
        if (e >= 0) a.part[(size_t)e * a.ntile + g] = pad ? 0.0 : acc[u][q];
      }
    }
  }
}

// ------------------------------------------------------- k_edge_reduce
// Wide rows: one wave per edge sums the edge's tile partials (contiguous,
// lane-strided, then the wave tree: a fixed order), then the same per-edge
// bookkeeping as the fused edge kernel.
__global__ __launch_bounds__(kEdgeBlock) void k_edge_reduce(ReduceArgs a) {
  const DevScalars *sc = a.sc;
  if (!a.init && sc->done) return;
  const Blk blk = hw_blk();
  const double pmine = a.init ? 0.0 : point_partial_load(a.psum, a.nbp, blk);
  const int pa = sc->pa;
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  double t3[kEdgeSums] = {0.0, 0.0, 0.0};
  for (int e = blockIdx.x * kEdgeWaves + wave; e < a.es.E; e += gridDim.x * kEdgeWaves) {
    EdgeIn in{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0};
    if (!a.init && lane == 0) in = edge_prefetch(a.es, e);
    const double *pe = a.part + (size_t)e * a.ntile;
    double nb2 = 0.0;
    // unrolled so that a lane's loads are in flight together; the sum keeps
    // its order
#pragma unroll 4
    for (int t = lane; t < a.ntile; t += kWave) nb2 += pe[t];
    nb2 = wave_sum(nb2);
    if (lane == 0) edge_update(a.es, e, nb2, in, a.init, pa, sc, t3);
  }
  if (a.init) return;
  edge_block_partials(t3, point_partial_sum(pmine, a.psum, a.nbp, blk), a.esum, blk);
}

// --------------------------------------------------------- small kernels
__global__ void k_set_params(DevScalars *sc, double mu, double rho, double eps,
                             double thr, int max_iter, int record, int K) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  sc->mu = mu; sc->rho = rho; sc->eps = eps; sc->thr = thr;
  sc->max_iter = max_iter; sc->record = record; sc->K = K;
  sc->m = 0; sc->done = 0; sc->converged = 0; sc->status = 0; sc->iters = 0;
  sc->d_prev = 0.0; sc->dA_prev = 0.0; sc->F_cur = 0.0;
  sc->F_last = 0.0; sc->d_last = 0.0; sc->rel_last = 0.0;
  sc->pending = 0; sc->path_k = 0; sc->finished = 0;
}

__global__ void k_reset_scalars(DevScalars *sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  memset(sc, 0, sizeof(DevScalars));
}

// Column statistics over observed entries: mean, ||x - mean||^2, and a count
// of non-finite observed entries.  One thread per column.
template <typename TI>
__global__ void k_colstats(int n, int p, const TI *X, int64_t ldx,
                           const uint8_t *M, int64_t ldm, double *mean,
                           double *dev2, int *nonfinite) {
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
  dev2[f] = ss;
  if (bad) atomicAdd(nonfinite, bad);
}

// Initial state: X-tilde (missing -> observed column mean), U = A = X-tilde,
// padding columns p..ld-1 zero and observed.
template <int PREC, typename TI>
__global__ void k_init_state(int n, int p, int ld, const TI *Xin, int64_t ldx,
                             const uint8_t *Min, int64_t ldm, const double *mean,
                             void *Xo, uint8_t *Mo, void *Uo, void *A0, void *G0) {
  using TS = typename Traits<PREC>::TS;
  using TG = typename Traits<PREC>::TG;
  using TX = typename Traits<PREC>::TX;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * ld) return;
  const int i = (int)(idx / ld), f = (int)(idx % ld);
  double x = 0.0, xt = 0.0;
  bool obs = true;
  if (f < p) {
    obs = Min ? (Min[(size_t)i * ldm + f] != 0) : true;
    x = obs ? (double)Xin[(size_t)i * ldx + f] : mean[f];
    xt = obs ? (double)(TX)x : mean[f];
  }
  reinterpret_cast<TX *>(Xo)[idx] = (TX)(obs ? x : xt);
  if (Mo) Mo[idx] = obs ? 1 : 0;
  reinterpret_cast<TS *>(Uo)[idx] = (TS)xt;
  double g, lo;
  const double a = state_round<PREC>(xt, g, lo);
  reinterpret_cast<typename Traits<PREC>::TA *>(A0)[idx] = (typename Traits<PREC>::TA)(Traits<PREC>::hilo ? lo : a);
  if (Traits<PREC>::mirror) reinterpret_cast<TG *>(G0)[idx] = (TG)g;
}

__global__ void k_fill(double *v, int64_t n, double val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = val;
}

template <typename TS, typename TO>
__global__ void k_copy_rows(int n, int p, const TS *src, int ld, TO *dst, int64_t ldo) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * p) return;
  const int i = (int)(idx / p), f = (int)(idx % p);
  dst[(size_t)i * ldo + f] = (TO)src[(size_t)i * ld + f];
}

template <int PREC>
__global__ void k_set_rows(int n, int p, int ld, const double *U, const double *A,
                           int64_t lds, void *Uo, void *Ao, void *Go) {
  using TS = typename Traits<PREC>::TS;
  using TG = typename Traits<PREC>::TG;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * ld) return;
  const int i = (int)(idx / ld), f = (int)(idx % ld);
  double u = 0.0, a = 0.0;
  if (f < p) { u = U[(size_t)i * lds + f]; a = A[(size_t)i * lds + f]; }
  reinterpret_cast<TS *>(Uo)[idx] = (TS)u;
  double g, lo;
  const double as = state_round<PREC>(a, g, lo);
  reinterpret_cast<typename Traits<PREC>::TA *>(Ao)[idx] = (typename Traits<PREC>::TA)(Traits<PREC>::hilo ? lo : as);
  if (Traits<PREC>::mirror) reinterpret_cast<TG *>(Go)[idx] = (TG)g;
}

// A of the mixed precision as FP64: the gather copy plus the low half.
__global__ void k_get_hilo(int n, int p, const float *G, const float *L, int ld, double *dst, int64_t ldo) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * p) return;
  const int i = (int)(idx / p), f = (int)(idx % p);
  const size_t k = (size_t)i * ld + f;
  dst[(size_t)i * ldo + f] = (double)G[k] + (double)L[k];
}

__global__ void k_fused_flags(int E, const double *s, uint8_t *out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) out[e] = (s[e] == 0.0) ? 1 : 0;
}

// Connected components of the kept edges (keep[e] != 0, or s[e] == 0 when
// keep is null), labelled by the smallest vertex index: min-label hooking
// with pointer jumping, one workgroup, at most n + 2 rounds.
__global__ __launch_bounds__(1024) void k_components(int n, int E, const int32_t *ei,
                                                     const int32_t *ej, const uint8_t *keep,
                                                     const double *s, int32_t *lab, int32_t *ncl) {
  __shared__ int changed;
  __shared__ int cnt_s[1024 / kWave];
  for (int i = threadIdx.x; i < n; i += blockDim.x) lab[i] = i;
  __syncthreads();
  for (int round = 0; round < n + 2; ++round) {
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    int local = 0;
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
      const bool fused = keep ? (keep[e] != 0) : (s[e] == 0.0);
      if (!fused) continue;
      const int a = ei[e], b = ej[e];
      const int la = __hip_atomic_load(&lab[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int lbv = __hip_atomic_load(&lab[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (la != lbv) {
        const int lo = min(la, lbv), hi = max(la, lbv);
        atomicMin(&lab[a], lo);
        atomicMin(&lab[b], lo);
        atomicMin(&lab[hi], lo);
        local = 1;
      }
    }
    if (local) changed = 1;
    __syncthreads();
    // pointer jumping
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      int l = __hip_atomic_load(&lab[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int ll = __hip_atomic_load(&lab[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (ll < l) {
        l = ll;
        ll = __hip_atomic_load(&lab[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      atomicMin(&lab[i], l);
    }
    __syncthreads();
    const int ch = changed;
    __syncthreads();
    if (!ch) break;
  }
  int c = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    c += (__hip_atomic_load(&lab[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == i) ? 1 : 0;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
  if (threadIdx.x % kWave == 0) cnt_s[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) tot += cnt_s[w];
    *ncl = tot;
  }
}

// ====================================================================== host
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int64_t kSlabBytes = 128 * 1024;  // LDS budget of the slab point sweep

static size_t ts_size(int prec) { return prec == kF32 ? 4 : 8; }
static size_t tx_size(int prec) { return prec == kF64 ? 8 : 4; }
static size_t tg_size(int prec) { return prec == kF64 ? 8 : 4; }
static size_t ta_size(int prec) { return prec == kF64 ? 8 : 4; }  // the stored A array

struct Launch {
  int blocks, chunk, nitems;
};

// Grid for a sweep over nitems wave-items with `waves` waves per block and
// about ipw items per wave: at most kMaxBlocks blocks, a multiple of the XCD
// count, each block owning a contiguous chunk.
static Launch sweep_grid(int64_t nitems, int waves = kWavesPerBlock, int ipw = 1) {
  Launch L;
  L.nitems = (int)nitems;
  int64_t want = cdiv(std::max<int64_t>(nitems, 1), (int64_t)waves * ipw);
  int64_t blocks = std::min<int64_t>(want, kMaxBlocks);
  // a multiple of the XCD count unless that would at least double the grid
  if (blocks > kXcds) blocks = cdiv(blocks, kXcds) * kXcds;
  L.blocks = (int)blocks;
  L.chunk = (int)cdiv(std::max<int64_t>(nitems, 1), blocks);
  return L;
}

// Event set for a sampled iteration (cc_profile), or null: start and end of
// the point sweep, then of the edge stage.
static hipEvent_t *prof_slot(Problem *P) {
  if (P->prof_every <= 0) return nullptr;
  const bool sample = (P->prof_iter++ % P->prof_every) == 0;
  if (!sample) return nullptr;
  const size_t need = 4 * (P->prof_used + 1);
  while (P->prof_events.size() < need) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    P->prof_events.push_back(ev);
  }
  return &P->prof_events[4 * P->prof_used++];
}

// Launch on a stream.  With events given, hipExtLaunchKernel stamps them with
// the kernel's own start (e0) and end (e1), so a sampled duration is the
// kernel's execution, not the gap between two markers around it.
template <typename... KArgs, typename... Args>
static void klaunch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds, hipStream_t stream,
                    hipEvent_t e0, hipEvent_t e1, Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, stream, e0, e1, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, args...);
}

// Arguments of a point sweep: it reads the current scalar slot and writes the
// other one.
static PointArgs point_args(Problem *P, const Launch &Lp) {
  return PointArgs{(int)P->n, (int)P->ld, P->ntile, Lp.nitems, Lp.chunk,
                   P->X, P->M, P->U, P->A[0], P->A[1], P->G[0], P->G[1], P->Usnap, P->Asnap,
                   P->ell_s, P->degE, P->colE, P->eidE, P->qE, P->s, P->cur_K, Lp.blocks,
                   P->psum, P->esum, P->nbe, P->trace, P->sc + P->slot, P->sc + (P->slot ^ 1), nullptr,
                   P->H, P->T[0], P->lazy_u ? 1 : 0, P->Umiss, P->moff};
}

// Projection sweeps 2..K after k_point_rhs (scalars: the slot the point
// sweep wrote).  Sweep k reads the increments of sweep k-1: T[0] holds the
// first sweep's, then T[0] and T[1] alternate; the last writes the gather
// copy of the state's A.
template <int PREC, int VEC>
static void launch_jacobi_t(Problem *P, const Launch &Lp) {
  JacArgs ja{(int)P->n, (int)P->ld, Lp.nitems, Lp.chunk, P->ell_s, P->cur_K, P->colE, P->H,
             nullptr, nullptr, P->U, P->A[0], P->A[1], P->G[0], P->G[1], P->Asnap, P->psum,
             P->sc + P->slot};
  for (int k = 2; k <= P->psweeps; ++k) {
    ja.Din = P->T[(k - 2) % 2];
    ja.Dout = P->T[(k - 1) % 2];
    if (k < P->psweeps)
      klaunch(k_jacobi<PREC, VEC, false>, dim3(Lp.blocks), dim3(kPointBlock), 0, P->stream, nullptr, nullptr, ja);
    else
      klaunch(k_jacobi<PREC, VEC, true>, dim3(Lp.blocks), dim3(kPointBlock), 0, P->stream, nullptr, nullptr, ja);
  }
}

template <int PREC, int VEC>
static void launch_point_t(Problem *P, const Launch &Lp) {
  if (P->psweeps > 1) {
    if (Lp.chunk > kPointWaves)
      klaunch(k_point_rhs<PREC, VEC, true>, dim3(Lp.blocks), dim3(kPointBlock), 0, P->stream, P->pev[0], P->pev[1],
              point_args(P, Lp));
    else
      klaunch(k_point_rhs<PREC, VEC, false>, dim3(Lp.blocks), dim3(kPointBlock), 0, P->stream, P->pev[0], P->pev[1],
              point_args(P, Lp));
    return;
  }
  // wider blocks: the mixed precision with 4 features per lane
  if constexpr (PREC == kMixed && VEC == 4) {
    if (P->pwaves == 8 || P->pwaves == 16) {
      const bool pf = Lp.chunk > P->pwaves;
      const dim3 t(kWave * P->pwaves);
      if (P->pwaves == 8) {
        if (pf) klaunch(k_point<PREC, VEC, true, 8>, dim3(Lp.blocks), t, 0, P->stream, P->pev[0], P->pev[1], point_args(P, Lp));
        else klaunch(k_point<PREC, VEC, false, 8>, dim3(Lp.blocks), t, 0, P->stream, P->pev[0], P->pev[1], point_args(P, Lp));
      } else {
        if (pf) klaunch(k_point<PREC, VEC, true, 16>, dim3(Lp.blocks), t, 0, P->stream, P->pev[0], P->pev[1], point_args(P, Lp));
        else klaunch(k_point<PREC, VEC, false, 16>, dim3(Lp.blocks), t, 0, P->stream, P->pev[0], P->pev[1], point_args(P, Lp));
      }
      return;
    }
  }
  // prefetching pays when a wave has more than one item
  if (Lp.chunk > kPointWaves)
    klaunch(k_point<PREC, VEC, true>, dim3(Lp.blocks), dim3(kPointBlock), 0, P->stream, P->pev[0], P->pev[1],
            point_args(P, Lp));
  else
    klaunch(k_point<PREC, VEC, false>, dim3(Lp.blocks), dim3(kPointBlock), 0, P->stream, P->pev[0], P->pev[1],
            point_args(P, Lp));
}

static EdgeState edge_state(Problem *P) {
  return EdgeState{(int)P->E, P->w, P->s, P->nb[0], P->nb[1], P->qe, P->qE, P->epos};
}

static EdgeArgs edge_args(Problem *P, const Launch &Le, int init, int nbp) {
  return EdgeArgs{(int)P->n, (int)P->ld, P->entile, Le.nitems, Le.chunk, init, nbp, Le.blocks,
                  P->G[0], P->G[1], P->ei, P->ej, P->itemI, P->itemJ, P->itemE,
                  P->rowptr, P->uptr, P->col, P->eid, P->part,
                  edge_state(P), P->esum, P->psum, P->sc + P->slot};
}

// Grid of the fused edge kernel: groups of 4 edges, one per wave, at most
// kEsumRows blocks (each leaves one partial row).
static Launch edge_fused_grid(int64_t E) {
  Launch L;
  const int64_t nitems = std::max<int64_t>(cdiv(E, 4), 1);
  L.nitems = (int)cdiv(E, 4);
  int64_t blocks = std::min<int64_t>(cdiv(nitems, kEdgeWaves), kEsumRows);
  blocks = std::min<int64_t>(cdiv(blocks, kXcds) * kXcds, kEsumRows);
  L.blocks = (int)blocks;
  L.chunk = (int)cdiv(nitems, blocks);
  return L;
}

// Grid of the item edge kernel: about ipw items per wave, at most kEsumRows
// blocks.
static Launch edge_items_grid(int64_t n_items, int ipw = 1) {
  Launch L;
  const int64_t nitems = std::max<int64_t>(n_items, 1);
  L.nitems = (int)n_items;
  int64_t blocks = std::min<int64_t>(cdiv(nitems, (int64_t)kEdgeWaves * ipw), kEsumRows);
  // a multiple of the XCD count unless that would at least double the grid
  if (blocks > kXcds) blocks = std::min<int64_t>(cdiv(blocks, kXcds) * kXcds, kEsumRows);
  L.blocks = (int)blocks;
  L.chunk = (int)cdiv(nitems, blocks);
  return L;
}

// Blocks of the edge-reduction kernel (wide rows): one wave per edge.
static int edge_reduce_blocks(int64_t E) {
  return (int)std::min<int64_t>(std::max<int64_t>(cdiv(E, kEdgeWaves), 1), kEsumRows);
}

// Partial rows the edge stage leaves for the next point sweep.
static int edge_rows(Problem *P) {
  if (P->eitems) return edge_items_grid(P->n_items, P->eipw).blocks;
  return P->efused ? edge_fused_grid(P->E).blocks : edge_reduce_blocks(P->E);
}

template <int PREC>
static void launch_edge_p(Problem *P, int init, int nbp) {
  if (P->eitems) {
    const Launch Li = edge_items_grid(P->n_items, P->eipw);
    const EdgeArgs ea = edge_args(P, Li, init, nbp);
    switch (P->item_nv) {
      case 1: klaunch(k_edge_items<PREC, 1>, dim3(Li.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
      case 2: klaunch(k_edge_items<PREC, 2>, dim3(Li.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
      case 4: klaunch(k_edge_items<PREC, 4>, dim3(Li.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
      case 8: klaunch(k_edge_items<PREC, 8>, dim3(Li.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
      default: klaunch(k_edge_items<PREC, 16>, dim3(Li.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
    }
    return;
  }
  if (P->efused) {
    const Launch Le = edge_fused_grid(P->E);
    const EdgeArgs ea = edge_args(P, Le, init, nbp);
    switch (P->npass) {
      case 1: klaunch(k_edge_fused<PREC, 1>, dim3(Le.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
      case 2: klaunch(k_edge_fused<PREC, 2>, dim3(Le.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
      case 4: klaunch(k_edge_fused<PREC, 4>, dim3(Le.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
      case 8: klaunch(k_edge_fused<PREC, 8>, dim3(Le.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
      default: klaunch(k_edge_fused<PREC, 16>, dim3(Le.blocks), dim3(kEdgeBlock), 0, P->stream, P->pev[2], P->pev[3], ea); break;
    }
    return;
  }
  if (P->eslab && P->eslab_items) {
    const Launch Ls{P->entile, 0, (int)P->n_items};
    const EdgeArgs ea = edge_args(P, Ls, init, nbp);
    const size_t lds = (size_t)P->n * (P->edge_f + kSlabPad) * sizeof(typename Traits<PREC>::TG);
    switch (P->edge_f) {
      case 4: klaunch(k_edge_slab_items<PREC, 4>, dim3(P->entile), dim3(1024), lds, P->stream, P->pev[2], nullptr, ea, P->eslab_tpg, P->eslab_ntf); break;
      case 8: klaunch(k_edge_slab_items<PREC, 8>, dim3(P->entile), dim3(1024), lds, P->stream, P->pev[2], nullptr, ea, P->eslab_tpg, P->eslab_ntf); break;
      case 16: klaunch(k_edge_slab_items<PREC, 16>, dim3(P->entile), dim3(1024), lds, P->stream, P->pev[2], nullptr, ea, P->eslab_tpg, P->eslab_ntf); break;
      default: klaunch(k_edge_slab_items<PREC, 32>, dim3(P->entile), dim3(1024), lds, P->stream, P->pev[2], nullptr, ea, P->eslab_tpg, P->eslab_ntf); break;
    }
  } else if (P->eslab) {
    const Launch Ls{P->entile, 0, 0};
    const EdgeArgs ea = edge_args(P, Ls, init, nbp);
    const size_t lds = (size_t)P->n * (P->edge_f + kSlabPad) * sizeof(typename Traits<PREC>::TG);
    switch (P->edge_f) {
      case 4: klaunch(k_edge_slab<PREC, 4>, dim3(P->entile), dim3(1024), lds, P->stream, P->pev[2], nullptr, ea, P->eslab_tpg, P->eslab_ntf); break;
      case 8: klaunch(k_edge_slab<PREC, 8>, dim3(P->entile), dim3(1024), lds, P->stream, P->pev[2], nullptr, ea, P->eslab_tpg, P->eslab_ntf); break;
      case 16: klaunch(k_edge_slab<PREC, 16>, dim3(P->entile), dim3(1024), lds, P->stream, P->pev[2], nullptr, ea, P->eslab_tpg, P->eslab_ntf); break;
      default: klaunch(k_edge_slab<PREC, 32>, dim3(P->entile), dim3(1024), lds, P->stream, P->pev[2], nullptr, ea, P->eslab_tpg, P->eslab_ntf); break;
    }
  } else {
    const Launch Le = sweep_grid(P->n * P->entile);
    klaunch(k_edge_tiles<PREC>, dim3(Le.blocks), dim3(kBlock), 0, P->stream, P->pev[2], nullptr,
            edge_args(P, Le, init, nbp));
  }
  const int rblocks = edge_reduce_blocks(P->E);
  ReduceArgs ra{P->entile, nbp, init, P->part, edge_state(P), P->esum, P->psum, P->sc + P->slot};
  klaunch(k_edge_reduce, dim3(rblocks), dim3(kEdgeBlock), 0, P->stream, nullptr, P->pev[3], ra);
}

template <int PREC, int F>
static void launch_point_slab_t(Problem *P, int blocks) {
  const PointArgs pa = point_args(P, Launch{blocks, 0, 0});
  const size_t lds = (size_t)P->n * F * sizeof(typename Traits<PREC>::TG);
  klaunch(k_point_slab<PREC, F>, dim3(blocks), dim3(kBlock), lds, P->stream, P->pev[0], P->pev[1], pa);
}

template <int PREC>
static void set_slab_attr() {
  (void)hipFuncSetAttribute((const void *)k_edge_slab<PREC, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSlabBytes);
  (void)hipFuncSetAttribute((const void *)k_edge_slab<PREC, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSlabBytes);
  (void)hipFuncSetAttribute((const void *)k_edge_slab<PREC, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSlabBytes);
  (void)hipFuncSetAttribute((const void *)k_edge_slab<PREC, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSlabBytes);
  (void)hipFuncSetAttribute((const void *)k_edge_slab_items<PREC, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSlabBytes);
  (void)hipFuncSetAttribute((const void *)k_edge_slab_items<PREC, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSlabBytes);
  (void)hipFuncSetAttribute((const void *)k_edge_slab_items<PREC, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSlabBytes);
  (void)hipFuncSetAttribute((const void *)k_edge_slab_items<PREC, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSlabBytes);
}

// Waves per block of the point sweep's launch.
static int point_waves(const Problem *P) {
  return (P->psweeps == 1 && P->precision == kMixed && P->vec == 4) ? P->pwaves : kPointWaves;
}

// Grid of the point sweep.
static Launch point_grid(const Problem *P) {
  return sweep_grid(P->n * P->ntile, point_waves(P), P->ipw);
}

// Blocks of the point sweep (its partials count).
static int point_blocks(Problem *P) {
  if (P->slab_f > 0) return (int)(cdiv(P->ntile * cdiv(P->n, kBlock), kXcds) * kXcds);
  return point_grid(P).blocks;
}

template <int PREC>
static void launch_point_p(Problem *P, const Launch &Lp) {
  if (P->slab_f > 0) {
    const int blocks = point_blocks(P);
    switch (P->slab_f) {
      case 4: launch_point_slab_t<PREC, 4>(P, blocks); break;
      case 8: launch_point_slab_t<PREC, 8>(P, blocks); break;
      case 16: launch_point_slab_t<PREC, 16>(P, blocks); break;
      default: launch_point_slab_t<PREC, 32>(P, blocks); break;
    }
    return;
  }
  switch (P->vec) {
    case 1: launch_point_t<PREC, 1>(P, Lp); break;
    case 2: launch_point_t<PREC, 2>(P, Lp); break;
    default: launch_point_t<PREC, 4>(P, Lp); break;
  }
}

// One launch pair: the point sweep (which first finishes the pending
// iteration) and the edge stage.  Advances the host's scalar slot.
// U of a lazily stored solve (after its last iteration).
template <int PREC>
static void launch_u_finish_p(Problem *P) {
  const Launch L = sweep_grid(P->n * P->ntile, kPointWaves);
  const PointArgs a = point_args(P, L);
  switch (P->vec) {
    case 1: klaunch(k_u_finish<PREC, 1>, dim3(L.blocks), dim3(kPointBlock), 0, P->stream, nullptr, nullptr, a); break;
    case 2: klaunch(k_u_finish<PREC, 2>, dim3(L.blocks), dim3(kPointBlock), 0, P->stream, nullptr, nullptr, a); break;
    default: klaunch(k_u_finish<PREC, 4>, dim3(L.blocks), dim3(kPointBlock), 0, P->stream, nullptr, nullptr, a); break;
  }
}
static void launch_u_finish(Problem *P) {
  if (P->precision == kF32) launch_u_finish_p<kF32>(P);
  else if (P->precision == kF64) launch_u_finish_p<kF64>(P);
  else launch_u_finish_p<kMixed>(P);
}

static void launch_iteration(Problem *P) {
  hipEvent_t *ev = prof_slot(P);
  for (int q = 0; q < 4; ++q) P->pev[q] = ev ? ev[q] : nullptr;
  const Launch Lp = point_grid(P);
  const int nbp = point_blocks(P);
  if (P->precision == kF32) launch_point_p<kF32>(P, Lp);
  else if (P->precision == kF64) launch_point_p<kF64>(P, Lp);
  else launch_point_p<kMixed>(P, Lp);
  P->slot ^= 1;
  if (P->psweeps > 1) {
    auto jac = [&](auto prec_tag) {
      constexpr int PR = decltype(prec_tag)::value;
      switch (P->vec) {
        case 1: launch_jacobi_t<PR, 1>(P, Lp); break;
        case 2: launch_jacobi_t<PR, 2>(P, Lp); break;
        default: launch_jacobi_t<PR, 4>(P, Lp); break;
      }
    };
    if (P->precision == kF32) jac(std::integral_constant<int, kF32>());
    else if (P->precision == kF64) jac(std::integral_constant<int, kF64>());
    else jac(std::integral_constant<int, kMixed>());
  }
  if (P->precision == kF32) launch_edge_p<kF32>(P, 0, nbp);
  else if (P->precision == kF64) launch_edge_p<kF64>(P, 0, nbp);
  else launch_edge_p<kMixed>(P, 0, nbp);
  for (int q = 0; q < 4; ++q) P->pev[q] = nullptr;
}

// Edge norms of the A in buffer pa (state set or reset).
static void launch_edge_init(Problem *P) {
  if (P->precision == kF32) launch_edge_p<kF32>(P, 1, 0);
  else if (P->precision == kF64) launch_edge_p<kF64>(P, 1, 0);
  else launch_edge_p<kMixed>(P, 1, 0);
}

cc_status profile(Problem *P, int32_t sample_every) {
  CC_HIP(hipStreamSynchronize(P->stream));
  P->prof_every = sample_every > 0 ? sample_every : 0;
  P->prof_iter = 0;
  P->prof_used = 0;
  for (int q = 0; q < 3; ++q) { P->prof_ms[q] = 0.0; P->prof_n[q] = 0; }
  return CC_OK;
}

// Fold the durations of every recorded event set into the statistics.  The
// caller has synchronised the stream, so every event is complete.
cc_status harvest_profile(Problem *P) {
  for (size_t k = 0; k < P->prof_used; ++k) {
    hipEvent_t *ev = &P->prof_events[4 * k];
    for (int q = 0; q < 2; ++q) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]) == hipSuccess) {
        P->prof_ms[q] += ms;
        P->prof_n[q] += 1;
      }
    }
  }
  P->prof_used = 0;
  return CC_OK;
}

void problem_free(Problem *P) {
  if (!P) return;
  void *bufs[] = {P->X, P->M, P->U, P->A[0], P->A[1], P->Usnap, P->Asnap, P->rowptr, P->col, P->eid, P->uptr,
                  P->itemI, P->itemJ, P->itemE,
                  P->ei, P->ej, P->w, P->s, P->nb[0], P->nb[1], P->qe, P->qE, P->epos, P->degE, P->colE,
                  P->eidE, P->part, P->psum,
                  P->esum, P->trace, P->sc, P->ncl_dev, P->H, P->T[0], P->T[1], P->Umiss, P->moff};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (Traits<kMixed>::mirror && P->precision == kMixed) {
    if (P->G[0]) (void)hipFree(P->G[0]);
    if (P->G[1]) (void)hipFree(P->G[1]);
  }
  for (hipEvent_t ev : P->prof_events) (void)hipEventDestroy(ev);
  if (P->sc_host) (void)hipHostFree(P->sc_host);
  if (P->flag_host) (void)hipHostFree(P->flag_host);
  delete P;
}

static cc_status dmalloc(void **p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    set_error(std::string("hipMalloc of ") + std::to_string(bytes) + " bytes failed: " +
              hipGetErrorString(e));
    return CC_ERR_OUT_OF_MEMORY;
  }
  return CC_OK;
}

#define CC_TRY(x)                       \
  do {                                  \
    cc_status _s = (x);                 \
    if (_s != CC_OK) return _s;         \
  } while (0)

static void choose_tiles(Problem *P) {
  // point sweep: the LDS slab variant when an n x F tile of the gather copy
  // fits (F = 32, 16, 8 or 4 features), else a wave per (point, 64*vec tile)
  // The wave kernel is the default: the slab variant runs one wave per SIMD
  // and measured slower on both the p = 500 and the p = 20000 workloads; it
  // is kept as an option (CCMI_SLAB_F = 4, 8, 16 or 32).
  const int64_t tg = (P->precision == kF64) ? 8 : 4;
  int slab = 0;
  const char *es = getenv("CCMI_SLAB_F");
  if (es) slab = atoi(es);
  if (slab != 4 && slab != 8 && slab != 16 && slab != 32) slab = 0;
  if (slab > 0 && P->n * slab * tg > kSlabBytes) slab = 0;
  P->slab_f = slab;
  P->ell_cm = slab > 0;
  // edge sweep over wide rows: LDS tile width (independent of the above)
  P->edge_f = 0;
  for (int f : {16, 8, 4}) {
    if (P->n * f * tg <= kSlabBytes / 2) { P->edge_f = f; break; }
  }
  const char *env = getenv("CCMI_VEC");
  int vec = 0;
  if (env) vec = atoi(env);
  if (vec != 1 && vec != 2 && vec != 4) vec = P->p > 256 ? 4 : (P->p > 96 ? 2 : 1);
  P->vec = vec;
  // items per wave of the point and item edge sweeps (CCMI_IPW = 1, 2 or 4)
  const char *ei = getenv("CCMI_IPW");
  const int ipw = ei ? atoi(ei) : 1;
  P->ipw = (ipw == 2 || ipw == 4) ? ipw : 1;
  // items per wave of the item edge sweep alone (CCMI_EDGE_IPW = 1, 2 or 4;
  // default: as the point sweep)
  const char *eiw = getenv("CCMI_EDGE_IPW");
  const int eipw = eiw ? atoi(eiw) : P->ipw;
  P->eipw = (eipw == 2 || eipw == 4) ? eipw : 1;
  P->tile_w = slab > 0 ? slab : kWave * vec;
  P->ntile = (int)cdiv(P->ld, P->tile_w);
  // waves per block of the point sweep (CCMI_POINT_WAVES = 4, 8 or 16; the
  // wider blocks for the mixed precision with 4 features per lane).  With
  // several items per wave (more items than 4-wave blocks on the capped grid
  // have waves) 8-wave blocks measured faster (genotype: 286 against 296 us),
  // with one item per wave 4-wave blocks (expression: 24.2 against 25.3 us)
  const char *pw = getenv("CCMI_POINT_WAVES");
  const bool several = P->n * P->ntile > (int64_t)kMaxBlocks * kPointWaves;
  const int pwv = pw ? atoi(pw) : (several ? 8 : kPointWaves);
  P->pwaves = (pwv == 8 || pwv == 16) ? pwv : kPointWaves;
  // edge sweep: work items of edges sharing a lower end when the whole row
  // fits a wave at up to 16 features per lane (CCMI_EDGE_ITEMS=0 turns this
  // off), else one tile over the whole row when it is at most 1024 wide
  const char *eit = getenv("CCMI_EDGE_ITEMS");
  P->eitems = P->ld <= 16 * kWave && !(eit && atoi(eit) == 0);
  P->item_nv = 1;
  while (P->item_nv * kWave < P->ld) P->item_nv <<= 1;
  if (P->ld <= 1024) {
    int np = 1;
    while (64 * np < P->ld) np <<= 1;
    P->npass = np;
    P->entile = 1;
    P->efused = true;
  } else {
    P->npass = 4;
    P->entile = (int)cdiv(P->ld, 256);
    P->efused = false;
    // small n: stage tiles in LDS and keep per-edge accumulators in registers
    const char *ee = getenv("CCMI_EDGE_SLAB");
    const bool allow = !ee || atoi(ee) != 0;
    if (allow && P->edge_f > 0 && P->E <= 1024 * 16 && P->n * (P->edge_f / 4) <= kSlabChunks * 1024 && P->n < 65536) {
      P->eslab = true;
      P->eslab_ntf = (int)cdiv(P->ld, P->edge_f);
      P->eslab_tpg = (int)cdiv(P->eslab_ntf, 256);
      const int64_t groups = cdiv(P->eslab_ntf, P->eslab_tpg);
      P->entile = (int)(cdiv(groups, kXcds) * kXcds);  // one partial column per block
    }
  }
}

cc_status reset_state(Problem *P);

cc_status problem_create(int64_t n, int64_t p, int32_t x_dtype, const void *X,
                         int64_t ldx, const uint8_t *mask, int64_t ldm,
                         int64_t n_edges, const int32_t *ei, const int32_t *ej,
                         const double *w, int32_t precision, hipStream_t stream,
                         Problem **out) {
  if (!out) { set_error("out is NULL"); return CC_ERR_INVALID_ARG; }
  *out = nullptr;
  if (n < 1 || p < 1) { set_error("need n >= 1 and p >= 1"); return CC_ERR_INVALID_ARG; }
  if (n > (int64_t)1 << 30 || p > (int64_t)1 << 30) { set_error("n or p too large"); return CC_ERR_INVALID_ARG; }
  if (x_dtype != CC_DTYPE_F32 && x_dtype != CC_DTYPE_F64) { set_error("x_dtype must be CC_DTYPE_F32 or CC_DTYPE_F64"); return CC_ERR_INVALID_ARG; }
  if (!X) { set_error("X is NULL"); return CC_ERR_INVALID_ARG; }
  if (ldx < p) { set_error("ldx < p"); return CC_ERR_INVALID_ARG; }
  if (mask && ldm < p) { set_error("ldm < p"); return CC_ERR_INVALID_ARG; }
  if (n_edges < 0) { set_error("n_edges < 0"); return CC_ERR_INVALID_ARG; }
  if (n_edges > 0 && (!ei || !ej || !w)) { set_error("edge arrays are NULL"); return CC_ERR_INVALID_ARG; }
  if (precision != kF32 && precision != kMixed && precision != kF64) { set_error("unknown precision"); return CC_ERR_INVALID_ARG; }
  if ((int64_t)n * ((p + 3) / 4 * 4) > ((int64_t)1 << 31) - 1) { set_error("n * p exceeds 2^31"); return CC_ERR_INVALID_ARG; }

  // ---- validate edges and weights on the host ----
  std::vector<int32_t> hi(n_edges), hj(n_edges);
  std::vector<double> hw(n_edges);
  if (n_edges > 0) {
    CC_HIP(hipMemcpyAsync(hi.data(), ei, n_edges * 4, hipMemcpyDeviceToHost, stream));
    CC_HIP(hipMemcpyAsync(hj.data(), ej, n_edges * 4, hipMemcpyDeviceToHost, stream));
    CC_HIP(hipMemcpyAsync(hw.data(), w, n_edges * 8, hipMemcpyDeviceToHost, stream));
    CC_HIP(hipStreamSynchronize(stream));
  }
  std::vector<int64_t> keys(n_edges);
  for (int64_t e = 0; e < n_edges; ++e) {
    if (hi[e] < 0 || hj[e] >= n || hi[e] >= hj[e]) {
      set_error("edge " + std::to_string(e) + " invalid: need 0 <= ei < ej < n");
      return CC_ERR_INVALID_ARG;
    }
    if (!std::isfinite(hw[e]) || !(hw[e] > 0.0)) {
      set_error("weight " + std::to_string(e) + " must be finite and > 0");
      return CC_ERR_INVALID_ARG;
    }
    keys[e] = (int64_t)hi[e] * n + hj[e];
  }
  {
    std::vector<int64_t> sk(keys);
    std::sort(sk.begin(), sk.end());
    for (size_t k = 1; k < sk.size(); ++k)
      if (sk[k] == sk[k - 1]) { set_error("duplicate edge"); return CC_ERR_INVALID_ARG; }
  }

  Problem *P = new (std::nothrow) Problem();
  if (!P) { set_error("host allocation failed"); return CC_ERR_OUT_OF_MEMORY; }
  P->n = n; P->p = p; P->E = n_edges; P->ld = (p + 3) / 4 * 4;
  P->precision = precision; P->stream = stream; P->has_mask = mask != nullptr;
  choose_tiles(P);
  if (P->slab_f > 0 || P->eslab) {
    if (precision == kF32) set_slab_attr<kF32>();
    else if (precision == kF64) set_slab_attr<kF64>();
    else set_slab_attr<kMixed>();
  }
  struct Guard { Problem *&P; bool ok = false; ~Guard() { if (!ok) problem_free(P); } } guard{P};

  const size_t nl = (size_t)n * P->ld;
  CC_TRY(dmalloc(&P->X, nl * tx_size(precision)));
  if (mask) CC_TRY(dmalloc((void **)&P->M, nl));
  CC_TRY(dmalloc(&P->U, nl * ts_size(precision)));
  CC_TRY(dmalloc(&P->A[0], nl * ta_size(precision)));
  CC_TRY(dmalloc(&P->A[1], nl * ta_size(precision)));
  CC_TRY(dmalloc(&P->Usnap, nl * ts_size(precision)));
  CC_TRY(dmalloc(&P->Asnap, nl * ts_size(precision)));
  if (precision == kMixed) {
    CC_TRY(dmalloc(&P->G[0], nl * tg_size(precision)));
    CC_TRY(dmalloc(&P->G[1], nl * tg_size(precision)));
  } else {
    P->G[0] = P->A[0]; P->G[1] = P->A[1];
  }
  const int64_t E = n_edges;
  CC_TRY(dmalloc((void **)&P->rowptr, (n + 1) * 4));
  CC_TRY(dmalloc((void **)&P->uptr, n * 4));
  CC_TRY(dmalloc((void **)&P->col, 2 * E * 4));
  CC_TRY(dmalloc((void **)&P->eid, 2 * E * 4));
  CC_TRY(dmalloc((void **)&P->ei, E * 4));
  CC_TRY(dmalloc((void **)&P->ej, E * 4));
  CC_TRY(dmalloc((void **)&P->w, E * 8));
  CC_TRY(dmalloc((void **)&P->s, E * 8));
  CC_TRY(dmalloc((void **)&P->nb[0], E * 8));
  CC_TRY(dmalloc((void **)&P->nb[1], E * 8));
  CC_TRY(dmalloc((void **)&P->qe, E * 8));
  CC_TRY(dmalloc((void **)&P->epos, 2 * E * 4));
  CC_TRY(dmalloc((void **)&P->part, E * (P->efused ? 1 : P->entile) * 8));
  // one row of point partials per block of the point sweep
  CC_TRY(dmalloc((void **)&P->psum, std::max<int64_t>(kMaxBlocks, point_blocks(P)) * 8 * 8));
  CC_TRY(dmalloc((void **)&P->esum, (size_t)kEsumRows * kEsumStride * 8));
  CC_TRY(dmalloc((void **)&P->sc, 2 * sizeof(DevScalars)));
  CC_TRY(dmalloc((void **)&P->ncl_dev, 4));
  CC_HIP(hipHostMalloc((void **)&P->sc_host, sizeof(DevScalars), hipHostMallocDefault));
  CC_HIP(hipHostMalloc((void **)&P->flag_host, 64, hipHostMallocDefault));

  // ---- symmetric CSR with sorted columns ----
  std::vector<int32_t> deg(n + 1, 0);
  for (int64_t e = 0; e < E; ++e) { deg[hi[e]]++; deg[hj[e]]++; }
  std::vector<int32_t> rp(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) rp[i + 1] = rp[i] + deg[i];
  std::vector<std::pair<int32_t, int32_t>> ent(2 * E);
  {
    std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
      ent[fill[hi[e]]++] = {hj[e], (int32_t)e};
      ent[fill[hj[e]]++] = {hi[e], (int32_t)e};
    }
  }
  std::vector<int32_t> hcol(2 * E), heid(2 * E), hup(n), hpos(2 * E);
  int64_t maxdeg = 0;
  for (int64_t i = 0; i < n; ++i) {
    std::sort(ent.begin() + rp[i], ent.begin() + rp[i + 1]);
    int32_t up = rp[i + 1];
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      hcol[k] = ent[k].first; heid[k] = ent[k].second;
      // entry (i -> j) of edge e sits in row ei[e] (slot 0) or ej[e] (slot 1)
      hpos[2 * (int64_t)ent[k].second + (hi[ent[k].second] == i ? 0 : 1)] = k;
      if (up == rp[i + 1] && ent[k].first > i) up = k;
    }
    hup[i] = up;
    maxdeg = std::max<int64_t>(maxdeg, rp[i + 1] - rp[i]);
  }
  P->max_deg = maxdeg;
  // edge work items: the upper neighbours of each point in runs of up to
  // kItemEdges (unused slots -1)
  {
    std::vector<int32_t> iI, iJ, iE;
    for (int64_t i = 0; i < n; ++i) {
      for (int32_t k = hup[i]; k < rp[i + 1]; k += kItemEdges) {
        iI.push_back((int32_t)i);
        for (int q = 0; q < kItemEdges; ++q) {
          const bool ok = k + q < rp[i + 1];
          iJ.push_back(ok ? hcol[k + q] : -1);
          iE.push_back(ok ? heid[k + q] : -1);
        }
      }
    }
    P->n_items = (int64_t)iI.size();
    if (P->eslab) {
      const char *es = getenv("CCMI_EDGE_SLAB_ITEMS");
      P->eslab_items = P->n_items <= (int64_t)kSlabItemSlots * 1024 && !(es && atoi(es) == 0);
    }
    CC_TRY(dmalloc((void **)&P->itemI, iI.size() * 4));
    CC_TRY(dmalloc((void **)&P->itemJ, iJ.size() * 4));
    CC_TRY(dmalloc((void **)&P->itemE, iE.size() * 4));
    if (!iI.empty()) {
      CC_HIP(hipMemcpyAsync(P->itemI, iI.data(), iI.size() * 4, hipMemcpyHostToDevice, stream));
      CC_HIP(hipMemcpyAsync(P->itemJ, iJ.data(), iJ.size() * 4, hipMemcpyHostToDevice, stream));
      CC_HIP(hipMemcpyAsync(P->itemE, iE.data(), iE.size() * 4, hipMemcpyHostToDevice, stream));
      CC_HIP(hipStreamSynchronize(stream));  // the host vectors go out of scope
    }
  }
  P->nbe = edge_rows(P);
  // ELL copy of the neighbour lists for the point sweep
  const int64_t S = std::max<int64_t>(maxdeg, 1);
  // the sweeps index ELL slots (n * S of them) in 32 bits: checked before
  // any of the n * S host or device arrays exists
  if (n * S > ((int64_t)1 << 31) - 1) {
    set_error("neighbour lists too large: n * max degree = " + std::to_string(n * S) + " >= 2^31");
    return CC_ERR_INVALID_ARG;
  }
  P->ell_s = (int)S;
  // unused slots: column -1 (the wave sweep counts neighbours by it), edge 0
  std::vector<int32_t> hdegE(n), hcolE(n * S, -1), heidE(n * S, 0), hposE(2 * E);
  // row-major (entry k of i at i*S + k) for the wave-per-point sweep,
  // column-major (k*n + i) for the slab sweep
  auto ell_slot = [&](int64_t i, int64_t k) -> int64_t { return P->ell_cm ? k * n + i : i * S + k; };
  for (int64_t i = 0; i < n; ++i) {
    hdegE[i] = rp[i + 1] - rp[i];
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int64_t slot = ell_slot(i, k - rp[i]);
      hcolE[slot] = hcol[k];
      heidE[slot] = heid[k];
    }
  }
  for (int64_t e2 = 0; e2 < 2 * E; ++e2) {
    // hpos holds CSR positions; map them to ELL slots
    const int32_t k = hpos[e2];
    const int64_t row = (e2 % 2 == 0) ? hi[e2 / 2] : hj[e2 / 2];
    hposE[e2] = (int32_t)ell_slot(row, k - rp[row]);
  }
  CC_TRY(dmalloc((void **)&P->degE, n * 4));
  CC_TRY(dmalloc((void **)&P->colE, n * S * 4));
  CC_TRY(dmalloc((void **)&P->eidE, n * S * 4));
  CC_TRY(dmalloc((void **)&P->qE, n * S * 8));
  CC_HIP(hipMemcpyAsync(P->degE, hdegE.data(), n * 4, hipMemcpyHostToDevice, stream));
  CC_HIP(hipMemcpyAsync(P->colE, hcolE.data(), n * S * 4, hipMemcpyHostToDevice, stream));
  CC_HIP(hipMemcpyAsync(P->eidE, heidE.data(), n * S * 4, hipMemcpyHostToDevice, stream));
  CC_HIP(hipMemcpyAsync(P->rowptr, rp.data(), (n + 1) * 4, hipMemcpyHostToDevice, stream));
  CC_HIP(hipMemcpyAsync(P->uptr, hup.data(), n * 4, hipMemcpyHostToDevice, stream));
  if (E > 0) {
    CC_HIP(hipMemcpyAsync(P->col, hcol.data(), 2 * E * 4, hipMemcpyHostToDevice, stream));
    CC_HIP(hipMemcpyAsync(P->eid, heid.data(), 2 * E * 4, hipMemcpyHostToDevice, stream));
    CC_HIP(hipMemcpyAsync(P->epos, hposE.data(), 2 * E * 4, hipMemcpyHostToDevice, stream));
    CC_HIP(hipMemcpyAsync(P->ei, hi.data(), E * 4, hipMemcpyHostToDevice, stream));
    CC_HIP(hipMemcpyAsync(P->ej, hj.data(), E * 4, hipMemcpyHostToDevice, stream));
    CC_HIP(hipMemcpyAsync(P->w, hw.data(), E * 8, hipMemcpyHostToDevice, stream));
  }
  double w2 = 0.0;
  for (int64_t e = 0; e < E; ++e) w2 += hw[e] * hw[e];
  P->w2 = w2;

  // ---- column statistics and the initial state ----
  double *mean = nullptr, *dev2 = nullptr;
  int *bad = nullptr;
  CC_TRY(dmalloc((void **)&mean, p * 8));
  struct Tmp { void *a, *b, *c; ~Tmp() { if (a) (void)hipFree(a); if (b) (void)hipFree(b); if (c) (void)hipFree(c); } } tmp{mean, nullptr, nullptr};
  CC_TRY(dmalloc((void **)&dev2, p * 8));
  tmp.b = dev2;
  CC_TRY(dmalloc((void **)&bad, 4));
  tmp.c = bad;
  CC_HIP(hipMemsetAsync(bad, 0, 4, stream));
  const int cb = (int)cdiv(p, 256);
  if (x_dtype == CC_DTYPE_F32)
    hipLaunchKernelGGL((k_colstats<float>), dim3(cb), dim3(256), 0, stream, (int)n, (int)p,
                       (const float *)X, ldx, mask, ldm, mean, dev2, bad);
  else
    hipLaunchKernelGGL((k_colstats<double>), dim3(cb), dim3(256), 0, stream, (int)n, (int)p,
                       (const double *)X, ldx, mask, ldm, mean, dev2, bad);
  CC_HIP(hipGetLastError());
  std::vector<double> hdev2(p);
  int hbad = 0;
  CC_HIP(hipMemcpyAsync(hdev2.data(), dev2, p * 8, hipMemcpyDeviceToHost, stream));
  CC_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, stream));
  CC_HIP(hipStreamSynchronize(stream));
  if (hbad) { set_error("observed X has non-finite entries"); return CC_ERR_INVALID_ARG; }
  P->dev2 = std::accumulate(hdev2.begin(), hdev2.end(), 0.0);

  const int ib = (int)cdiv(nl, 256);
#define CC_INIT(PR, TI)                                                                    \
  hipLaunchKernelGGL((k_init_state<PR, TI>), dim3(ib), dim3(256), 0, stream, (int)n, (int)p, \
                     (int)P->ld, (const TI *)X, ldx, mask, ldm, mean, P->X, P->M, P->U,     \
                     P->A[0], P->G[0])
  if (x_dtype == CC_DTYPE_F32) {
    if (precision == kF32) CC_INIT(kF32, float);
    else if (precision == kF64) CC_INIT(kF64, float);
    else CC_INIT(kMixed, float);
  } else {
    if (precision == kF32) CC_INIT(kF32, double);
    else if (precision == kF64) CC_INIT(kF64, double);
    else CC_INIT(kMixed, double);
  }
#undef CC_INIT
  CC_HIP(hipGetLastError());
  CC_HIP(hipStreamSynchronize(stream));
  CC_TRY(reset_state(P));
  guard.ok = true;
  *out = P;
  return CC_OK;
}

// Back to the initial state U = A' = X-tilde, s = 1 (stored in buffer 0).
cc_status reset_state(Problem *P) {
  const size_t nl = (size_t)P->n * P->ld;
  const size_t bytes = nl * ts_size(P->precision);
  // U and A[0] are rebuilt from the stored X-tilde copy
  if (P->precision == kF64) {
    CC_HIP(hipMemcpyAsync(P->U, P->X, bytes, hipMemcpyDeviceToDevice, P->stream));
    CC_HIP(hipMemcpyAsync(P->A[0], P->X, bytes, hipMemcpyDeviceToDevice, P->stream));
  } else if (P->precision == kF32) {
    CC_HIP(hipMemcpyAsync(P->U, P->X, bytes, hipMemcpyDeviceToDevice, P->stream));
    CC_HIP(hipMemcpyAsync(P->A[0], P->X, bytes, hipMemcpyDeviceToDevice, P->stream));
  } else {
    const int b = (int)cdiv(nl, 256);
    hipLaunchKernelGGL((k_copy_rows<float, double>), dim3(b), dim3(256), 0, P->stream,
                       (int)P->n, (int)P->ld, (const float *)P->X, (int)P->ld, (double *)P->U,
                       (int64_t)P->ld);
    // A = X-tilde as hi + lo: the entries are FP32 values, so lo = 0
    CC_HIP(hipMemsetAsync(P->A[0], 0, nl * ta_size(P->precision), P->stream));
    CC_HIP(hipMemcpyAsync(P->G[0], P->X, nl * 4, hipMemcpyDeviceToDevice, P->stream));
  }
  if (P->E > 0) {
    hipLaunchKernelGGL(k_fill, dim3((int)cdiv(P->E, 256)), dim3(256), 0, P->stream, P->s,
                       P->E, 1.0);
  }
  P->slot = 0;
  hipLaunchKernelGGL(k_reset_scalars, dim3(1), dim3(1), 0, P->stream, P->sc);
  CC_HIP(hipGetLastError());
  launch_edge_init(P);
  CC_HIP(hipGetLastError());
  CC_HIP(hipStreamSynchronize(P->stream));
  P->state_valid = true;
  return CC_OK;
}

static cc_status read_scalars(Problem *P) {
  CC_HIP(hipMemcpyAsync(P->sc_host, P->sc + P->slot, sizeof(DevScalars), hipMemcpyDeviceToHost, P->stream));
  CC_HIP(hipStreamSynchronize(P->stream));
  return CC_OK;
}

// rho, eps and the stop threshold tol * eta of a solve at gamma (eta the
// effective sqrt(eps) / rho when eps is given).
static void solve_constants(const Problem *P, double gamma, const cc_solve_opts &o, double *rho,
                            double *eps, double *thr) {
  double r = o.rho > 0 ? o.rho : 2.0 * std::sqrt(P->dev2 + gamma * gamma * P->w2);
  if (!(r > 0.0)) r = 1.0;
  const double e = o.eps > 0 ? o.eps : (o.eta * r) * (o.eta * r);
  const double eta = std::sqrt(e) / r;
  *rho = r;
  *eps = e;
  *thr = o.tol > 0 ? o.tol * eta : 0.0;
}

// Offsets of the missing entries of each (point, tile) work item at the
// current tile width, in item order, and the side array they index.
static cc_status build_miss_index(Problem *P) {
  if (P->moff) (void)hipFree(P->moff);
  if (P->Umiss) (void)hipFree(P->Umiss);
  P->moff = nullptr;
  P->Umiss = nullptr;
  P->n_miss = 0;
  const int64_t n = P->n, ld = P->ld, W = (int64_t)kWave * P->vec, nt = P->ntile;
  std::vector<uint8_t> m((size_t)(n * ld));
  CC_HIP(hipMemcpyAsync(m.data(), P->M, m.size(), hipMemcpyDeviceToHost, P->stream));
  CC_HIP(hipStreamSynchronize(P->stream));
  std::vector<int32_t> off((size_t)(n * nt + 1));
  int64_t tot = 0;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t f1 = std::min(ld, (t + 1) * W);
    for (int64_t i = 0; i < n; ++i) {
      off[(size_t)(t * n + i)] = (int32_t)tot;
      const uint8_t *r = m.data() + i * ld;
      for (int64_t f = t * W; f < f1; ++f) tot += r[f] == 0;
      if (tot > INT32_MAX) { set_error("too many missing entries for the lazy U index"); return CC_ERR_INVALID_ARG; }
    }
  }
  off[(size_t)(n * nt)] = (int32_t)tot;
  CC_TRY(dmalloc((void **)&P->moff, off.size() * 4));
  CC_TRY(dmalloc(&P->Umiss, (size_t)std::max<int64_t>(tot, 1) * ts_size(P->precision)));
  CC_HIP(hipMemcpyAsync(P->moff, off.data(), off.size() * 4, hipMemcpyHostToDevice, P->stream));
  CC_HIP(hipStreamSynchronize(P->stream));  // the host vector goes out of scope
  P->n_miss = tot;
  P->moff_vec = P->vec;
  return CC_OK;
}

cc_status solve(Problem *P, double gamma, const cc_solve_opts &o, cc_solve_info *info) {
  if (!(gamma >= 0.0) || !std::isfinite(gamma)) { set_error("gamma must be finite and >= 0"); return CC_ERR_INVALID_ARG; }
  if (o.max_iter < 1) { set_error("max_iter must be >= 1"); return CC_ERR_INVALID_ARG; }
  if (o.test_every < 1) { set_error("test_every must be >= 1"); return CC_ERR_INVALID_ARG; }
  if (!(o.tol >= 0.0)) { set_error("tol must be >= 0"); return CC_ERR_INVALID_ARG; }
  if (!(o.eta > 0.0) && !(o.eps > 0.0)) { set_error("need eta > 0 or eps > 0"); return CC_ERR_INVALID_ARG; }
  if (o.proj_sweeps < 1 || o.proj_sweeps > kMaxProjSweeps) {
    set_error("proj_sweeps must be in 1.." + std::to_string(kMaxProjSweeps));
    return CC_ERR_INVALID_ARG;
  }
  if (o.proj_sweeps > 1 && P->slab_f > 0) {
    set_error("proj_sweeps > 1 needs the wave point sweep (not the LDS-slab option)");
    return CC_ERR_INVALID_ARG;
  }
  if (o.proj_sweeps > 1 && !P->H) {
    const size_t nl = (size_t)P->n * P->ld;
    CC_TRY(dmalloc((void **)&P->H, nl * 8));
    CC_TRY(dmalloc(&P->T[0], nl * tg_size(P->precision)));
    CC_TRY(dmalloc(&P->T[1], nl * tg_size(P->precision)));
  }
  P->psweeps = o.proj_sweeps;
  // U stored lazily by the wave point sweep with one projection sweep.
  // With missing data the sweep then reads and writes a side array at
  // dependent offsets, which pays only where waves take several items (the
  // sweep streams bytes); waves with one item wait on latency, not bytes.
  // CCMI_LAZY_U: 0 never, 2 always, else that rule.
  const char *lz = getenv("CCMI_LAZY_U");
  const int lzmode = lz ? atoi(lz) : 1;
  P->lazy_u = P->psweeps == 1 && P->slab_f == 0 && lzmode != 0 &&
              (!P->M || lzmode == 2 || point_grid(P).chunk > point_waves(P));
  if (P->lazy_u && P->M && (!P->moff || P->moff_vec != P->vec)) {
    if (build_miss_index(P) != CC_OK) P->lazy_u = false;  // store U every iteration
  }
  const auto t0 = std::chrono::steady_clock::now();
  if (!o.warm_start || !P->state_valid) CC_TRY(reset_state(P));
  double rho, eps, thr;
  solve_constants(P, gamma, o, &rho, &eps, &thr);
  P->cur_K = o.test_every;
  if (o.record_objective) {
    const int64_t need = (int64_t)o.max_iter + 2;
    if (P->trace_cap < need) {
      if (P->trace) (void)hipFree(P->trace);
      P->trace = nullptr;
      P->trace_cap = 0;
      CC_TRY(dmalloc((void **)&P->trace, need * 8));
      P->trace_cap = need;
    }
  }
  const int record = o.record_objective ? 1 : 0;
  hipLaunchKernelGGL(k_set_params, dim3(1), dim3(1), 0, P->stream, P->sc + P->slot, gamma, rho,
                     eps, thr, o.max_iter, record, o.test_every);
  CC_HIP(hipGetLastError());
  const int check = std::max(1, o.check_every);
  // sweeps m = 0 .. max_iter, each finished by the next launch pair; the
  // last pair only finishes (the stop rule ends the solve by then)
  const int64_t last = (int64_t)o.max_iter + 1;
  for (int64_t it = 0; it <= last; ++it) {
    launch_iteration(P);
    if ((it + 1) % check == 0 || it == last) {
      CC_HIP(hipGetLastError());
      CC_HIP(hipMemcpyAsync(P->flag_host, &P->sc[P->slot].done, 4, hipMemcpyDeviceToHost, P->stream));
      CC_HIP(hipStreamSynchronize(P->stream));
      if (P->prof_used) harvest_profile(P);
      if (P->flag_host[0]) break;
    }
  }
  if (P->lazy_u) {
    launch_u_finish(P);
    CC_HIP(hipGetLastError());
  }
  CC_TRY(read_scalars(P));
  const DevScalars &h = *P->sc_host;
  P->trace_count = record ? h.iters : 0;
  cc_status st = h.status == 0 ? CC_OK : (cc_status)h.status;
  if (!h.done) { set_error("solver did not finish"); st = CC_ERR_STATE; }
  if (st == CC_ERR_NUMERIC) {
    set_error("d or the objective became non-finite");
    P->state_valid = false;
  }
  if (info) {
    info->iters = h.iters;
    info->converged = h.converged;
    info->status = st;
    info->gamma = gamma;
    info->objective = h.F_last;
    info->d = h.d_last;
    info->rel_change = h.rel_last;
    info->rho = rho;
    info->eps = eps;
    info->n_clusters = 0;
    if (st == CC_OK) {
      int32_t ncl = 0;
      // labels of the final state into scratch space reused from part
      int32_t *lab = nullptr;
      CC_TRY(dmalloc((void **)&lab, P->n * 4));
      cc_status ls = write_labels(P, lab, &ncl);
      (void)hipFree(lab);
      if (ls != CC_OK) return ls;
      info->n_clusters = ncl;
    }
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

cc_status components(int64_t n, int64_t E, const int32_t *ei, const int32_t *ej,
                     const uint8_t *keep, const double *s, int32_t *labels,
                     int32_t *ncl_dev, hipStream_t stream) {
  hipLaunchKernelGGL(k_components, dim3(1), dim3(1024), 0, stream, (int)n, (int)E, ei, ej, keep,
                     s, labels, ncl_dev);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

cc_status write_labels(Problem *P, int32_t *labels, int32_t *ncl_host) {
  CC_TRY(components(P->n, P->E, P->ei, P->ej, nullptr, P->s, labels, P->ncl_dev, P->stream));
  if (ncl_host) {
    CC_HIP(hipMemcpyAsync(P->flag_host, P->ncl_dev, 4, hipMemcpyDeviceToHost, P->stream));
    CC_HIP(hipStreamSynchronize(P->stream));
    *ncl_host = P->flag_host[0];
  }
  return CC_OK;
}

cc_status copy_U(Problem *P, int32_t out_dtype, void *dst, int64_t ldu) {
  const size_t np = (size_t)P->n * P->p;
  const int b = (int)cdiv(np, 256);
  if (P->precision == kF32) {
    if (out_dtype == CC_DTYPE_F32)
      hipLaunchKernelGGL((k_copy_rows<float, float>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const float *)P->U, (int)P->ld, (float *)dst, ldu);
    else
      hipLaunchKernelGGL((k_copy_rows<float, double>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const float *)P->U, (int)P->ld, (double *)dst, ldu);
  } else {
    if (out_dtype == CC_DTYPE_F32)
      hipLaunchKernelGGL((k_copy_rows<double, float>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const double *)P->U, (int)P->ld, (float *)dst, ldu);
    else
      hipLaunchKernelGGL((k_copy_rows<double, double>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const double *)P->U, (int)P->ld, (double *)dst, ldu);
  }
  CC_HIP(hipGetLastError());
  return CC_OK;
}

cc_status get_fused(Problem *P, uint8_t *fused) {
  if (P->E == 0) return CC_OK;
  hipLaunchKernelGGL(k_fused_flags, dim3((int)cdiv(P->E, 256)), dim3(256), 0, P->stream,
                     (int)P->E, P->s, fused);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

cc_status set_state(Problem *P, const double *U, const double *A, int64_t ld, const double *s) {
  // the state goes to buffer 0 (pa = 0 after the scalar reset)
  const size_t nl = (size_t)P->n * P->ld;
  const int b = (int)cdiv(nl, 256);
  if (P->precision == kF32)
    hipLaunchKernelGGL((k_set_rows<kF32>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (int)P->ld, U, A, ld, P->U, P->A[0], P->G[0]);
  else if (P->precision == kF64)
    hipLaunchKernelGGL((k_set_rows<kF64>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (int)P->ld, U, A, ld, P->U, P->A[0], P->G[0]);
  else
    hipLaunchKernelGGL((k_set_rows<kMixed>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (int)P->ld, U, A, ld, P->U, P->A[0], P->G[0]);
  if (P->E > 0) CC_HIP(hipMemcpyAsync(P->s, s, P->E * 8, hipMemcpyDeviceToDevice, P->stream));
  P->slot = 0;
  hipLaunchKernelGGL(k_reset_scalars, dim3(1), dim3(1), 0, P->stream, P->sc);
  CC_HIP(hipGetLastError());
  launch_edge_init(P);
  CC_HIP(hipGetLastError());
  CC_HIP(hipStreamSynchronize(P->stream));
  P->state_valid = true;
  return CC_OK;
}

cc_status get_state(Problem *P, double *U, double *A, int64_t ld, double *s) {
  CC_TRY(read_scalars(P));
  const int pa = P->sc_host->pa;
  const size_t np = (size_t)P->n * P->p;
  const int b = (int)cdiv(np, 256);
  if (P->precision == kF32) {
    hipLaunchKernelGGL((k_copy_rows<float, double>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const float *)P->U, (int)P->ld, U, ld);
    hipLaunchKernelGGL((k_copy_rows<float, double>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const float *)P->A[pa], (int)P->ld, A, ld);
  } else {
    hipLaunchKernelGGL((k_copy_rows<double, double>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const double *)P->U, (int)P->ld, U, ld);
    if (P->precision == kMixed)
      hipLaunchKernelGGL(k_get_hilo, dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const float *)P->G[pa], (const float *)P->A[pa], (int)P->ld, A, ld);
    else
      hipLaunchKernelGGL((k_copy_rows<double, double>), dim3(b), dim3(256), 0, P->stream, (int)P->n, (int)P->p, (const double *)P->A[pa], (int)P->ld, A, ld);
  }
  if (P->E > 0) CC_HIP(hipMemcpyAsync(s, P->s, P->E * 8, hipMemcpyDeviceToDevice, P->stream));
  CC_HIP(hipGetLastError());
  return CC_OK;
}


// ============================================================ batched solves
// Instances advance together: per MM iteration one point-sweep launch and
// one edge-sweep launch cover every instance (a block table maps each block
// to an instance and its local block); each instance keeps its own scalars,
// partial rows and stop rule and moves along its own gamma path on the
// device.  Graph replays of graph_iters iterations run until every path is
// done.

// Slot 0 of every instance: the first gamma of its path (the state and its
// buffer index pa stay, as for a warm-started solve).
__global__ void k_batch_init(int n_inst, const BatchInst *bi, int max_iter, int K,
                             unsigned long long *ticks, int *n_finished) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) {
    ticks[0] = wall_clock64();
    *n_finished = 0;
  }
  if (b >= n_inst) return;
  DevScalars *sc = bi[b].sc0;
  sc->mu = bi[b].mu[0]; sc->rho = bi[b].rho[0]; sc->eps = bi[b].eps[0]; sc->thr = bi[b].thr[0];
  sc->max_iter = max_iter; sc->record = 0; sc->K = K;
  sc->m = 0; sc->done = 0; sc->converged = 0; sc->status = 0; sc->iters = 0;
  sc->d_prev = 0.0; sc->dA_prev = 0.0; sc->F_cur = 0.0;
  sc->F_last = 0.0; sc->d_last = 0.0; sc->rel_last = 0.0;
  sc->pending = 0; sc->path_k = 0; sc->finished = 0;
}

__global__ void k_batch_done_ticks(int n_inst, const BatchInst *bi, unsigned long long *out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_inst) out[b] = *bi[b].t_done;
}

template <int PREC>
static void launch_point_class(const PointClass &c, int par, hipStream_t st) {
  const dim3 g(c.nblk), t(kPointBlock);
  if (c.ipw > 1) {
    switch (c.vec) {
      case 1: hipLaunchKernelGGL((k_point_batch<PREC, 1, true>), g, t, 0, st, c.pargs[par], c.ptab); break;
      case 2: hipLaunchKernelGGL((k_point_batch<PREC, 2, true>), g, t, 0, st, c.pargs[par], c.ptab); break;
      default: hipLaunchKernelGGL((k_point_batch<PREC, 4, true>), g, t, 0, st, c.pargs[par], c.ptab); break;
    }
  } else {
    switch (c.vec) {
      case 1: hipLaunchKernelGGL((k_point_batch<PREC, 1, false>), g, t, 0, st, c.pargs[par], c.ptab); break;
      case 2: hipLaunchKernelGGL((k_point_batch<PREC, 2, false>), g, t, 0, st, c.pargs[par], c.ptab); break;
      default: hipLaunchKernelGGL((k_point_batch<PREC, 4, false>), g, t, 0, st, c.pargs[par], c.ptab); break;
    }
  }
}

template <int PREC>
static void launch_edge_class(const EdgeClass &c, int par, hipStream_t s) {
  const dim3 g(c.nblk), t(kEdgeBlock);
  switch (c.nv) {
    case 1: hipLaunchKernelGGL((k_edge_items_batch<PREC, 1>), g, t, 0, s, c.eargs[par], c.etab); break;
    case 2: hipLaunchKernelGGL((k_edge_items_batch<PREC, 2>), g, t, 0, s, c.eargs[par], c.etab); break;
    case 4: hipLaunchKernelGGL((k_edge_items_batch<PREC, 4>), g, t, 0, s, c.eargs[par], c.etab); break;
    case 8: hipLaunchKernelGGL((k_edge_items_batch<PREC, 8>), g, t, 0, s, c.eargs[par], c.etab); break;
    default: hipLaunchKernelGGL((k_edge_items_batch<PREC, 16>), g, t, 0, s, c.eargs[par], c.etab); break;
  }
}

// Launches of one class list; with side streams and events (graph capture)
// the classes after the first run on their own streams as parallel branches
// forked from and joined back into st (they cover disjoint instances).
template <typename Cls, typename Fn>
static void launch_branches(const std::vector<Cls> &cls, hipStream_t st, const hipStream_t *side,
                            const hipEvent_t *ev, Fn launch) {
  const int nc = (int)cls.size();
  if (side && nc > 1) (void)hipEventRecord(ev[0], st);
  for (int k = 0; k < nc; ++k) {
    hipStream_t s = st;
    if (side && k > 0) {
      s = side[k - 1];
      (void)hipStreamWaitEvent(s, ev[0], 0);
    }
    launch(cls[k], s);
    if (side && k > 0) (void)hipEventRecord(ev[k], s);
  }
  if (side)
    for (int k = 1; k < nc; ++k) (void)hipStreamWaitEvent(st, ev[k], 0);
}

// One iteration of a launch set: every point class, then every edge class.
template <int PREC>
static void launch_set_p(const LaunchSet &L, int par, hipStream_t st, const hipStream_t *side,
                         const hipEvent_t *ev) {
  launch_branches(L.pcls, st, side, ev, [&](const PointClass &c, hipStream_t s) {
    if (c.nblk > 0) launch_point_class<PREC>(c, par, s);
  });
  launch_branches(L.ecls, st, side, ev, [&](const EdgeClass &c, hipStream_t s) {
    launch_edge_class<PREC>(c, par, s);
  });
}

// One MM iteration of every problem of the set (scalar-slot parity par).
static void launch_set_iteration(const LaunchSet &L, int prec, int par, hipStream_t st,
                                 const hipStream_t *side = nullptr, const hipEvent_t *ev = nullptr) {
  if (prec == kF32) launch_set_p<kF32>(L, par, st, side, ev);
  else if (prec == kF64) launch_set_p<kF64>(L, par, st, side, ev);
  else launch_set_p<kMixed>(L, par, st, side, ev);
}

template <typename T>
static cc_status upload(T **dst, const std::vector<T> &v, hipStream_t st) {
  if (*dst) (void)hipFree(*dst);
  *dst = nullptr;
  CC_TRY(dmalloc((void **)dst, std::max<size_t>(v.size(), 1) * sizeof(T)));
  if (!v.empty()) CC_HIP(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return CC_OK;
}

static void free_launch_set(LaunchSet &L) {
  for (PointClass &c : L.pcls) {
    void *pb[] = {c.pargs[0], c.pargs[1], c.ptab};
    for (void *b : pb)
      if (b) (void)hipFree(b);
  }
  for (EdgeClass &c : L.ecls) {
    void *eb[] = {c.eargs[0], c.eargs[1], c.etab};
    for (void *b : eb)
      if (b) (void)hipFree(b);
  }
  L = LaunchSet();
}

// Launch tables for problems probs[k] (device descriptors bis[k]), blocks
// laid out in the given order of instances: instance k gets tile shape
// vec_of[k] (64 * vec features per wave) and about ipw_of[k] items per wave
// (waves with several items prefetch the next); point launches are grouped
// by (vec, ipw), edge launches by each instance's features per lane.  Sets
// the problems' tile fields and scalar slot 0.
constexpr int kBatchEdgeItems = 4;  // items per wave of the batched item edge sweep

static cc_status build_launch_set(LaunchSet &L, const std::vector<Problem *> &probs,
                                  const std::vector<const BatchInst *> &bis,
                                  const std::vector<int> &order, const std::vector<int> &vec_of,
                                  const std::vector<int> &ipw_of, int K, hipStream_t st) {
  free_launch_set(L);
  const int n_inst = (int)probs.size();
  std::vector<PointArgs> pa[2];
  std::vector<EdgeArgs> ea[2];
  std::vector<int> pblocks(n_inst), eblocks(n_inst);
  for (int b = 0; b < n_inst; ++b) {
    Problem *P = probs[b];
    P->vec = vec_of[b];
    P->tile_w = kWave * P->vec;
    P->ntile = (int)cdiv(P->ld, P->tile_w);
    P->cur_K = K;
    P->ipw = ipw_of[b];
    // the item edge sweep takes kBatchEdgeItems items per wave whatever the
    // point sweep's choice (measured: 4 against 1 and 16, and against
    // following the point sweep)
    P->eipw = kBatchEdgeItems;
    P->nbe = edge_rows(P);
    const Launch Lp = sweep_grid(P->n * P->ntile, kPointWaves, P->ipw);
    const Launch Li = edge_items_grid(P->n_items, P->eipw);
    pblocks[b] = Lp.blocks;
    eblocks[b] = Li.blocks;
    for (int par = 0; par < 2; ++par) {
      P->slot = par;
      PointArgs x = point_args(P, Lp);
      x.bi = bis[b];
      x.lazy = 0;  // batched sweeps store U every iteration
      pa[par].push_back(x);
      P->slot = par ^ 1;
      ea[par].push_back(edge_args(P, Li, 0, Lp.blocks));
    }
    P->slot = 0;
  }
  // point classes in order of first appearance along the instance order
  std::vector<std::pair<int, int>> keys;
  for (int b : order) {
    const std::pair<int, int> k{vec_of[b], ipw_of[b]};
    if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
  }
  for (const auto &k : keys) {
    std::vector<int2> pt;
    for (int b : order)
      if (vec_of[b] == k.first && ipw_of[b] == k.second)
        for (int q = 0; q < pblocks[b]; ++q) pt.push_back(make_int2(b, q));
    PointClass c;
    c.vec = k.first;
    c.ipw = k.second;
    c.nblk = (int)pt.size();
    for (int par = 0; par < 2; ++par) CC_TRY(upload(&c.pargs[par], pa[par], st));
    CC_TRY(upload(&c.ptab, pt, st));
    L.pcls.push_back(c);
  }
  for (int nv : {1, 2, 4, 8, 16}) {
    std::vector<int2> et;
    for (int b : order)
      if (probs[b]->item_nv == nv)
        for (int q = 0; q < eblocks[b]; ++q) et.push_back(make_int2(b, q));
    if (et.empty()) continue;
    EdgeClass c;
    c.nv = nv;
    c.nblk = (int)et.size();
    for (int par = 0; par < 2; ++par) CC_TRY(upload(&c.eargs[par], ea[par], st));
    CC_TRY(upload(&c.etab, et, st));
    L.ecls.push_back(c);
  }
  CC_HIP(hipStreamSynchronize(st));
  return CC_OK;
}

// Launch tables and the graph of graph_iters iterations for the instances'
// tile shapes (inst_vec, inst_ipw), over the given instances (default all).
static cc_status batch_configure(Batch *B, const std::vector<int> *order = nullptr) {
  std::vector<const BatchInst *> bis;
  for (size_t b = 0; b < B->probs.size(); ++b) bis.push_back(B->bi + b);
  CC_TRY(build_launch_set(B->ls, B->probs, bis, order ? *order : B->order, B->inst_vec, B->inst_ipw,
                          B->opts.test_every, B->stream));
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->gexec = nullptr;
  B->graph = nullptr;
  const size_t nc = std::max(B->ls.ecls.size(), B->ls.pcls.size());
  while (B->side.size() + 1 < nc) {
    hipStream_t s;
    CC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    B->side.push_back(s);
  }
  while (B->ev.size() < std::max<size_t>(nc, 1)) {
    hipEvent_t e;
    CC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    B->ev.push_back(e);
  }
  CC_HIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
  for (int it = 0; it < B->graph_iters; ++it)
    launch_set_iteration(B->ls, B->precision, it & 1, B->stream, B->side.data(), B->ev.data());
  CC_HIP(hipStreamEndCapture(B->stream, &B->graph));
  CC_HIP(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
  return CC_OK;
}

// Every instance to scalar slot 0 with the first gamma of its path.
static cc_status batch_start(Batch *B) {
  for (Problem *P : B->probs) {
    CC_HIP(hipStreamSynchronize(P->stream));
    if (P->slot != 0) {
      CC_HIP(hipMemcpyAsync(P->sc, P->sc + 1, sizeof(DevScalars), hipMemcpyDeviceToDevice, B->stream));
      P->slot = 0;
    }
  }
  const int n_inst = (int)B->probs.size();
  hipLaunchKernelGGL(k_batch_init, dim3((int)cdiv(n_inst, 256)), dim3(256), 0, B->stream, n_inst,
                     (const BatchInst *)B->bi, B->opts.max_iter, B->opts.test_every, B->ticks,
                     B->n_finished);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// Autotuner candidates: (vec, items per wave) = (1,1), (1,4), (1,16), (2,1), ...
constexpr int kTuneConfigs = 9;
// Features per lane of a batched point sweep without tuning: the whole row
// in one wave where it fits.
static int natural_vec(int64_t ld) { return ld > 128 ? 4 : (ld > 64 ? 2 : 1); }
static int tune_vec(int c) { return 1 << (c / 3); }
static int tune_ipw(int c) { return c % 3 == 0 ? 1 : (c % 3 == 1 ? 4 : 16); }

static cc_status check_opts(const cc_solve_opts &o) {
  if (o.proj_sweeps != 1) { set_error("batched and served solves run one projection sweep per MM iteration (proj_sweeps = 1)"); return CC_ERR_INVALID_ARG; }
  if (o.max_iter < 1) { set_error("max_iter must be >= 1"); return CC_ERR_INVALID_ARG; }
  if (o.test_every < 1) { set_error("test_every must be >= 1"); return CC_ERR_INVALID_ARG; }
  if (!(o.tol >= 0.0)) { set_error("tol must be >= 0"); return CC_ERR_INVALID_ARG; }
  if (!(o.eta > 0.0) && !(o.eps > 0.0)) { set_error("need eta > 0 or eps > 0"); return CC_ERR_INVALID_ARG; }
  return CC_OK;
}

void batch_free(Batch *B) {
  if (!B) return;
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  free_launch_set(B->ls);
  void *bufs[] = {B->bi, B->gconst, B->fused, B->info, B->ticks, B->n_finished, B->ncl};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (B->fin_host) (void)hipHostFree(B->fin_host);
  if (B->stream) (void)hipStreamDestroy(B->stream);
  for (hipStream_t s : B->side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : B->ev) (void)hipEventDestroy(e);
  delete B;
}

// Runs the batch from the instances' current states; returns us per MM
// iteration over `iters` iterations (graph replays).
static cc_status batch_time(Batch *B, int replays, double *us) {
  CC_TRY(batch_start(B));
  hipEvent_t e0, e1;
  CC_HIP(hipEventCreate(&e0));
  CC_HIP(hipEventCreate(&e1));
  CC_HIP(hipGraphLaunch(B->gexec, B->stream));  // warm-up
  CC_HIP(hipEventRecord(e0, B->stream));
  for (int r = 0; r < replays; ++r) CC_HIP(hipGraphLaunch(B->gexec, B->stream));
  CC_HIP(hipEventRecord(e1, B->stream));
  CC_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  CC_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us = 1e3 * ms / ((double)replays * B->graph_iters);
  return CC_OK;
}

cc_status batch_create(int32_t n_inst, Problem *const *probs, const int32_t *n_gamma,
                       const double *gammas, const cc_solve_opts &o, int32_t autotune,
                       Batch **out) {
  if (!out) { set_error("out is NULL"); return CC_ERR_INVALID_ARG; }
  *out = nullptr;
  if (n_inst < 1 || !probs || !n_gamma || !gammas) { set_error("need n_inst >= 1 and non-NULL arrays"); return CC_ERR_INVALID_ARG; }
  CC_TRY(check_opts(o));
  int64_t total = 0;
  for (int b = 0; b < n_inst; ++b) {
    const Problem *P = probs[b];
    if (!P) { set_error("problem " + std::to_string(b) + " is NULL"); return CC_ERR_INVALID_ARG; }
    if (P->precision != probs[0]->precision) { set_error("all problems of a batch need the same precision"); return CC_ERR_INVALID_ARG; }
    if (!P->eitems || P->slab_f > 0) {
      set_error("problem " + std::to_string(b) + ": rows wider than a batched sweep takes (p <= 1024)");
      return CC_ERR_INVALID_ARG;
    }
    if (n_gamma[b] < 1) { set_error("every instance needs at least one gamma"); return CC_ERR_INVALID_ARG; }
    for (int b2 = 0; b2 < b; ++b2)
      if (probs[b2] == P) { set_error("a problem appears twice in the batch"); return CC_ERR_INVALID_ARG; }
    total += n_gamma[b];
  }
  for (int64_t k = 0; k < total; ++k)
    if (!(gammas[k] >= 0.0) || !std::isfinite(gammas[k])) { set_error("gammas must be finite and >= 0"); return CC_ERR_INVALID_ARG; }

  Batch *B = new (std::nothrow) Batch();
  if (!B) { set_error("host allocation failed"); return CC_ERR_OUT_OF_MEMORY; }
  struct Guard { Batch *&B; bool ok = false; ~Guard() { if (!ok) batch_free(B); } } guard{B};
  B->probs.assign(probs, probs + n_inst);
  B->precision = probs[0]->precision;
  B->opts = o;
  B->n_gamma.assign(n_gamma, n_gamma + n_inst);
  B->total_gamma = total;
  CC_HIP(hipStreamCreate(&B->stream));
  int dev = 0, khz = 0;
  CC_HIP(hipGetDevice(&dev));
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
    B->tick_khz = khz;

  // per-(instance, gamma) constants, computed as a single solve does
  std::vector<double> hmu(total), hrho(total), heps(total), hthr(total);
  B->goff.resize(n_inst);
  B->foff.resize(n_inst);
  int64_t g = 0, f = 0;
  for (int b = 0; b < n_inst; ++b) {
    B->goff[b] = g;
    B->foff[b] = f;
    for (int k = 0; k < n_gamma[b]; ++k, ++g) {
      hmu[g] = gammas[g];
      solve_constants(probs[b], gammas[g], o, &hrho[g], &heps[g], &hthr[g]);
    }
    f += (int64_t)n_gamma[b] * probs[b]->E;
  }
  B->total_fused = f;
  B->gammas = hmu;
  B->rho = hrho;
  B->eps = heps;
  std::vector<double> gc;
  gc.insert(gc.end(), hmu.begin(), hmu.end());
  gc.insert(gc.end(), hrho.begin(), hrho.end());
  gc.insert(gc.end(), heps.begin(), heps.end());
  gc.insert(gc.end(), hthr.begin(), hthr.end());
  CC_TRY(upload(&B->gconst, gc, B->stream));
  CC_TRY(dmalloc((void **)&B->fused, std::max<int64_t>(f, 1)));
  CC_TRY(dmalloc((void **)&B->info, total * kInfoVals * 8));
  CC_TRY(dmalloc((void **)&B->ticks, (1 + 2 * (size_t)n_inst) * 8));
  CC_TRY(dmalloc((void **)&B->n_finished, 4));
  CC_TRY(dmalloc((void **)&B->ncl, total * 4));
  CC_HIP(hipHostMalloc((void **)&B->fin_host, 64, hipHostMallocDefault));
  std::vector<BatchInst> bis(n_inst);
  for (int b = 0; b < n_inst; ++b) {
    const int64_t g0 = B->goff[b];
    Problem *P = probs[b];
    bis[b] = BatchInst{n_gamma[b], (int)P->E, P->sc, B->gconst + g0, B->gconst + total + g0,
                       B->gconst + 2 * total + g0, B->gconst + 3 * total + g0, P->s,
                       B->fused + B->foff[b], B->info + g0 * kInfoVals, B->ticks + 1 + n_inst + b,
                       B->n_finished};
  }
  CC_TRY(upload(&B->bi, bis, B->stream));
  // bigger instances first in the block tables
  B->order.resize(n_inst);
  std::iota(B->order.begin(), B->order.end(), 0);
  std::stable_sort(B->order.begin(), B->order.end(), [&](int a, int b) {
    return probs[a]->n * probs[a]->ld + 2 * probs[a]->E * probs[a]->ld >
           probs[b]->n * probs[b]->ld + 2 * probs[b]->E * probs[b]->ld;
  });

  // the tile shape a single solve would take: 64 * vec features per wave
  // with vec from the row width, one item per wave
  B->inst_vec.resize(n_inst);
  B->inst_ipw.assign(n_inst, 1);
  B->inst_class.assign(n_inst, -1);
  for (int b = 0; b < n_inst; ++b) B->inst_vec[b] = natural_vec(probs[b]->ld);
  if (autotune) {
    // classes by row width and point-sweep work; per class, coordinate
    // descent over (vec, items per wave) in {1, 2, 4} x {1, 4, 16}: each
    // candidate is timed over a few graph replays of the whole batch from
    // the initial states, the others keeping their current choice; classes
    // with more work are tuned first
    std::vector<int> wsum;
    for (int b = 0; b < n_inst; ++b) {
      const Problem *P = probs[b];
      const int width = P->ld <= 64 ? 0 : (P->ld <= 128 ? 1 : (P->ld <= 256 ? 2 : 3));
      const int64_t items = P->n * cdiv(P->ld, kWave * B->inst_vec[b]);
      const int size = items <= 512 ? 0 : (items <= 2048 ? 1 : 2);
      int c = -1;
      for (size_t k = 0; k < B->classes.size(); ++k)
        if (B->classes[k].width == width && B->classes[k].size == size) c = (int)k;
      if (c < 0) {
        TuneClass tc;
        tc.width = width;
        tc.size = size;
        B->classes.push_back(tc);
        wsum.push_back(0);
        c = (int)B->classes.size() - 1;
      }
      B->classes[c].instances += 1;
      wsum[c] += (int)std::min<int64_t>(P->n * P->ld + 2 * P->E * P->ld, 1 << 30);
      B->inst_class[b] = c;
    }
    std::vector<int> cord(B->classes.size());
    std::iota(cord.begin(), cord.end(), 0);
    std::stable_sort(cord.begin(), cord.end(), [&](int a, int b) { return wsum[a] > wsum[b]; });
    for (int c : cord) {
      TuneClass &tc = B->classes[c];
      tc.tried.assign(kTuneConfigs, 0.0);
      double best = 1e300;
      int best_k = 0;
      for (int k = 0; k < kTuneConfigs; ++k) {
        for (int b = 0; b < n_inst; ++b)
          if (B->inst_class[b] == c) { B->inst_vec[b] = tune_vec(k); B->inst_ipw[b] = tune_ipw(k); }
        for (Problem *P : B->probs) CC_TRY(reset_state(P));
        CC_TRY(batch_configure(B));
        double us = 0.0;
        CC_TRY(batch_time(B, 2, &us));
        tc.tried[k] = us;
        if (us < best) { best = us; best_k = k; }
      }
      tc.vec = tune_vec(best_k);
      tc.ipw = tune_ipw(best_k);
      tc.us = best;
      for (int b = 0; b < n_inst; ++b)
        if (B->inst_class[b] == c) { B->inst_vec[b] = tc.vec; B->inst_ipw[b] = tc.ipw; }
    }
    for (Problem *P : B->probs) CC_TRY(reset_state(P));
  }
  CC_TRY(batch_configure(B));
  guard.ok = true;
  *out = B;
  return CC_OK;
}

// Path-finished flag of each instance, read from its scalar slot 0.
__global__ void k_gather_finished(int n, DevScalars *const *sc0, int *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = sc0[k]->finished;
}

cc_status batch_run(Batch *B, int32_t *labels, cc_solve_info *infos, double *latency_ms) {
  const int n_inst = (int)B->probs.size();
  CC_TRY(batch_start(B));
  // every path ends by its iteration caps: sum over its gammas of max_iter + 2
  int64_t budget = 0;
  for (int b = 0; b < n_inst; ++b)
    budget = std::max<int64_t>(budget, (int64_t)B->n_gamma[b] * ((int64_t)B->opts.max_iter + 2));
  const int64_t max_replays = cdiv(budget, B->graph_iters) + 2;
  // Compaction: once half of the instances in the current launch tables have
  // finished their paths, the tables and the graph are rebuilt over the
  // active ones (after a replay every instance is back on scalar slot 0), so
  // finished instances stop taking blocks.  Each instance's blocks do the
  // same work either way.
  struct Bufs {
    void *a = nullptr, *b = nullptr;
    ~Bufs() { if (a) (void)hipFree(a); if (b) (void)hipFree(b); }
  } tmp;
  CC_TRY(dmalloc(&tmp.a, (size_t)n_inst * 4));
  CC_TRY(dmalloc(&tmp.b, (size_t)n_inst * sizeof(DevScalars *)));
  int32_t *d_fin = (int32_t *)tmp.a;
  DevScalars **d_sc0 = (DevScalars **)tmp.b;
  std::vector<DevScalars *> hsc(n_inst);
  for (int b = 0; b < n_inst; ++b) hsc[b] = B->probs[b]->sc;
  CC_HIP(hipMemcpyAsync(d_sc0, hsc.data(), hsc.size() * sizeof(DevScalars *), hipMemcpyHostToDevice, B->stream));
  std::vector<int32_t> hfin(n_inst);
  int in_set = n_inst;
  bool finished = false, compacted = false;
  for (int64_t r = 0; r < max_replays; ++r) {
    CC_HIP(hipGraphLaunch(B->gexec, B->stream));
    CC_HIP(hipMemcpyAsync(B->fin_host, B->n_finished, 4, hipMemcpyDeviceToHost, B->stream));
    CC_HIP(hipStreamSynchronize(B->stream));
    const int done = B->fin_host[0];
    if (done >= n_inst) { finished = true; break; }
    if (n_inst - done <= in_set / 2) {
      hipLaunchKernelGGL(k_gather_finished, dim3((int)cdiv(n_inst, 256)), dim3(256), 0, B->stream, n_inst,
                         (DevScalars *const *)d_sc0, d_fin);
      CC_HIP(hipGetLastError());
      CC_HIP(hipMemcpyAsync(hfin.data(), d_fin, (size_t)n_inst * 4, hipMemcpyDeviceToHost, B->stream));
      CC_HIP(hipStreamSynchronize(B->stream));
      std::vector<int> active;
      for (int b : B->order)
        if (!hfin[b]) active.push_back(b);
      if (!active.empty()) {
        CC_TRY(batch_configure(B, &active));
        in_set = (int)active.size();
        compacted = true;
      }
    }
  }
  // the next run starts from the full tables
  if (compacted) CC_TRY(batch_configure(B));
  if (!finished) { set_error("batch did not finish within its iteration caps"); return CC_ERR_STATE; }
  // graph_iters is even: every instance is back on scalar slot 0
  std::vector<double> hinfo(B->total_gamma * kInfoVals);
  CC_HIP(hipMemcpyAsync(hinfo.data(), B->info, hinfo.size() * 8, hipMemcpyDeviceToHost, B->stream));
  std::vector<unsigned long long> ticks(1 + 2 * (size_t)n_inst);
  hipLaunchKernelGGL(k_batch_done_ticks, dim3((int)cdiv(n_inst, 256)), dim3(256), 0, B->stream, n_inst,
                     (const BatchInst *)B->bi, B->ticks + 1);
  CC_HIP(hipMemcpyAsync(ticks.data(), B->ticks, ticks.size() * 8, hipMemcpyDeviceToHost, B->stream));
  // labels of every (instance, gamma) from its recorded fusion flags
  int64_t loff = 0;
  for (int b = 0; b < n_inst; ++b) {
    Problem *P = B->probs[b];
    for (int k = 0; k < B->n_gamma[b]; ++k) {
      const int64_t gk = B->goff[b] + k;
      if (labels)
        CC_TRY(components(P->n, P->E, P->ei, P->ej, B->fused + B->foff[b] + (int64_t)k * P->E, nullptr,
                          labels + loff, B->ncl + gk, B->stream));
      loff += P->n;
    }
  }
  std::vector<int32_t> hncl(B->total_gamma, 0);
  if (labels) CC_HIP(hipMemcpyAsync(hncl.data(), B->ncl, hncl.size() * 4, hipMemcpyDeviceToHost, B->stream));
  CC_HIP(hipStreamSynchronize(B->stream));
  cc_status st = CC_OK;
  for (int b = 0; b < n_inst; ++b) {
    Problem *P = B->probs[b];
    for (int k = 0; k < B->n_gamma[b]; ++k) {
      const int64_t gk = B->goff[b] + k;
      const double *v = &hinfo[gk * kInfoVals];
      const int status = (int)v[2];
      if (status != 0) {
        st = (cc_status)status;
        set_error("instance " + std::to_string(b) + ": d or the objective became non-finite");
        P->state_valid = false;
      }
      if (infos) {
        cc_solve_info &in = infos[gk];
        in.iters = (int32_t)v[0];
        in.converged = (int32_t)v[1];
        in.n_clusters = hncl[gk];
        in.status = status;
        in.gamma = B->gammas[gk];
        in.objective = v[3];
        in.d = v[4];
        in.rel_change = v[5];
        in.rho = B->rho[gk];
        in.eps = B->eps[gk];
        in.seconds = (v[7] - (double)ticks[0]) / (B->tick_khz * 1e3);
      }
    }
    if (latency_ms) latency_ms[b] = (double)(ticks[1 + b] - ticks[0]) / B->tick_khz;
  }
  return st;
}


// ============================================================ served solves
// Requests wait on the host until the HBM budget admits them (first come,
// first served); an admitted request gets its kNN weights and problem on
// the device and joins the shared launches; rounds of round_iters MM
// iterations run every admitted request; a request whose path is done on
// the device leaves the launches, its result stays until released.

__global__ void k_inst_init(const BatchInst *bi, int max_iter, int K) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  DevScalars *sc = bi->sc0;
  sc->mu = bi->mu[0]; sc->rho = bi->rho[0]; sc->eps = bi->eps[0]; sc->thr = bi->thr[0];
  sc->max_iter = max_iter; sc->record = 0; sc->K = K;
  sc->m = 0; sc->done = 0; sc->converged = 0; sc->status = 0; sc->iters = 0;
  sc->d_prev = 0.0; sc->dA_prev = 0.0; sc->F_cur = 0.0;
  sc->F_last = 0.0; sc->d_last = 0.0; sc->rel_last = 0.0;
  sc->pending = 0; sc->path_k = 0; sc->finished = 0;
}

static double host_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device bytes a request will hold: the problem's arrays (edges bounded by
// n * k, neighbour lists by 2k per point on average) and the per-gamma
// outputs.
static int64_t request_bytes(int64_t n, int64_t p, int32_t k, bool mask, int precision, int64_t n_gamma) {
  const int64_t ld = (p + 3) / 4 * 4;
  const int64_t ts = precision == kF32 ? 4 : 8, tx = precision == kF64 ? 8 : 4;
  const int64_t tg = precision == kMixed ? 4 : 0, ta = precision == kF64 ? 8 : 4;
  const int64_t E = n * k;
  return n * ld * (tx + (mask ? 1 : 0) + 3 * ts + 2 * ta + 2 * tg) + E * (128 + n_gamma) + n * 2 * k * 16 +
         n_gamma * kInfoVals * 8 + (int64_t)kMaxBlocks * 64;
}

static void free_request_device(Request *R);

void server_free(Server *S) {
  if (!S) return;
  for (Request *R : S->all) {
    free_request_device(R);
    delete R;
  }
  free_launch_set(S->ls);
  void *bufs[] = {S->d_sc0, S->d_fin, S->n_finished};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (S->h_fin) (void)hipHostFree(S->h_fin);
  delete S;
}

cc_status server_create(int32_t precision, const cc_solve_opts &o, int64_t budget, int32_t max_active,
                        int32_t round_iters, hipStream_t stream, Server **out) {
  if (!out) { set_error("out is NULL"); return CC_ERR_INVALID_ARG; }
  *out = nullptr;
  if (precision != kF32 && precision != kMixed && precision != kF64) { set_error("unknown precision"); return CC_ERR_INVALID_ARG; }
  if (budget < 1) { set_error("need an HBM budget >= 1 byte"); return CC_ERR_INVALID_ARG; }
  if (max_active < 1 || max_active > 4096) { set_error("need 1 <= max_active <= 4096"); return CC_ERR_INVALID_ARG; }
  if (round_iters < 2 || round_iters % 2) { set_error("round_iters must be even and >= 2"); return CC_ERR_INVALID_ARG; }
  CC_TRY(check_opts(o));
  Server *S = new (std::nothrow) Server();
  if (!S) { set_error("host allocation failed"); return CC_ERR_OUT_OF_MEMORY; }
  struct Guard { Server *&S; bool ok = false; ~Guard() { if (!ok) server_free(S); } } guard{S};
  S->precision = precision;
  S->opts = o;
  S->budget = budget;
  S->max_active = max_active;
  S->round_iters = round_iters;
  S->stream = stream;
  CC_TRY(dmalloc((void **)&S->d_sc0, (size_t)max_active * sizeof(DevScalars *)));
  CC_TRY(dmalloc((void **)&S->d_fin, (size_t)max_active * 4));
  CC_TRY(dmalloc((void **)&S->n_finished, 4));
  CC_HIP(hipHostMalloc((void **)&S->h_fin, (size_t)max_active * 4, hipHostMallocDefault));
  S->t0 = host_seconds();
  guard.ok = true;
  *out = S;
  return CC_OK;
}

cc_status server_submit(Server *S, int64_t n, int64_t p, const float *X, const uint8_t *mask, int32_t k,
                        double phi, int32_t n_gamma, const double *gammas, int64_t *ticket) {
  if (n < 2 || p < 1 || !X) { set_error("need n >= 2, p >= 1 and X"); return CC_ERR_INVALID_ARG; }
  if ((p + 3) / 4 * 4 > 16 * kWave) { set_error("served requests take p <= 1024"); return CC_ERR_INVALID_ARG; }
  if (n > 16384) { set_error("served requests take n <= 16384"); return CC_ERR_INVALID_ARG; }
  if (k < 1 || k >= n) { set_error("need 1 <= k < n"); return CC_ERR_INVALID_ARG; }
  if (!std::isfinite(phi)) { set_error("phi must be finite"); return CC_ERR_INVALID_ARG; }
  if (n_gamma < 1 || !gammas) { set_error("need at least one gamma"); return CC_ERR_INVALID_ARG; }
  for (int32_t g = 0; g < n_gamma; ++g)
    if (!(gammas[g] >= 0.0) || !std::isfinite(gammas[g])) { set_error("gammas must be finite and >= 0"); return CC_ERR_INVALID_ARG; }
  Request *R = new (std::nothrow) Request();
  if (!R) { set_error("host allocation failed"); return CC_ERR_OUT_OF_MEMORY; }
  R->ticket = S->next_ticket++;
  R->state = CC_REQ_WAITING;
  R->n = n;
  R->p = p;
  R->k = k;
  R->phi = phi;
  R->X.assign(X, X + n * p);
  if (mask) R->mask.assign(mask, mask + n * p);
  R->gammas.assign(gammas, gammas + n_gamma);
  R->footprint = request_bytes(n, p, k, mask != nullptr, S->precision, n_gamma);
  R->t_submit = host_seconds() - S->t0;
  S->waiting.push_back(R);
  S->all.push_back(R);
  if (ticket) *ticket = R->ticket;
  return CC_OK;
}

// Device memory of a request (problem, descriptor, per-gamma outputs).
static void free_request_device(Request *R) {
  if (R->P) problem_free(R->P);
  R->P = nullptr;
  void *bufs[] = {R->bi, R->gconst, R->fused, R->info, R->tdone};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  R->bi = nullptr;
  R->gconst = nullptr;
  R->fused = nullptr;
  R->info = nullptr;
  R->tdone = nullptr;
}

// Weights, problem and device descriptor of a request; its host copies go.
static cc_status admit(Server *S, Request *R) {
  const int64_t n = R->n, p = R->p;
  float *dX = nullptr;
  uint8_t *dM = nullptr;
  int32_t *ei = nullptr, *ej = nullptr;
  double *w = nullptr;
  struct Tmp {
    void *b[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~Tmp() { for (void *x : b) if (x) (void)hipFree(x); }
  } tmp;
  CC_TRY(dmalloc((void **)&dX, n * p * 4));
  tmp.b[0] = dX;
  CC_HIP(hipMemcpyAsync(dX, R->X.data(), n * p * 4, hipMemcpyHostToDevice, S->stream));
  if (!R->mask.empty()) {
    CC_TRY(dmalloc((void **)&dM, n * p));
    tmp.b[1] = dM;
    CC_HIP(hipMemcpyAsync(dM, R->mask.data(), n * p, hipMemcpyHostToDevice, S->stream));
  }
  const int64_t cap = n * R->k;
  CC_TRY(dmalloc((void **)&ei, cap * 4));
  tmp.b[2] = ei;
  CC_TRY(dmalloc((void **)&ej, cap * 4));
  tmp.b[3] = ej;
  CC_TRY(dmalloc((void **)&w, cap * 8));
  tmp.b[4] = w;
  int64_t E = 0;
  double phi_used = 0.0;
  CC_TRY(build_knn_weights(n, p, CC_DTYPE_F32, dX, p, dM, p, R->k, R->phi, 0, ei, ej, w, cap, &E,
                           &phi_used, S->stream));
  CC_TRY(problem_create(n, p, CC_DTYPE_F32, dX, p, dM, p, E, ei, ej, w, S->precision, S->stream, &R->P));
  Problem *P = R->P;
  const int ng = (int)R->gammas.size();
  R->rho.resize(ng);
  R->eps.resize(ng);
  R->thr.resize(ng);
  for (int g = 0; g < ng; ++g) solve_constants(P, R->gammas[g], S->opts, &R->rho[g], &R->eps[g], &R->thr[g]);
  std::vector<double> gc;
  for (const auto *v : {&R->gammas, &R->rho, &R->eps, &R->thr}) gc.insert(gc.end(), v->begin(), v->end());
  CC_TRY(upload(&R->gconst, gc, S->stream));
  CC_TRY(dmalloc((void **)&R->fused, std::max<int64_t>((int64_t)ng * P->E, 1)));
  CC_TRY(dmalloc((void **)&R->info, (size_t)ng * kInfoVals * 8));
  CC_TRY(dmalloc((void **)&R->tdone, 8));
  const BatchInst bi{ng, (int)P->E, P->sc, R->gconst, R->gconst + ng, R->gconst + 2 * ng, R->gconst + 3 * ng,
                     P->s, R->fused, R->info, R->tdone, S->n_finished};
  CC_TRY(upload(&R->bi, std::vector<BatchInst>{bi}, S->stream));
  hipLaunchKernelGGL(k_inst_init, dim3(1), dim3(1), 0, S->stream, (const BatchInst *)R->bi, S->opts.max_iter,
                     S->opts.test_every);
  CC_HIP(hipGetLastError());
  CC_HIP(hipStreamSynchronize(S->stream));
  P->slot = 0;
  R->X.clear();
  R->X.shrink_to_fit();
  R->mask.clear();
  R->mask.shrink_to_fit();
  R->state = CC_REQ_ACTIVE;
  R->t_admit = host_seconds() - S->t0;
  return CC_OK;
}

cc_status server_step(Server *S, int32_t *n_active, int32_t *n_waiting, int32_t *n_done) {
  // admission: first come, first served, while the budget allows (a request
  // alone on the device is admitted whatever its size)
  while (!S->waiting.empty() && (int)S->active.size() < S->max_active) {
    Request *R = S->waiting.front();
    if (!S->active.empty() && S->used + R->footprint > S->budget) break;
    S->waiting.erase(S->waiting.begin());
    cc_status st = admit(S, R);
    if (st != CC_OK) {
      // a failed admission keeps no device memory and is never charged
      R->error = cc_last_error_message();
      free_request_device(R);
      R->state = CC_REQ_FAILED;
      R->status = st;
      R->t_done = host_seconds() - S->t0;
      continue;
    }
    S->used += R->footprint;
    R->charged = true;
    S->active.push_back(R);
    S->dirty = true;
  }
  int done_now = 0;
  if (!S->active.empty()) {
    const int na = (int)S->active.size();
    if (S->dirty) {
      std::vector<Problem *> probs;
      std::vector<const BatchInst *> bis;
      std::vector<DevScalars *> sc0;
      for (Request *R : S->active) {
        probs.push_back(R->P);
        bis.push_back(R->bi);
        sc0.push_back(R->P->sc);
      }
      std::vector<int> order(na);
      std::iota(order.begin(), order.end(), 0);
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return probs[a]->n * probs[a]->ld > probs[b]->n * probs[b]->ld;
      });
      CC_TRY(build_launch_set(S->ls, probs, bis, order, std::vector<int>(na, S->vec),
                              std::vector<int>(na, S->ipw), S->opts.test_every, S->stream));
      CC_HIP(hipMemcpyAsync(S->d_sc0, sc0.data(), sc0.size() * sizeof(DevScalars *), hipMemcpyHostToDevice, S->stream));
      S->dirty = false;
    }
    for (int it = 0; it < S->round_iters; ++it) launch_set_iteration(S->ls, S->precision, it & 1, S->stream);
    hipLaunchKernelGGL(k_gather_finished, dim3((int)cdiv(na, 256)), dim3(256), 0, S->stream, na,
                       (DevScalars *const *)S->d_sc0, S->d_fin);
    CC_HIP(hipGetLastError());
    CC_HIP(hipMemcpyAsync(S->h_fin, S->d_fin, (size_t)na * 4, hipMemcpyDeviceToHost, S->stream));
    CC_HIP(hipStreamSynchronize(S->stream));
    const double now = host_seconds() - S->t0;
    std::vector<Request *> still;
    for (int k = 0; k < na; ++k) {
      Request *R = S->active[k];
      if (!S->h_fin[k]) {
        still.push_back(R);
        continue;
      }
      R->hinfo.resize(R->gammas.size() * kInfoVals);
      CC_HIP(hipMemcpy(R->hinfo.data(), R->info, R->hinfo.size() * 8, hipMemcpyDeviceToHost));
      R->state = CC_REQ_DONE;
      R->t_done = now;
      for (size_t g = 0; g < R->gammas.size(); ++g)
        if (R->hinfo[g * kInfoVals + 2] != 0.0) R->status = (int)R->hinfo[g * kInfoVals + 2];
      ++done_now;
    }
    if ((int)still.size() != na) {
      S->active = still;
      S->dirty = true;
    }
  }
  if (n_active) *n_active = (int)S->active.size();
  if (n_waiting) *n_waiting = (int)S->waiting.size();
  if (n_done) *n_done = done_now;
  return CC_OK;
}

Request *server_find(Server *S, int64_t ticket) {
  for (Request *R : S->all)
    if (R->ticket == ticket) return R;
  return nullptr;
}

cc_status server_result(Server *S, Request *R, int32_t *labels, cc_solve_info *infos) {
  if (R->state == CC_REQ_FAILED) { set_error("admission failed: " + R->error); return (cc_status)R->status; }
  if (R->state != CC_REQ_DONE) { set_error("request not done"); return CC_ERR_STATE; }
  Problem *P = R->P;
  const int ng = (int)R->gammas.size();
  int32_t *scratch = nullptr;
  struct Tmp { int32_t *&p; ~Tmp() { if (p) (void)hipFree(p); } } tmp{scratch};
  if (!labels && infos) CC_TRY(dmalloc((void **)&scratch, P->n * 4));
  for (int g = 0; g < ng; ++g) {
    int32_t ncl = 0;
    if (labels || infos) {
      CC_TRY(components(P->n, P->E, P->ei, P->ej, R->fused + (int64_t)g * P->E, nullptr,
                        labels ? labels + (int64_t)g * P->n : scratch, P->ncl_dev, S->stream));
      CC_HIP(hipMemcpyAsync(P->flag_host, P->ncl_dev, 4, hipMemcpyDeviceToHost, S->stream));
      CC_HIP(hipStreamSynchronize(S->stream));
      ncl = P->flag_host[0];
    }
    if (infos) {
      const double *v = &R->hinfo[(size_t)g * kInfoVals];
      cc_solve_info &in = infos[g];
      in.iters = (int32_t)v[0];
      in.converged = (int32_t)v[1];
      in.n_clusters = ncl;
      in.status = (int32_t)v[2];
      in.gamma = R->gammas[g];
      in.objective = v[3];
      in.d = v[4];
      in.rel_change = v[5];
      in.rho = R->rho[g];
      in.eps = R->eps[g];
      in.seconds = R->t_done - R->t_admit;
    }
  }
  return R->status == 0 ? CC_OK : (cc_status)R->status;
}

cc_status server_release(Server *S, Request *R) {
  if (R->state == CC_REQ_ACTIVE) { set_error("request still running"); return CC_ERR_STATE; }
  if (R->state == CC_REQ_WAITING) S->waiting.erase(std::find(S->waiting.begin(), S->waiting.end(), R));
  if (R->charged) {
    S->used -= R->footprint;
    R->charged = false;
  }
  free_request_device(R);
  S->all.erase(std::find(S->all.begin(), S->all.end(), R));
  delete R;
  return CC_OK;
}

}  // namespace ccmi
