// Internal declarations shared by the libccmi translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ccmi.h"

namespace ccmi {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kPointWaves = 4;  // waves per block of the wave-per-item point sweep
constexpr int kPointBlock = kWave * kPointWaves;
constexpr int kXcds = 8;         // MI355X: 8 accelerator complex dies
constexpr int kMaxBlocks = 2048; // grid cap for the grid-stride sweeps
constexpr int kPointSums = 6;    // per-block FP64 partial sums of the point pass
constexpr int kEdgeSums = 3;     // per-block FP64 partial sums of the edge pass
constexpr int kIterSums = kPointSums + kEdgeSums;
constexpr int kEdgeBlock = 512;  // threads per block of the edge-stage kernels
constexpr int kEdgeWaves = kEdgeBlock / kWave;
constexpr int kEsumRows = 512;   // max partial rows the edge stage leaves
constexpr int kEsumStride = 10;  // doubles per partial row (kIterSums, padded to 16 B)
constexpr int kItemEdges = 8;    // edges per work item of the item edge sweep
constexpr int kMaxProjSweeps = 64;  // Jacobi sweeps of the projection per MM iteration

// Device-resident iteration scalars, in two slots.  Written by the host
// only through the set-parameters and reset kernels.  A point sweep reads
// one slot, finishes the previous MM iteration (when one is pending) and its
// block 0 writes the advanced scalars to the other slot, which the edge stage
// and the next point sweep read.
struct DevScalars {
  // per-solve constants
  double mu, rho, eps, thr;  // thr = tol * eta (0 disables the stop test)
  int max_iter, record, K;   // K = stop-test window
  int pending;    // a sweep ran with these scalars and is not yet finished
  // iteration state
  int m;          // MM iteration index within the current solve
  int pa;         // buffer index holding A_{m-1} (and its edge norms)
  int done, converged, status, iters;
  double d_prev;  // d_{m-1}
  double dA_prev; // ||A_{m-1} - A_{m-1-K}||^2 of the last A window
  double F_cur;   // F_{m-1} once iteration m-1 has finished
  double F_last, d_last, rel_last;
  int path_k;     // batched: index of the gamma in progress
  int finished;   // batched: the whole gamma path is done
  // the last point sweep that ran: its iteration index, the buffer of its
  // A' and its U-update weight theta (U is rebuilt from these when the
  // sweep does not store it)
  int m_run, pa_run;
  double theta_run;
};

// Batched solves: what the device needs to move an instance along its gamma
// path without the host.  Per-gamma constants are computed on the host with
// the same arithmetic as a single solve.
constexpr int kInfoVals = 8;  // iters, converged, status, F, d, rel, gamma, t (ticks)
struct BatchInst {
  int n_gamma, E;
  DevScalars *sc0;                     // the instance's scalar slot 0
  const double *mu, *rho, *eps, *thr;  // per gamma
  const double *s;                     // the instance's shrink factors
  uint8_t *fused;                      // n_gamma x E: s == 0 at the end of each gamma
  double *info;                        // n_gamma x kInfoVals
  unsigned long long *t_done;          // wall-clock ticks when the path finished
  int *n_finished;                     // batch-wide count of finished paths
};

enum Prec { kF32 = CC_PREC_F32, kMixed = CC_PREC_MIXED, kF64 = CC_PREC_F64 };

struct Problem {
  int64_t n = 0, p = 0, E = 0, ld = 0;
  int precision = kMixed;
  hipStream_t stream = nullptr;
  int ntile = 1;      // point-sweep feature tiles of width tile_w
  int tile_w = 256;   // features per tile (64 lanes x vec)
  int vec = 4;
  int ipw = 1;        // about this many items per wave in the point and item edge sweeps
  int pwaves = kPointWaves;  // waves per block of the point sweep
  int eipw = 1;       // about this many items per wave in the item edge sweep
  int entile = 1;     // edge-sweep tiles (1: the fused edge kernel)
  int npass = 4;      // 64-feature passes per edge tile
  bool efused = true;
  bool eitems = false;       // rows up to 512 wide: edge work items by lower end
  int item_nv = 8;           // features per lane of the item edge sweep
  int64_t n_items = 0;       // edge work items (up to kItemEdges edges each)
  bool eslab = false;        // wide rows, small n: LDS-slab edge sweep
  bool eslab_items = false;  // the slab sweep takes edges in work items
  // U stored lazily (single solves with one projection sweep): the point
  // sweep keeps U only at missing entries, in a side array (Umiss, FP state
  // type) indexed from per-item offsets (moff, built for tile width vec)
  bool lazy_u = false;
  void *Umiss = nullptr;
  int32_t *moff = nullptr;
  int64_t n_miss = 0;
  int moff_vec = 0;
  int eslab_tpg = 1;         // feature tiles per block of the slab edge sweep
  int eslab_ntf = 1;         // feature tiles of width edge_f
  int edge_f = 0;            // LDS tile width of the slab edge sweep
  // device buffers
  void *X = nullptr;         // n x ld, float (f32/mixed) or double (f64)
  uint8_t *M = nullptr;      // n x ld or null
  void *U = nullptr;         // n x ld, state type
  void *A[2] = {nullptr, nullptr};  // n x ld, state type
  void *G[2] = {nullptr, nullptr};  // gather mirrors (== A when no mirror)
  void *Usnap = nullptr, *Asnap = nullptr;  // stop-test window snapshots
  int32_t *rowptr = nullptr, *col = nullptr, *eid = nullptr, *uptr = nullptr;
  int32_t *ei = nullptr, *ej = nullptr;
  int32_t *itemI = nullptr;  // lower end of each edge work item
  int32_t *itemJ = nullptr, *itemE = nullptr;  // kItemEdges upper ends / edge ids per item (-1 pad)
  double *w = nullptr, *s = nullptr, *nb[2] = {nullptr, nullptr};
  double *qe = nullptr;     // mu w / (rho ||b||) per edge
  // point-sweep neighbour lists, fixed stride ell_s per point (ELL layout):
  // entries i*ell_s .. i*ell_s + degE[i] - 1 hold the neighbours of i
  int ell_s = 1;
  int32_t *degE = nullptr, *colE = nullptr, *eidE = nullptr;
  double *qE = nullptr;     // q per ELL entry
  int32_t *epos = nullptr;  // ELL positions of (i->j) and (j->i) per edge
  int psweeps = 1;          // projection sweeps per MM iteration (this solve)
  double *H = nullptr;       // several sweeps: h_i = sum_j s_ij (a'_i - a'_j), n x ld FP64
  void *T[2] = {nullptr, nullptr};  // several sweeps: gather copies of the sweeps' increments
  int slab_f = 0;           // > 0: LDS-slab point sweep with F-feature tiles
  bool ell_cm = false;      // ELL stored column-major (entry k of i at k*n + i)
  int cur_K = 64;
  double *part = nullptr;    // E x entile edge partials
  double *psum = nullptr;    // point-sweep blocks x 8 point partials
  double *esum = nullptr;    // kEsumRows x kEsumStride: partial rows of the
                             // edge stage (point sums gathered in)
  int nbe = 1;               // partial rows the edge stage writes
  double *trace = nullptr;   // objective per iteration (record mode)
  int64_t trace_cap = 0, trace_count = 0;
  DevScalars *sc = nullptr;  // two slots
  int slot = 0;              // slot holding the current scalars
  DevScalars *sc_host = nullptr; // pinned mirror
  int32_t *flag_host = nullptr;  // pinned
  int32_t *ncl_dev = nullptr;
  // host-side constants
  double dev2 = 0.0;   // ||M o (X - xbar)||^2
  double w2 = 0.0;     // sum_e w_e^2
  int64_t max_deg = 0;
  bool has_mask = false;
  bool state_valid = true;
  // sampled kernel timing (cc_profile)
  int prof_every = 0;
  int64_t prof_iter = 0;
  std::vector<hipEvent_t> prof_events;  // 4 per sampled iteration
  hipEvent_t pev[4] = {nullptr, nullptr, nullptr, nullptr};  // events of the launch being enqueued
  size_t prof_used = 0;                 // event sets recorded, not yet harvested
  double prof_ms[3] = {0, 0, 0};
  int64_t prof_n[3] = {0, 0, 0};
};

struct PointArgs;  // kernel argument blocks (solver.hip)
struct EdgeArgs;

// Launch tables of problems that share launches: one point-sweep launch per
// class of (features per lane, items per wave) and one item edge-sweep
// launch per features-per-lane class of the edge sweep; block -> (instance,
// local block) tables and per-instance argument blocks for both scalar-slot
// parities.  The classes cover disjoint instances.
struct PointClass {
  int vec = 4, ipw = 1, nblk = 0;
  PointArgs *pargs[2] = {nullptr, nullptr};
  int2 *ptab = nullptr;
};
struct EdgeClass {
  int nv = 1, nblk = 0;
  EdgeArgs *eargs[2] = {nullptr, nullptr};
  int2 *etab = nullptr;
};
struct LaunchSet {
  std::vector<PointClass> pcls;
  std::vector<EdgeClass> ecls;
};

// Autotuner: instances are grouped by the width of their rows (p <= 64,
// <= 128, <= 256, wider) and the number of point-sweep work items at their
// natural tile width (<= 512, <= 2048, more); each group gets its own
// (features per lane, items per wave).
struct TuneClass {
  int width = 0, size = 0, instances = 0, vec = 4, ipw = 1;
  double us = 0.0;                // us per batched iteration with the choice
  std::vector<double> tried;      // us for the 9 candidates (in order)
};

// Many problems solved along their own gamma paths in the same launches.
struct Batch {
  std::vector<Problem *> probs;   // not owned
  int precision = kMixed;
  LaunchSet ls;
  int graph_iters = 32;           // MM iterations per graph replay (even)
  cc_solve_opts opts{};
  hipStream_t stream = nullptr;   // private: graphs are captured on it
  std::vector<hipStream_t> side;  // point and edge classes beyond the first, as graph branches
  std::vector<hipEvent_t> ev;      // fork and join events of those branches
  std::vector<int> order;         // instances by decreasing work
  BatchInst *bi = nullptr;
  std::vector<int> n_gamma;
  std::vector<int64_t> goff;      // first (instance, gamma) slot of each instance
  std::vector<int64_t> foff;      // offset of each instance's fused flags
  int64_t total_gamma = 0, total_fused = 0;
  std::vector<double> gammas, rho, eps;
  double *gconst = nullptr;       // mu, rho, eps, thr: 4 x total_gamma
  uint8_t *fused = nullptr;
  double *info = nullptr;         // total_gamma x kInfoVals
  unsigned long long *ticks = nullptr;  // [0] start, [1 + b] path done
  int *n_finished = nullptr;
  int32_t *ncl = nullptr;         // clusters per (instance, gamma)
  int32_t *fin_host = nullptr;    // pinned
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double tick_khz = 100000.0;     // wall-clock counter rate
  std::vector<int> inst_vec, inst_ipw;  // per instance: point-sweep tile shape
  std::vector<int> inst_class;    // per instance: its autotuner class
  std::vector<TuneClass> classes; // autotuner classes (empty without autotuning)
};

// ---- error reporting (thread-local message) ----
void set_error(const std::string &msg);
cc_status hip_fail(hipError_t e, const char *what);
#define CC_HIP(call)                                  \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) return ::ccmi::hip_fail(_e, #call); \
  } while (0)

// ---- solver (solver.hip) ----
cc_status problem_create(int64_t n, int64_t p, int32_t x_dtype, const void *X,
                         int64_t ldx, const uint8_t *mask, int64_t ldm,
                         int64_t n_edges, const int32_t *ei, const int32_t *ej,
                         const double *w, int32_t precision, hipStream_t stream,
                         Problem **out);
void problem_free(Problem *P);
cc_status reset_state(Problem *P);
cc_status solve(Problem *P, double gamma, const cc_solve_opts &o,
                cc_solve_info *info);
cc_status write_labels(Problem *P, int32_t *labels, int32_t *ncl_host);
cc_status copy_U(Problem *P, int32_t out_dtype, void *dst, int64_t ldu);
cc_status get_fused(Problem *P, uint8_t *fused);
cc_status set_state(Problem *P, const double *U, const double *A, int64_t ld,
                    const double *s);
cc_status get_state(Problem *P, double *U, double *A, int64_t ld, double *s);
cc_status profile(Problem *P, int32_t sample_every);
cc_status harvest_profile(Problem *P);
cc_status components(int64_t n, int64_t E, const int32_t *ei,
                     const int32_t *ej, const uint8_t *keep, const double *s,
                     int32_t *labels, int32_t *ncl_dev, hipStream_t stream);

// Served solves: requests queue on the host, are admitted while the HBM
// budget allows, and share launches with the other admitted requests.
struct Request {
  int64_t ticket = 0;
  int state = 0;                   // CC_REQ_*
  int64_t n = 0, p = 0;
  int32_t k = 10;
  double phi = -0.5;
  std::vector<float> X;            // host copies until admission
  std::vector<uint8_t> mask;
  std::vector<double> gammas, rho, eps, thr;
  Problem *P = nullptr;            // owned once admitted
  int64_t footprint = 0;           // bytes counted against the budget
  bool charged = false;            // footprint counted in the server's used bytes
  BatchInst *bi = nullptr;         // device descriptor and its arrays
  double *gconst = nullptr;
  uint8_t *fused = nullptr;
  double *info = nullptr;
  unsigned long long *tdone = nullptr;
  std::vector<double> hinfo;       // per-gamma info once done
  double t_submit = 0, t_admit = 0, t_done = 0;  // seconds since server creation
  int status = 0;
  std::string error;               // message of a failed admission
};

struct Server {
  int precision = kMixed;
  cc_solve_opts opts{};
  int64_t budget = 0, used = 0;
  int max_active = 64;
  int round_iters = 32;            // MM iterations per round (even)
  int vec = 4, ipw = 4;
  hipStream_t stream = nullptr;    // not owned
  LaunchSet ls;
  bool dirty = false;
  int64_t next_ticket = 1;
  std::vector<Request *> waiting;  // FIFO
  std::vector<Request *> active;
  std::vector<Request *> all;      // every request not yet released
  DevScalars **d_sc0 = nullptr;    // slot 0 of each active request
  int *d_fin = nullptr;
  int *h_fin = nullptr;            // pinned
  int *n_finished = nullptr;
  double t0 = 0;
};

cc_status server_create(int32_t precision, const cc_solve_opts &o, int64_t budget, int32_t max_active,
                        int32_t round_iters, hipStream_t stream, Server **out);
cc_status server_submit(Server *S, int64_t n, int64_t p, const float *X, const uint8_t *mask, int32_t k,
                        double phi, int32_t n_gamma, const double *gammas, int64_t *ticket);
cc_status server_step(Server *S, int32_t *n_active, int32_t *n_waiting, int32_t *n_done);
Request *server_find(Server *S, int64_t ticket);
cc_status server_result(Server *S, Request *R, int32_t *labels, cc_solve_info *infos);
cc_status server_release(Server *S, Request *R);
void server_free(Server *S);

cc_status batch_create(int32_t n_inst, Problem *const *probs, const int32_t *n_gamma,
                       const double *gammas, const cc_solve_opts &o, int32_t autotune,
                       Batch **out);
cc_status batch_run(Batch *B, int32_t *labels, cc_solve_info *infos, double *latency_ms);
void batch_free(Batch *B);

// ---- weights and preparation (knn.hip) ----
cc_status build_knn_weights(int64_t n, int64_t p, int32_t x_dtype,
                            const void *X, int64_t ldx, const uint8_t *mask,
                            int64_t ldm, int32_t k, double phi,
                            int32_t normalize, int32_t *ei, int32_t *ej,
                            double *w, int64_t capacity, int64_t *n_edges,
                            double *phi_used, hipStream_t stream);
cc_status standardize_columns(int64_t n, int64_t p, int32_t x_dtype, void *X,
                              int64_t ldx, const uint8_t *mask, int64_t ldm,
                              hipStream_t stream);
cc_status standardize_columns_noalloc(int64_t n, int64_t p, int32_t x_dtype, void *X,
                                      int64_t ldx, const uint8_t *mask, int64_t ldm,
                                      hipStream_t stream);
cc_status min_connected_k(int64_t n, int64_t p, int32_t x_dtype, const void *X,
                          int64_t ldx, const uint8_t *mask, int64_t ldm,
                          int32_t k_max, int32_t *k_min, int32_t *n_components,
                          hipStream_t stream);
cc_status composite_weights(int64_t n, int64_t n_edges, const int32_t *ei,
                            const int32_t *ej, int64_t p, int32_t x_dtype,
                            const void *X, int64_t ldx, const uint8_t *mask,
                            int64_t ldm, int32_t q,
                            const double *Y, int64_t ldy, const double *period,
                            int32_t geodesic, double radius, double alpha,
                            double phi, int32_t normalize, double *w,
                            double *phi_used, hipStream_t stream);

// ---- principal components and path projection (extras.hip) ----
cc_status pca(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
              const uint8_t *mask, int64_t ldm, int32_t r, int32_t iters,
              double *V, double *sval, double *center, hipStream_t stream);
cc_status project_U(Problem *P, int32_t r, const double *V, const double *center,
                    double *out);

}  // namespace ccmi
