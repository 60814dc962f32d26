// extern "C" entry points of libccmi (declared in include/ccmi.h).  Argument
// checks happen here, before anything is launched; no exception crosses the
// ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <string>
#include <vector>

#include "ccmi_internal.h"

namespace ccmi {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

cc_status hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return CC_ERR_HIP;
}

static bool opts_ok(const cc_solve_opts *o) {
  return o == nullptr || o->struct_size == (int32_t)sizeof(cc_solve_opts);
}

static cc_solve_opts resolve(const cc_solve_opts *o) {
  cc_solve_opts r;
  cc_default_opts(&r);
  if (o) r = *o;
  return r;
}

struct StateHeader {
  uint64_t magic;
  int64_t n, p, E;
  int32_t precision, pad;
};
static constexpr uint64_t kStateMagic = 0x4343'4d49'5354'0001ull;  // "CCMIST" v1

}  // namespace ccmi

using namespace ccmi;

#define CC_GUARD_BEGIN try {
#define CC_GUARD_END                                          \
  }                                                           \
  catch (const std::bad_alloc &) {                            \
    set_error("host allocation failed");                      \
    return CC_ERR_OUT_OF_MEMORY;                              \
  }                                                           \
  catch (const std::exception &ex) {                          \
    set_error(std::string("internal error: ") + ex.what());   \
    return CC_ERR_STATE;                                      \
  }                                                           \
  catch (...) {                                               \
    set_error("internal error");                              \
    return CC_ERR_STATE;                                      \
  }

extern "C" {

const char *cc_status_string(cc_status s) {
  switch (s) {
    case CC_OK: return "CC_OK";
    case CC_ERR_INVALID_ARG: return "CC_ERR_INVALID_ARG";
    case CC_ERR_OUT_OF_MEMORY: return "CC_ERR_OUT_OF_MEMORY";
    case CC_ERR_HIP: return "CC_ERR_HIP";
    case CC_ERR_NUMERIC: return "CC_ERR_NUMERIC";
    case CC_ERR_STATE: return "CC_ERR_STATE";
    default: return "CC_ERR_UNKNOWN";
  }
}

const char *cc_last_error_message(void) { return g_last_error.c_str(); }

int32_t cc_version(void) { return 100; }

void cc_default_opts(cc_solve_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(cc_solve_opts);
  o->eta = 1e-2;
  o->rho = 0.0;
  o->eps = 0.0;
  o->tol = 1e-6;
  o->max_iter = 200000;
  o->check_every = 256;
  o->warm_start = 1;
  o->record_objective = 0;
  o->test_every = 64;
  o->proj_sweeps = 1;
}

cc_status cc_problem_create(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                            const uint8_t *mask, int64_t ldm, int64_t n_edges,
                            const int32_t *ei, const int32_t *ej, const double *w,
                            int32_t precision, void *stream, cc_problem_t *out) {
  CC_GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return CC_ERR_INVALID_ARG; }
  *out = nullptr;
  Problem *P = nullptr;
  cc_status s = problem_create(n, p, x_dtype, X, ldx, mask, ldm, n_edges, ei, ej, w, precision,
                               (hipStream_t)stream, &P);
  if (s == CC_OK) *out = reinterpret_cast<cc_problem_t>(P);
  return s;
  CC_GUARD_END
}

cc_status cc_problem_destroy(cc_problem_t prob) {
  CC_GUARD_BEGIN
  if (!prob) return CC_OK;
  Problem *P = reinterpret_cast<Problem *>(prob);
  (void)hipStreamSynchronize(P->stream);
  problem_free(P);
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_problem_dims(cc_problem_t prob, int64_t *n, int64_t *p, int64_t *n_edges,
                          int32_t *precision) {
  if (!prob) { set_error("problem is NULL"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  if (n) *n = P->n;
  if (p) *p = P->p;
  if (n_edges) *n_edges = P->E;
  if (precision) *precision = P->precision;
  return CC_OK;
}

cc_status cc_solve(cc_problem_t prob, double gamma, const cc_solve_opts *opts,
                   cc_solve_info *info) {
  CC_GUARD_BEGIN
  if (!prob) { set_error("problem is NULL"); return CC_ERR_INVALID_ARG; }
  if (!opts_ok(opts)) { set_error("opts->struct_size mismatch"); return CC_ERR_INVALID_ARG; }
  return solve(reinterpret_cast<Problem *>(prob), gamma, resolve(opts), info);
  CC_GUARD_END
}

cc_status cc_solve_path(cc_problem_t prob, int32_t n_gamma, const double *gammas,
                        const cc_solve_opts *opts, int32_t *labels, float *U_path,
                        cc_solve_info *infos) {
  CC_GUARD_BEGIN
  if (!prob) { set_error("problem is NULL"); return CC_ERR_INVALID_ARG; }
  if (n_gamma < 0 || (n_gamma > 0 && !gammas)) { set_error("bad gamma array"); return CC_ERR_INVALID_ARG; }
  if (!opts_ok(opts)) { set_error("opts->struct_size mismatch"); return CC_ERR_INVALID_ARG; }
  for (int32_t g = 0; g < n_gamma; ++g)
    if (!(gammas[g] >= 0.0) || !std::isfinite(gammas[g])) {
      set_error("gammas must be finite and >= 0");
      return CC_ERR_INVALID_ARG;
    }
  Problem *P = reinterpret_cast<Problem *>(prob);
  cc_solve_opts o = resolve(opts);
  for (int32_t g = 0; g < n_gamma; ++g) {
    cc_solve_info info;
    std::memset(&info, 0, sizeof(info));
    cc_status s = solve(P, gammas[g], o, &info);
    if (infos) infos[g] = info;
    if (s != CC_OK) return s;
    if (labels) {
      s = write_labels(P, labels + (size_t)g * P->n, nullptr);
      if (s != CC_OK) return s;
    }
    if (U_path) {
      s = copy_U(P, CC_DTYPE_F32, U_path + (size_t)g * P->n * P->p, P->p);
      if (s != CC_OK) return s;
    }
    o.warm_start = 1;
  }
  if (hipStreamSynchronize(P->stream) != hipSuccess) { set_error("stream sync failed"); return CC_ERR_HIP; }
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_solve_path_pc(cc_problem_t prob, int32_t n_gamma, const double *gammas,
                           const cc_solve_opts *opts, int32_t *labels, int32_t r,
                           const double *V, const double *center, double *proj,
                           cc_solve_info *infos) {
  CC_GUARD_BEGIN
  if (!prob) { set_error("problem is NULL"); return CC_ERR_INVALID_ARG; }
  if (n_gamma < 0 || (n_gamma > 0 && !gammas)) { set_error("bad gamma array"); return CC_ERR_INVALID_ARG; }
  if (!opts_ok(opts)) { set_error("opts->struct_size mismatch"); return CC_ERR_INVALID_ARG; }
  if (r < 1 || r > 16 || !V || !proj) { set_error("need 1 <= r <= 16 and V, proj"); return CC_ERR_INVALID_ARG; }
  for (int32_t g = 0; g < n_gamma; ++g)
    if (!(gammas[g] >= 0.0) || !std::isfinite(gammas[g])) {
      set_error("gammas must be finite and >= 0");
      return CC_ERR_INVALID_ARG;
    }
  Problem *P = reinterpret_cast<Problem *>(prob);
  cc_solve_opts o = resolve(opts);
  for (int32_t g = 0; g < n_gamma; ++g) {
    cc_solve_info info;
    std::memset(&info, 0, sizeof(info));
    cc_status s = solve(P, gammas[g], o, &info);
    if (infos) infos[g] = info;
    if (s != CC_OK) return s;
    if (labels) {
      s = write_labels(P, labels + (size_t)g * P->n, nullptr);
      if (s != CC_OK) return s;
    }
    s = project_U(P, r, V, center, proj + (size_t)g * P->n * r);
    if (s != CC_OK) return s;
    o.warm_start = 1;
  }
  if (hipStreamSynchronize(P->stream) != hipSuccess) { set_error("stream sync failed"); return CC_ERR_HIP; }
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_batch_create(int32_t n_inst, const cc_problem_t *problems, const int32_t *n_gamma,
                          const double *gammas, const cc_solve_opts *opts, int32_t autotune,
                          cc_batch_t *out) {
  CC_GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return CC_ERR_INVALID_ARG; }
  *out = nullptr;
  if (!opts_ok(opts)) { set_error("opts->struct_size mismatch"); return CC_ERR_INVALID_ARG; }
  if (n_inst < 1 || !problems) { set_error("need n_inst >= 1 problems"); return CC_ERR_INVALID_ARG; }
  for (int32_t b = 0; b < n_inst; ++b)
    if (!problems[b]) { set_error("problem " + std::to_string(b) + " is NULL"); return CC_ERR_INVALID_ARG; }
  const cc_solve_opts o = resolve(opts);
  std::vector<Problem *> probs(n_inst);
  for (int32_t b = 0; b < n_inst; ++b) probs[b] = reinterpret_cast<Problem *>(problems[b]);
  Batch *B = nullptr;
  cc_status s = batch_create(n_inst, probs.data(), n_gamma, gammas, o, autotune, &B);
  if (s != CC_OK) return s;
  *out = reinterpret_cast<cc_batch_t>(B);
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_batch_run(cc_batch_t batch, int32_t *labels, cc_solve_info *infos, double *latency_ms) {
  CC_GUARD_BEGIN
  if (!batch) { set_error("batch is NULL"); return CC_ERR_INVALID_ARG; }
  return batch_run(reinterpret_cast<Batch *>(batch), labels, infos, latency_ms);
  CC_GUARD_END
}

cc_status cc_batch_config(cc_batch_t batch, int32_t *vec, int32_t *items_per_wave,
                          int32_t *graph_iters, double *tune_us) {
  CC_GUARD_BEGIN
  if (!batch) { set_error("batch is NULL"); return CC_ERR_INVALID_ARG; }
  const Batch *B = reinterpret_cast<const Batch *>(batch);
  // the instance with the most work (first in the block tables) and its class
  const int b0 = B->order.empty() ? 0 : B->order[0];
  if (vec) *vec = B->inst_vec.empty() ? 0 : B->inst_vec[b0];
  if (items_per_wave) *items_per_wave = B->inst_ipw.empty() ? 0 : B->inst_ipw[b0];
  if (graph_iters) *graph_iters = B->graph_iters;
  if (tune_us) {
    const TuneClass *tc = nullptr;
    if (!B->inst_class.empty() && B->inst_class[b0] >= 0) tc = &B->classes[B->inst_class[b0]];
    for (int c = 0; c < 9; ++c) tune_us[c] = (tc && c < (int)tc->tried.size()) ? tc->tried[c] : 0.0;
  }
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_batch_tuning(cc_batch_t batch, int32_t cap, int32_t *n_classes, int32_t *classes,
                          double *us, int32_t *inst_class) {
  CC_GUARD_BEGIN
  if (!batch) { set_error("batch is NULL"); return CC_ERR_INVALID_ARG; }
  if (cap < 0 || (cap > 0 && !classes)) { set_error("need cap >= 0 and classes for cap > 0"); return CC_ERR_INVALID_ARG; }
  const Batch *B = reinterpret_cast<const Batch *>(batch);
  const int nc = (int)B->classes.size();
  if (n_classes) *n_classes = nc;
  for (int c = 0; c < std::min(nc, (int)cap); ++c) {
    const TuneClass &t = B->classes[c];
    int32_t *o = classes + 5 * c;
    o[0] = t.width; o[1] = t.size; o[2] = t.instances; o[3] = t.vec; o[4] = t.ipw;
    if (us) us[c] = t.us;
  }
  if (inst_class)
    for (size_t b = 0; b < B->probs.size(); ++b) inst_class[b] = B->inst_class.empty() ? -1 : B->inst_class[b];
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_batch_destroy(cc_batch_t batch) {
  CC_GUARD_BEGIN
  batch_free(reinterpret_cast<Batch *>(batch));
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_server_create(int32_t precision, const cc_solve_opts *opts, int64_t hbm_budget,
                           int32_t max_active, int32_t round_iters, void *stream, cc_server_t *out) {
  CC_GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return CC_ERR_INVALID_ARG; }
  *out = nullptr;
  if (!opts_ok(opts)) { set_error("opts->struct_size mismatch"); return CC_ERR_INVALID_ARG; }
  Server *S = nullptr;
  cc_status s = server_create(precision, resolve(opts), hbm_budget, max_active, round_iters,
                              (hipStream_t)stream, &S);
  if (s != CC_OK) return s;
  *out = reinterpret_cast<cc_server_t>(S);
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_server_submit(cc_server_t server, int64_t n, int64_t p, const float *X, const uint8_t *mask,
                           int32_t k, double phi, int32_t n_gamma, const double *gammas, int64_t *ticket) {
  CC_GUARD_BEGIN
  if (!server) { set_error("server is NULL"); return CC_ERR_INVALID_ARG; }
  return server_submit(reinterpret_cast<Server *>(server), n, p, X, mask, k, phi, n_gamma, gammas, ticket);
  CC_GUARD_END
}

cc_status cc_server_step(cc_server_t server, int32_t *n_active, int32_t *n_waiting, int32_t *n_done) {
  CC_GUARD_BEGIN
  if (!server) { set_error("server is NULL"); return CC_ERR_INVALID_ARG; }
  return server_step(reinterpret_cast<Server *>(server), n_active, n_waiting, n_done);
  CC_GUARD_END
}

cc_status cc_server_status(cc_server_t server, int64_t ticket, int32_t *state, double *t_submit,
                           double *t_admit, double *t_done) {
  CC_GUARD_BEGIN
  if (!server) { set_error("server is NULL"); return CC_ERR_INVALID_ARG; }
  Request *R = server_find(reinterpret_cast<Server *>(server), ticket);
  if (!R) { set_error("unknown ticket"); return CC_ERR_INVALID_ARG; }
  if (state) *state = R->state;
  if (t_submit) *t_submit = R->t_submit;
  if (t_admit) *t_admit = R->t_admit;
  if (t_done) *t_done = R->t_done;
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_server_result(cc_server_t server, int64_t ticket, int32_t *labels, cc_solve_info *infos,
                           float *U) {
  CC_GUARD_BEGIN
  if (!server) { set_error("server is NULL"); return CC_ERR_INVALID_ARG; }
  Server *S = reinterpret_cast<Server *>(server);
  Request *R = server_find(S, ticket);
  if (!R) { set_error("unknown ticket"); return CC_ERR_INVALID_ARG; }
  cc_status s = server_result(S, R, labels, infos);
  if (U && R->state == CC_REQ_DONE) {
    cc_status su = copy_U(R->P, CC_DTYPE_F32, U, R->p);
    if (su != CC_OK) return su;
    if (hipStreamSynchronize(S->stream) != hipSuccess) { set_error("stream sync failed"); return CC_ERR_HIP; }
  }
  return s;
  CC_GUARD_END
}

cc_status cc_server_release(cc_server_t server, int64_t ticket) {
  CC_GUARD_BEGIN
  if (!server) { set_error("server is NULL"); return CC_ERR_INVALID_ARG; }
  Server *S = reinterpret_cast<Server *>(server);
  Request *R = server_find(S, ticket);
  if (!R) { set_error("unknown ticket"); return CC_ERR_INVALID_ARG; }
  return server_release(S, R);
  CC_GUARD_END
}

cc_status cc_server_memory(cc_server_t server, int64_t *used, int64_t *budget) {
  CC_GUARD_BEGIN
  if (!server) { set_error("server is NULL"); return CC_ERR_INVALID_ARG; }
  const Server *S = reinterpret_cast<const Server *>(server);
  if (used) *used = S->used;
  if (budget) *budget = S->budget;
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_server_destroy(cc_server_t server) {
  CC_GUARD_BEGIN
  server_free(reinterpret_cast<Server *>(server));
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_get_U(cc_problem_t prob, int32_t out_dtype, void *U, int64_t ldu) {
  CC_GUARD_BEGIN
  if (!prob || !U) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  if (out_dtype != CC_DTYPE_F32 && out_dtype != CC_DTYPE_F64) { set_error("bad out_dtype"); return CC_ERR_INVALID_ARG; }
  if (ldu < P->p) { set_error("ldu < p"); return CC_ERR_INVALID_ARG; }
  return copy_U(P, out_dtype, U, ldu);
  CC_GUARD_END
}

cc_status cc_get_labels(cc_problem_t prob, int32_t *labels, int32_t *n_clusters) {
  CC_GUARD_BEGIN
  if (!prob || !labels) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  return write_labels(reinterpret_cast<Problem *>(prob), labels, n_clusters);
  CC_GUARD_END
}

cc_status cc_get_fused_edges(cc_problem_t prob, uint8_t *fused) {
  CC_GUARD_BEGIN
  if (!prob) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  if (P->E > 0 && !fused) { set_error("fused is NULL"); return CC_ERR_INVALID_ARG; }
  return get_fused(P, fused);
  CC_GUARD_END
}

cc_status cc_get_trace(cc_problem_t prob, double *F, int64_t cap, int64_t *count) {
  CC_GUARD_BEGIN
  if (!prob || !count || (cap > 0 && !F)) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  const int64_t c = std::min(cap, P->trace_count);
  if (c > 0) {
    if (hipMemcpyAsync(F, P->trace, c * 8, hipMemcpyDeviceToHost, P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess) {
      set_error("trace copy failed");
      return CC_ERR_HIP;
    }
  }
  *count = c;
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_profile(cc_problem_t prob, int32_t sample_every) {
  CC_GUARD_BEGIN
  if (!prob) { set_error("problem is NULL"); return CC_ERR_INVALID_ARG; }
  if (sample_every < 0) { set_error("sample_every < 0"); return CC_ERR_INVALID_ARG; }
  return profile(reinterpret_cast<Problem *>(prob), sample_every);
  CC_GUARD_END
}

cc_status cc_kernel_stats(cc_problem_t prob, double *avg_ms, int64_t *launches) {
  CC_GUARD_BEGIN
  if (!prob || !avg_ms) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  if (hipStreamSynchronize(P->stream) != hipSuccess) { set_error("stream sync failed"); return CC_ERR_HIP; }
  harvest_profile(P);
  for (int q = 0; q < 2; ++q) {
    avg_ms[q] = P->prof_n[q] ? P->prof_ms[q] / (double)P->prof_n[q] : 0.0;
    if (launches) launches[q] = P->prof_n[q];
  }
  return CC_OK;
  CC_GUARD_END
}

cc_status cc_state_size(cc_problem_t prob, size_t *bytes) {
  if (!prob || !bytes) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  *bytes = sizeof(StateHeader) + (size_t)(2 * P->n * P->p + P->E) * sizeof(double);
  return CC_OK;
}

cc_status cc_export_state(cc_problem_t prob, void *buf, size_t bytes) {
  CC_GUARD_BEGIN
  if (!prob || !buf) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  size_t need = 0;
  cc_state_size(prob, &need);
  if (bytes < need) { set_error("buffer too small"); return CC_ERR_INVALID_ARG; }
  const size_t np = (size_t)P->n * P->p;
  double *d = nullptr;
  if (hipMalloc((void **)&d, (2 * np + P->E + 1) * sizeof(double)) != hipSuccess) {
    set_error("hipMalloc failed"); return CC_ERR_OUT_OF_MEMORY;
  }
  cc_status s = get_state(P, d, d + np, P->p, d + 2 * np);
  if (s == CC_OK) {
    StateHeader h{kStateMagic, P->n, P->p, P->E, P->precision, 0};
    std::memcpy(buf, &h, sizeof(h));
    if (hipMemcpyAsync((char *)buf + sizeof(h), d, (2 * np + P->E) * sizeof(double),
                       hipMemcpyDeviceToHost, P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess) {
      set_error("state copy failed"); s = CC_ERR_HIP;
    }
  }
  (void)hipFree(d);
  return s;
  CC_GUARD_END
}

cc_status cc_import_state(cc_problem_t prob, const void *buf, size_t bytes) {
  CC_GUARD_BEGIN
  if (!prob || !buf) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  size_t need = 0;
  cc_state_size(prob, &need);
  if (bytes < need) { set_error("buffer too small"); return CC_ERR_INVALID_ARG; }
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kStateMagic || h.n != P->n || h.p != P->p || h.E != P->E ||
      h.precision != P->precision) {
    set_error("state does not match this problem"); return CC_ERR_INVALID_ARG;
  }
  const size_t np = (size_t)P->n * P->p;
  const double *src = reinterpret_cast<const double *>((const char *)buf + sizeof(h));
  for (int64_t e = 0; e < P->E; ++e) {
    const double sv = src[2 * np + e];
    if (!(sv >= 0.0 && sv <= 1.0)) { set_error("shrink factor outside [0, 1]"); return CC_ERR_INVALID_ARG; }
  }
  double *d = nullptr;
  if (hipMalloc((void **)&d, (2 * np + P->E + 1) * sizeof(double)) != hipSuccess) {
    set_error("hipMalloc failed"); return CC_ERR_OUT_OF_MEMORY;
  }
  cc_status s = CC_OK;
  if (hipMemcpyAsync(d, src, (2 * np + P->E) * sizeof(double), hipMemcpyHostToDevice,
                     P->stream) != hipSuccess) {
    set_error("state copy failed"); s = CC_ERR_HIP;
  }
  if (s == CC_OK) s = set_state(P, d, d + np, P->p, d + 2 * np);
  (void)hipStreamSynchronize(P->stream);
  (void)hipFree(d);
  return s;
  CC_GUARD_END
}

cc_status cc_reset_state(cc_problem_t prob) {
  CC_GUARD_BEGIN
  if (!prob) { set_error("problem is NULL"); return CC_ERR_INVALID_ARG; }
  return reset_state(reinterpret_cast<Problem *>(prob));
  CC_GUARD_END
}

cc_status cc_set_state(cc_problem_t prob, const double *U, const double *A, int64_t ld,
                       const double *s) {
  CC_GUARD_BEGIN
  if (!prob || !U || !A) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  if (ld < P->p) { set_error("ld < p"); return CC_ERR_INVALID_ARG; }
  if (P->E > 0) {
    if (!s) { set_error("s is NULL"); return CC_ERR_INVALID_ARG; }
    std::vector<double> hs(P->E);
    if (hipMemcpyAsync(hs.data(), s, P->E * 8, hipMemcpyDeviceToHost, P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess) {
      set_error("copy of s failed"); return CC_ERR_HIP;
    }
    for (double v : hs)
      if (!(v >= 0.0 && v <= 1.0)) { set_error("shrink factor outside [0, 1]"); return CC_ERR_INVALID_ARG; }
  }
  return set_state(P, U, A, ld, s);
  CC_GUARD_END
}

cc_status cc_get_state(cc_problem_t prob, double *U, double *A, int64_t ld, double *s) {
  CC_GUARD_BEGIN
  if (!prob || !U || !A) { set_error("NULL argument"); return CC_ERR_INVALID_ARG; }
  Problem *P = reinterpret_cast<Problem *>(prob);
  if (ld < P->p) { set_error("ld < p"); return CC_ERR_INVALID_ARG; }
  if (P->E > 0 && !s) { set_error("s is NULL"); return CC_ERR_INVALID_ARG; }
  return get_state(P, U, A, ld, s);
  CC_GUARD_END
}

cc_status cc_build_knn_weights(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                               const uint8_t *mask, int64_t ldm, int32_t k, double phi,
                               int32_t normalize, int32_t *ei, int32_t *ej, double *w,
                               int64_t capacity, int64_t *n_edges, double *phi_used,
                               void *stream) {
  CC_GUARD_BEGIN
  return build_knn_weights(n, p, x_dtype, X, ldx, mask, ldm, k, phi, normalize, ei, ej, w,
                           capacity, n_edges, phi_used, (hipStream_t)stream);
  CC_GUARD_END
}

cc_status cc_standardize_columns(int64_t n, int64_t p, int32_t x_dtype, void *X, int64_t ldx,
                                 const uint8_t *mask, int64_t ldm, void *stream) {
  CC_GUARD_BEGIN
  return standardize_columns(n, p, x_dtype, X, ldx, mask, ldm, (hipStream_t)stream);
  CC_GUARD_END
}

cc_status cc_standardize_columns_noalloc(int64_t n, int64_t p, int32_t x_dtype, void *X, int64_t ldx,
                                         const uint8_t *mask, int64_t ldm, void *stream) {
  CC_GUARD_BEGIN
  return standardize_columns_noalloc(n, p, x_dtype, X, ldx, mask, ldm, (hipStream_t)stream);
  CC_GUARD_END
}

cc_status cc_pca(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                 const uint8_t *mask, int64_t ldm, int32_t r, int32_t iters, double *V,
                 double *sval, double *center, void *stream) {
  CC_GUARD_BEGIN
  return pca(n, p, x_dtype, X, ldx, mask, ldm, r, iters, V, sval, center, (hipStream_t)stream);
  CC_GUARD_END
}

cc_status cc_min_connected_k(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                             const uint8_t *mask, int64_t ldm, int32_t k_max, int32_t *k_min,
                             int32_t *n_components, void *stream) {
  CC_GUARD_BEGIN
  return min_connected_k(n, p, x_dtype, X, ldx, mask, ldm, k_max, k_min, n_components,
                         (hipStream_t)stream);
  CC_GUARD_END
}

cc_status cc_composite_weights(int64_t n, int64_t n_edges, const int32_t *ei, const int32_t *ej,
                               int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                               const uint8_t *mask, int64_t ldm, int32_t q,
                               const double *Y, int64_t ldy, const double *period,
                               int32_t geodesic, double radius, double alpha, double phi,
                               int32_t normalize, double *w, double *phi_used, void *stream) {
  CC_GUARD_BEGIN
  return composite_weights(n, n_edges, ei, ej, p, x_dtype, X, ldx, mask, ldm, q, Y, ldy, period, geodesic,
                           radius, alpha, phi, normalize, w, phi_used, (hipStream_t)stream);
  CC_GUARD_END
}

cc_status cc_components(int64_t n, int64_t n_edges, const int32_t *ei, const int32_t *ej,
                        const uint8_t *keep, int32_t *labels, int32_t *n_components,
                        void *stream) {
  CC_GUARD_BEGIN
  if (n < 1 || n_edges < 0 || !labels || (n_edges > 0 && (!ei || !ej))) {
    set_error("bad argument"); return CC_ERR_INVALID_ARG;
  }
  if (n > ((int64_t)1 << 31) - 1 || n_edges > ((int64_t)1 << 31) - 1) {
    set_error("n or n_edges too large"); return CC_ERR_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int32_t *ncl = nullptr;
  if (hipMalloc((void **)&ncl, 4) != hipSuccess) { set_error("hipMalloc failed"); return CC_ERR_OUT_OF_MEMORY; }
  uint8_t *ones = nullptr;
  const uint8_t *kp = keep;
  if (!kp && n_edges > 0) {
    if (hipMalloc((void **)&ones, n_edges) != hipSuccess) { (void)hipFree(ncl); set_error("hipMalloc failed"); return CC_ERR_OUT_OF_MEMORY; }
    (void)hipMemsetAsync(ones, 1, n_edges, st);
    kp = ones;
  }
  cc_status s = components(n, n_edges, ei, ej, kp, nullptr, labels, ncl, st);
  int32_t h = 0;
  if (s == CC_OK) {
    if (hipMemcpyAsync(&h, ncl, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) { set_error("copy failed"); s = CC_ERR_HIP; }
  }
  if (n_components) *n_components = h;
  (void)hipFree(ncl);
  if (ones) (void)hipFree(ones);
  return s;
  CC_GUARD_END
}

}  // extern "C"
