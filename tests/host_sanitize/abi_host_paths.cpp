// Host-side paths of the C ABI, for a build of the library's host code
// with AddressSanitizer and UndefinedBehaviorSanitizer: argument validation
// of every entry point, error strings, and (on a machine without a GPU,
// where every HIP call fails) the clean-up after a failed device call.
// Exit status: the number of failed expectations.
#include <cstdio>
#include <cstring>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "ccmi.h"

static int g_fail = 0;

static void expect(bool ok, const char *what, cc_status s) {
  const char *msg = cc_last_error_message();
  const size_t len = msg ? std::strlen(msg) : 0;
  if (!ok) {
    ++g_fail;
    std::printf("FAIL %s: status %s, message '%s'\n", what, cc_status_string(s), msg ? msg : "(null)");
  } else {
    std::printf("ok   %s: %s (%zu-byte message)\n", what, cc_status_string(s), len);
  }
}
#define INVALID(call) do { cc_status s_ = (call); expect(s_ == CC_ERR_INVALID_ARG, #call, s_); } while (0)
#define NOT_OK(call) do { cc_status s_ = (call); expect(s_ != CC_OK, #call, s_); } while (0)

int main() {
  // the cases past host validation pass host memory where device memory is
  // expected: they run only where no GPU is present (every HIP call fails)
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
  const bool no_gpu = ndev == 0;
  // strings and defaults
  for (int s = -1; s <= 7; ++s) {
    const char *t = cc_status_string((cc_status)s);
    if (!t || !*t) { ++g_fail; std::printf("FAIL status string %d\n", s); }
  }
  cc_solve_opts o;
  cc_default_opts(&o);
  expect(o.struct_size == (int32_t)sizeof(cc_solve_opts) && o.proj_sweeps == 1 && o.max_iter > 0,
         "cc_default_opts", CC_OK);
  expect(cc_version() >= 100, "cc_version", CC_OK);

  // fake device addresses: host validation rejects before any device access
  std::vector<float> X(64 * 8, 1.0f);
  std::vector<int32_t> ei(16, 0), ej(16, 1);
  std::vector<double> w(16, 1.0), g(4, 1.0);
  std::vector<uint8_t> m(64 * 8, 1);
  cc_problem_t pr = nullptr;
  INVALID(cc_problem_create(0, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 0, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, &pr));
  INVALID(cc_problem_create(4, 0, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 0, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, &pr));
  INVALID(cc_problem_create(4, 3, CC_DTYPE_F32, X.data(), 2, nullptr, 3, 0, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, &pr));
  INVALID(cc_problem_create(4, 3, 7, X.data(), 3, nullptr, 3, 0, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, &pr));
  INVALID(cc_problem_create(4, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 0, nullptr, nullptr, nullptr, 9, nullptr, &pr));
  INVALID(cc_problem_create(4, 3, CC_DTYPE_F32, nullptr, 3, nullptr, 3, 0, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, &pr));
  INVALID(cc_problem_create(4, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 0, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, nullptr));
  INVALID(cc_problem_create(4, 3, CC_DTYPE_F32, X.data(), 3, m.data(), 2, 0, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, &pr));
  INVALID(cc_problem_create(4, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, -1, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, &pr));
  INVALID(cc_problem_create(4, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 2, nullptr, ej.data(), w.data(), CC_PREC_MIXED, nullptr, &pr));
  INVALID(cc_problem_create(1LL << 20, 1LL << 12, CC_DTYPE_F32, X.data(), 1LL << 12, nullptr, 0, 0, nullptr, nullptr, nullptr, CC_PREC_MIXED, nullptr, &pr));
  expect(pr == nullptr, "no handle after a rejected create", CC_OK);
  // past host validation: the first device call fails without a GPU
  if (no_gpu) {
    NOT_OK(cc_problem_create(4, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 2, ei.data(), ej.data(), w.data(), CC_PREC_MIXED, nullptr, &pr));
    expect(pr == nullptr, "no handle after a failed create", CC_OK);
  }

  // null handles
  cc_solve_info info;
  int64_t n64 = 0;
  int32_t i32 = 0;
  size_t sz = 0;
  INVALID(cc_solve(nullptr, 1.0, nullptr, &info));
  INVALID(cc_solve_path(nullptr, 4, g.data(), nullptr, nullptr, nullptr, &info));
  INVALID(cc_get_U(nullptr, CC_DTYPE_F32, X.data(), 8));
  INVALID(cc_get_labels(nullptr, ei.data(), &i32));
  INVALID(cc_get_fused_edges(nullptr, m.data()));
  INVALID(cc_get_trace(nullptr, w.data(), 4, &n64));
  INVALID(cc_profile(nullptr, 4));
  INVALID(cc_kernel_stats(nullptr, w.data(), &n64));
  INVALID(cc_state_size(nullptr, &sz));
  INVALID(cc_export_state(nullptr, X.data(), 16));
  INVALID(cc_import_state(nullptr, X.data(), 16));
  INVALID(cc_reset_state(nullptr));
  INVALID(cc_set_state(nullptr, w.data(), w.data(), 4, w.data()));
  INVALID(cc_get_state(nullptr, w.data(), w.data(), 4, w.data()));
  INVALID(cc_problem_dims(nullptr, &n64, &n64, &n64, &i32));
  INVALID(cc_solve_path_pc(nullptr, 4, g.data(), nullptr, nullptr, 2, w.data(), w.data(), w.data(), &info));
  expect(cc_problem_destroy(nullptr) != CC_ERR_HIP, "cc_problem_destroy(nullptr)", CC_OK);

  // weights, standardisation, components, extras
  INVALID(cc_build_knn_weights(5, 2, CC_DTYPE_F32, X.data(), 2, nullptr, 2, 5, 0.5, 0, ei.data(), ej.data(), w.data(), 25, &n64, nullptr, nullptr));
  INVALID(cc_build_knn_weights(5, 2, CC_DTYPE_F32, X.data(), 1, nullptr, 2, 2, 0.5, 0, ei.data(), ej.data(), w.data(), 10, &n64, nullptr, nullptr));
  // a capacity below the edge count is found only after the build: fails on the device call here
  if (no_gpu) NOT_OK(cc_build_knn_weights(5, 2, CC_DTYPE_F32, X.data(), 2, nullptr, 2, 2, 0.5, 0, ei.data(), ej.data(), w.data(), 1, &n64, nullptr, nullptr));
  INVALID(cc_build_knn_weights(5, 2, CC_DTYPE_F32, nullptr, 2, nullptr, 2, 2, 0.5, 0, ei.data(), ej.data(), w.data(), 10, &n64, nullptr, nullptr));
  INVALID(cc_standardize_columns(0, 2, CC_DTYPE_F32, X.data(), 2, nullptr, 2, nullptr));
  INVALID(cc_standardize_columns(4, 2, CC_DTYPE_F32, X.data(), 1, nullptr, 2, nullptr));
  INVALID(cc_standardize_columns_noalloc(4, 70000, CC_DTYPE_F32, X.data(), 70000, nullptr, 70000, nullptr));
  INVALID(cc_standardize_columns_noalloc(4, 2, CC_DTYPE_F32, nullptr, 2, nullptr, 2, nullptr));
  INVALID(cc_components(0, 0, nullptr, nullptr, nullptr, ei.data(), &i32, nullptr));
  INVALID(cc_components(4, 2, nullptr, ej.data(), nullptr, ei.data(), &i32, nullptr));
  INVALID(cc_pca(4, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 0, 10, w.data(), w.data(), w.data(), nullptr));
  INVALID(cc_pca(4, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 5, 10, w.data(), w.data(), w.data(), nullptr));
  INVALID(cc_min_connected_k(4, 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 9, &i32, &i32, nullptr));
  INVALID(cc_composite_weights(4, 2, ei.data(), ej.data(), 3, CC_DTYPE_F32, X.data(), 3, nullptr, 3, 2, w.data(), 2, nullptr, 1, 1.0, 1.5, 0.5, 0, w.data(), nullptr, nullptr));

  // batched and served
  cc_batch_t bt = nullptr;
  int32_t ng = 4;
  INVALID(cc_batch_create(0, nullptr, &ng, g.data(), nullptr, 0, &bt));
  INVALID(cc_batch_create(1, nullptr, &ng, g.data(), nullptr, 0, &bt));
  cc_problem_t none[2] = {nullptr, nullptr};
  INVALID(cc_batch_create(2, none, &ng, g.data(), nullptr, 0, &bt));
  INVALID(cc_batch_create(2, none, &ng, g.data(), nullptr, 0, nullptr));
  expect(bt == nullptr, "no batch after a rejected create", CC_OK);
  INVALID(cc_batch_run(nullptr, nullptr, nullptr, nullptr));
  INVALID(cc_batch_config(nullptr, &i32, &i32, &i32, nullptr));
  INVALID(cc_batch_tuning(nullptr, 0, &i32, nullptr, nullptr, nullptr));
  cc_server_t sv = nullptr;
  INVALID(cc_server_create(9, nullptr, 1 << 20, 4, 64, nullptr, &sv));
  INVALID(cc_server_create(CC_PREC_MIXED, nullptr, 1 << 20, 4, 64, nullptr, nullptr));
  INVALID(cc_server_create(CC_PREC_MIXED, nullptr, 1 << 20, 0, 64, nullptr, &sv));
  INVALID(cc_server_create(CC_PREC_MIXED, nullptr, 1 << 20, 4, 63, nullptr, &sv));
  cc_solve_opts bad = o;
  bad.proj_sweeps = 2;
  INVALID(cc_server_create(CC_PREC_MIXED, &bad, 1 << 20, 4, 64, nullptr, &sv));
  INVALID(cc_server_submit(nullptr, 8, 3, X.data(), nullptr, 2, 0.5, 4, g.data(), &n64));
  INVALID(cc_server_step(nullptr, &i32, &i32, &i32));
  INVALID(cc_server_status(nullptr, 0, &i32, nullptr, nullptr, nullptr));
  INVALID(cc_server_result(nullptr, 0, nullptr, &info, nullptr));
  INVALID(cc_server_release(nullptr, 0));
  INVALID(cc_server_memory(nullptr, &n64, &n64));
  expect(cc_server_destroy(nullptr) != CC_ERR_HIP, "cc_server_destroy(nullptr)", CC_OK);
  // a server with valid arguments: its first device call fails without a GPU
  if (no_gpu) {
    NOT_OK(cc_server_create(CC_PREC_MIXED, nullptr, 1 << 20, 4, 64, nullptr, &sv));
    expect(sv == nullptr, "no server after a failed create", CC_OK);
  }

  std::printf("%d failed\n", g_fail);
  return g_fail;
}
