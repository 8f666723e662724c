// Learned strategy selector: host side.  Holds the network's parameters on
// the device, loads and saves them, and exposes the training kernels (forward,
// masked-MSE gradient, Adam) on device buffers the caller owns.
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cstdio>
#include <cstring>
#include <vector>

#include "scan_internal.h"

namespace scan_dev {
hipError_t launch_mlp_forward(const float* theta, const float* X, uint32_t rows, float* out, hipStream_t st);
uint32_t mlp_grad_partials(uint32_t rows);
hipError_t launch_mlp_grad(const float* theta, const float* X, const float* Y, const float* M, uint32_t rows,
                           float inv_denom, float* partials, float* grad, float* loss, hipStream_t st);
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, uint32_t count, int step, float lr,
                       float beta1, float beta2, float eps, hipStream_t st);
}  // namespace scan_dev

namespace {
constexpr uint32_t kParamCount = 5128;  // 6 -> 64 -> 64 -> 8
constexpr const char* kMagic = "scan-mlp-v1";
}  // namespace

struct SelectorState {
  float* theta = nullptr;     // kParamCount floats (device)
  float* partials = nullptr;  // gradient work space (device)
  size_t partials_floats = 0;
};

static SelectorState* state(scan_ctx* ctx) {
  if (!ctx->selector) ctx->selector = new SelectorState();
  return ctx->selector;
}

const float* selector_theta(scan_ctx* ctx) { return ctx->selector ? ctx->selector->theta : nullptr; }

void destroy_selector(scan_ctx* ctx) {
  if (ctx->selector) {
    if (ctx->selector->theta) (void)hipFree(ctx->selector->theta);
    if (ctx->selector->partials) (void)hipFree(ctx->selector->partials);
    delete ctx->selector;
    ctx->selector = nullptr;
  }
  ctx->selector_ready = false;
}

extern "C" {

int scan_mlp_param_count(void) { return (int)kParamCount; }

scan_status scan_selector_set(scan_ctx* ctx, const float* theta_host, size_t count) {
  if (!ctx) return SCAN_EINVAL;
  if (!theta_host) return fail(ctx, SCAN_EINVAL, "theta is NULL");
  if (count != kParamCount) return fail(ctx, SCAN_EINVAL, "selector needs %u parameters, got %zu", kParamCount, count);
  for (size_t i = 0; i < count; ++i)
    if (!(theta_host[i] == theta_host[i]) || theta_host[i] > 3.0e38f || theta_host[i] < -3.0e38f)
      return fail(ctx, SCAN_EINVAL, "selector parameter %zu is not finite", i);
  SelectorState* s = state(ctx);
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess && !s->theta) e = hipMalloc(&s->theta, sizeof(float) * kParamCount);
  if (e == hipSuccess) e = hipMemcpy(s->theta, theta_host, sizeof(float) * kParamCount, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "selector upload");
  ctx->selector_ready = true;
  return SCAN_OK;
}

scan_status scan_selector_clear(scan_ctx* ctx) {
  if (!ctx) return SCAN_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  ctx->selector_ready = false;
  return SCAN_OK;
}

int scan_selector_loaded(const scan_ctx* ctx) { return ctx && ctx->selector_ready ? 1 : 0; }

scan_status scan_selector_load(scan_ctx* ctx, const char* path) {
  if (!ctx) return SCAN_EINVAL;
  if (!path) return fail(ctx, SCAN_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(ctx, SCAN_EINVAL, "cannot open %s: %s", path, std::strerror(errno));
  char magic[32] = {0};
  unsigned count = 0;
  std::vector<float> theta;
  bool ok = std::fscanf(f, "%31s %u", magic, &count) == 2 && std::strcmp(magic, kMagic) == 0 && count == kParamCount;
  if (ok) {
    theta.resize(count);
    for (unsigned i = 0; i < count && ok; ++i) ok = std::fscanf(f, "%f", &theta[i]) == 1;
  }
  // optional last line: "margin <x>" (files without it select by plain argmin)
  float margin = 0.0f;
  if (ok) {
    char key[16] = {0};
    float x = 0.0f;
    const int got = std::fscanf(f, "%15s %f", key, &x);
    if (got == 2 && std::strcmp(key, "margin") == 0) margin = x;
    else if (got != EOF) ok = false;
  }
  std::fclose(f);
  if (!ok) return fail(ctx, SCAN_EINVAL, "%s is not a selector file ('%s %u', %u numbers, optionally 'margin x')",
                       path, kMagic, kParamCount, kParamCount);
  if (!(margin >= 0.0f && margin < 1e30f)) return fail(ctx, SCAN_EINVAL, "%s: margin must be >= 0", path);
  const scan_status st = scan_selector_set(ctx, theta.data(), theta.size());
  if (st == SCAN_OK) ctx->selector_margin = margin;
  return st;
}

scan_status scan_selector_set_margin(scan_ctx* ctx, float margin) {
  if (!ctx) return SCAN_EINVAL;
  if (!(margin >= 0.0f && margin < 1e30f)) return fail(ctx, SCAN_EINVAL, "margin must be finite and >= 0");
  ctx->selector_margin = margin;
  return SCAN_OK;
}

scan_status scan_selector_save(scan_ctx* ctx, const char* path) {
  if (!ctx) return SCAN_EINVAL;
  if (!path) return fail(ctx, SCAN_EINVAL, "path is NULL");
  if (!ctx->selector_ready) return fail(ctx, SCAN_EINVAL, "no selector loaded");
  std::vector<float> theta(kParamCount);
  hipError_t e = hipMemcpy(theta.data(), ctx->selector->theta, sizeof(float) * kParamCount, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "selector download");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(ctx, SCAN_EINVAL, "cannot write %s: %s", path, std::strerror(errno));
  std::fprintf(f, "%s %u\n", kMagic, kParamCount);
  for (float x : theta) std::fprintf(f, "%.9g\n", (double)x);
  std::fprintf(f, "margin %.9g\n", (double)ctx->selector_margin);
  const bool ok = std::fclose(f) == 0;
  return ok ? SCAN_OK : fail(ctx, SCAN_EINVAL, "write failed: %s", path);
}

scan_status scan_mlp_forward(scan_ctx* ctx, const float* theta, const float* X, uint32_t rows, float* out) {
  if (!ctx) return SCAN_EINVAL;
  if (rows == 0) return SCAN_OK;
  if (!theta || !X || !out) return fail(ctx, SCAN_EINVAL, "theta, X and out must not be NULL");
  const hipError_t e = scan_dev::launch_mlp_forward(theta, X, rows, out, ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "mlp forward");
}

scan_status scan_mlp_loss_grad(scan_ctx* ctx, const float* theta, const float* X, const float* Y, const float* M,
                               uint32_t rows, float inv_denom, float* grad, float* loss) {
  if (!ctx) return SCAN_EINVAL;
  if (rows == 0) return fail(ctx, SCAN_EINVAL, "rows must be positive");
  if (!theta || !X || !Y || !M || !grad) return fail(ctx, SCAN_EINVAL, "theta, X, Y, M and grad must not be NULL");
  SelectorState* s = state(ctx);
  const size_t need = (size_t)scan_dev::mlp_grad_partials(rows) * (kParamCount + 1);
  hipError_t e = hipSuccess;
  if (need > s->partials_floats) {
    // The old buffer may still be read by queued work.
    e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && s->partials) e = hipFree(s->partials);
    s->partials = nullptr;
    s->partials_floats = 0;
    if (e == hipSuccess) e = hipMalloc(&s->partials, sizeof(float) * need);
    if (e != hipSuccess) return hip_fail(ctx, e, "gradient work space");
    s->partials_floats = need;
  }
  e = scan_dev::launch_mlp_grad(theta, X, Y, M, rows, inv_denom, s->partials, grad, loss, ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "mlp gradient");
}

scan_status scan_adam_step(scan_ctx* ctx, float* theta, const float* grad, float* m, float* v, uint32_t count,
                           int32_t step, float lr, float beta1, float beta2, float eps) {
  if (!ctx) return SCAN_EINVAL;
  if (!theta || !grad || !m || !v) return fail(ctx, SCAN_EINVAL, "theta, grad, m and v must not be NULL");
  if (step < 1) return fail(ctx, SCAN_EINVAL, "Adam steps count from 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f))
    return fail(ctx, SCAN_EINVAL, "beta1 and beta2 must lie in [0, 1)");
  if (count == 0) return SCAN_OK;
  const hipError_t e = scan_dev::launch_adam(theta, grad, m, v, count, step, lr, beta1, beta2, eps, ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "adam");
}

}  // extern "C"
