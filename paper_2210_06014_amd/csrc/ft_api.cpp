// C-ABI entry points: argument checks on the host, then kernel launches on the
// caller's stream.
#include <string>

#include "ft_internal.h"

namespace ft {
const char* last_error();
}
using namespace ft;

namespace {

ft_status check_plan(const ft_plan* P) {
  if (!P) return fail(FT_ERR_ARG, "null plan");
  if (!P->uploaded) return fail(FT_ERR_STATE, "plan not uploaded (call ft_plan_upload)");
  return FT_OK;
}

ft_status check_params(const ft_plan* P, const ft_params* p) {
  if (!p) return fail(FT_ERR_ARG, "null params");
  if (p->storage != FT_STORE_F32 && p->storage != FT_STORE_BF16) return fail(FT_ERR_ARG, "unknown storage");
  const bool b16 = p->storage == FT_STORE_BF16;
  if (b16 && P->no_c_cache) return fail(FT_ERR_UNSUPPORTED, "FT_NO_C_CACHE is built for FP32 storage only");
  for (int n = 0; n < P->N; ++n) {
    if (!p->A[n] || !p->B[n] || (!b16 && !p->C[n]) || (b16 && (!p->A16[n] || !p->B16[n] || !p->C16[n])))
      return fail(FT_ERR_ARG, "null parameter pointer for mode " + std::to_string(n));
  }
  return FT_OK;
}

// the parameter set's scratch buffer, for the calls that write scratch
ft_status check_scratch(const ft_plan* P, const ft_params* p) {
  if (!p->scratch || p->scratch_bytes < P->scratch_bytes)
    return fail(FT_ERR_WORKSPACE, "parameter scratch of " + std::to_string(p->scratch ? p->scratch_bytes : 0) +
                                      " bytes, the plan needs " + std::to_string(P->scratch_bytes));
  if (reinterpret_cast<uintptr_t>(p->scratch) % kAlign)
    return fail(FT_ERR_WORKSPACE, "parameter scratch not 256-byte aligned");
  return FT_OK;
}

ft_status check_mode(const ft_plan* P, int32_t m) {
  if (m < 0 || m >= P->N) return fail(FT_ERR_ARG, "mode out of range");
  return FT_OK;
}

ft_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return FT_OK;
  return fail(FT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

ft_status check_lr(double lr, double lam) {
  if (!(lr >= 0.0) || !(lam >= 0.0) || !(lr * lam < 1.0))
    return fail(FT_ERR_ARG, "need lr >= 0, lam >= 0 and lr * lam < 1");
  return FT_OK;
}

}  // namespace

#define FT_TRY(x)                   \
  do {                              \
    ft_status _s = (x);             \
    if (_s != FT_OK) return _s;     \
  } while (0)

extern "C" const char* ft_status_str(ft_status s) {
  switch (s) {
    case FT_OK: return "FT_OK";
    case FT_ERR_ARG: return "FT_ERR_ARG";
    case FT_ERR_SHAPE: return "FT_ERR_SHAPE";
    case FT_ERR_INDEX: return "FT_ERR_INDEX";
    case FT_ERR_UNSUPPORTED: return "FT_ERR_UNSUPPORTED";
    case FT_ERR_STATE: return "FT_ERR_STATE";
    case FT_ERR_NOMEM: return "FT_ERR_NOMEM";
    case FT_ERR_HIP: return "FT_ERR_HIP";
    case FT_ERR_WORKSPACE: return "FT_ERR_WORKSPACE";
  }
  return "FT_ERR_UNKNOWN";
}

extern "C" const char* ft_last_error(void) { return ft::last_error(); }

extern "C" int32_t ft_supported(int32_t order, int32_t J, int32_t R) { return supported(order, J, R) ? 1 : 0; }

extern "C" ft_status ft_refresh(const ft_plan* P, const ft_params* p, int32_t mode, void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  if (mode >= P->N) return fail(FT_ERR_ARG, "mode out of range");
  hipStream_t s = (hipStream_t)stream;
  for (int n = 0; n < P->N; ++n) {
    if (mode >= 0 && n != mode) continue;
    FT_TRY(hip_status(launch_refresh(P, n, p, s), "refresh"));
  }
  return FT_OK;
}

extern "C" ft_status ft_predict(const ft_plan* P, const ft_params* p, const int32_t* d_coords, int64_t q,
                                float* d_out, void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  if (q < 0) return fail(FT_ERR_ARG, "negative query count");
  if (q == 0) return FT_OK;
  if (!d_coords || !d_out) return fail(FT_ERR_ARG, "null coords or output");
  return hip_status(launch_predict(P, p, d_coords, q, d_out, (hipStream_t)stream), "predict");
}

extern "C" ft_status ft_factor_pass(const ft_plan* P, const ft_params* p, int32_t mode, double lr, double lam,
                                    void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  FT_TRY(check_scratch(P, p));
  FT_TRY(check_mode(P, mode));
  FT_TRY(check_lr(lr, lam));
  return hip_status(launch_factor(P, mode, p, scratch_of(P, p), lr, lam, (hipStream_t)stream), "factor pass");
}

extern "C" ft_status ft_factor_epoch(const ft_plan* P, const ft_params* p, double lr, double lam, void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  FT_TRY(check_scratch(P, p));
  FT_TRY(check_lr(lr, lam));
  hipStream_t s = (hipStream_t)stream;
  const Scratch S = scratch_of(P, p);
  for (int m = 0; m < P->N; ++m) {
    FT_TRY(hip_status(launch_factor(P, m, p, S, lr, lam, s), "factor pass"));
    FT_TRY(hip_status(launch_refresh(P, m, p, s), "refresh"));
  }
  return FT_OK;
}

extern "C" ft_status ft_core_grad(const ft_plan* P, const ft_params* p, int32_t mode, float* d_G, void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  FT_TRY(check_scratch(P, p));
  FT_TRY(check_mode(P, mode));
  if (!d_G) return fail(FT_ERR_ARG, "null output");
  return hip_status(launch_core_grad(P, mode, p, scratch_of(P, p), d_G, (hipStream_t)stream), "core gradient");
}

extern "C" ft_status ft_core_pass(const ft_plan* P, const ft_params* p, int32_t mode, double lr, double lam,
                                  void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  FT_TRY(check_scratch(P, p));
  FT_TRY(check_mode(P, mode));
  FT_TRY(check_lr(lr, lam));
  return hip_status(launch_core_update(P, mode, p, scratch_of(P, p), lr, lam, (hipStream_t)stream), "core pass");
}

extern "C" ft_status ft_core_epoch(const ft_plan* P, const ft_params* p, double lr, double lam, void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  FT_TRY(check_scratch(P, p));
  FT_TRY(check_lr(lr, lam));
  hipStream_t s = (hipStream_t)stream;
  const Scratch S = scratch_of(P, p);
  for (int m = 0; m < P->N; ++m) {
    FT_TRY(hip_status(launch_core_update(P, m, p, S, lr, lam, s), "core pass"));
    FT_TRY(hip_status(launch_refresh(P, m, p, s), "refresh"));
  }
  return FT_OK;
}

extern "C" ft_status ft_epoch(const ft_plan* P, const ft_params* p, double lr_a, double lam_a, double lr_b,
                              double lam_b, void* stream) {
  FT_TRY(ft_factor_epoch(P, p, lr_a, lam_a, stream));
  return ft_core_epoch(P, p, lr_b, lam_b, stream);
}

extern "C" ft_status ft_loss(const ft_plan* P, const ft_params* p, double lam_a, double lam_b, double* d_out4,
                             void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  FT_TRY(check_scratch(P, p));
  if (!d_out4) return fail(FT_ERR_ARG, "null output");
  return hip_status(launch_loss(P, p, scratch_of(P, p), lam_a, lam_b, d_out4, (hipStream_t)stream), "loss");
}

extern "C" ft_status ft_loss_noalloc(const ft_plan* P, const ft_params* p, double lam_a, double lam_b,
                                     double* d_out4, void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  if (!d_out4) return fail(FT_ERR_ARG, "null output");
  if (noalloc_loss_need(P) > noalloc_loss_capacity())
    return fail(FT_ERR_WORKSPACE, "ft_loss_noalloc needs " + std::to_string(noalloc_loss_need(P)) +
                                      " bytes of static scratch, the library holds " +
                                      std::to_string(noalloc_loss_capacity()));
  return hip_status(launch_loss_noalloc(P, p, lam_a, lam_b, d_out4, (hipStream_t)stream), "loss (no allocation)");
}

extern "C" ft_status ft_forward(const ft_plan* P, const ft_params* p, float* d_out, void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  if (!d_out) return fail(FT_ERR_ARG, "null output");
  if (!(P->desc.flags & FT_WITH_PERM)) return fail(FT_ERR_STATE, "ft_forward needs a plan built with FT_WITH_PERM");
  return hip_status(launch_forward(P, p, Scratch{}, d_out, (hipStream_t)stream), "forward");
}

extern "C" ft_status ft_grad(const ft_plan* P, const ft_params* p, const float* d_upstream, float* const* d_gA,
                             float* const* d_gB, void* stream) {
  FT_TRY(check_plan(P));
  FT_TRY(check_params(P, p));
  FT_TRY(check_scratch(P, p));
  if (!d_gA || !d_gB) return fail(FT_ERR_ARG, "null gradient arrays");
  for (int n = 0; n < P->N; ++n)
    if (!d_gA[n] || !d_gB[n]) return fail(FT_ERR_ARG, "null gradient pointer");
  if (d_upstream && !(P->desc.flags & FT_WITH_PERM))
    return fail(FT_ERR_STATE, "an upstream gradient needs a plan built with FT_WITH_PERM");
  return hip_status(launch_grad(P, p, scratch_of(P, p), d_upstream, d_gA, d_gB, (hipStream_t)stream), "gradient");
}

static void prof_clear(ft_plan* P) {
  for (auto& r : P->prof) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  P->prof.clear();
}

extern "C" ft_status ft_profile_enable(ft_plan* P, int32_t enable) {
  if (!P) return fail(FT_ERR_ARG, "null plan");
  if (!P->prof.empty()) {
    for (auto& r : P->prof) (void)hipEventSynchronize(r.stop);
    prof_clear(P);
  }
  P->prof_on = enable != 0;
  return FT_OK;
}

extern "C" ft_status ft_profile_read(ft_plan* P, double* ms, int64_t* launches) {
  if (!P) return fail(FT_ERR_ARG, "null plan");
  double acc[FT_K_COUNT] = {0};
  int64_t cnt[FT_K_COUNT] = {0};
  ft_status st = FT_OK;
  for (auto& r : P->prof) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
    if (e != hipSuccess && st == FT_OK) st = fail(FT_ERR_HIP, std::string("event timing: ") + hipGetErrorString(e));
    acc[r.kid] += t;
    cnt[r.kid] += 1;
  }
  prof_clear(P);
  for (int k = 0; k < FT_K_COUNT; ++k) {
    if (ms) ms[k] = acc[k];
    if (launches) launches[k] = cnt[k];
  }
  return st;
}
