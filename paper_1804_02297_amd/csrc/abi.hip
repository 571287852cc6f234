// C ABI entry points (include/ls.h).  Argument checking and dispatch only;
// the arithmetic lives in the kernels of the other translation units.
#include <new>

#include "common.h"

using namespace ls;

static inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

const char* ls_status_string(ls_status s) {
  switch (s) {
    case LS_OK: return "ok";
    case LS_EINVAL: return "invalid argument";
    case LS_ENOMEM: return "out of memory";
    case LS_EHIP: return "HIP runtime error";
    case LS_ENOCONV: return "FGMRES did not converge";
    case LS_EHOST: return "host factorisation exceeds the memory cap";
    case LS_ESTATE: return "call out of order";
    case LS_EIO: return "weights file unreadable or malformed";
  }
  return "unknown status";
}

ls_status ls_plan_create(const ls_plan_desc* desc, const void* m_dev, void* hip_stream,
                         ls_plan** out) {
  if (!desc || !m_dev || !out) return LS_EINVAL;
  *out = nullptr;
  if (desc->n < 3 || desc->n > 192 || !(desc->k > 0.0) || desc->max_rhs < 1) return LS_EINVAL;
  ls_plan* p = new (std::nothrow) ls_plan();
  if (!p) return LS_ENOMEM;
  p->host_mem_cap = desc->host_mem_cap;
  if (desc->tune_cache) p->tune_cache = desc->tune_cache;
  ls_status st = apply_plan_init(p->ap, desc->n, desc->k, desc->max_rhs, m_dev, as_stream(hip_stream));
  if (st == LS_OK && hipStreamSynchronize(as_stream(hip_stream)) != hipSuccess) st = LS_EHIP;
  if (st != LS_OK) {
    delete p;
    return st;
  }
  *out = p;
  return LS_OK;
}

ls_status ls_apply(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                   void* hip_stream) {
  if (!plan || !x_dev || !y_dev || nrhs < 1) return LS_EINVAL;
  if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
  const size_t es = (prec == LS_C64) ? 8 : 16;
  const size_t per = (size_t)3 * plan->ap.n * plan->ap.n * plan->ap.n * es;
  for (int b0 = 0; b0 < nrhs; b0 += plan->ap.max_rhs) {
    const int nb = (nrhs - b0 < plan->ap.max_rhs) ? nrhs - b0 : plan->ap.max_rhs;
    const char* x = static_cast<const char*>(x_dev) + (size_t)b0 * per;
    char* y = static_cast<char*>(y_dev) + (size_t)b0 * per;
    LS_TRY(apply_run(plan->ap, x, y, nb, prec, as_stream(hip_stream)));
  }
  return LS_OK;
}

ls_status ls_apply_timed(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                         void* hip_stream, double* pass_ms) {
  if (!plan || !x_dev || !y_dev || nrhs < 1 || !pass_ms) return LS_EINVAL;
  if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      return LS_EHIP;
    }
  for (int i = 0; i < 5; ++i) pass_ms[i] = 0.0;
  const size_t es = (prec == LS_C64) ? 8 : 16;
  const size_t per = (size_t)3 * plan->ap.n * plan->ap.n * plan->ap.n * es;
  ls_status st = LS_OK;
  for (int b0 = 0; b0 < nrhs && st == LS_OK; b0 += plan->ap.max_rhs) {
    const int nb = (nrhs - b0 < plan->ap.max_rhs) ? nrhs - b0 : plan->ap.max_rhs;
    st = apply_run(plan->ap, static_cast<const char*>(x_dev) + (size_t)b0 * per,
                   static_cast<char*>(y_dev) + (size_t)b0 * per, nb, prec, s, false, ev);
    if (st == LS_OK && hipEventSynchronize(ev[5]) != hipSuccess) st = LS_EHIP;
    for (int i = 0; i < 5 && st == LS_OK; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) st = LS_EHIP;
      pass_ms[i] += ms;
    }
  }
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
  return st;
}

ls_status ls_rhs_from_incident(ls_plan* plan, const void* Ei_dev, void* g_dev, int nrhs,
                               void* hip_stream) {
  if (!plan || !Ei_dev || !g_dev || nrhs < 1) return LS_EINVAL;
  const size_t per = (size_t)3 * plan->ap.n * plan->ap.n * plan->ap.n * 16;
  for (int b0 = 0; b0 < nrhs; b0 += plan->ap.max_rhs) {
    const int nb = (nrhs - b0 < plan->ap.max_rhs) ? nrhs - b0 : plan->ap.max_rhs;
    LS_TRY(apply_run(plan->ap, static_cast<const char*>(Ei_dev) + (size_t)b0 * per,
                     static_cast<char*>(g_dev) + (size_t)b0 * per, nb, LS_C128,
                     as_stream(hip_stream), /*minus_conv=*/true));
  }
  return LS_OK;
}

int ls_plan_fft_size(const ls_plan* plan) { return plan ? plan->ap.P : 0; }

void ls_plan_destroy(ls_plan* plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  delete plan;
}

}  // extern "C"
