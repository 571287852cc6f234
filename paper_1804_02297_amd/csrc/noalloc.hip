// The apply without any allocation, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).
//
// ls_apply runs its five passes through the plan's workspace.  This variant
// runs the same kernels with the pass intermediates in one fixed device
// array of kScratchBytes, so it calls no hipMalloc or hipFree and no
// allocating library routine.  Every GPU that the library runs on holds its
// own copy of the array until the process ends; its device address is looked
// up once per device, on the first call there.  All calls on one GPU share
// that array: two calls that overlap in time on the same GPU (different
// streams, or different host threads) race on it.  The passes write every
// intermediate before reading it, so nothing needs clearing between calls.
#include <algorithm>
#include <mutex>

#include "plan.h"

namespace ls {
namespace {

constexpr size_t kScratchBytes = 128ull << 20;      // 128 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch array (looked up on first use).
ls_status scratch_for_current_device(void** out) {
  int dev = 0;
  LS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return LS_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LS_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LS_OK;
}

}  // namespace
}  // namespace ls

using namespace ls;

extern "C" ls_status ls_apply_noalloc(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                                      void* hip_stream) {
  if (!plan || !x_dev || !y_dev || nrhs < 1) return LS_EINVAL;
  if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
  if (plan->ap.form != 0) return LS_ESTATE;
  const size_t per = apply_work_bytes(plan->ap, prec);
  if (per > kScratchBytes) return LS_ENOMEM;           // one right-hand side does not fit
  void* work = nullptr;
  LS_TRY(scratch_for_current_device(&work));
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const int chunk = (int)std::min<size_t>(kScratchBytes / per, (size_t)nrhs);
  const size_t es = (prec == LS_C64) ? 8 : 16;
  const size_t field = (size_t)3 * plan->ap.n * plan->ap.n * plan->ap.n * es;
  for (int b0 = 0; b0 < nrhs; b0 += chunk) {
    const int nb = std::min(chunk, nrhs - b0);
    LS_TRY(apply_run(plan->ap, static_cast<const char*>(x_dev) + (size_t)b0 * field,
                     static_cast<char*>(y_dev) + (size_t)b0 * field, nb, prec, s, false, nullptr, work));
  }
  return LS_OK;
}
