// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ls.h"
#include "cplx.h"

namespace ls {

#define LS_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return LS_EHIP;              \
  } while (0)

#define LS_TRY(call)                                   \
  do {                                                 \
    ls_status s_ = (call);                             \
    if (s_ != LS_OK) return s_;                        \
  } while (0)

// Supported padded FFT lengths (even, 2^a 3^b); P is the smallest of these >= 2n - 1.
int choose_fft_size(int n);
bool fft_size_supported(int P);

// Device buffer with RAII release.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  ls_status alloc(size_t b) {
    release();
    if (b == 0) return LS_OK;
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      return LS_ENOMEM;
    }
    bytes = b;
    return LS_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

// Operator data owned by a plan: contrast, Khat in both precisions, twiddles
// and the pass workspace of the FFT apply.
// Launch choices of the apply for one precision, picked by the autotuner.
// 0 = the built-in default.
struct ApplyTune {
  int chunk = 0;                 // right-hand sides per apply launch set (<= max_rhs)
  int kmul_w = 0;                // pass-3 teams per workgroup (1, 2, 4)
  int half_runs = 0;             // bit i set: strided pass i (0 dim-1 forward, 1 dim-2
                                 // forward, 2 dim-2 inverse, 3 dim-1 inverse) works on
                                 // half-length row runs (128 bytes instead of 256)
  int persist = 0;               // bit 0: the four strided passes, bit 1: pass 3 launch
                                 // only the workgroups the device holds at once, and
                                 // each takes work items grid-stride
};

struct ApplyPlan {
  int n = 0, P = 0, H = 0;       // H = P/2 + 1 (octant extent)
  double k = 0.0, h = 0.0;
  int max_rhs = 1;
  DevBuf m64, m32;               // contrast, complex128 / complex64, [n][n][n]
  DevBuf kh64, kh32;             // octant symbol / P^3: [H][H][6][H]
  DevBuf tw64, tw32;             // exp(-2 pi i t / P), t in [0, P)
  DevBuf work;                   // pass intermediates
  size_t work_per_rhs64 = 0;     // bytes per rhs in FP64
  ApplyTune tune[3];             // per ls_prec
  // the paper's own 3x4 form (selected by form = 1), built on first use
  int form = 0;
  DevBuf kp64, kp32;             // octant symbol / P^3 of (k^2 G, G^1, G^2, G^3): [H][H][4][H]
  DevBuf p64, p32;               // p^d = (dm/dx_d) / (1 - m), [3][n][n][n]
  DevBuf work34;                 // four transformed fields per rhs, and p.x
};

ls_status apply_plan_init(ApplyPlan& ap, int n, double k, int max_rhs, const void* m_dev,
                          hipStream_t s);
// y = x + K*(m x), or y = -K*(m x) when minus_conv; prec selects the kernel set.
// nrhs <= max_rhs.  ev, when given, holds 6 events recorded around the 5 passes.
// work, when given, replaces the plan's pass workspace (apply_work_bytes per
// rhs; the dyadic form only) and lifts the max_rhs limit.
ls_status apply_run(ApplyPlan& ap, const void* x, void* y, int nrhs, ls_prec prec, hipStream_t s,
                    bool minus_conv = false, hipEvent_t* ev = nullptr, void* work = nullptr);
// Bytes of pass workspace one rhs needs at prec: 3 (P n^2 + P^2 n) complex values.
inline size_t apply_work_bytes(const ApplyPlan& ap, ls_prec prec) {
  const size_t es = (prec == LS_C128) ? 16 : 8;
  return (size_t)3 * ((size_t)ap.P * ap.n * ap.n + (size_t)ap.P * ap.P * ap.n) * es;
}
// apply_run over any number of right-hand sides, ap.tune[prec].chunk (default
// max_rhs) at a time.
ls_status apply_batched(ApplyPlan& ap, const void* x, void* y, int nrhs, ls_prec prec, hipStream_t s,
                        bool minus_conv = false);
// Select the operator form: 0 the dyadic form y = x + K*(m x); 1 the paper's
// form y_d = x_d + k^2 G*(m x_d) + G^d*(p.x) (its symbol, p and workspace are
// built on the first selection).
ls_status apply_plan_set_form(ApplyPlan& ap, int form, hipStream_t s);
// Pass-3 team counts the plan's FFT size supports (1 always; 2 and 4 when a
// team is one wavefront).
std::vector<int> kmul_team_choices(const ApplyPlan& ap);

}  // namespace ls
