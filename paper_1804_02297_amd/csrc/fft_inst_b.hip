// The FFT apply instantiated for P = 64, 96 (one unit per group of lengths,
// so that the lengths compile in parallel).
#include "fft_kernels.h"

namespace ls {

template ls_status apply_dispatch<64>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, hipEvent_t*,
                                          void*);
template ls_status apply_dispatch<96>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, hipEvent_t*,
                                          void*);

}  // namespace ls
