// The FFT apply instantiated for P = 8, 12, 16, 24, 32, 48 (one unit per group of lengths,
// so that the lengths compile in parallel).
#include "fft_kernels.h"

namespace ls {

template ls_status apply_dispatch<8>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, hipEvent_t*,
                                          void*);
template ls_status apply_dispatch<12>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, hipEvent_t*,
                                          void*);
template ls_status apply_dispatch<16>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, hipEvent_t*,
                                          void*);
template ls_status apply_dispatch<24>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, hipEvent_t*,
                                          void*);
template ls_status apply_dispatch<32>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, hipEvent_t*,
                                          void*);
template ls_status apply_dispatch<48>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, hipEvent_t*,
                                          void*);

}  // namespace ls
