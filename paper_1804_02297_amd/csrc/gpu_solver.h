// GPU multifrontal sparse LU of the sparsified system S, fronts in HBM.
#pragma once

#include "common.h"

namespace ls {

struct GpuSolver;

// rows_dev: device array [n^3][3 rows][27 slots][3 comps] of complex128 (the
// layout of the plan's assembled rows).  fp32: keep the factor in complex64.
// Synchronises the stream before returning.
ls_status gpu_factor(int n, const C<double>* rows_dev, bool fp32, hipStream_t s, GpuSolver** out);
// The same for a d0 x d1 x d2 grid with nc unknowns per point (nc = 2 or 3;
// the 2-D variant: dims = {n, n, 1}, nc = 2): rows_dev [points][nc rows][27
// slots][nc comps]; solves take b, x as [nrhs][nc][points].
ls_status gpu_factor_grid(const int dims[3], int nc, const C<double>* rows_dev, bool fp32, hipStream_t s,
                          GpuSolver** out);
// Solve S x = b on the device; b, x are [nrhs][3][n^3] complex128 and may be
// the same array (stream-ordered: b is read completely before x is written).
ls_status gpu_solve(GpuSolver* gs, const C<double>* b_dev, C<double>* x_dev, int nrhs, hipStream_t s);
size_t gpu_factor_bytes(const GpuSolver* gs);
double gpu_factor_flops(const GpuSolver* gs);
bool gpu_factor_is_fp32(const GpuSolver* gs);
void gpu_free(GpuSolver* gs);

}  // namespace ls
