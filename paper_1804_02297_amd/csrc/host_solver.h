// Host multifrontal sparse LU for the sparsified system S (nested dissection).
#pragma once

#include <complex>
#include <cstddef>

#include "../../include/ls.h"

namespace ls {

struct HostSolver;

// rows: host array [n^3][3 rows][27 slots][3 comps] of complex128; slot
// 9 (s1+1) + 3 (s2+1) + (s3+1) holds the 3x3 block coupling point i to i + s.
// mem_cap: bytes the factor may use (0 = unlimited); LS_EHOST if exceeded.
// fp32: keep the factor in single precision (a preconditioner for FP64 FGMRES).
ls_status host_factor(int n, const std::complex<double>* rows, size_t mem_cap, bool fp32, HostSolver** out);
// The same for a d0 x d1 x d2 grid with nc unknowns per point (the 2-D
// variant: dims = {n, n, 1}, nc = 2): rows [points][nc rows][27 slots][nc
// comps], slot 9 (s1+1) + 3 (s2+1) + (s3+1) as above (offsets outside the
// grid are ignored); b is [nrhs][nc][points].
ls_status host_factor_grid(const int dims[3], int nc, const std::complex<double>* rows, size_t mem_cap, bool fp32,
                           HostSolver** out);
// Solve S x = b in place; b is [nrhs][3][n^3] (component-major, like the fields).
ls_status host_solve(HostSolver* hs, std::complex<double>* b, int nrhs);
size_t host_factor_bytes(const HostSolver* hs);
double host_factor_flops(const HostSolver* hs);
bool host_factor_is_fp32(const HostSolver* hs);
void host_free(HostSolver* hs);

}  // namespace ls
