// FGMRES driver interface.
#pragma once

#include <functional>
#include <vector>

#include "common.h"

namespace ls {

struct GmresContext {
  long len = 0;                 // 3 n^3 complex entries per rhs
  DevBuf V, Z, W, partial, hdev;
};

struct GmresOps {
  // y = A x for nrhs contiguous fields (device)
  std::function<ls_status(const C<double>*, C<double>*, int, ls_prec, hipStream_t)> apply;
  // in place z <- P^-1 z for the listed rhs (ptr(b) gives rhs b's vector); t_host: host seconds
  std::function<ls_status(const std::vector<int>&, const std::function<C<double>*(int)>&, hipStream_t, double*)>
      precond_batch;
};

ls_status gmres_solve(GmresContext& ctx, const GmresOps& ops, const C<double>* g, C<double>* x, int nrhs,
                      double tol, int restart, int maxit, ls_prec prec, ls_solve_info* info, hipStream_t s);

}  // namespace ls
