// Medium-dependent per-point stencil fit (project extension of Section 3).
#pragma once

#include "common.h"
#include "stencil.h"

namespace ls {

// Block inverse iterations of the per-point eigensolver, from the class Ritz
// vectors.  On these Grams lambda_3 / lambda_9 is 0.03-0.04 (n = 12 and 24,
// six-bump media), so eight steps shrink the error of the three-dimensional
// subspace by about 1e-11 even from an unrelated start.
constexpr int kPointIters = 8;

// Interior points: alpha_i = three smallest eigenvectors of the medium-weighted
// Gram (shell weights w = 1 + |m| / m0), beta_i = B^H alpha_i; boundary points
// copy their class stencils.  Needs class_fit first.  batch: points per Gram
// batch; iters: inverse iterations from the class Ritz vectors.
ls_status point_fit(StencilData& sd, int n, double k, const C<double>* m, double m0, int batch, int iters,
                    hipStream_t s);

// The same fit in pieces, for point lists (training samples, learned-fit fallback).
struct PointFitCtx {
  int n = 0, batch = 0;
  DevBuf Hr, Gcls, Bint, coef, Gb;
};
// allocates per-point stencils (initialised to the class stencils) and the shell data
ls_status pointfit_prepare(PointFitCtx& ctx, StencilData& sd, int n, double k, int batch, hipStream_t s);
// weighted Grams of cnt <= batch interior points (device list) into ctx.Gb
ls_status pointfit_grams(PointFitCtx& ctx, const C<double>* m, double m0, const int* dpts, int cnt, hipStream_t s);
// exact stencils of those points into sd.palpha; the Gram of point q is ctx.Gb's
// entry dslots[q] (device list) when dslots is given, else entry q
ls_status pointfit_solve(PointFitCtx& ctx, StencilData& sd, const int* dpts, int cnt, int iters, hipStream_t s,
                         const int* dslots = nullptr);
// beta = B^H alpha of those points into sd.pbeta
ls_status pointfit_beta(PointFitCtx& ctx, StencilData& sd, const int* dpts, int cnt, hipStream_t s);

}  // namespace ls
