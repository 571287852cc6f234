// Medium-dependent per-point stencil fit (project extension of Section 3).
#pragma once

#include "common.h"
#include "stencil.h"

namespace ls {

// Interior points: alpha_i = three smallest eigenvectors of the medium-weighted
// Gram (shell weights w = 1 + |m| / m0), beta_i = B^H alpha_i; boundary points
// copy their class stencils.  Needs class_fit first.  batch: points per Gram
// batch; iters: inverse iterations from the class Ritz vectors.
ls_status point_fit(StencilData& sd, int n, double k, const C<double>* m, double m0, int batch, int iters,
                    hipStream_t s);

}  // namespace ls
