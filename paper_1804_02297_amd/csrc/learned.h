// Learned stencils: training samples, training loop and the learned fit.
#pragma once

#include "common.h"
#include "mlp.h"
#include "pointfit.h"
#include "stencil.h"

namespace ls {

// Exact per-point fits at the listed interior points become training samples.
ls_status mlp_add_samples(MlpState& st, StencilData& sd, int n, double k, const C<double>* m, double m0,
                          const int* pts_host, int npts, hipStream_t s);
// Adam on minibatches drawn from a seeded permutation of the samples.
ls_status mlp_train(MlpState& st, int steps, int batch, double lr, unsigned seed, double* loss_hist, hipStream_t s);
// Interior stencils from the network; rejected points fall back to the exact per-point fit.
ls_status learned_fit(StencilData& sd, MlpState& st, int n, double k, const C<double>* m, double m0,
                      int* n_fallback, hipStream_t s);

}  // namespace ls
