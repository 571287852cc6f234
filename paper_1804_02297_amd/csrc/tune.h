// Autotuner of the batched apply (launch choices per plan and precision).
#pragma once
#include <string>

#include "common.h"

namespace ls {

struct TuneOutcome {
  ApplyTune t;
  double ms_per_rhs = 0.0, ms_default_per_rhs = 0.0;
  int from_cache = 0, n_tried = 0, cache_write_failed = 0;
};

// Picks ap.tune[prec] for batches of nrhs: from the cache file when it holds
// this key, else by timing every choice; cache == "" disables the file.
ls_status apply_tune(ApplyPlan& ap, const std::string& cache, int nrhs, ls_prec prec, hipStream_t s,
                     TuneOutcome* out);

}  // namespace ls
