// The plan behind the opaque ls_plan handle.
#pragma once

#include "common.h"
#include "gmres.h"
#include "host_solver.h"
#include "learned.h"
#include "mlp.h"
#include "pointfit.h"
#include "stencil.h"

namespace ls {
constexpr double kPointFitM0 = 0.1;   // medium scale of the per-point weights w = 1 + |m| / m0
}

struct ls_plan {
  ls::ApplyPlan ap;
  ls::StencilData sd;
  ls::HostSolver* hs = nullptr;
  ls::GmresContext gctx;
  ls::DevBuf qtmp;              // Q v scratch for the preconditioner
  std::vector<std::complex<double>> hbuf;   // host staging of preconditioner vectors
  std::string tune_cache;
  size_t host_mem_cap = 0;
  ~ls_plan() { ls::host_free(hs); }
};

struct ls_sparse {
  ls::HostSolver* hs = nullptr;
  ~ls_sparse() { ls::host_free(hs); }
};

struct ls_mlp {
  ls::MlpState st;
};
