// The plan behind the opaque ls_plan handle.
#pragma once

#include "common.h"
#include "gmres.h"
#include "gpu_solver.h"
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
  ls::GpuSolver* gs = nullptr;   // the GPU factor, when it is the current one
  ls::GmresContext gctx;
  ls::DevBuf qtmp;              // Q v scratch for the preconditioner
  std::vector<std::complex<double>> hbuf;   // host staging of preconditioner vectors
  std::string tune_cache;
  size_t host_mem_cap = 0;
  ~ls_plan() {
    ls::host_free(hs);
    ls::gpu_free(gs);
  }
};

struct ls_sparse {
  ls::HostSolver* hs = nullptr;   // exactly one of hs, gs is set
  ls::GpuSolver* gs = nullptr;
  ~ls_sparse() {
    ls::host_free(hs);
    ls::gpu_free(gs);
  }
};

struct ls_mlp {
  ls::MlpState st;
};
