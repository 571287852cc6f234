// C ABI entry points (include/ls.h).  Argument checking and dispatch only;
// the arithmetic lives in the kernels of the other translation units.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>

#include "plan.h"
#include "tune.h"

using namespace ls;

// Host allocations inside an entry point (vectors of the symbolic phase, host
// staging, plan objects) may throw; no exception crosses the C boundary.
template <typename F>
static ls_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return LS_ENOMEM;
  } catch (const std::length_error&) {
    return LS_ENOMEM;
  }
}

static inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
static inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// y = A x over nrhs fields, chunked by the plan's max_rhs
static ls_status apply_chunked(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                               hipStream_t s, bool minus_conv = false) {
  return apply_batched(plan->ap, x_dev, y_dev, nrhs, prec, s, minus_conv);
}

// z <- S^-1 Q z for the listed right-hand sides (device vectors), host solve in one block
static ls_status precond_list(ls_plan* plan, const std::vector<int>& lb,
                              const std::function<C<double>*(int)>& ptr, hipStream_t s, double* t_host) {
  const long len = 3L * plan->ap.n * plan->ap.n * plan->ap.n;
  const size_t vb = (size_t)len * sizeof(C<double>);
  const int nb = (int)lb.size();
  if (plan->gs) {   // GPU factor: Q v into a contiguous block, solve it in HBM
    if (plan->qtmp.bytes < (size_t)nb * vb) LS_TRY(plan->qtmp.alloc((size_t)nb * vb));
    C<double>* blk = plan->qtmp.as<C<double>>();
    C<double>* v0 = ptr(lb[0]);
    bool contiguous = true;   // the vectors one after another (every rhs of a lockstep block)
    for (int q = 1; q < nb && contiguous; ++q) contiguous = ptr(lb[q]) == v0 + (size_t)q * len;
    if (t_host) *t_host = 0.0;
    if (contiguous) {
      LS_TRY(q_apply(plan->sd, plan->ap.n, v0, blk, nb, s));
      return gpu_solve(plan->gs, blk, v0, nb, s);
    }
    for (int q = 0; q < nb; ++q) LS_TRY(q_apply(plan->sd, plan->ap.n, ptr(lb[q]), blk + (size_t)q * len, 1, s));
    LS_TRY(gpu_solve(plan->gs, blk, blk, nb, s));
    for (int q = 0; q < nb; ++q)
      LS_HIP(hipMemcpyAsync(ptr(lb[q]), blk + (size_t)q * len, vb, hipMemcpyDeviceToDevice, s));
    return LS_OK;
  }
  if (plan->qtmp.bytes < vb) LS_TRY(plan->qtmp.alloc(vb));
  plan->hbuf.resize((size_t)nb * len);
  for (int q = 0; q < nb; ++q) {
    LS_TRY(q_apply(plan->sd, plan->ap.n, ptr(lb[q]), plan->qtmp.as<C<double>>(), 1, s));
    LS_HIP(hipMemcpyAsync(plan->hbuf.data() + (size_t)q * len, plan->qtmp.p, vb, hipMemcpyDeviceToHost, s));
  }
  LS_HIP(hipStreamSynchronize(s));
  const double t0 = now_s();
  LS_TRY(host_solve(plan->hs, plan->hbuf.data(), nb));
  if (t_host) *t_host = now_s() - t0;
  for (int q = 0; q < nb; ++q)
    LS_HIP(hipMemcpyAsync(ptr(lb[q]), plan->hbuf.data() + (size_t)q * len, vb, hipMemcpyHostToDevice, s));
  LS_HIP(hipStreamSynchronize(s));
  return LS_OK;
}

extern "C" {

const char* ls_status_string(ls_status s) {
  switch (s) {
    case LS_OK: return "ok";
    case LS_EINVAL: return "invalid argument";
    case LS_ENOMEM: return "out of memory";
    case LS_EHIP: return "HIP runtime error";
    case LS_ENOCONV: return "FGMRES did not converge";
    case LS_EHOST: return "host factorisation exceeds the memory cap";
    case LS_ESTATE: return "call out of order";
    case LS_EIO: return "weights file unreadable or malformed";
  }
  return "unknown status";
}

ls_status ls_plan_create(const ls_plan_desc* desc, const void* m_dev, void* hip_stream,
                         ls_plan** out) {
  return guarded([&]() -> ls_status {
    if (!desc || !m_dev || !out) return LS_EINVAL;
    *out = nullptr;
    if (desc->n < 3 || desc->n > 192 || !(desc->k > 0.0) || desc->max_rhs < 1) return LS_EINVAL;
    std::unique_ptr<ls_plan> p(new (std::nothrow) ls_plan());
    if (!p) return LS_ENOMEM;
    p->host_mem_cap = desc->host_mem_cap;
    if (desc->tune_cache) p->tune_cache = desc->tune_cache;
    ls_status st = apply_plan_init(p->ap, desc->n, desc->k, desc->max_rhs, m_dev, as_stream(hip_stream));
    if (st == LS_OK && hipStreamSynchronize(as_stream(hip_stream)) != hipSuccess) st = LS_EHIP;
    if (st != LS_OK) return st;
    p->gctx.len = 3L * desc->n * desc->n * desc->n;
    *out = p.release();
    return LS_OK;
  });
}

ls_status ls_apply(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                   void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan || !x_dev || !y_dev || nrhs < 1) return LS_EINVAL;
    if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
    return apply_chunked(plan, x_dev, y_dev, nrhs, prec, as_stream(hip_stream));
  });
}

ls_status ls_apply_timed(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                         void* hip_stream, double* pass_ms) {
  return guarded([&]() -> ls_status {
    if (!plan || !x_dev || !y_dev || nrhs < 1 || !pass_ms) return LS_EINVAL;
    if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
    hipStream_t s = as_stream(hip_stream);
    hipEvent_t ev[6];
    for (int i = 0; i < 6; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
        return LS_EHIP;
      }
    for (int i = 0; i < 5; ++i) pass_ms[i] = 0.0;
    const size_t es = (prec == LS_C64) ? 8 : 16;
    const size_t per = (size_t)3 * plan->ap.n * plan->ap.n * plan->ap.n * es;
    ls_status st = LS_OK;
    int chunk = plan->ap.form == 0 ? plan->ap.tune[prec].chunk : 0;   // as apply_batched
    if (chunk <= 0 || chunk > plan->ap.max_rhs) chunk = plan->ap.max_rhs;
    for (int b0 = 0; b0 < nrhs && st == LS_OK; b0 += chunk) {
      const int nb = (nrhs - b0 < chunk) ? nrhs - b0 : chunk;
      st = apply_run(plan->ap, static_cast<const char*>(x_dev) + (size_t)b0 * per,
                     static_cast<char*>(y_dev) + (size_t)b0 * per, nb, prec, s, false, ev);
      if (st == LS_OK && hipEventSynchronize(ev[5]) != hipSuccess) st = LS_EHIP;
      for (int i = 0; i < 5 && st == LS_OK; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) st = LS_EHIP;
        pass_ms[i] += ms;
      }
    }
    for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
    return st;
  });
}

ls_status ls_plan_tune(ls_plan* plan, int nrhs, ls_prec prec, void* hip_stream, ls_tune_info* info) {
  return guarded([&]() -> ls_status {
    if (!plan || nrhs < 1) return LS_EINVAL;
    if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
    TuneOutcome r;
    LS_TRY(apply_tune(plan->ap, plan->tune_cache, nrhs, prec, as_stream(hip_stream), &r));
    if (info) {
      info->chunk = r.t.chunk;
      info->kmul_w = r.t.kmul_w;
      info->half_runs = r.t.half_runs;
      info->persist = r.t.persist;
      info->ms_per_rhs = r.ms_per_rhs;
      info->ms_default_per_rhs = r.ms_default_per_rhs;
      info->from_cache = r.from_cache;
      info->n_tried = r.n_tried;
    }
    return LS_OK;
  });
}

ls_status ls_plan_set_tune(ls_plan* plan, ls_prec prec, int chunk, int kmul_w, int half_runs, int persist) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
    if (chunk < 0 || chunk > plan->ap.max_rhs) return LS_EINVAL;
    if (kmul_w != 0 && kmul_w != 1 && kmul_w != 2 && kmul_w != 4) return LS_EINVAL;
    if (half_runs < 0 || half_runs > 15 || persist < 0 || persist > 3) return LS_EINVAL;
    plan->ap.tune[prec].chunk = chunk;
    plan->ap.tune[prec].kmul_w = kmul_w;
    plan->ap.tune[prec].half_runs = half_runs;
    plan->ap.tune[prec].persist = persist;
    return LS_OK;
  });
}

ls_status ls_rhs_from_incident(ls_plan* plan, const void* Ei_dev, void* g_dev, int nrhs,
                               void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan || !Ei_dev || !g_dev || nrhs < 1) return LS_EINVAL;
    return apply_chunked(plan, Ei_dev, g_dev, nrhs, LS_C128, as_stream(hip_stream), /*minus_conv=*/true);
  });
}

ls_status ls_stencil_fit(ls_plan* plan, ls_fit_mode mode, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan || (mode != LS_FIT_CLASS && mode != LS_FIT_POINT)) return LS_EINVAL;
    if (plan->ap.n < 4) return LS_EINVAL;     // n = 3: the interior complement is empty
    hipStream_t s = as_stream(hip_stream);
    host_free(plan->hs);
    plan->hs = nullptr;
    gpu_free(plan->gs);
    plan->gs = nullptr;
    plan->sd.have_point = false;
    plan->sd.have_rows = false;
    plan->sd.have_learned = false;
    // the class stencils depend on (n, k) only: computed once per plan
    if (!plan->sd.have_class) LS_TRY(class_fit(plan->sd, plan->ap.n, plan->ap.k, s));
    if (mode == LS_FIT_POINT)
      LS_TRY(point_fit(plan->sd, plan->ap.n, plan->ap.k, plan->ap.m64.as<C<double>>(), kPointFitM0, 16384, kPointIters, s));
    LS_TRY(assemble_rows(plan->sd, plan->ap.n, plan->ap.m64.as<C<double>>(), s));
    LS_HIP(hipStreamSynchronize(s));
    plan->sd.have_rows = true;
    return LS_OK;
  });
}

ls_status ls_get_point_stencils(const ls_plan* plan, void* alpha_host, double* eig_host) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    if (!plan->sd.have_point) return LS_ESTATE;
    if (alpha_host) LS_HIP(hipMemcpy(alpha_host, plan->sd.palpha.p, plan->sd.palpha.bytes, hipMemcpyDeviceToHost));
    if (eig_host) LS_HIP(hipMemcpy(eig_host, plan->sd.peval.p, plan->sd.peval.bytes, hipMemcpyDeviceToHost));
    return LS_OK;
  });
}

ls_status ls_get_learned_info(const ls_plan* plan, int* accept_host, double* ratio_host) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    if (!plan->sd.have_learned || !plan->sd.have_point) return LS_ESTATE;
    const auto& a = plan->sd.learned_accept;
    const auto& r = plan->sd.learned_ratio;
    if (accept_host) std::memcpy(accept_host, a.data(), a.size() * sizeof(int));
    if (ratio_host) std::memcpy(ratio_host, r.data(), r.size() * sizeof(double));
    return LS_OK;
  });
}

ls_status ls_get_class_stencils(const ls_plan* plan, void* alpha_host, void* beta_host, double* eig_host,
                                void* gram_host) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    if (!plan->sd.have_class) return LS_ESTATE;
    if (alpha_host) LS_HIP(hipMemcpy(alpha_host, plan->sd.alpha.p, plan->sd.alpha.bytes, hipMemcpyDeviceToHost));
    if (beta_host) LS_HIP(hipMemcpy(beta_host, plan->sd.beta.p, plan->sd.beta.bytes, hipMemcpyDeviceToHost));
    if (eig_host) LS_HIP(hipMemcpy(eig_host, plan->sd.evals.p, plan->sd.evals.bytes, hipMemcpyDeviceToHost));
    if (gram_host) LS_HIP(hipMemcpy(gram_host, plan->sd.gram.p, plan->sd.gram.bytes, hipMemcpyDeviceToHost));
    return LS_OK;
  });
}

ls_status ls_get_rows(const ls_plan* plan, void* rows_host) {
  return guarded([&]() -> ls_status {
    if (!plan || !rows_host) return LS_EINVAL;
    if (!plan->sd.have_rows) return LS_ESTATE;
    LS_HIP(hipMemcpy(rows_host, plan->sd.rows.p, plan->sd.rows.bytes, hipMemcpyDeviceToHost));
    return LS_OK;
  });
}

ls_status ls_factor(ls_plan* plan, double* seconds_out) { return ls_factor_prec(plan, LS_C128, seconds_out); }

ls_status ls_factor_prec(ls_plan* plan, ls_prec factor_prec, double* seconds_out) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    if (factor_prec != LS_C128 && factor_prec != LS_C64 && factor_prec != LS_MIXED) return LS_EINVAL;
    if (!plan->sd.have_rows) return LS_ESTATE;
    const double t0 = now_s();
    std::vector<std::complex<double>> rows(plan->sd.rows.bytes / sizeof(std::complex<double>));
    LS_HIP(hipMemcpy(rows.data(), plan->sd.rows.p, plan->sd.rows.bytes, hipMemcpyDeviceToHost));
    host_free(plan->hs);
    plan->hs = nullptr;
    gpu_free(plan->gs);
    plan->gs = nullptr;
    LS_TRY(host_factor(plan->ap.n, rows.data(), plan->host_mem_cap, factor_prec != LS_C128, &plan->hs));
    if (seconds_out) *seconds_out = now_s() - t0;
    return LS_OK;
  });
}

ls_status ls_factor_gpu(ls_plan* plan, ls_prec factor_prec, void* hip_stream, double* seconds_out) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    if (factor_prec != LS_C128 && factor_prec != LS_C64 && factor_prec != LS_MIXED) return LS_EINVAL;
    if (!plan->sd.have_rows) return LS_ESTATE;
    hipStream_t s = as_stream(hip_stream);
    LS_HIP(hipStreamSynchronize(s));
    const double t0 = now_s();
    host_free(plan->hs);
    plan->hs = nullptr;
    gpu_free(plan->gs);
    plan->gs = nullptr;
    LS_TRY(gpu_factor(plan->ap.n, plan->sd.rows.as<C<double>>(), factor_prec != LS_C128, s, &plan->gs));
    if (seconds_out) *seconds_out = now_s() - t0;
    return LS_OK;
  });
}

ls_status ls_precond_apply(ls_plan* plan, const void* v_dev, void* z_dev, int nrhs, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan || !v_dev || !z_dev || nrhs < 1) return LS_EINVAL;
    if (!plan->hs && !plan->gs) return LS_ESTATE;
    hipStream_t s = as_stream(hip_stream);
    const long len = plan->gctx.len;
    if (v_dev != z_dev)
      LS_HIP(hipMemcpyAsync(z_dev, v_dev, (size_t)nrhs * len * sizeof(C<double>), hipMemcpyDeviceToDevice, s));
    std::vector<int> lb(nrhs);
    for (int b = 0; b < nrhs; ++b) lb[b] = b;
    C<double>* z = static_cast<C<double>*>(z_dev);
    return precond_list(plan, lb, [&](int b) { return z + (long)b * len; }, s, nullptr);
  });
}

ls_status ls_gmres_solve(ls_plan* plan, const void* g_dev, void* x_dev, int nrhs, double tol, int restart,
                         int maxit, ls_prec apply_prec, ls_solve_info* info, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan || !g_dev || !x_dev || nrhs < 1 || !info || restart < 1 || maxit < 1 || !(tol > 0.0))
      return LS_EINVAL;
    if (apply_prec != LS_C128 && apply_prec != LS_MIXED) return LS_EINVAL;
    if (!plan->hs && !plan->gs) return LS_ESTATE;
    hipStream_t s = as_stream(hip_stream);
    GmresOps ops;
    ops.apply = [plan](const C<double>* x, C<double>* y, int nb, ls_prec pr, hipStream_t st) {
      return apply_chunked(plan, x, y, nb, pr, st);
    };
    ops.precond_batch = [plan](const std::vector<int>& lb, const std::function<C<double>*(int)>& ptr, hipStream_t st,
                               double* th) { return precond_list(plan, lb, ptr, st, th); };
    const double t0 = now_s();
    ls_status st = gmres_solve(plan->gctx, ops, static_cast<const C<double>*>(g_dev), static_cast<C<double>*>(x_dev),
                               nrhs, tol, restart, maxit, apply_prec, info, s);
    const double tt = now_s() - t0;
    for (int b = 0; b < nrhs; ++b) info[b].t_gpu = tt / nrhs - info[b].t_host;
    return st;
  });
}

// ---- learned stencils -------------------------------------------------------------

ls_status ls_mlp_create(const float* params_host, ls_mlp** out) {
  return guarded([&]() -> ls_status {
    if (!params_host || !out) return LS_EINVAL;
    *out = nullptr;
    ls_mlp* p = new (std::nothrow) ls_mlp();
    if (!p) return LS_ENOMEM;
    ls_status st = mlp_init(p->st, params_host, nullptr);
    if (st == LS_OK && hipStreamSynchronize(nullptr) != hipSuccess) st = LS_EHIP;
    if (st != LS_OK) {
      delete p;
      return st;
    }
    *out = p;
    return LS_OK;
  });
}

ls_status ls_mlp_get_params(const ls_mlp* mlp, float* params_host) {
  return guarded([&]() -> ls_status {
    if (!mlp || !params_host) return LS_EINVAL;
    LS_HIP(hipMemcpy(params_host, mlp->st.w.p, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    return LS_OK;
  });
}

ls_status ls_mlp_forward_backward(ls_mlp* mlp, const float* x_host, const float* t_host, int B, float* y_host,
                                  float* grad_host, double* loss_out, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!mlp || !x_host || !t_host || B < 1) return LS_EINVAL;
    hipStream_t s = as_stream(hip_stream);
    std::vector<float> xpad((size_t)B * MLP_IP, 0.f);
    for (int b = 0; b < B; ++b)
      for (int f = 0; f < MLP_I; ++f) xpad[(size_t)b * MLP_IP + f] = x_host[(size_t)b * MLP_I + f];
    // host rounding of the inputs to bf16 (nearest, ties to even), as the features kernel does
    std::vector<unsigned short> xb(xpad.size());
    for (size_t i = 0; i < xpad.size(); ++i) {
      unsigned u;
      std::memcpy(&u, &xpad[i], 4);
      u += 0x7FFFu + ((u >> 16) & 1u);
      xb[i] = (unsigned short)(u >> 16);
    }
    DevBuf dx, dt;
    LS_TRY(dx.alloc(xb.size() * 2));
    LS_TRY(dt.alloc((size_t)B * MLP_O * 4));
    LS_HIP(hipMemcpyAsync(dx.p, xb.data(), xb.size() * 2, hipMemcpyHostToDevice, s));
    LS_HIP(hipMemcpyAsync(dt.p, t_host, (size_t)B * MLP_O * 4, hipMemcpyHostToDevice, s));
    LS_TRY(mlp_forward(mlp->st, dx.as<unsigned short>(), B, s));
    double loss = 0.0;
    LS_TRY(mlp_backward(mlp->st, dx.as<unsigned short>(), dt.as<float>(), B, &loss, s));
    if (y_host) {
      std::vector<float> y((size_t)B * MLP_OP);
      LS_HIP(hipMemcpyAsync(y.data(), mlp->st.y.p, y.size() * 4, hipMemcpyDeviceToHost, s));
      LS_HIP(hipStreamSynchronize(s));
      for (int b = 0; b < B; ++b)
        std::memcpy(y_host + (size_t)b * MLP_O, y.data() + (size_t)b * MLP_OP, MLP_O * 4);
    }
    if (grad_host) LS_HIP(hipMemcpyAsync(grad_host, mlp->st.grad.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost, s));
    LS_HIP(hipStreamSynchronize(s));
    if (loss_out) *loss_out = loss;
    return LS_OK;
  });
}

ls_status ls_mlp_forward(ls_mlp* mlp, const float* x_host, int B, float* y_host, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!mlp || !x_host || !y_host || B < 1) return LS_EINVAL;
    hipStream_t s = as_stream(hip_stream);
    std::vector<unsigned short> xb((size_t)B * MLP_IP, 0);
    for (int b = 0; b < B; ++b)
      for (int f = 0; f < MLP_I; ++f) {
        unsigned u;
        std::memcpy(&u, &x_host[(size_t)b * MLP_I + f], 4);
        u += 0x7FFFu + ((u >> 16) & 1u);            // to bf16, nearest, ties to even
        xb[(size_t)b * MLP_IP + f] = (unsigned short)(u >> 16);
      }
    DevBuf dx;
    LS_TRY(dx.alloc(xb.size() * 2));
    LS_HIP(hipMemcpyAsync(dx.p, xb.data(), xb.size() * 2, hipMemcpyHostToDevice, s));
    LS_TRY(mlp_infer(mlp->st, dx.as<unsigned short>(), B, s));
    std::vector<float> y((size_t)B * MLP_OP);
    LS_HIP(hipMemcpyAsync(y.data(), mlp->st.y.p, y.size() * 4, hipMemcpyDeviceToHost, s));
    LS_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < B; ++b) std::memcpy(y_host + (size_t)b * MLP_O, y.data() + (size_t)b * MLP_OP, MLP_O * 4);
    return LS_OK;
  });
}

ls_status ls_mlp_adam_step(ls_mlp* mlp, double lr, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!mlp || !(lr > 0.0) || !std::isfinite(lr)) return LS_EINVAL;
    if (!mlp->st.have_grad) return LS_ESTATE;
    LS_TRY(mlp_adam(mlp->st, lr, as_stream(hip_stream)));
    LS_HIP(hipStreamSynchronize(as_stream(hip_stream)));
    return LS_OK;
  });
}

ls_status ls_mlp_add_samples(ls_mlp* mlp, ls_plan* plan, const int* points_host, int npts, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!mlp || !plan || !points_host || npts < 1 || plan->ap.n < 4) return LS_EINVAL;
    return mlp_add_samples(mlp->st, plan->sd, plan->ap.n, plan->ap.k, plan->ap.m64.as<C<double>>(), kPointFitM0,
                           points_host, npts, as_stream(hip_stream));
  });
}

long ls_mlp_num_samples(const ls_mlp* mlp) { return mlp ? mlp->st.nsamples : 0; }

ls_status ls_mlp_get_samples(const ls_mlp* mlp, float* x_host, float* t_host) {
  return guarded([&]() -> ls_status {
    if (!mlp) return LS_EINVAL;
    const long N = mlp->st.nsamples;
    if (N == 0) return LS_OK;
    if (x_host) {
      std::vector<unsigned short> xb((size_t)N * MLP_IP);
      LS_HIP(hipMemcpy(xb.data(), mlp->st.xs.p, xb.size() * 2, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < xb.size(); ++i) {
        const unsigned u = ((unsigned)xb[i]) << 16;
        std::memcpy(&x_host[i], &u, 4);
      }
    }
    if (t_host) LS_HIP(hipMemcpy(t_host, mlp->st.ts.p, (size_t)N * MLP_O * 4, hipMemcpyDeviceToHost));
    return LS_OK;
  });
}

ls_status ls_mlp_train(ls_mlp* mlp, int steps, int batch, double lr, unsigned seed, double* loss_out,
                       void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!mlp || !(lr > 0.0) || !std::isfinite(lr)) return LS_EINVAL;
    return mlp_train(mlp->st, steps, batch, lr, seed, loss_out, as_stream(hip_stream));
  });
}

ls_status ls_mlp_save(const ls_mlp* mlp, const char* path) {
  return guarded([&]() -> ls_status {
    if (!mlp || !path) return LS_EINVAL;
    std::vector<float> buf(3 * (size_t)MLP_NPARAM);
    LS_HIP(hipMemcpy(buf.data(), mlp->st.w.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost));
    LS_HIP(hipMemcpy(buf.data() + MLP_NPARAM, mlp->st.m.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost));
    LS_HIP(hipMemcpy(buf.data() + 2 * MLP_NPARAM, mlp->st.v.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) return LS_EIO;
    std::fprintf(f,
                 "{\"format\": \"ls_mlp\", \"version\": 1, \"nparam\": %ld, \"adam_t\": %d, \"layout\": "
                 "\"W1[250][256] b1[256] W2[256][256] b2[256] W3[256][468] b3[468]; then Adam m, v\"}\n",
                 (long)MLP_NPARAM, mlp->st.t);
    const size_t wr = std::fwrite(buf.data(), 4, buf.size(), f);
    std::fclose(f);
    return wr == buf.size() ? LS_OK : LS_EIO;
  });
}

ls_status ls_mlp_load(const char* path, ls_mlp** out) {
  return guarded([&]() -> ls_status {
    if (!path || !out) return LS_EINVAL;
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return LS_EIO;
    char line[512];
    if (!std::fgets(line, sizeof(line), f)) {
      std::fclose(f);
      return LS_EIO;
    }
    long np = 0;
    int t = 0;
    const char* pn = std::strstr(line, "\"nparam\":");
    const char* pt = std::strstr(line, "\"adam_t\":");
    if (!std::strstr(line, "\"ls_mlp\"") || !pn || !pt || std::sscanf(pn + 9, "%ld", &np) != 1 ||
        std::sscanf(pt + 9, "%d", &t) != 1 || np != MLP_NPARAM) {
      std::fclose(f);
      return LS_EIO;
    }
    std::vector<float> buf(3 * (size_t)MLP_NPARAM);
    const size_t rd = std::fread(buf.data(), 4, buf.size(), f);
    std::fclose(f);
    if (rd != buf.size()) return LS_EIO;
    ls_mlp* p = nullptr;
    LS_TRY(ls_mlp_create(buf.data(), &p));
    if (hipMemcpy(p->st.m.p, buf.data() + MLP_NPARAM, MLP_NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->st.v.p, buf.data() + 2 * MLP_NPARAM, MLP_NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess) {
      delete p;
      return LS_EHIP;
    }
    p->st.t = t;
    *out = p;
    return LS_OK;
  });
}

void ls_mlp_destroy(ls_mlp* mlp) {
  if (!mlp) return;
  (void)hipDeviceSynchronize();
  delete mlp;
}

ls_status ls_stencil_fit_learned(ls_plan* plan, ls_mlp* mlp, int* n_fallback_out, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan || !mlp || plan->ap.n < 4) return LS_EINVAL;
    hipStream_t s = as_stream(hip_stream);
    host_free(plan->hs);
    plan->hs = nullptr;
    gpu_free(plan->gs);
    plan->gs = nullptr;
    plan->sd.have_point = false;
    plan->sd.have_rows = false;
    LS_TRY(learned_fit(plan->sd, mlp->st, plan->ap.n, plan->ap.k, plan->ap.m64.as<C<double>>(), kPointFitM0,
                       n_fallback_out, s));
    LS_TRY(assemble_rows(plan->sd, plan->ap.n, plan->ap.m64.as<C<double>>(), s));
    LS_HIP(hipStreamSynchronize(s));
    plan->sd.have_rows = true;
    return LS_OK;
  });
}

ls_status ls_sparse_factor_host(int n, const void* rows_host, size_t host_mem_cap, ls_prec factor_prec,
                                ls_sparse** out) {
  return guarded([&]() -> ls_status {
    if (n < 1 || !rows_host || !out) return LS_EINVAL;
    if (factor_prec != LS_C128 && factor_prec != LS_C64 && factor_prec != LS_MIXED) return LS_EINVAL;
    *out = nullptr;
    ls_sparse* sp = new (std::nothrow) ls_sparse();
    if (!sp) return LS_ENOMEM;
    ls_status st = host_factor(n, static_cast<const std::complex<double>*>(rows_host), host_mem_cap,
                               factor_prec != LS_C128, &sp->hs);
    if (st != LS_OK) {
      delete sp;
      return st;
    }
    *out = sp;
    return LS_OK;
  });
}

ls_status ls_sparse_solve_host(ls_sparse* sp, void* b_host, int nrhs) {
  return guarded([&]() -> ls_status {
    if (!sp || !b_host || nrhs < 1) return LS_EINVAL;
    if (!sp->hs) return LS_ESTATE;
    return host_solve(sp->hs, static_cast<std::complex<double>*>(b_host), nrhs);
  });
}

ls_status ls_sparse_factor_gpu(int n, const void* rows_host, ls_prec factor_prec, void* hip_stream, ls_sparse** out) {
  return guarded([&]() -> ls_status {
    if (!rows_host || !out || n < 3 || n > 192) return LS_EINVAL;
    if (factor_prec != LS_C128 && factor_prec != LS_C64 && factor_prec != LS_MIXED) return LS_EINVAL;
    *out = nullptr;
    hipStream_t s = as_stream(hip_stream);
    const size_t rb = (size_t)n * n * n * 243 * sizeof(C<double>);
    DevBuf rows;
    LS_TRY(rows.alloc(rb));
    LS_HIP(hipMemcpyAsync(rows.p, rows_host, rb, hipMemcpyHostToDevice, s));
    ls_sparse* sp = new (std::nothrow) ls_sparse();
    if (!sp) return LS_ENOMEM;
    ls_status st = gpu_factor(n, rows.as<C<double>>(), factor_prec != LS_C128, s, &sp->gs);
    if (st != LS_OK) {
      delete sp;
      return st;
    }
    *out = sp;
    return LS_OK;
  });
}

ls_status ls_sparse_solve_gpu(ls_sparse* sp, void* b_dev, int nrhs, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!sp || !b_dev || nrhs < 1) return LS_EINVAL;
    if (!sp->gs) return LS_ESTATE;
    return gpu_solve(sp->gs, static_cast<C<double>*>(b_dev), static_cast<C<double>*>(b_dev), nrhs,
                     as_stream(hip_stream));
  });
}

ls_status ls_sparse_info(const ls_sparse* sp, size_t* bytes, double* flops) {
  return guarded([&]() -> ls_status {
    if (!sp) return LS_EINVAL;
    if (bytes) *bytes = sp->gs ? gpu_factor_bytes(sp->gs) : host_factor_bytes(sp->hs);
    if (flops) *flops = sp->gs ? gpu_factor_flops(sp->gs) : host_factor_flops(sp->hs);
    return LS_OK;
  });
}

void ls_sparse_destroy(ls_sparse* sp) { delete sp; }

ls_status ls_plan_set_form(ls_plan* plan, ls_form form, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan || (form != LS_FORM_DYADIC && form != LS_FORM_PAPER)) return LS_EINVAL;
    return apply_plan_set_form(plan->ap, (int)form, as_stream(hip_stream));
  });
}

int ls_plan_fft_size(const ls_plan* plan) { return plan ? plan->ap.P : 0; }

void ls_plan_destroy(ls_plan* plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  delete plan;
}

}  // extern "C"
