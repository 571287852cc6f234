// Learned stencils: training samples from the exact per-point fit, training,
// and the learned fit with exact-fit fallback (project extension of Section 3).
//
//   features_kernel : x = Re, Im of m on the 5^3 patch / 0.3 (BF16, 256 wide)
//   gauge_kernel    : alpha~ = alpha (alpha_centre)^-1 (centre block = I)
//   encode_kernel   : target = off-centre blocks of (alpha~_i - alpha~_class) / T_SCALE (468 reals)
//   decode_kernel   : alpha^_i = alpha~_class + T_SCALE * network output (centre block I)
//   locality_kernel : Q = orthonormal basis of alpha^_i; accept when
//                     tr(Q^H Gram_i Q) <= tr(alpha_c^H Gram_i alpha_c)
#include <algorithm>
#include <cmath>
#include <random>
#include <vector>

#include "common.h"
#include "learned.h"

namespace ls {

namespace {

constexpr int R81 = 81;
constexpr int CENTRE = 13;          // index of offset (0,0,0) in the interior tau
constexpr double kGaugeCondMax = 1e6;   // training samples need a well-conditioned centre block

__device__ __forceinline__ unsigned short f2bf_l(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// xb[q] = features of point pts[sel[q]] (sel == nullptr: q itself), q < np
__global__ void features_kernel(int n, const C<double>* __restrict__ m, const int* __restrict__ pts,
                                const int* __restrict__ sel, int np, unsigned short* __restrict__ xb) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)np * MLP_IP) return;
  const int p = (int)(id / MLP_IP), f = (int)(id % MLP_IP);
  float v = 0.f;
  if (f < MLP_I) {
    const int t = f / 2, part = f % 2;
    const int o1 = t / 25 - 2, o2 = (t / 5) % 5 - 2, o3 = t % 5 - 2;
    const int i = pts[sel ? sel[p] : p];
    const int i3 = i % n, i2 = (i / n) % n, i1 = i / (n * n);
    const int j1 = i1 + o1, j2 = i2 + o2, j3 = i3 + o3;
    if (j1 >= 0 && j1 < n && j2 >= 0 && j2 < n && j3 >= 0 && j3 < n) {
      const C<double> mv = m[((long)j1 * n + j2) * n + j3];
      v = (float)((part ? mv.im : mv.re) / MLP_M_SCALE);
    }
  }
  xb[id] = f2bf_l(v);
}

// 3x3 complex inverse by cofactors
__device__ inline void inv3(const C<double> a[3][3], C<double> r[3][3]) {
  C<double> cof[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      cof[i][j] = a[i1][j1] * a[i2][j2] - a[i1][j2] * a[i2][j1];
    }
  const C<double> det = a[0][0] * cof[0][0] + a[0][1] * cof[0][1] + a[0][2] * cof[0][2];
  const double dd = det.re * det.re + det.im * det.im;
  const C<double> idet = cmk(det.re / dd, -det.im / dd);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r[i][j] = cof[j][i] * idet;
}

// out[p] = alpha[p] (alpha[p]_centre)^-1 for cnt stencils given by row pointers;
// ok[p] (when given) = 1 if the centre block's Frobenius condition number
// |A0|_F |A0^-1|_F is at most kGaugeCondMax (the gauge is then well defined)
__global__ void gauge_kernel(const C<double>* __restrict__ alpha, const int* __restrict__ pts, int cnt,
                             C<double>* __restrict__ out, int* __restrict__ ok) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= cnt) return;
  const C<double>* a = alpha + (long)(pts ? pts[p] : p) * 243;
  C<double> A0[3][3], Ai[3][3];
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) A0[c][r] = a[(3 * CENTRE + c) * 3 + r];
  inv3(A0, Ai);
  if (ok) {
    double f0 = 0.0, f1 = 0.0;
    for (int c = 0; c < 3; ++c)
      for (int r = 0; r < 3; ++r) {
        f0 += A0[c][r].re * A0[c][r].re + A0[c][r].im * A0[c][r].im;
        f1 += Ai[c][r].re * Ai[c][r].re + Ai[c][r].im * Ai[c][r].im;
      }
    const double cf = sqrt(f0 * f1);
    ok[p] = (cf == cf && cf <= kGaugeCondMax) ? 1 : 0;     // NaN (singular block) fails too
  }
  C<double>* o = out + (long)p * 243;
  for (int row = 0; row < R81; ++row)
    for (int r = 0; r < 3; ++r) {
      C<double> s = cmk(0.0, 0.0);
      for (int q = 0; q < 3; ++q) s = s + a[row * 3 + q] * Ai[q][r];
      o[row * 3 + r] = s;
    }
}

// targets[p][2 (9 t + 3 c + r) + {0,1}] = Re, Im of (gt[p] - gclass)[(a, c), r], a != centre
// targets[q] from gt[sel[q]], q < cnt
__global__ void encode_kernel(const C<double>* __restrict__ gt, const C<double>* __restrict__ gclass,
                              const int* __restrict__ sel, int cnt, float* __restrict__ targets) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)cnt * 234) return;
  const long p = id / 234;
  const long src = sel[p];
  const int e = (int)(id % 234);
  const int t = e / 9, c = (e % 9) / 3, r = e % 3;
  const int a = t < CENTRE ? t : t + 1;
  const C<double> d = gt[src * 243 + (3 * a + c) * 3 + r] - gclass[(3 * a + c) * 3 + r];
  targets[p * MLP_O + 2 * e] = (float)(d.re / MLP_T_SCALE);
  targets[p * MLP_O + 2 * e + 1] = (float)(d.im / MLP_T_SCALE);
}

// alpha^[pts[p]] = gclass + y[p] (centre block stays the identity of gclass)
__global__ void decode_kernel(const float* __restrict__ y, const C<double>* __restrict__ gclass, const int* __restrict__ pts,
                              int cnt, C<double>* __restrict__ alpha) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)cnt * 243) return;
  const long p = id / 243;
  const int row = (int)(id % 243) / 3, r = (int)(id % 3);
  const int a = row / 3, c = row % 3;
  C<double> v = gclass[row * 3 + r];
  if (a != CENTRE) {
    const int t = a < CENTRE ? a : a - 1;
    const int e = 9 * t + 3 * c + r;
    v = v + cmk(MLP_T_SCALE * (double)y[p * MLP_OP + 2 * e], MLP_T_SCALE * (double)y[p * MLP_OP + 2 * e + 1]);
  }
  alpha[(long)pts[p] * 243 + row * 3 + r] = v;
}

__device__ __forceinline__ void wsync_l() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// One wavefront per point.  Orthonormalises alpha[pts[p]] in place (MGS) and
// sets accept[p] = 1 when its trace against the packed Gram is <= the class
// stencil's; writes the ratio.
__global__ __launch_bounds__(64) void locality_kernel(const C<double>* __restrict__ Gall, const int* __restrict__ pts,
                                                      int cnt, const C<double>* __restrict__ aclass,
                                                      C<double>* __restrict__ alpha, int* __restrict__ accept,
                                                      double* __restrict__ ratio) {
  __shared__ C<double> Q[R81][3];
  __shared__ C<double> A[R81][3];
  const int p = blockIdx.x, l = threadIdx.x;
  if (p >= cnt) return;
  C<double>* ap = alpha + (long)pts[p] * 243;
  const C<double>* G = Gall + (long)p * 3321;
  for (int e = l; e < 243; e += 64) {
    Q[e / 3][e % 3] = ap[e];
    A[e / 3][e % 3] = aclass[e];
  }
  wsync_l();
  for (int pass = 0; pass < 2; ++pass)
    for (int c = 0; c < 3; ++c) {
      for (int d = 0; d < c; ++d) {
        double pr = 0.0, pi = 0.0;
        for (int i = l; i < R81; i += 64) {
          const C<double> a = Q[i][d], b = Q[i][c];
          pr += a.re * b.re + a.im * b.im;
          pi += a.re * b.im - a.im * b.re;
        }
        for (int o = 32; o > 0; o >>= 1) {
          pr += __shfl_xor(pr, o);
          pi += __shfl_xor(pi, o);
        }
        for (int i = l; i < R81; i += 64) Q[i][c] = Q[i][c] - Q[i][d] * cmk(pr, pi);
        wsync_l();
      }
      double nr = 0.0;
      for (int i = l; i < R81; i += 64) nr += Q[i][c].re * Q[i][c].re + Q[i][c].im * Q[i][c].im;
      for (int o = 32; o > 0; o >>= 1) nr += __shfl_xor(nr, o);
      const double sc = 1.0 / sqrt(nr);
      for (int i = l; i < R81; i += 64) Q[i][c] = cscale(Q[i][c], sc);
      wsync_l();
    }
  // traces tr(X^H G X) for X = Q and X = A (the class stencil, orthonormal),
  // walking the packed lower triangle of G in order (lane l takes entries
  // l, l + 64, ..., so every load of the wave is one contiguous kilobyte):
  // the entry (i, j), j < i, and its mirror (j, i) = conj(G_ij) contribute
  // 2 Re(sum_v conj(X_iv) G_ij X_jv), the diagonal once
  double tq = 0.0, ta = 0.0;
  int i = 0;
  for (int e = l; e < 3321; e += 64) {
    while ((i + 1) * (i + 2) / 2 <= e) ++i;           // row of entry e (advances monotonically)
    const int j = e - i * (i + 1) / 2;
    const C<double> g = G[e];
    const double w = (j < i) ? 2.0 : 1.0;
    double sq = 0.0, sa = 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      sq += (cconj(Q[i][v]) * (g * Q[j][v])).re;
      sa += (cconj(A[i][v]) * (g * A[j][v])).re;
    }
    tq += w * sq;
    ta += w * sa;
  }
  for (int o = 32; o > 0; o >>= 1) {
    tq += __shfl_xor(tq, o);
    ta += __shfl_xor(ta, o);
  }
  // strictly more local than the class stencil (so a network that only
  // reproduces the class stencil falls back to the exact fit)
  const bool ok = tq < ta * (1.0 - 1e-9);
  if (ok)
    for (int e = l; e < 243; e += 64) ap[e] = Q[e / 3][e % 3];
  if (l == 0) {
    accept[p] = ok ? 1 : 0;
    ratio[p] = tq / ta;
  }
}

inline unsigned nbl(long len, int t) { return (unsigned)((len + t - 1) / t); }

std::vector<int> interior_points(int n) {
  std::vector<int> pts;
  for (int a = 1; a < n - 1; ++a)
    for (int b = 1; b < n - 1; ++b)
      for (int c = 1; c < n - 1; ++c) pts.push_back((a * n + b) * n + c);
  return pts;
}

}  // namespace

// gauge-fixed class stencil alpha~_class (interior class) into out (81 x 3)
static ls_status class_gauge(StencilData& sd, DevBuf& out, hipStream_t s) {
  LS_TRY(out.alloc(243 * sizeof(C<double>)));
  hipLaunchKernelGGL(gauge_kernel, dim3(1), dim3(64), 0, s, sd.alpha.as<C<double>>() + 13L * 243, nullptr, 1,
                     out.as<C<double>>(), nullptr);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status mlp_add_samples(MlpState& st, StencilData& sd, int n, double k, const C<double>* m, double m0,
                          const int* pts_host, int npts, hipStream_t s) {
  if (npts <= 0) return LS_EINVAL;
  for (int q = 0; q < npts; ++q) {
    const int i = pts_host[q];
    const int i3 = i % n, i2 = (i / n) % n, i1 = i / (n * n);
    if (i < 0 || i >= n * n * n || i1 == 0 || i1 == n - 1 || i2 == 0 || i2 == n - 1 || i3 == 0 || i3 == n - 1)
      return LS_EINVAL;   // samples are interior points only
  }
  if (!sd.have_class) LS_TRY(class_fit(sd, n, k, s));
  const long need = st.nsamples + npts;
  if (need > st.cap) {
    const long cap = std::max(need, 2 * st.cap + 4096);
    DevBuf nx, nt;
    LS_TRY(nx.alloc((size_t)cap * MLP_IP * 2));
    LS_TRY(nt.alloc((size_t)cap * MLP_O * 4));
    if (st.nsamples) {
      LS_HIP(hipMemcpyAsync(nx.p, st.xs.p, (size_t)st.nsamples * MLP_IP * 2, hipMemcpyDeviceToDevice, s));
      LS_HIP(hipMemcpyAsync(nt.p, st.ts.p, (size_t)st.nsamples * MLP_O * 4, hipMemcpyDeviceToDevice, s));
    }
    LS_HIP(hipStreamSynchronize(s));
    std::swap(st.xs.p, nx.p);
    std::swap(st.xs.bytes, nx.bytes);
    std::swap(st.ts.p, nt.p);
    std::swap(st.ts.bytes, nt.bytes);
    st.cap = cap;
  }
  PointFitCtx ctx;
  const int B = std::min(npts, 8192);
  LS_TRY(pointfit_prepare(ctx, sd, n, k, B, s));
  DevBuf dpts, gclass, gt, dok, dsel;
  LS_TRY(dpts.alloc((size_t)npts * sizeof(int)));
  LS_HIP(hipMemcpyAsync(dpts.p, pts_host, (size_t)npts * sizeof(int), hipMemcpyHostToDevice, s));
  LS_TRY(class_gauge(sd, gclass, s));
  LS_TRY(gt.alloc((size_t)B * 243 * sizeof(C<double>)));
  LS_TRY(dok.alloc((size_t)B * sizeof(int)));
  LS_TRY(dsel.alloc((size_t)B * sizeof(int)));
  std::vector<int> ok(B), sel;
  long added = 0;
  for (int p0 = 0; p0 < npts; p0 += B) {
    const int cnt = std::min(B, npts - p0);
    const int* dp = dpts.as<int>() + p0;
    LS_TRY(pointfit_grams(ctx, m, m0, dp, cnt, s));
    LS_TRY(pointfit_solve(ctx, sd, dp, cnt, kPointIters, s));
    hipLaunchKernelGGL(gauge_kernel, dim3(nbl(cnt, 64)), dim3(64), 0, s, sd.palpha.as<C<double>>(), dp, cnt,
                       gt.as<C<double>>(), dok.as<int>());
    LS_HIP(hipGetLastError());
    LS_HIP(hipMemcpyAsync(ok.data(), dok.p, cnt * sizeof(int), hipMemcpyDeviceToHost, s));
    LS_HIP(hipStreamSynchronize(s));
    sel.clear();
    for (int q = 0; q < cnt; ++q)
      if (ok[q]) sel.push_back(q);
    const int cg = (int)sel.size();
    if (cg == 0) continue;
    LS_HIP(hipMemcpyAsync(dsel.p, sel.data(), cg * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(encode_kernel, dim3(nbl((long)cg * 234, 256)), dim3(256), 0, s, gt.as<C<double>>(),
                       gclass.as<C<double>>(), dsel.as<int>(), cg, st.ts.as<float>() + (st.nsamples + added) * MLP_O);
    hipLaunchKernelGGL(features_kernel, dim3(nbl((long)cg * MLP_IP, 256)), dim3(256), 0, s, n, m, dp,
                       dsel.as<int>(), cg, st.xs.as<unsigned short>() + (st.nsamples + added) * MLP_IP);
    LS_HIP(hipGetLastError());
    added += cg;
  }
  LS_HIP(hipStreamSynchronize(s));
  st.nsamples += added;
  sd.have_point = false;      // palpha now holds a partial fit: not a usable per-point stencil set
  return LS_OK;
}

namespace {
__global__ void gather_rows_kernel(const unsigned short* __restrict__ xs, const float* __restrict__ ts,
                                   const int* __restrict__ idx, int Bm, unsigned short* __restrict__ xb,
                                   float* __restrict__ tb) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < (long)Bm * MLP_IP) xb[id] = xs[(long)idx[id / MLP_IP] * MLP_IP + id % MLP_IP];
  if (id < (long)Bm * MLP_O) tb[id] = ts[(long)idx[id / MLP_O] * MLP_O + id % MLP_O];
}
}  // namespace

ls_status mlp_train(MlpState& st, int steps, int batch, double lr, unsigned seed, double* loss_hist, hipStream_t s) {
  if (st.nsamples < 1 || steps < 1 || batch < 1) return LS_EINVAL;
  const int Bm = (int)std::min<long>(batch, st.nsamples);
  LS_TRY(mlp_workspace(st, Bm));
  DevBuf xb, tb, didx;
  LS_TRY(xb.alloc((size_t)Bm * MLP_IP * 2));
  LS_TRY(tb.alloc((size_t)Bm * MLP_O * 4));
  LS_TRY(didx.alloc((size_t)Bm * sizeof(int)));
  std::mt19937_64 rng(seed);
  std::vector<int> perm(st.nsamples);
  for (long i = 0; i < st.nsamples; ++i) perm[i] = (int)i;
  long pos = st.nsamples;
  std::vector<int> idx(Bm);
  for (int it = 0; it < steps; ++it) {
    for (int b = 0; b < Bm; ++b) {          // epochs of a seeded permutation
      if (pos >= st.nsamples) {
        std::shuffle(perm.begin(), perm.end(), rng);
        pos = 0;
      }
      idx[b] = perm[pos++];
    }
    LS_HIP(hipMemcpyAsync(didx.p, idx.data(), Bm * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_rows_kernel, dim3(nbl((long)Bm * MLP_O, 256)), dim3(256), 0, s,
                       st.xs.as<unsigned short>(), st.ts.as<float>(), didx.as<int>(), Bm, xb.as<unsigned short>(),
                       tb.as<float>());
    LS_HIP(hipGetLastError());
    LS_TRY(mlp_forward(st, xb.as<unsigned short>(), Bm, s));
    double loss = 0.0;
    LS_TRY(mlp_backward(st, xb.as<unsigned short>(), tb.as<float>(), Bm, loss_hist ? &loss : nullptr, s));
    if (loss_hist) loss_hist[it] = loss;
    LS_TRY(mlp_adam(st, lr, s));
  }
  LS_HIP(hipStreamSynchronize(s));
  return LS_OK;
}

ls_status learned_fit(StencilData& sd, MlpState& st, int n, double k, const C<double>* m, double m0,
                      int* n_fallback, hipStream_t s) {
  if (!sd.have_class) LS_TRY(class_fit(sd, n, k, s));
  std::vector<int> pts = interior_points(n);
  const int npts = (int)pts.size();
  const int B = std::min(npts, 8192);
  PointFitCtx ctx;
  LS_TRY(pointfit_prepare(ctx, sd, n, k, B, s));
  DevBuf dpts, gclass, xb, acc, rat, dfail, dslot;
  LS_TRY(dpts.alloc((size_t)npts * sizeof(int)));
  LS_HIP(hipMemcpyAsync(dpts.p, pts.data(), (size_t)npts * sizeof(int), hipMemcpyHostToDevice, s));
  LS_TRY(class_gauge(sd, gclass, s));
  LS_TRY(xb.alloc((size_t)B * MLP_IP * 2));
  LS_TRY(acc.alloc((size_t)B * sizeof(int)));
  LS_TRY(rat.alloc((size_t)B * sizeof(double)));
  LS_TRY(dfail.alloc((size_t)B * sizeof(int)));
  LS_TRY(dslot.alloc((size_t)B * sizeof(int)));
  std::vector<int> accept(B), fail, fslot;
  std::vector<double> ratio(B);
  const long N3 = (long)n * n * n;
  sd.have_learned = false;
  sd.learned_accept.assign(N3, -1);
  sd.learned_ratio.assign(N3, 0.0);
  int nfb = 0;
  for (int p0 = 0; p0 < npts; p0 += B) {
    const int cnt = std::min(B, npts - p0);
    const int* dp = dpts.as<int>() + p0;
    hipLaunchKernelGGL(features_kernel, dim3(nbl((long)cnt * MLP_IP, 256)), dim3(256), 0, s, n, m, dp, nullptr,
                       cnt, xb.as<unsigned short>());
    LS_HIP(hipGetLastError());
    LS_TRY(mlp_infer(st, xb.as<unsigned short>(), cnt, s));
    hipLaunchKernelGGL(decode_kernel, dim3(nbl((long)cnt * 243, 256)), dim3(256), 0, s, st.y.as<float>(),
                       gclass.as<C<double>>(), dp, cnt, sd.palpha.as<C<double>>());
    LS_HIP(hipGetLastError());
    LS_TRY(pointfit_grams(ctx, m, m0, dp, cnt, s));
    hipLaunchKernelGGL(locality_kernel, dim3(cnt), dim3(64), 0, s, ctx.Gb.as<C<double>>(), dp, cnt,
                       sd.alpha.as<C<double>>() + 13L * 243, sd.palpha.as<C<double>>(), acc.as<int>(),
                       rat.as<double>());
    LS_HIP(hipGetLastError());
    LS_HIP(hipMemcpyAsync(accept.data(), acc.p, cnt * sizeof(int), hipMemcpyDeviceToHost, s));
    LS_HIP(hipMemcpyAsync(ratio.data(), rat.p, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    LS_HIP(hipStreamSynchronize(s));
    fail.clear();
    fslot.clear();
    for (int q = 0; q < cnt; ++q) {
      sd.learned_accept[pts[p0 + q]] = accept[q] ? 1 : 0;
      sd.learned_ratio[pts[p0 + q]] = ratio[q];
      if (!accept[q]) {
        fail.push_back(pts[p0 + q]);
        fslot.push_back(q);
      }
    }
    nfb += (int)fail.size();
    if (!fail.empty()) {
      // exact fit for the rejected points from the Grams already in the batch
      LS_HIP(hipMemcpyAsync(dfail.p, fail.data(), fail.size() * sizeof(int), hipMemcpyHostToDevice, s));
      LS_HIP(hipMemcpyAsync(dslot.p, fslot.data(), fslot.size() * sizeof(int), hipMemcpyHostToDevice, s));
      LS_TRY(pointfit_solve(ctx, sd, dfail.as<int>(), (int)fail.size(), kPointIters, s, dslot.as<int>()));
    }
    LS_TRY(pointfit_beta(ctx, sd, dp, cnt, s));
  }
  LS_HIP(hipStreamSynchronize(s));
  if (n_fallback) *n_fallback = nfb;
  sd.have_point = true;
  sd.have_learned = true;
  return LS_OK;
}

}  // namespace ls
