// FFT-based Nystrom apply  y = x + K * (m x)  on gfx950.
//
// Paper: Eq. (5) and Eq. (6) - the convolution (Toeplitz) matrices are
// applied by FFT on the uniform grid (Section 2; Section 3.3 gives the
// O(N log N) cost).  Here the 3x3 dyadic tensor K is embedded in a circulant
// of length P >= 2n - 1 per dimension, its FFT Khat is computed once per
// plan in FP64, and every apply runs five HBM-streaming passes:
//
//   pass 1  dim 1 forward  (x, m) -> X1[b][c][q1][i2 i3]   n rows in, P out, u = m x fused
//   pass 2  dim 2 forward  X1 -> X2[b][c][q1][q2][i3]       n rows in, P out
//   pass 3  dim 3 forward, 3x3 multiply by Khat(q), dim 3 inverse, in place in X2
//   pass 4  dim 2 inverse  X2 -> Y1[b][c][q1][i2][i3]       P rows in, n out
//   pass 5  dim 1 inverse  y = x + Y1                      P rows in, n out, identity fused
//
// Zero padding is never materialised: forward passes read only the n
// non-zero rows, inverse passes write only the n rows that are kept.
//
// Every 1-D transform is a four-step FFT of length P = N1 N2 held in
// registers: a length-N2 DFT per thread, a twiddle by W_P^{j q}, one LDS
// exchange, a length-N1 DFT per thread.  Passes 1, 2, 4, 5 transform along a
// strided dimension: a workgroup owns T consecutive lines, so every global
// access is a run of T consecutive elements (T = 16 or 32, 256 B) and the LDS
// exchange is bank-conflict free (the line index is the fastest lane index).
// Pass 3 transforms along the contiguous dimension; a workgroup owns one
// octant line (f1, f2) of Khat and the up-to-four grid lines
// (+-f1, +-f2) that share it, so Khat is read from HBM once per apply.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "common.h"
#include "fft_kernels.h"

namespace ls {

static const int kSizes[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768};

int choose_fft_size(int n) {
  for (int P : kSizes)
    if (P >= 2 * n - 1) return P;
  return 0;
}
bool fft_size_supported(int P) {
  for (int s : kSizes)
    if (s == P) return true;
  return false;
}

// ---- Nystrom weights ----------------------------------------------------------
// Component cidx of K(r) on the P^3 circulant embedding: index r mod P for
// |r_d| <= n-1, zero elsewhere.  cidx: 0 xx, 1 yy, 2 zz, 3 xy, 4 xz, 5 yz.
__global__ void embed_kernel_component(C<double>* __restrict__ E, int n, int P, double k, double h,
                                       int cidx) {
  const long tot = (long)P * P * P;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= tot) return;
  const int e3 = (int)(id % P);
  const int e2 = (int)((id / P) % P);
  const int e1 = (int)(id / ((long)P * P));
  const int r1 = e1 <= P / 2 ? e1 : e1 - P;
  const int r2 = e2 <= P / 2 ? e2 : e2 - P;
  const int r3 = e3 <= P / 2 ? e3 : e3 - P;
  C<double> val = cmk(0.0, 0.0);
  if (abs(r1) <= n - 1 && abs(r2) <= n - 1 && abs(r3) <= n - 1) {
    const int ia = (cidx < 3) ? cidx : (cidx == 5 ? 1 : 0);
    const int ib = (cidx < 3) ? cidx : (cidx == 3 ? 1 : 2);
    if (r1 == 0 && r2 == 0 && r3 == 0) {
      if (ia == ib) {
        // equal-volume ball: a = h (3/(4 pi))^(1/3); K(0) = (2/3)[(1 - ika)e^{ika} - 1] - 1/3
        const double a = h * cbrt(3.0 / (4.0 * kPi));
        double sn, cs;
        sincos(k * a, &sn, &cs);
        // (1 - i k a)(cs + i sn) = (cs + k a sn) + i (sn - k a cs)
        const double br = cs + k * a * sn - 1.0, bi = sn - k * a * cs;
        val = cmk((2.0 / 3.0) * br - 1.0 / 3.0, (2.0 / 3.0) * bi);
      }
    } else {
      const double x[3] = {h * r1, h * r2, h * r3};
      const double R2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      const double R = sqrt(R2);
      double sn, cs;
      sincos(k * R, &sn, &cs);
      const double g = 1.0 / (4.0 * kPi * R);
      const C<double> G = cmk(cs * g, sn * g);
      const C<double> ciso = G * cmk(k * k - 1.0 / R2, k / R);
      const C<double> crad = G * cmk(-k * k + 3.0 / R2, -3.0 * k / R);
      const double xa = x[ia] / R, xb = x[ib] / R;
      const double h3 = h * h * h;
      C<double> v = cscale(crad, xa * xb);
      if (ia == ib) v = v + ciso;
      val = cscale(v, h3);
    }
  }
  E[id] = val;
}

// Octant gather: Kh[f1][f2][cidx][f3] = E[f1][f2][f3] * inv
__global__ void gather_octant(const C<double>* __restrict__ E, C<double>* __restrict__ kh64,
                              C<float>* __restrict__ kh32, int P, int cidx, double inv) {
  const int H = P / 2 + 1;
  const long tot = (long)H * H * H;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= tot) return;
  const int f3 = (int)(id % H);
  const int f2 = (int)((id / H) % H);
  const int f1 = (int)(id / ((long)H * H));
  C<double> v = cscale(E[((long)f1 * P + f2) * P + f3], inv);
  const long o = (((long)f1 * H + f2) * 6 + cidx) * H + f3;
  kh64[o] = v;
  kh32[o] = ccast<float>(v);
}

__global__ void to_c64(const C<double>* __restrict__ a, C<float>* __restrict__ b, long cnt) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < cnt) b[id] = ccast<float>(a[id]);
}

// ---- the paper's own form (Section 2): y_d = x_d + k^2 G*(m x_d) + G^d*(p.x) ----
// Component cidx of (k^2 G, G^1, G^2, G^3) on the P^3 circulant embedding
// (index r mod P for |r_d| <= n-1, zero elsewhere).  Off the origin:
// k^2 h^3 G(hr) and h^3 dG/dx_d(hr) = h^3 G (ik - 1/R) x_d / R.  At the
// origin: k^2 times the integral of G over the ball of volume h^3,
// e^{ika}(1 - ika) - 1, and 0 for the odd G^d.
__global__ void embed_paper_component(C<double>* __restrict__ E, int n, int P, double k, double h, int cidx) {
  const long tot = (long)P * P * P;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= tot) return;
  const int e3 = (int)(id % P);
  const int e2 = (int)((id / P) % P);
  const int e1 = (int)(id / ((long)P * P));
  const int r1 = e1 <= P / 2 ? e1 : e1 - P;
  const int r2 = e2 <= P / 2 ? e2 : e2 - P;
  const int r3 = e3 <= P / 2 ? e3 : e3 - P;
  C<double> val = cmk(0.0, 0.0);
  if (abs(r1) <= n - 1 && abs(r2) <= n - 1 && abs(r3) <= n - 1) {
    if (r1 == 0 && r2 == 0 && r3 == 0) {
      if (cidx == 0) {
        const double a = h * cbrt(3.0 / (4.0 * kPi));
        double sn, cs;
        sincos(k * a, &sn, &cs);
        val = cmk(cs + k * a * sn - 1.0, sn - k * a * cs);   // (1 - ika) e^{ika} - 1
      }
    } else {
      const double x[3] = {h * r1, h * r2, h * r3};
      const double R = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      double sn, cs;
      sincos(k * R, &sn, &cs);
      const double g = h * h * h / (4.0 * kPi * R);
      const C<double> G = cmk(cs * g, sn * g);                // h^3 G(hr)
      if (cidx == 0)
        val = cscale(G, k * k);
      else
        val = cscale(G * cmk(-1.0 / R, k), x[cidx - 1] / R);
    }
  }
  E[id] = val;
}

// Kp[f1][f2][cidx][f3] = E[f1][f2][f3] * inv
__global__ void gather_octant4(const C<double>* __restrict__ E, C<double>* __restrict__ kp64,
                               C<float>* __restrict__ kp32, int P, int cidx, double inv) {
  const int H = P / 2 + 1;
  const long tot = (long)H * H * H;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= tot) return;
  const int f3 = (int)(id % H);
  const int f2 = (int)((id / H) % H);
  const int f1 = (int)(id / ((long)H * H));
  const C<double> v = cscale(E[((long)f1 * P + f2) * P + f3], inv);
  const long o = (((long)f1 * H + f2) * 4 + cidx) * H + f3;
  kp64[o] = v;
  kp32[o] = ccast<float>(v);
}

// p^d = (m_{i+e_d} - m_{i-e_d}) / (2h) / (1 - m_i), m = 0 outside the grid
__global__ void gradient_p_kernel(const C<double>* __restrict__ m, int n, double h, C<double>* __restrict__ p64,
                                  C<float>* __restrict__ p32) {
  const long n3 = (long)n * n * n;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n3) return;
  const int i3 = (int)(id % n), i2 = (int)((id / n) % n), i1 = (int)(id / ((long)n * n));
  const int ii[3] = {i1, i2, i3};
  const long st[3] = {(long)n * n, (long)n, 1};
  const C<double> mi = m[id];
  const double dr = 1.0 - mi.re, di = -mi.im, dd = dr * dr + di * di;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const C<double> mp = ii[d] + 1 < n ? m[id + st[d]] : cmk(0.0, 0.0);
    const C<double> mm = ii[d] > 0 ? m[id - st[d]] : cmk(0.0, 0.0);
    const C<double> g = cscale(mp - mm, 0.5 / h);
    // g / (1 - m)
    const C<double> q = cmk((g.re * dr + g.im * di) / dd, (g.im * dr - g.re * di) / dd);
    p64[d * n3 + id] = q;
    p32[d * n3 + id] = ccast<float>(q);
  }
}

template <int P>
static ls_status build_symbol(ApplyPlan& ap, hipStream_t s) {
  const long P3 = (long)P * P * P;
  DevBuf E, scr;
  LS_TRY(E.alloc(P3 * sizeof(C<double>)));
  LS_TRY(scr.alloc(P3 * sizeof(C<double>)));
  const int H = P / 2 + 1;
  const long H3 = (long)H * H * H;
  const double inv = 1.0 / (double)P3;
  for (int c = 0; c < 6; ++c) {
    hipLaunchKernelGGL(embed_kernel_component, dim3((unsigned)((P3 + 255) / 256)), dim3(256), 0, s,
                       E.as<C<double>>(), ap.n, P, ap.k, ap.h, c);
    LS_HIP(hipGetLastError());
    LS_TRY(fft3d_f64<P>(E.as<C<double>>(), scr.as<C<double>>(), ap.tw64.as<C<double>>(), s));
    hipLaunchKernelGGL(gather_octant, dim3((unsigned)((H3 + 255) / 256)), dim3(256), 0, s,
                       E.as<C<double>>(), ap.kh64.as<C<double>>(), ap.kh32.as<C<float>>(), P, c, inv);
    LS_HIP(hipGetLastError());
  }
  LS_HIP(hipStreamSynchronize(s));   // E and scr are released on return
  return LS_OK;
}

template <int P>
static ls_status build_paper_symbol(ApplyPlan& ap, hipStream_t s) {
  const long P3 = (long)P * P * P;
  DevBuf E, scr;
  LS_TRY(E.alloc(P3 * sizeof(C<double>)));
  LS_TRY(scr.alloc(P3 * sizeof(C<double>)));
  const int H = P / 2 + 1;
  const long H3 = (long)H * H * H;
  const double inv = 1.0 / (double)P3;
  for (int c = 0; c < 4; ++c) {
    hipLaunchKernelGGL(embed_paper_component, dim3((unsigned)((P3 + 255) / 256)), dim3(256), 0, s,
                       E.as<C<double>>(), ap.n, P, ap.k, ap.h, c);
    LS_HIP(hipGetLastError());
    LS_TRY(fft3d_f64<P>(E.as<C<double>>(), scr.as<C<double>>(), ap.tw64.as<C<double>>(), s));
    hipLaunchKernelGGL(gather_octant4, dim3((unsigned)((H3 + 255) / 256)), dim3(256), 0, s,
                       E.as<C<double>>(), ap.kp64.as<C<double>>(), ap.kp32.as<C<float>>(), P, c, inv);
    LS_HIP(hipGetLastError());
  }
  LS_HIP(hipStreamSynchronize(s));
  return LS_OK;
}

ls_status apply_plan_init(ApplyPlan& ap, int n, double k, int max_rhs, const void* m_dev,
                          hipStream_t s) {
  const int P = choose_fft_size(n);
  if (P == 0 || P > 384) return LS_EINVAL;
  ap.n = n;
  ap.P = P;
  ap.H = P / 2 + 1;
  ap.k = k;
  ap.h = 1.0 / (n + 1);
  ap.max_rhs = max_rhs;
  const long n3 = (long)n * n * n;
  const long H3 = (long)ap.H * ap.H * ap.H;
  LS_TRY(ap.m64.alloc(n3 * sizeof(C<double>)));
  LS_TRY(ap.m32.alloc(n3 * sizeof(C<float>)));
  LS_TRY(ap.kh64.alloc(H3 * 6 * sizeof(C<double>)));
  LS_TRY(ap.kh32.alloc(H3 * 6 * sizeof(C<float>)));
  LS_TRY(ap.tw64.alloc(P * sizeof(C<double>)));
  LS_TRY(ap.tw32.alloc(P * sizeof(C<float>)));
  ap.work_per_rhs64 = (size_t)3 * ((size_t)P * n * n + (size_t)P * P * n) * sizeof(C<double>);
  LS_TRY(ap.work.alloc(ap.work_per_rhs64 * (size_t)max_rhs));
  // twiddles exp(-2 pi i t / P), evaluated in long double on the host
  std::vector<C<double>> t64(P);
  std::vector<C<float>> t32(P);
  for (int t = 0; t < P; ++t) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * t / P;
    t64[t] = cmk((double)cosl(ang), (double)sinl(ang));
    t32[t] = cmk((float)cosl(ang), (float)sinl(ang));
  }
  LS_HIP(hipMemcpyAsync(ap.tw64.p, t64.data(), P * sizeof(C<double>), hipMemcpyHostToDevice, s));
  LS_HIP(hipMemcpyAsync(ap.tw32.p, t32.data(), P * sizeof(C<float>), hipMemcpyHostToDevice, s));
  LS_HIP(hipMemcpyAsync(ap.m64.p, m_dev, n3 * sizeof(C<double>), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(to_c64, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s,
                     ap.m64.as<C<double>>(), ap.m32.as<C<float>>(), n3);
  LS_HIP(hipGetLastError());
  switch (P) {
#define X(SZ) \
  case SZ: return build_symbol<SZ>(ap, s);
    LS_FOR_SIZES(X)
#undef X
  }
  return LS_EINVAL;
}

ls_status apply_plan_set_form(ApplyPlan& ap, int form, hipStream_t s) {
  if (form != 0 && form != 1) return LS_EINVAL;
  if (form == 1 && !ap.kp64.p) {
    const int n = ap.n, P = ap.P, H = ap.H;
    const long n3 = (long)n * n * n, H3 = (long)H * H * H;
    LS_TRY(ap.kp64.alloc(H3 * 4 * sizeof(C<double>)));
    LS_TRY(ap.kp32.alloc(H3 * 4 * sizeof(C<float>)));
    LS_TRY(ap.p64.alloc(3 * n3 * sizeof(C<double>)));
    LS_TRY(ap.p32.alloc(3 * n3 * sizeof(C<float>)));
    // FP64 sizes: X1 and X2 of four fields and W of one, per rhs
    const size_t per = ((size_t)4 * P * n * n + (size_t)4 * P * P * n + (size_t)n3) * sizeof(C<double>);
    LS_TRY(ap.work34.alloc(per * (size_t)ap.max_rhs));
    hipLaunchKernelGGL(gradient_p_kernel, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s,
                       ap.m64.as<C<double>>(), n, ap.h, ap.p64.as<C<double>>(), ap.p32.as<C<float>>());
    LS_HIP(hipGetLastError());
    ls_status st = LS_EINVAL;
    switch (P) {
#define X(SZ) \
  case SZ: st = build_paper_symbol<SZ>(ap, s); break;
      LS_FOR_SIZES(X)
#undef X
    }
    if (st != LS_OK) {
      ap.kp64.release();
      return st;
    }
  }
  ap.form = form;
  return LS_OK;
}

std::vector<int> kmul_team_choices(const ApplyPlan& ap) {
  const Fac f = col_factors(ap.P);
  if (4 * cmax(f.n1, f.n2) == 64) return {1, 2, 4};
  if (job_lanes(cmax(f.n1, f.n2)) == 32) return {1, 2};
  return {1};
}

ls_status apply_run(ApplyPlan& ap, const void* x, void* y, int nrhs, ls_prec prec, hipStream_t s,
                    bool minus_conv, hipEvent_t* ev, void* work) {
  if (nrhs < 1 || (!work && nrhs > ap.max_rhs)) return LS_EINVAL;
  if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
  switch (ap.P) {
#define X(SZ) \
  case SZ: return apply_dispatch<SZ>(ap, x, y, nrhs, prec, minus_conv, s, ev, work);
    LS_FOR_SIZES(X)
#undef X
  }
  return LS_EINVAL;
}

ls_status apply_batched(ApplyPlan& ap, const void* x, void* y, int nrhs, ls_prec prec, hipStream_t s,
                        bool minus_conv) {
  if (nrhs < 1) return LS_EINVAL;
  if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
  const size_t es = (prec == LS_C64) ? 8 : 16;
  const size_t per = (size_t)3 * ap.n * ap.n * ap.n * es;
  int chunk = ap.form == 0 ? ap.tune[prec].chunk : 0;   // the tuned choices are the dyadic form's
  if (chunk <= 0 || chunk > ap.max_rhs) chunk = ap.max_rhs;
  for (int b0 = 0; b0 < nrhs; b0 += chunk) {
    const int nb = std::min(chunk, nrhs - b0);
    LS_TRY(apply_run(ap, static_cast<const char*>(x) + (size_t)b0 * per, static_cast<char*>(y) + (size_t)b0 * per,
                     nb, prec, s, minus_conv));
  }
  return LS_OK;
}

}  // namespace ls
