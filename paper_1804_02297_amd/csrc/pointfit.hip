// Medium-dependent per-point stencil fit (a project extension of Section 3).
//
// The paper's stencils depend only on the position class (Section 3.2).  The
// term the sparse rows drop is alpha^H M diag(m) E over the complement
// (Eq. (9)); it grows with |m| (Section 4 relates larger |m| to more
// iterations).  The per-point fit weights the complement by the local medium:
//
//   Gram_i = sum_{j in tau^c} w_j^2 K_{tau,j} K_{tau,j}^H
//          = Gram_class + sum_{s in shell} (w_s^2 - 1) H_s ,   H_s = K_{tau,s} K_{tau,s}^H,
//
// with w_s = 1 + |m_{i+s}| / m0 on the 98 offsets of the 5^3 shell around i
// (m = 0 off the grid) and w = 1 beyond; alpha_i = the three eigenvectors of
// Gram_i with the smallest eigenvalues, beta_i = B^H alpha_i.  It is applied
// to interior points; boundary points keep their class stencils.  With m = 0
// on the shell it is exactly the class fit.
//
//   shell_h_kernel     : H_s for the 98 shell offsets, packed lower triangles
//   shell_coef_kernel  : c[p][s] = w_s^2 - 1 for a batch of interior points
//   gram_batch_kernel  : Gram_p = Gram_class + C H on FP64 MFMA (batch x 98 x 6642)
//   heev_wave_kernel   : one wavefront per point: Cholesky in LDS, block inverse
//                        iteration warm-started from the class Ritz vectors,
//                        Rayleigh-Ritz with a lane-parallel 8x8 Jacobi
//   point_beta_kernel  : beta_p = B^H alpha_p
#include "common.h"
#include "kernel_eval.h"
#include "pointfit.h"
#include "stencil.h"

namespace ls {

namespace {

constexpr int R81 = 81;
constexpr int NPK = 3321;          // packed lower triangle of 81 x 81
constexpr int NPKR = 2 * NPK;      // as reals
constexpr int NCOL = 6656;         // NPKR padded to a multiple of 256
constexpr int KSH = 98;            // shell offsets
constexpr int KPAD = 100;          // padded to a multiple of 4
constexpr int EBW = 8;             // block size of the per-point inverse iteration

__host__ __device__ inline int LI(int i, int j) { return i * (i + 1) / 2 + j; }

// shell offsets: the 5^3 patch minus {-1,0,1}^3, lexicographic, last dimension fastest
__device__ inline void shell_offset(int s, int* o) {
  int c = 0;
  for (int a = -2; a <= 2; ++a)
    for (int b = -2; b <= 2; ++b)
      for (int e = -2; e <= 2; ++e) {
        if (abs(a) <= 1 && abs(b) <= 1 && abs(e) <= 1) continue;
        if (c == s) {
          o[0] = a;
          o[1] = b;
          o[2] = e;
          return;
        }
        ++c;
      }
}

__device__ inline void interior_tau(int a, int* t) {
  t[0] = a / 9 - 1;
  t[1] = (a / 3) % 3 - 1;
  t[2] = a % 3 - 1;
}

// Hr[s][2 LI(u,v) + {0,1}] = H_s[u][v] (v <= u); rows >= 98 and columns >= 6642 are zero.
__global__ void shell_h_kernel(double k, double h, double* __restrict__ Hr) {
  const int s = blockIdx.x;
  __shared__ C<double> Kt[R81][3];
  int o[3];
  shell_offset(s, o);
  for (int a = threadIdx.x; a < 27; a += blockDim.x) {
    int t[3];
    interior_tau(a, t);
    C<double> Kv[6];
    dyadic_K(t[0] - o[0], t[1] - o[1], t[2] - o[2], k, h, Kv);
    for (int c = 0; c < 3; ++c)
      for (int e = 0; e < 3; ++e) Kt[3 * a + c][e] = Kv[sym_index(c, e)];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NPK; idx += blockDim.x) {
    int u = (int)((sqrt(8.0 * idx + 1.0) - 1.0) / 2.0);
    while (LI(u + 1, 0) <= idx) ++u;
    while (LI(u, 0) > idx) --u;
    const int v = idx - LI(u, 0);
    C<double> acc = cmk(0.0, 0.0);
    for (int e = 0; e < 3; ++e) acc = acc + Kt[u][e] * cconj(Kt[v][e]);
    Hr[(long)s * NCOL + 2 * idx] = acc.re;
    Hr[(long)s * NCOL + 2 * idx + 1] = acc.im;
  }
}

// c[p][s] = (1 + |m_{i+s}| / m0)^2 - 1 for interior points i = pts[p]
__global__ void shell_coef_kernel(int n, const C<double>* __restrict__ m, const int* __restrict__ pts, int np,
                                  double inv_m0, double* __restrict__ coef) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)np * KPAD) return;
  const int p = (int)(id / KPAD), s = (int)(id % KPAD);
  double c = 0.0;
  if (s < KSH) {
    const int i = pts[p];
    const int i3 = i % n, i2 = (i / n) % n, i1 = i / (n * n);
    int o[3];
    shell_offset(s, o);
    const int j1 = i1 + o[0], j2 = i2 + o[1], j3 = i3 + o[2];
    if (j1 >= 0 && j1 < n && j2 >= 0 && j2 < n && j3 >= 0 && j3 < n) {
      const C<double> mv = m[((long)j1 * n + j2) * n + j3];
      const double w = 1.0 + sqrt(mv.re * mv.re + mv.im * mv.im) * inv_m0;
      c = w * w - 1.0;
    }
  }
  coef[id] = c;
}

// G[p][col] = Gclass[col] + sum_s coef[p][s] Hr[s][col], col < 6642 (packed reals).
// Block: 4 waves, tile of 16 points x 256 columns (4 MFMA tiles per wave).
__global__ __launch_bounds__(256) void gram_batch_kernel(const double* __restrict__ coef, const double* __restrict__ Hr,
                                                         const double* __restrict__ Gclass, int np,
                                                         double* __restrict__ G) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p0 = blockIdx.y * 16;
  const int col0 = blockIdx.x * 256 + wave * 64;
  v4d acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  const int prow = p0 + (lane & 15);
  for (int k0 = 0; k0 < KPAD; k0 += 4) {
    const int kk = k0 + (lane >> 4);
    const double a = (prow < np) ? coef[(long)prow * KPAD + kk] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double b = Hr[(long)kk * NCOL + col0 + 16 * t + (lane & 15)];
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pi = p0 + 4 * r + (lane >> 4);
      const int col = col0 + 16 * t + (lane & 15);
      if (pi < np && col < NPKR) G[(long)pi * NPKR + col] = acc[t][r] + Gclass[col];
    }
}

__device__ __forceinline__ void wsync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// One wavefront per point.  G: packed lower triangles [np][3321] complex.
// X0: [81][8] warm start (class Ritz vectors).  Writes alpha [pts[p]][81][3].
__global__ __launch_bounds__(64) void heev_wave_kernel(const C<double>* __restrict__ Gall, int np,
                                                       const C<double>* __restrict__ X0, int iters,
                                                       const int* __restrict__ pts, C<double>* __restrict__ alpha_out,
                                                       double* __restrict__ eval_out) {
  __shared__ C<double> L[NPK];
  __shared__ C<double> X[R81][EBW];
  __shared__ C<double> Yk[EBW];
  __shared__ C<double> T[EBW][EBW];
  __shared__ C<double> V[EBW][EBW];
  __shared__ double red[64];
  const int p = blockIdx.x;
  if (p >= np) return;
  const int l = threadIdx.x;
  const C<double>* G = Gall + (long)p * NPK;

  // load, shift, Cholesky
  double tr = 0.0;
  for (int i = l; i < R81; i += 64) tr += G[LI(i, i)].re;
  red[l] = tr;
  wsync();
  double trace = 0.0;
  for (int q = 0; q < 64; ++q) trace += red[q];
  const double shift = 1e-15 * trace;
  for (int e = l; e < NPK; e += 64) L[e] = G[e];
  wsync();
  if (l == 0)
    for (int i = 0; i < R81; ++i) L[LI(i, i)].re += shift;
  wsync();
  for (int kk = 0; kk < R81; ++kk) {
    if (l == 0) L[LI(kk, kk)] = cmk(sqrt(fmax(L[LI(kk, kk)].re, 1e-300)), 0.0);
    wsync();
    const double dinv = 1.0 / L[LI(kk, kk)].re;
    for (int i = kk + 1 + l; i < R81; i += 64) L[LI(i, kk)] = cscale(L[LI(i, kk)], dinv);
    wsync();
    const int m = R81 - kk - 1;
    const int tot = m * (m + 1) / 2;
    for (int e = l; e < tot; e += 64) {
      int ii = (int)((sqrt(8.0 * e + 1.0) - 1.0) / 2.0);
      while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
      while (ii * (ii + 1) / 2 > e) --ii;
      const int jj = e - ii * (ii + 1) / 2;
      const int i = kk + 1 + ii, j = kk + 1 + jj;
      L[LI(i, j)] = L[LI(i, j)] - L[LI(i, kk)] * cconj(L[LI(j, kk)]);
    }
    wsync();
  }
  for (int e = l; e < R81 * EBW; e += 64) X[e / EBW][e % EBW] = X0[e];
  wsync();
  for (int it = 0; it < iters; ++it) {
    for (int kk = 0; kk < R81; ++kk) {               // L Y = X
      if (l < EBW) Yk[l] = cscale(X[kk][l], 1.0 / L[LI(kk, kk)].re);
      wsync();
      if (l < EBW) X[kk][l] = Yk[l];
      for (int e = l; e < (R81 - kk - 1) * EBW; e += 64) {
        const int i = kk + 1 + e / EBW, c = e % EBW;
        X[i][c] = X[i][c] - L[LI(i, kk)] * Yk[c];
      }
      wsync();
    }
    for (int kk = R81 - 1; kk >= 0; --kk) {          // L^H Z = Y
      if (l < EBW) Yk[l] = cscale(X[kk][l], 1.0 / L[LI(kk, kk)].re);
      wsync();
      if (l < EBW) X[kk][l] = Yk[l];
      for (int e = l; e < kk * EBW; e += 64) {
        const int i = e / EBW, c = e % EBW;
        X[i][c] = X[i][c] - cconj(L[LI(kk, i)]) * Yk[c];
      }
      wsync();
    }
    for (int pass = 0; pass < 2; ++pass)              // modified Gram-Schmidt, twice
      for (int c = 0; c < EBW; ++c) {
        double nr = 0.0;
        for (int i = l; i < R81; i += 64) nr += X[i][c].re * X[i][c].re + X[i][c].im * X[i][c].im;
        for (int o = 32; o > 0; o >>= 1) nr += __shfl_xor(nr, o);
        const double sc = 1.0 / sqrt(nr);
        for (int i = l; i < R81; i += 64) X[i][c] = cscale(X[i][c], sc);
        wsync();
        for (int d = c + 1; d < EBW; ++d) {
          double pr = 0.0, pi = 0.0;
          for (int i = l; i < R81; i += 64) {
            const C<double> a = X[i][c], b = X[i][d];
            pr += a.re * b.re + a.im * b.im;
            pi += a.re * b.im - a.im * b.re;
          }
          for (int o = 32; o > 0; o >>= 1) {
            pr += __shfl_xor(pr, o);
            pi += __shfl_xor(pi, o);
          }
          const C<double> pc = cmk(pr, pi);
          for (int i = l; i < R81; i += 64) X[i][d] = X[i][d] - X[i][c] * pc;
          wsync();
        }
      }
  }
  // Rayleigh-Ritz with the unshifted G: GX (81 x 8) into the space of L, then
  // T = X^H (G X), lane (pp, qq) of the 8x8
  C<double>* GX = L;
  for (int i = l; i < R81; i += 64) {
    C<double> acc[EBW];
    for (int q = 0; q < EBW; ++q) acc[q] = cmk(0.0, 0.0);
    for (int j = 0; j < R81; ++j) {
      const C<double> gij = (j <= i) ? G[LI(i, j)] : cconj(G[LI(j, i)]);
      for (int q = 0; q < EBW; ++q) acc[q] = acc[q] + gij * X[j][q];
    }
    for (int q = 0; q < EBW; ++q) GX[i * EBW + q] = acc[q];
  }
  wsync();
  {
    const int pp = l / EBW, qq = l % EBW;
    C<double> s = cmk(0.0, 0.0);
    for (int i = 0; i < R81; ++i) s = s + cconj(X[i][pp]) * GX[i * EBW + qq];
    T[pp][qq] = s;
    V[pp][qq] = cmk(pp == qq ? 1.0 : 0.0, 0.0);
  }
  wsync();
  {
    const int pp = l / EBW, qq = l % EBW;
    const C<double> a = T[pp][qq], b = cconj(T[qq][pp]);
    wsync();
    T[pp][qq] = cmk(0.5 * (a.re + b.re), 0.5 * (a.im + b.im));
    wsync();
  }
  // cyclic Jacobi, one rotation at a time, every lane owns one entry (i, j)
  for (int sweep = 0; sweep < 12; ++sweep) {
    for (int p1 = 0; p1 < EBW; ++p1)
      for (int q1 = p1 + 1; q1 < EBW; ++q1) {
        const C<double> apq = T[p1][q1];
        const double ab = sqrt(apq.re * apq.re + apq.im * apq.im);
        if (ab <= 1e-300) continue;                       // uniform across the wave
        const C<double> ph = cmk(apq.re / ab, apq.im / ab);
        const double tau = (T[q1][q1].re - T[p1][p1].re) / (2.0 * ab);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        const int i = l / EBW, j = l % EBW;
        // T' = U^H T U with U = identity except columns p1, q1:
        //   U[:,p1] = c e_p1 - sn conj(ph) e_q1 ,  U[:,q1] = sn ph e_p1 + c e_q1
        auto ucol = [&](int col, int row) -> C<double> {
          if (col == p1) return row == p1 ? cmk(c, 0.0) : (row == q1 ? cscale(cconj(ph), -sn) : cmk(0.0, 0.0));
          if (col == q1) return row == p1 ? cscale(ph, sn) : (row == q1 ? cmk(c, 0.0) : cmk(0.0, 0.0));
          return cmk(row == col ? 1.0 : 0.0, 0.0);
        };
        // (T U)[r][j] for r in {i, p1, q1} needed: compute new entry directly
        C<double> tu_i, tu_p, tu_q;
        // column j of T U, rows i, p1, q1
        auto tu = [&](int r, int cj) -> C<double> {
          if (cj == p1) return T[r][p1] * ucol(p1, p1) + T[r][q1] * ucol(p1, q1);
          if (cj == q1) return T[r][p1] * ucol(q1, p1) + T[r][q1] * ucol(q1, q1);
          return T[r][cj];
        };
        tu_i = tu(i, j);
        tu_p = tu(p1, j);
        tu_q = tu(q1, j);
        C<double> nv;
        if (i == p1)
          nv = cconj(ucol(p1, p1)) * tu_p + cconj(ucol(p1, q1)) * tu_q;
        else if (i == q1)
          nv = cconj(ucol(q1, p1)) * tu_p + cconj(ucol(q1, q1)) * tu_q;
        else
          nv = tu_i;
        // V U
        C<double> vnew;
        if (j == p1)
          vnew = V[i][p1] * ucol(p1, p1) + V[i][q1] * ucol(p1, q1);
        else if (j == q1)
          vnew = V[i][p1] * ucol(q1, p1) + V[i][q1] * ucol(q1, q1);
        else
          vnew = V[i][j];
        wsync();
        T[i][j] = nv;
        V[i][j] = vnew;
        wsync();
        if (l == 0) {
          T[p1][q1] = cmk(0.0, 0.0);
          T[q1][p1] = cmk(0.0, 0.0);
        }
        wsync();
      }
  }
  // the three smallest Ritz values
  int idx[EBW];
  for (int q = 0; q < EBW; ++q) idx[q] = q;
  for (int a = 0; a < EBW; ++a)
    for (int b = a + 1; b < EBW; ++b)
      if (T[idx[b]][idx[b]].re < T[idx[a]][idx[a]].re) {
        const int t = idx[a];
        idx[a] = idx[b];
        idx[b] = t;
      }
  const long pt = pts[p];
  C<double>* out = alpha_out + pt * (R81 * 3);
  for (int e = l; e < R81 * 3; e += 64) {
    const int i = e / 3, v = e % 3;
    C<double> s = cmk(0.0, 0.0);
    for (int q = 0; q < EBW; ++q) s = s + X[i][q] * V[q][idx[v]];
    out[e] = s;
  }
  if (eval_out && l < 3) eval_out[pt * 3 + l] = T[idx[l]][idx[l]].re;
}

// beta_p = B^H alpha_p for the listed points; B: interior local block (81 x 81, row-major)
__global__ void point_beta_kernel(const C<double>* __restrict__ B, const int* __restrict__ pts, int np,
                                  const C<double>* __restrict__ alpha, C<double>* __restrict__ beta) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long)np * 243) return;
  const long pt = pts[id / 243];
  const int e = (int)(id % 243), row = e / 3, v = e % 3;
  const C<double>* al = alpha + pt * 243;
  C<double> s = cmk(0.0, 0.0);
  for (int a = 0; a < R81; ++a) s = s + cconj(B[a * R81 + row]) * al[a * 3 + v];
  beta[pt * 243 + e] = s;
}

__global__ void interior_block_kernel(double k, double h, C<double>* __restrict__ B) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= R81 * R81) return;
  const int u = id / R81, v = id % R81;
  int ta[3], tb[3];
  interior_tau(u / 3, ta);
  interior_tau(v / 3, tb);
  C<double> Kv[6];
  dyadic_K(ta[0] - tb[0], ta[1] - tb[1], ta[2] - tb[2], k, h, Kv);
  B[id] = Kv[sym_index(u % 3, v % 3)];
}

// per-point stencils of every point from the class stencils (boundary points keep them)
__global__ void broadcast_class_kernel(int n, const C<double>* __restrict__ calpha, const C<double>* __restrict__ cbeta,
                                       C<double>* __restrict__ palpha, C<double>* __restrict__ pbeta) {
  const long n3 = (long)n * n * n;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n3 * 243) return;
  const long p = id / 243;
  const int e = (int)(id % 243);
  const int i3 = (int)(p % n), i2 = (int)((p / n) % n), i1 = (int)(p / ((long)n * n));
  auto cd = [n](int i) { return i == 0 ? CLS_LO : (i == n - 1 ? CLS_HI : CLS_IN); };
  const int kappa = 9 * cd(i1) + 3 * cd(i2) + cd(i3);
  palpha[id] = calpha[kappa * 243 + e];
  pbeta[id] = cbeta[kappa * 243 + e];
}

__global__ void pack_lower_kernel(const C<double>* __restrict__ G81, double* __restrict__ Gp) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NPK) return;
  int u = (int)((sqrt(8.0 * idx + 1.0) - 1.0) / 2.0);
  while (LI(u + 1, 0) <= idx) ++u;
  while (LI(u, 0) > idx) --u;
  const int v = idx - LI(u, 0);
  Gp[2 * idx] = G81[u * R81 + v].re;
  Gp[2 * idx + 1] = G81[u * R81 + v].im;
}

inline unsigned nb(long len, int t) { return (unsigned)((len + t - 1) / t); }

}  // namespace

ls_status point_fit(StencilData& sd, int n, double k, const C<double>* m, double m0, int batch, int iters,
                    hipStream_t s) {
  if (!sd.have_class || n < 4 || !(m0 > 0.0)) return LS_ESTATE;
  const double h = 1.0 / (n + 1);
  const long n3 = (long)n * n * n;
  LS_TRY(sd.palpha.alloc((size_t)n3 * 243 * sizeof(C<double>)));
  LS_TRY(sd.pbeta.alloc((size_t)n3 * 243 * sizeof(C<double>)));
  LS_TRY(sd.peval.alloc((size_t)n3 * 3 * sizeof(double)));
  LS_HIP(hipMemsetAsync(sd.peval.p, 0, sd.peval.bytes, s));
  hipLaunchKernelGGL(broadcast_class_kernel, dim3(nb(n3 * 243, 256)), dim3(256), 0, s, n, sd.alpha.as<C<double>>(),
                     sd.beta.as<C<double>>(), sd.palpha.as<C<double>>(), sd.pbeta.as<C<double>>());
  LS_HIP(hipGetLastError());
  // interior points
  std::vector<int> pts;
  pts.reserve((size_t)(n - 2) * (n - 2) * (n - 2));
  for (int a = 1; a < n - 1; ++a)
    for (int b = 1; b < n - 1; ++b)
      for (int c = 1; c < n - 1; ++c) pts.push_back((a * n + b) * n + c);
  const int npts = (int)pts.size();
  DevBuf dpts, Hr, Gcls, coef, Gb, Bint;
  LS_TRY(dpts.alloc(npts * sizeof(int)));
  LS_HIP(hipMemcpyAsync(dpts.p, pts.data(), npts * sizeof(int), hipMemcpyHostToDevice, s));
  LS_TRY(Hr.alloc((size_t)KPAD * NCOL * sizeof(double)));
  LS_HIP(hipMemsetAsync(Hr.p, 0, Hr.bytes, s));
  hipLaunchKernelGGL(shell_h_kernel, dim3(KSH), dim3(256), 0, s, k, h, Hr.as<double>());
  LS_HIP(hipGetLastError());
  LS_TRY(Gcls.alloc((size_t)NCOL * sizeof(double)));
  LS_HIP(hipMemsetAsync(Gcls.p, 0, Gcls.bytes, s));
  hipLaunchKernelGGL(pack_lower_kernel, dim3(nb(NPK, 256)), dim3(256), 0, s,
                     sd.gram.as<C<double>>() + 13L * R81 * R81, Gcls.as<double>());
  LS_HIP(hipGetLastError());
  LS_TRY(Bint.alloc((size_t)R81 * R81 * sizeof(C<double>)));
  hipLaunchKernelGGL(interior_block_kernel, dim3(nb(R81 * R81, 256)), dim3(256), 0, s, k, h, Bint.as<C<double>>());
  LS_HIP(hipGetLastError());
  const int B = batch < npts ? batch : npts;
  LS_TRY(coef.alloc((size_t)B * KPAD * sizeof(double)));
  LS_TRY(Gb.alloc((size_t)B * NPKR * sizeof(double)));
  const C<double>* X0 = sd.ritz8.as<C<double>>() + 13L * R81 * EBW;
  for (int p0 = 0; p0 < npts; p0 += B) {
    const int cnt = (npts - p0 < B) ? npts - p0 : B;
    const int* dp = dpts.as<int>() + p0;
    hipLaunchKernelGGL(shell_coef_kernel, dim3(nb((long)cnt * KPAD, 256)), dim3(256), 0, s, n, m, dp, cnt, 1.0 / m0,
                       coef.as<double>());
    LS_HIP(hipGetLastError());
    hipLaunchKernelGGL(gram_batch_kernel, dim3(NCOL / 256, (cnt + 15) / 16), dim3(256), 0, s, coef.as<double>(),
                       Hr.as<double>(), Gcls.as<double>(), cnt, Gb.as<double>());
    LS_HIP(hipGetLastError());
    hipLaunchKernelGGL(heev_wave_kernel, dim3(cnt), dim3(64), 0, s, Gb.as<C<double>>(), cnt, X0, iters, dp,
                       sd.palpha.as<C<double>>(), sd.peval.as<double>());
    LS_HIP(hipGetLastError());
    hipLaunchKernelGGL(point_beta_kernel, dim3(nb((long)cnt * 243, 256)), dim3(256), 0, s, Bint.as<C<double>>(), dp,
                       cnt, sd.palpha.as<C<double>>(), sd.pbeta.as<C<double>>());
    LS_HIP(hipGetLastError());
  }
  LS_HIP(hipStreamSynchronize(s));
  sd.have_point = true;
  return LS_OK;
}

// ---- pieces of the per-point fit for callers that work on point lists ----------

ls_status pointfit_prepare(PointFitCtx& ctx, StencilData& sd, int n, double k, int batch, hipStream_t s) {
  if (!sd.have_class || n < 4) return LS_ESTATE;
  const double h = 1.0 / (n + 1);
  const long n3 = (long)n * n * n;
  ctx.n = n;
  ctx.batch = batch;
  LS_TRY(sd.palpha.alloc((size_t)n3 * 243 * sizeof(C<double>)));
  LS_TRY(sd.pbeta.alloc((size_t)n3 * 243 * sizeof(C<double>)));
  LS_TRY(sd.peval.alloc((size_t)n3 * 3 * sizeof(double)));
  LS_HIP(hipMemsetAsync(sd.peval.p, 0, sd.peval.bytes, s));
  hipLaunchKernelGGL(broadcast_class_kernel, dim3(nb(n3 * 243, 256)), dim3(256), 0, s, n, sd.alpha.as<C<double>>(),
                     sd.beta.as<C<double>>(), sd.palpha.as<C<double>>(), sd.pbeta.as<C<double>>());
  LS_HIP(hipGetLastError());
  LS_TRY(ctx.Hr.alloc((size_t)KPAD * NCOL * sizeof(double)));
  LS_HIP(hipMemsetAsync(ctx.Hr.p, 0, ctx.Hr.bytes, s));
  hipLaunchKernelGGL(shell_h_kernel, dim3(KSH), dim3(256), 0, s, k, h, ctx.Hr.as<double>());
  LS_HIP(hipGetLastError());
  LS_TRY(ctx.Gcls.alloc((size_t)NCOL * sizeof(double)));
  LS_HIP(hipMemsetAsync(ctx.Gcls.p, 0, ctx.Gcls.bytes, s));
  hipLaunchKernelGGL(pack_lower_kernel, dim3(nb(NPK, 256)), dim3(256), 0, s,
                     sd.gram.as<C<double>>() + 13L * R81 * R81, ctx.Gcls.as<double>());
  LS_HIP(hipGetLastError());
  LS_TRY(ctx.Bint.alloc((size_t)R81 * R81 * sizeof(C<double>)));
  hipLaunchKernelGGL(interior_block_kernel, dim3(nb(R81 * R81, 256)), dim3(256), 0, s, k, h, ctx.Bint.as<C<double>>());
  LS_HIP(hipGetLastError());
  LS_TRY(ctx.coef.alloc((size_t)batch * KPAD * sizeof(double)));
  LS_TRY(ctx.Gb.alloc((size_t)batch * NPKR * sizeof(double)));
  return LS_OK;
}

// weighted Grams of cnt <= batch points (device list) into ctx.Gb (packed lower triangles)
ls_status pointfit_grams(PointFitCtx& ctx, const C<double>* m, double m0, const int* dpts, int cnt, hipStream_t s) {
  if (cnt > ctx.batch) return LS_EINVAL;
  hipLaunchKernelGGL(shell_coef_kernel, dim3(nb((long)cnt * KPAD, 256)), dim3(256), 0, s, ctx.n, m, dpts, cnt,
                     1.0 / m0, ctx.coef.as<double>());
  LS_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram_batch_kernel, dim3(NCOL / 256, (cnt + 15) / 16), dim3(256), 0, s, ctx.coef.as<double>(),
                     ctx.Hr.as<double>(), ctx.Gcls.as<double>(), cnt, ctx.Gb.as<double>());
  LS_HIP(hipGetLastError());
  return LS_OK;
}

// exact per-point stencils for cnt points whose Grams are in ctx.Gb
ls_status pointfit_solve(PointFitCtx& ctx, StencilData& sd, const int* dpts, int cnt, int iters, hipStream_t s) {
  const C<double>* X0 = sd.ritz8.as<C<double>>() + 13L * R81 * EBW;
  hipLaunchKernelGGL(heev_wave_kernel, dim3(cnt), dim3(64), 0, s, ctx.Gb.as<C<double>>(), cnt, X0, iters, dpts,
                     sd.palpha.as<C<double>>(), sd.peval.as<double>());
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status pointfit_beta(PointFitCtx& ctx, StencilData& sd, const int* dpts, int cnt, hipStream_t s) {
  hipLaunchKernelGGL(point_beta_kernel, dim3(nb((long)cnt * 243, 256)), dim3(256), 0, s, ctx.Bint.as<C<double>>(),
                     dpts, cnt, sd.palpha.as<C<double>>(), sd.pbeta.as<C<double>>());
  LS_HIP(hipGetLastError());
  return LS_OK;
}

}  // namespace ls
