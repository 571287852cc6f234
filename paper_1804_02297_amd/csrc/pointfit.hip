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
//   heev_block_kernel  : one workgroup per point: Cholesky and triangular inverse
//                        in LDS, block inverse iteration warm-started from the
//                        class Ritz vectors as dense triangular products,
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

// accb[r][j] = sum_{j <= k < i0} Lp[LI(i0 + r, k)] Lp[LI(k, j)] for r < rows and
// j < i0 (i0 a multiple of 8): the block rows i0.. of the Cholesky factor times
// the finished rows of W = L^-1 (Lp rows < i0 already hold W), on FP64 MFMA
// in realified form as in mm81x8 below.  A 16-row band (rows >= `rows` zero)
// times 8-column groups of W, the groups shared round-robin by the four
// waves; group g starts at k = 8 g, where W's lower-triangular columns start.
__device__ __forceinline__ void band_times_w(const C<double>* __restrict__ Lp, int i0, int rows,
                                             C<double>* __restrict__ accb, int wave, int lane) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  const int col = lane & 15, c8 = col & 7, kl = lane >> 4, rr = lane & 15;
  for (int g = wave; 8 * g < i0; g += 4) {
    const int j = 8 * g + c8;
    v4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k4 = 8 * g; k4 < i0; k4 += 4) {
      const int k = k4 + kl;
      C<double> a = cmk(0.0, 0.0), w = cmk(0.0, 0.0);
      if (k < i0) {
        if (rr < rows) a = Lp[LI(i0 + rr, k)];
        if (j <= k) w = Lp[LI(k, j)];
      }
      const double b1 = (col < EBW) ? w.re : w.im;
      const double b2 = (col < EBW) ? -w.im : w.re;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b1, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b2, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * r + kl;
      if (row < rows) {
        if (col < EBW)
          accb[row * R81 + j].re = acc[r];
        else
          accb[row * R81 + j].im = acc[r];
      }
    }
  }
}

// Y = op(A) X for the 81 x 8 complex blocks X, Y in LDS (rows padded to EBW + 1)
// and A given by its packed lower triangle Lp: OP 0 A = Lp (lower triangular),
// 1 A = Lp^H (upper triangular), 2 A = the Hermitian matrix with lower
// triangle Lp.  On FP64 MFMA (16x16x4) in realified form: a 16-row tile of
// [Re Y | Im Y] (16 columns) accumulates Re A [Re X | Im X] + Im A [-Im X | Re X]
// over k in steps of 4 (lane l holds A(row l%16, k l/16) and B(k l/16, col
// l%16); result D(4r + l/16, l%16) in register r).  The six row tiles are
// shared by the four wavefronts so that each does about the same number of
// nonzero k steps.
template <int OP>
__device__ __forceinline__ void mm81x8(const C<double>* __restrict__ Lp, const C<double> (*X)[EBW + 1],
                                       C<double> (*Y)[EBW + 1], int wave, int lane) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  // tiles of each wave: OP 0 needs (mt + 1) k blocks, OP 1 (6 - mt), OP 2 six
  constexpr int T0[3][4][2] = {{{5, -1}, {4, 0}, {3, 1}, {2, -1}},
                               {{0, -1}, {1, 5}, {2, 4}, {3, -1}},
                               {{0, 4}, {1, 5}, {2, -1}, {3, -1}}};
  const int col = lane & 15, c8 = col & 7, kl = lane >> 4;
  for (int ti = 0; ti < 2; ++ti) {
    const int mt = T0[OP][wave][ti];
    if (mt < 0) break;                                  // uniform over the wave
    const int row = 16 * mt + (lane & 15);
    const int kb = (OP == 1) ? 16 * mt : 0;
    const int ke = (OP == 0) ? min(R81, 16 * mt + 16) : R81;
    v4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k4 = kb; k4 < ke; k4 += 4) {
      const int k = k4 + kl;
      C<double> a = cmk(0.0, 0.0);
      if (row < R81 && k < R81) {
        if (OP == 0) {
          if (k <= row) a = Lp[LI(row, k)];
        } else if (OP == 1) {
          if (k >= row) a = cconj(Lp[LI(k, row)]);
        } else {
          a = (k <= row) ? Lp[LI(row, k)] : cconj(Lp[LI(k, row)]);
        }
      }
      const C<double> x = (k < R81) ? X[k][c8] : cmk(0.0, 0.0);
      const double b1 = (col < EBW) ? x.re : x.im;
      const double b2 = (col < EBW) ? -x.im : x.re;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b1, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b2, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = 16 * mt + 4 * r + kl;
      if (rr < R81) {
        if (col < EBW)
          Y[rr][c8].re = acc[r];
        else
          Y[rr][c8].im = acc[r];
      }
    }
  }
}

// One workgroup of four wavefronts per point.  G: packed lower triangles
// [np][3321] complex; X0: [81][8] warm start (class Ritz vectors).  Writes
// alpha [pts[p]][81][3] and the three smallest Ritz values:
//   1. Cholesky G + shift I = L L^H in 9 x 9 blocks, packed in LDS;
//   2. W = L^-1 in place, eight rows per step (the products with the
//      finished rows on FP64 MFMA);
//   3. `iters` block inverse iterations X <- W^H (W X) (products on FP64
//      MFMA), every second one followed by a Cholesky QR of the 8 columns
//      (twice after the last);
//   4. Rayleigh-Ritz with the unshifted G and an 8x8 parallel cyclic Jacobi
//      (wavefront 0).
// The products of step 3 have no sequential dependency, so all four SIMDs of
// the CU share them; only the factorisation and the 8x8 work are sequential.
constexpr int HB = 256;           // threads per point
constexpr int RBW = 8;            // rows per step of the triangular inverse
constexpr int CB = 9;             // block size of the Cholesky factorisation
__global__ __launch_bounds__(HB) void heev_block_kernel(const C<double>* __restrict__ Gall, int np,
                                                        const C<double>* __restrict__ X0, int iters,
                                                        const int* __restrict__ pts,
                                                        const int* __restrict__ slots,
                                                        C<double>* __restrict__ alpha_out,
                                                        double* __restrict__ eval_out) {
  // rows of X and Y padded to 9 entries: lanes that walk rows then hit
  // distinct LDS banks (a 128-byte row stride puts them all on two)
  __shared__ C<double> L[NPK];
  __shared__ C<double> X[R81][EBW + 1];
  __shared__ C<double> Y[R81][EBW + 1];
  __shared__ C<double> T[EBW][EBW];
  __shared__ C<double> V[EBW][EBW];
  __shared__ double red[R81];
  const int p = blockIdx.x;
  if (p >= np) return;                 // uniform over the workgroup
  const int t = threadIdx.x;
  const C<double>* G = Gall + (long)(slots ? slots[p] : p) * NPK;   // point p's Gram

  if (t < R81) red[t] = G[LI(t, t)].re;
  for (int e = t; e < NPK; e += HB) L[e] = G[e];
  __syncthreads();
  double trace = 0.0;
  for (int q = 0; q < R81; ++q) trace += red[q];
  if (t < R81) L[LI(t, t)].re += 1e-15 * trace;
  __syncthreads();

  // 1. Cholesky in 9 x 9 blocks: (a) the diagonal block on wavefront 0,
  // one lane per entry of its lower triangle; (b) the block column below by
  // substitution, one thread per row; (c) the trailing triangle, K = 9.
  for (int k0 = 0; k0 < R81; k0 += CB) {
    if (t < 64) {
      int ii = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
      while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
      while (ii * (ii + 1) / 2 > t) --ii;
      const int jj = t - ii * (ii + 1) / 2;
      const bool own = t < CB * (CB + 1) / 2;
      for (int j = 0; j < CB; ++j) {
        if (own && ii == j && jj == j) L[LI(k0 + j, k0 + j)] = cmk(sqrt(fmax(L[LI(k0 + j, k0 + j)].re, 1e-300)), 0.0);
        wsync();
        if (own && jj == j && ii > j) L[LI(k0 + ii, k0 + j)] = cscale(L[LI(k0 + ii, k0 + j)], 1.0 / L[LI(k0 + j, k0 + j)].re);
        wsync();
        if (own && jj > j) L[LI(k0 + ii, k0 + jj)] = L[LI(k0 + ii, k0 + jj)] - L[LI(k0 + ii, k0 + j)] * cconj(L[LI(k0 + jj, k0 + j)]);
        wsync();
      }
    }
    __syncthreads();
    const int nbl = R81 - k0 - CB;
    if (t < nbl) {
      const int i = k0 + CB + t;
      C<double> row[CB];
#pragma unroll
      for (int q = 0; q < CB; ++q) row[q] = L[LI(i, k0 + q)];
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        C<double> s = row[j];
#pragma unroll
        for (int q = 0; q < j; ++q) s = s - row[q] * cconj(L[LI(k0 + j, k0 + q)]);
        row[j] = cscale(s, 1.0 / L[LI(k0 + j, k0 + j)].re);
      }
#pragma unroll
      for (int q = 0; q < CB; ++q) L[LI(i, k0 + q)] = row[q];
    }
    __syncthreads();
    const int tot = nbl * (nbl + 1) / 2;
    for (int e = t; e < tot; e += HB) {
      int ii = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
      while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
      while (ii * (ii + 1) / 2 > e) --ii;
      const int i = k0 + CB + ii, j = k0 + CB + (e - ii * (ii + 1) / 2);
      C<double> acc = L[LI(i, j)];
#pragma unroll
      for (int q = 0; q < CB; ++q) acc = acc - L[LI(i, k0 + q)] * cconj(L[LI(j, k0 + q)]);
      L[LI(i, j)] = acc;
    }
    __syncthreads();
  }

  // 2. W = L^-1 in place, rows [i0, i1) per step: (a) the partial sums
  // acc[r][j] = sum_{j <= k < i0} L[i0+r][k] W[k][j] over the finished rows
  // of W (MFMA); (b) thread j runs the block rows in order; (c) the block
  // rows of W replace those of L.  X holds acc, Y the new rows.
  const int wave = t >> 6, lane = t & 63;
  C<double>* accb = &X[0][0];                       // RBW x 81
  C<double>* tmp = &Y[0][0];                        // RBW x 81
  for (int i0 = 0; i0 < R81; i0 += RBW) {
    const int i1 = min(R81, i0 + RBW);
    band_times_w(L, i0, i1 - i0, accb, wave, lane);
    __syncthreads();
    if (t < i1) {
      const int j = t;
      C<double> wb[RBW];
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
        const int i = i0 + r;
        C<double> v = cmk(0.0, 0.0);
        if (i < i1 && i >= j) {
          const double lii = L[LI(i, i)].re;
          if (i == j) {
            v = cmk(1.0 / lii, 0.0);
          } else {
            C<double> sacc = (j < i0) ? accb[r * R81 + j] : cmk(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < r; ++q)
              if (i0 + q >= j) sacc = sacc + L[LI(i, i0 + q)] * wb[q];
            v = cscale(sacc, -1.0 / lii);
          }
        }
        wb[r] = v;
        if (i < i1) tmp[r * R81 + j] = v;
      }
    }
    __syncthreads();
    for (int e = t; e < (i1 - i0) * R81; e += HB) {
      const int i = i0 + e / R81, j = e % R81;
      if (j <= i) L[LI(i, j)] = tmp[e];
    }
    __syncthreads();
  }

  // 3. block inverse iteration with (G + shift)^-1 = W^H W; after every
  // second step the block is orthonormalised by Cholesky QR: the 8 x 8 Gram
  // from four partial sums, its Cholesky factor R and R^-1 on wavefront 0,
  // then X R^-1 into the other buffer.  Two steps scale the columns apart by
  // at most (lambda_8 / lambda_1)^2, about 1e4 on these Grams, so the
  // Cholesky of their Gram (condition 1e8) is safe and leaves them
  // orthonormal to about 1e-8, which the next steps do not need better (the
  // span is what they refine); the last step orthonormalises twice for the
  // Rayleigh-Ritz.
  C<double>(*PX)[EBW + 1] = X;
  C<double>(*PY)[EBW + 1] = Y;
  for (int e = t; e < R81 * EBW; e += HB) PX[e / EBW][e % EBW] = X0[e];
  __syncthreads();
  const int c = t & (EBW - 1), rg = t / EBW;      // column, row group (32 groups)
  const int l = t;                                 // lane index inside wavefront 0
  for (int it = 0; it < iters; ++it) {
    mm81x8<0>(L, PX, PY, wave, lane);              // Y = W X
    __syncthreads();
    mm81x8<1>(L, PY, PX, wave, lane);              // X = W^H Y
    __syncthreads();
    const int npass = (it + 1 == iters) ? 2 : (it & 1);
    for (int pass = 0; pass < npass; ++pass) {
      {
        const int pq = t & 63, part = t >> 6, pp = pq >> 3, qq = pq & 7;
        C<double> h = cmk(0.0, 0.0);
        for (int i = part; i < R81; i += 4) h = h + cconj(PX[i][pp]) * PX[i][qq];
        (&PY[0][0])[part * 64 + pq] = h;
      }
      __syncthreads();
      if (t < 64) {
        const int pp = l >> 3, qq = l & 7;
        const C<double>* pa = &PY[0][0];
        T[pp][qq] = pa[l] + pa[64 + l] + pa[128 + l] + pa[192 + l];
        wsync();
        // T = R^H R, R upper in the upper triangle of T
        for (int j = 0; j < EBW; ++j) {
          if (pp == j && qq == j) T[j][j] = cmk(sqrt(fmax(T[j][j].re, 1e-300)), 0.0);
          wsync();
          if (pp == j && qq > j) T[j][qq] = cscale(T[j][qq], 1.0 / T[j][j].re);
          wsync();
          if (pp > j && qq >= pp) T[pp][qq] = T[pp][qq] - cconj(T[j][pp]) * T[j][qq];
          wsync();
        }
        // V = R^-1 (upper), one column per lane
        if (l < EBW) {
          const int q = l;
          for (int r = EBW - 1; r >= 0; --r) {
            C<double> s = cmk(r == q ? 1.0 : 0.0, 0.0);
            for (int k = r + 1; k <= q; ++k) s = s - T[r][k] * V[k][q];
            V[r][q] = (r <= q) ? cscale(s, 1.0 / T[r][r].re) : cmk(0.0, 0.0);
          }
        }
        wsync();
      }
      __syncthreads();
      for (int i = rg; i < R81; i += HB / EBW) {
        C<double> acc = cmk(0.0, 0.0);
        for (int d = 0; d <= c; ++d) acc = acc + PX[i][d] * V[d][c];
        PY[i][c] = acc;
      }
      __syncthreads();
      C<double>(*sw)[EBW + 1] = PX;
      PX = PY;
      PY = sw;
    }
  }


  // 4. Rayleigh-Ritz with the unshifted G (reloaded into L): GX (81 x 8)
  // into Y, T = X^H (G X)
  for (int e = t; e < NPK; e += HB) L[e] = G[e];
  __syncthreads();
  mm81x8<2>(L, PX, PY, wave, lane);
  __syncthreads();
  if (t >= 64) return;                              // the 8x8 work is one wavefront's
  {
    const int pp = l / EBW, qq = l % EBW;
    C<double> sacc = cmk(0.0, 0.0);
    for (int i = 0; i < R81; ++i) sacc = sacc + cconj(PX[i][pp]) * PY[i][qq];
    T[pp][qq] = sacc;
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
  // parallel cyclic Jacobi: a sweep is seven rounds of four disjoint
  // rotations (round r pairs 7 with r and i with (2r - i) mod 7), which
  // commute, so a round is one update T <- U^H T U, V <- V U.  Lanes 0..7
  // form the column of U of their index (U[i][i] and U[partner][i]), then
  // every lane updates its entry (i, j).
  __shared__ double Ud[EBW];
  __shared__ C<double> Uo[EBW];
  for (int sweep = 0; sweep < 12; ++sweep) {
    {
      // converged: off-diagonal mass below 1e-30 of the diagonal's (uniform)
      const int i = l / EBW, j = l % EBW;
      double off = (i < j) ? T[i][j].re * T[i][j].re + T[i][j].im * T[i][j].im : 0.0;
      double dia = (i == j) ? T[i][i].re * T[i][i].re : 0.0;
      for (int o = 32; o > 0; o >>= 1) {
        off += __shfl_xor(off, o);
        dia += __shfl_xor(dia, o);
      }
      // lanes may round the butterfly sums differently: decide on lane 0's
      off = __shfl(off, 0);
      dia = __shfl(dia, 0);
      if (off <= 1e-30 * dia) break;
    }
    for (int r = 0; r < EBW - 1; ++r) {
      auto partner = [r](int i) { return i == EBW - 1 ? r : (i == r ? EBW - 1 : (2 * r - i + 2 * (EBW - 1)) % (EBW - 1)); };
      if (l < EBW) {
        // both lanes of a pair compute its rotation from the same entries
        const int pi = partner(l), p1 = min(l, pi), q1 = max(l, pi);
        const C<double> apq = T[p1][q1];
        const double ab = sqrt(apq.re * apq.re + apq.im * apq.im);
        double ud = 1.0;
        C<double> uo = cmk(0.0, 0.0);
        if (ab > 1e-300) {
          const C<double> ph = cmk(apq.re / ab, apq.im / ab);
          const double tau = (T[q1][q1].re - T[p1][p1].re) / (2.0 * ab);
          const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          const double c = 1.0 / sqrt(1.0 + tt * tt), sn = tt * c;
          // U[:,p1] = c e_p1 - sn conj(ph) e_q1 ,  U[:,q1] = sn ph e_p1 + c e_q1
          ud = c;
          uo = (l == p1) ? cscale(cconj(ph), -sn) : cscale(ph, sn);
        }
        Ud[l] = ud;
        Uo[l] = uo;
      }
      wsync();
      const int i = l / EBW, j = l % EBW, pi = partner(i), pj = partner(j);
      const double di = Ud[i], dj = Ud[j];
      const C<double> oi = Uo[i], oj = Uo[j];
      C<double> nv;
      if (j == pi && (oi.re != 0.0 || oi.im != 0.0)) {
        nv = cmk(0.0, 0.0);                                 // the rotated pair's entry
      } else {
        const C<double> ri = cscale(T[i][j], dj) + T[i][pj] * oj;
        const C<double> rp = cscale(T[pi][j], dj) + T[pi][pj] * oj;
        nv = cscale(ri, di) + cconj(oi) * rp;
      }
      const C<double> vnew = cscale(V[i][j], dj) + V[i][pj] * oj;
      wsync();
      T[i][j] = nv;
      V[i][j] = vnew;
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
    for (int q = 0; q < EBW; ++q) s = s + PX[i][q] * V[q][idx[v]];
    out[e] = s;
  }
  if (eval_out && l < 3) eval_out[pt * 3 + l] = T[idx[l]][idx[l]].re;
}

// beta_p = B^H alpha_p for the listed points; B: interior local block (81 x 81,
// row-major).  A workgroup takes BPTS points: their alpha in LDS, thread e <
// 243 forms entry e = (row, v) of all of them, so each B entry is loaded once
// per BPTS points (one thread per entry and point re-read B and alpha 81 times
// each from the caches).
constexpr int BPTS = 8;
__global__ __launch_bounds__(256) void point_beta_kernel(const C<double>* __restrict__ B,
                                                         const int* __restrict__ pts, int np,
                                                         const C<double>* __restrict__ alpha,
                                                         C<double>* __restrict__ beta) {
  __shared__ C<double> al[BPTS][243];
  const int p0 = blockIdx.x * BPTS, t = threadIdx.x;
  const int npb = min(BPTS, np - p0);
  for (int e = t; e < npb * 243; e += 256) al[e / 243][e % 243] = alpha[(long)pts[p0 + e / 243] * 243 + e % 243];
  __syncthreads();
  if (t >= 243) return;
  const int row = t / 3, v = t % 3;
  C<double> acc[BPTS];
#pragma unroll
  for (int q = 0; q < BPTS; ++q) acc[q] = cmk(0.0, 0.0);
  for (int a = 0; a < R81; ++a) {
    const C<double> b = cconj(B[a * R81 + row]);
#pragma unroll
    for (int q = 0; q < BPTS; ++q) acc[q] = acc[q] + b * al[q][a * 3 + v];
  }
#pragma unroll
  for (int q = 0; q < BPTS; ++q)
    if (q < npb) beta[(long)pts[p0 + q] * 243 + t] = acc[q];
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
    hipLaunchKernelGGL(heev_block_kernel, dim3(cnt), dim3(HB), 0, s, Gb.as<C<double>>(), cnt, X0, iters, dp,
                       (const int*)nullptr, sd.palpha.as<C<double>>(), sd.peval.as<double>());
    LS_HIP(hipGetLastError());
    hipLaunchKernelGGL(point_beta_kernel, dim3(nb(cnt, BPTS)), dim3(256), 0, s, Bint.as<C<double>>(), dp, cnt,
                       sd.palpha.as<C<double>>(), sd.pbeta.as<C<double>>());
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
ls_status pointfit_solve(PointFitCtx& ctx, StencilData& sd, const int* dpts, int cnt, int iters, hipStream_t s,
                         const int* dslots) {
  const C<double>* X0 = sd.ritz8.as<C<double>>() + 13L * R81 * EBW;
  hipLaunchKernelGGL(heev_block_kernel, dim3(cnt), dim3(HB), 0, s, ctx.Gb.as<C<double>>(), cnt, X0, iters, dpts,
                     dslots, sd.palpha.as<C<double>>(), sd.peval.as<double>());
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status pointfit_beta(PointFitCtx& ctx, StencilData& sd, const int* dpts, int cnt, hipStream_t s) {
  hipLaunchKernelGGL(point_beta_kernel, dim3(nb(cnt, BPTS)), dim3(256), 0, s, ctx.Bint.as<C<double>>(), dpts, cnt,
                     sd.palpha.as<C<double>>(), sd.pbeta.as<C<double>>());
  LS_HIP(hipGetLastError());
  return LS_OK;
}

}  // namespace ls
