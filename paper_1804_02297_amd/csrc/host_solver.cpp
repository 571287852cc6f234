// Host multifrontal sparse LU of the sparsified system S.
//
// Paper: the assembled local rows form a sparse system that is factored by
// nested dissection and used as the preconditioner (end of Section 3.1;
// costs in Section 3.3).  Here: geometric nested dissection of the n^3 grid
// (planar separators of thickness one, which separate a 27-point stencil),
// a multifrontal LU with partial pivoting inside each front's pivot block,
// and multifrontal forward / backward solves for many right-hand sides.
//
// Front of a node = its pivot points (the separator; all points of the box
// for a leaf) followed by its boundary points (the one-point shell of its
// box, which lies on ancestor separators).  Entry (i, j) of S is assembled
// at the node that eliminates i or j first.  Fronts are dense, row-major,
// with real and imaginary parts stored apart (vectorises on AVX2/AVX-512);
// the subtree recursion and the Schur-complement updates of large fronts
// run as OpenMP tasks.
//
// The factor is kept in FP64 or FP32 (R = double / float).  An FP32 factor
// is a preconditioner for the FP64 flexible GMRES: half the memory and twice
// the SIMD width for the factorisation and every solve.
#include "host_solver.h"
#include "nd_tree.h"

#include <omp.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <vector>

#if defined(__x86_64__)
#include <xmmintrin.h>
#endif

// LS_NO_TARGET_CLONES: one code path, for the ThreadSanitizer build (the
// ifunc resolvers of target clones run before its runtime starts)
#if defined(__x86_64__) && !defined(LS_NO_TARGET_CLONES)
#define LS_CLONES __attribute__((target_clones("avx512f", "avx2", "default")))
#else
#define LS_CLONES
#endif
#define LS_INLINE __attribute__((always_inline)) inline

namespace ls {

namespace {

constexpr int kNB = 32;         // panel width of the blocked partial LU
constexpr long kPanelTask = 65536;   // panel updates above this many entries run as row tasks

// numeric data of one node
template <typename R>
struct Vals {
  std::vector<R> l11r, l11i;    // np x np: L (unit, below) and U (on and above)
  std::vector<R> u12r, u12i;    // np x nb
  std::vector<R> l21r, l21i;    // nb x np
  std::vector<int> ipiv;        // np
  std::vector<R> updr, updi;    // nb x nb update matrix, freed once the parent took it
};

// Subnormal inputs and results (fill-in decays below FP32's normal range)
// take a slow path on x86; every thread of the factor and solve regions runs
// with flush-to-zero and denormals-are-zero and restores its own mode after.
struct FlushDenormals {
#if defined(__x86_64__)
  unsigned saved;
  FlushDenormals() : saved(_mm_getcsr()) { _mm_setcsr(saved | 0x8040u); }
  ~FlushDenormals() { _mm_setcsr(saved); }
#endif
};

using Geom = NdNode;
inline int pos_in(const std::vector<int>& v, int p) { return nd_pos_in(v, p); }
inline int front_pos(const Geom& nd, int p) { return nd_front_pos(nd, p); }

// ---- kernels: one template body, multiversioned per real type -------------------

// Y[a][r] -= sum_k A[a][k] X[k][r] for MR rows a, RB right-hand sides r.
template <typename R, int MR, int RB>
LS_INLINE void mk_sub(const R* __restrict__ Ar, const R* __restrict__ Ai, long lda, long K,
                      const R* __restrict__ Xr, const R* __restrict__ Xi, long ldx, R* __restrict__ Yr,
                      R* __restrict__ Yi) {
  R cr[MR][RB], ci[MR][RB];
  for (int a = 0; a < MR; ++a)
    for (int r = 0; r < RB; ++r) cr[a][r] = ci[a][r] = 0;
  for (long k = 0; k < K; ++k) {
    const R* xr = Xr + k * ldx;
    const R* xi = Xi + k * ldx;
    for (int a = 0; a < MR; ++a) {
      const R ar = Ar[a * lda + k], ai = Ai[a * lda + k];
#pragma omp simd
      for (int r = 0; r < RB; ++r) {
        cr[a][r] += ar * xr[r] - ai * xi[r];
        ci[a][r] += ar * xi[r] + ai * xr[r];
      }
    }
  }
  for (int a = 0; a < MR; ++a)
#pragma omp simd
    for (int r = 0; r < RB; ++r) {
      Yr[a * ldx + r] -= cr[a][r];
      Yi[a * ldx + r] -= ci[a][r];
    }
}

// C[i][j] -= sum_k A[i][k] B[k][j] over rows [r0, r1), cols [c0, c1), k in [k0, k1)
// of one row-major planar matrix F (A = F[.][k], B = F[k][.], C = F, lda = nf):
// 4 x 16 blocks of C stay in registers across the panel (mk_sub), column
// blocks of 256 outside so the panel rows they read stay in L2.
template <typename R>
LS_INLINE void gemm_rows_t(R* __restrict__ Fr, R* __restrict__ Fi, long nf, long r0, long r1, long c0, long c1,
                           long k0, long k1) {
  const long K = k1 - k0;
  const R* Ar = Fr + k0;
  const R* Ai = Fi + k0;
  const R* Br = Fr + k0 * nf;
  const R* Bi = Fi + k0 * nf;
  constexpr long JB = 256;
  for (long jb = c0; jb < c1; jb += JB) {
    const long je = std::min(c1, jb + JB);
    for (long i = r0; i < r1;) {
      const bool quad = i + 4 <= r1;
      long j = jb;
      if (quad) {
        for (; j + 16 <= je; j += 16)
          mk_sub<R, 4, 16>(Ar + i * nf, Ai + i * nf, nf, K, Br + j, Bi + j, nf, Fr + i * nf + j, Fi + i * nf + j);
        for (; j + 4 <= je; j += 4)
          mk_sub<R, 4, 4>(Ar + i * nf, Ai + i * nf, nf, K, Br + j, Bi + j, nf, Fr + i * nf + j, Fi + i * nf + j);
      } else {
        for (; j + 16 <= je; j += 16)
          mk_sub<R, 1, 16>(Ar + i * nf, Ai + i * nf, nf, K, Br + j, Bi + j, nf, Fr + i * nf + j, Fi + i * nf + j);
        for (; j + 4 <= je; j += 4)
          mk_sub<R, 1, 4>(Ar + i * nf, Ai + i * nf, nf, K, Br + j, Bi + j, nf, Fr + i * nf + j, Fi + i * nf + j);
      }
      const long rows = quad ? 4 : 1;
      for (; j < je; ++j)                  // fewer than four columns left
        for (long a = i; a < i + rows; ++a) {
          R sr = 0, si = 0;
          for (long k = 0; k < K; ++k) {
            const R ar = Ar[a * nf + k], ai = Ai[a * nf + k];
            const R br = Br[k * nf + j], bi = Bi[k * nf + j];
            sr += ar * br - ai * bi;
            si += ar * bi + ai * br;
          }
          Fr[a * nf + j] -= sr;
          Fi[a * nf + j] -= si;
        }
      i += rows;
    }
  }
}
LS_CLONES void gemm_rows_d(double* Fr, double* Fi, long nf, long r0, long r1, long c0, long c1, long k0, long k1) {
  gemm_rows_t<double>(Fr, Fi, nf, r0, r1, c0, c1, k0, k1);
}
LS_CLONES void gemm_rows_f(float* Fr, float* Fi, long nf, long r0, long r1, long c0, long c1, long k0, long k1) {
  gemm_rows_t<float>(Fr, Fi, nf, r0, r1, c0, c1, k0, k1);
}
inline void gemm_rows(double* Fr, double* Fi, long nf, long r0, long r1, long c0, long c1, long k0, long k1) {
  gemm_rows_d(Fr, Fi, nf, r0, r1, c0, c1, k0, k1);
}
inline void gemm_rows(float* Fr, float* Fi, long nf, long r0, long r1, long c0, long c1, long k0, long k1) {
  gemm_rows_f(Fr, Fi, nf, r0, r1, c0, c1, k0, k1);
}

// sum_k (ar + i ai)[k] (xr + i xi)[k]
template <typename R>
LS_INLINE void cdot_t(const R* __restrict__ ar, const R* __restrict__ ai, const R* __restrict__ xr,
                      const R* __restrict__ xi, long len, R* outr, R* outi) {
  R sr = 0, si = 0;
#pragma omp simd reduction(+ : sr, si)
  for (long k = 0; k < len; ++k) {
    sr += ar[k] * xr[k] - ai[k] * xi[k];
    si += ar[k] * xi[k] + ai[k] * xr[k];
  }
  *outr = sr;
  *outi = si;
}
LS_CLONES void cdot_d(const double* ar, const double* ai, const double* xr, const double* xi, long len,
                      double* outr, double* outi) {
  cdot_t<double>(ar, ai, xr, xi, len, outr, outi);
}
LS_CLONES void cdot_f(const float* ar, const float* ai, const float* xr, const float* xi, long len, float* outr,
                      float* outi) {
  cdot_t<float>(ar, ai, xr, xi, len, outr, outi);
}
inline void cdot(const double* ar, const double* ai, const double* xr, const double* xi, long len, double* outr,
                 double* outi) {
  cdot_d(ar, ai, xr, xi, len, outr, outi);
}
inline void cdot(const float* ar, const float* ai, const float* xr, const float* xi, long len, float* outr,
                 float* outi) {
  cdot_f(ar, ai, xr, xi, len, outr, outi);
}

// ---- many right-hand sides: block vectors [dof][ldx], ldx a multiple of 4 -------
// With the right-hand sides interleaved (entry (k, r) at k ldx + r), a factor
// entry is broadcast against a short vector of right-hand sides, so each
// factor row is streamed once per 16 (FP64) or 32 (FP32) right-hand sides and
// the arithmetic vectorises over r.

// rows [i0, i1) of Y -= A X; A row-major (lda), K columns; X, Y block vectors
template <typename R>
LS_INLINE void gemm_sub_rows_t(const R* Ar, const R* Ai, long lda, long i0, long i1, long K, const R* Xr,
                               const R* Xi, long ldx, R* Yr, R* Yi) {
  long i = i0;
  for (; i + 4 <= i1; i += 4)
    for (long r0 = 0; r0 < ldx;) {
      if (sizeof(R) == 4 && ldx - r0 >= 32) {     // FP32: a 4 x 32 tile still fits the registers
        mk_sub<R, 4, 32>(Ar + i * lda, Ai + i * lda, lda, K, Xr + r0, Xi + r0, ldx, Yr + i * ldx + r0,
                         Yi + i * ldx + r0);
        r0 += 32;
      } else if (ldx - r0 >= 16) {
        mk_sub<R, 4, 16>(Ar + i * lda, Ai + i * lda, lda, K, Xr + r0, Xi + r0, ldx, Yr + i * ldx + r0,
                         Yi + i * ldx + r0);
        r0 += 16;
      } else if (ldx - r0 >= 8) {
        mk_sub<R, 4, 8>(Ar + i * lda, Ai + i * lda, lda, K, Xr + r0, Xi + r0, ldx, Yr + i * ldx + r0,
                        Yi + i * ldx + r0);
        r0 += 8;
      } else {
        mk_sub<R, 4, 4>(Ar + i * lda, Ai + i * lda, lda, K, Xr + r0, Xi + r0, ldx, Yr + i * ldx + r0,
                        Yi + i * ldx + r0);
        r0 += 4;
      }
    }
  for (; i < i1; ++i)
    for (long r0 = 0; r0 < ldx; r0 += 4)
      mk_sub<R, 1, 4>(Ar + i * lda, Ai + i * lda, lda, K, Xr + r0, Xi + r0, ldx, Yr + i * ldx + r0,
                      Yi + i * ldx + r0);
}
LS_CLONES void gemm_sub_rows_d(const double* Ar, const double* Ai, long lda, long i0, long i1, long K,
                               const double* Xr, const double* Xi, long ldx, double* Yr, double* Yi) {
  gemm_sub_rows_t<double>(Ar, Ai, lda, i0, i1, K, Xr, Xi, ldx, Yr, Yi);
}
LS_CLONES void gemm_sub_rows_f(const float* Ar, const float* Ai, long lda, long i0, long i1, long K, const float* Xr,
                               const float* Xi, long ldx, float* Yr, float* Yi) {
  gemm_sub_rows_t<float>(Ar, Ai, lda, i0, i1, K, Xr, Xi, ldx, Yr, Yi);
}
inline void gemm_sub_rows(const double* Ar, const double* Ai, long lda, long i0, long i1, long K, const double* Xr,
                          const double* Xi, long ldx, double* Yr, double* Yi) {
  gemm_sub_rows_d(Ar, Ai, lda, i0, i1, K, Xr, Xi, ldx, Yr, Yi);
}
inline void gemm_sub_rows(const float* Ar, const float* Ai, long lda, long i0, long i1, long K, const float* Xr,
                          const float* Xi, long ldx, float* Yr, float* Yi) {
  gemm_sub_rows_f(Ar, Ai, lda, i0, i1, K, Xr, Xi, ldx, Yr, Yi);
}

// W[i][r] -= L[i][k] W[k][r] for k in [b0, i), i in [b0, b1)  (within a diagonal block).
// Row i of W is held in local accumulators for RB right-hand sides at a time
// (rows i and k of W share one array, so the compiler cannot keep it in
// registers on its own).
template <typename R, int RB>
LS_INLINE void lower_block_chunk(const R* __restrict__ Lr, const R* __restrict__ Li, long np, long b0, long b1,
                                 R* __restrict__ Wr, R* __restrict__ Wi, long ldx, long r0) {
  for (long i = b0; i < b1; ++i) {
    R yr[RB], yi[RB];
#pragma omp simd
    for (int r = 0; r < RB; ++r) {
      yr[r] = Wr[i * ldx + r0 + r];
      yi[r] = Wi[i * ldx + r0 + r];
    }
    for (long k = b0; k < i; ++k) {
      const R ar = Lr[i * np + k], ai = Li[i * np + k];
      const R* xr = Wr + k * ldx + r0;
      const R* xi = Wi + k * ldx + r0;
#pragma omp simd
      for (int r = 0; r < RB; ++r) {
        yr[r] -= ar * xr[r] - ai * xi[r];
        yi[r] -= ar * xi[r] + ai * xr[r];
      }
    }
#pragma omp simd
    for (int r = 0; r < RB; ++r) {
      Wr[i * ldx + r0 + r] = yr[r];
      Wi[i * ldx + r0 + r] = yi[r];
    }
  }
}
template <typename R>
LS_INLINE void lower_block_multi_t(const R* __restrict__ Lr, const R* __restrict__ Li, long np, long b0, long b1,
                                   R* __restrict__ Wr, R* __restrict__ Wi, long ldx) {
  for (long r0 = 0; r0 < ldx;) {
    if (ldx - r0 >= 16) {
      lower_block_chunk<R, 16>(Lr, Li, np, b0, b1, Wr, Wi, ldx, r0);
      r0 += 16;
    } else if (ldx - r0 >= 8) {
      lower_block_chunk<R, 8>(Lr, Li, np, b0, b1, Wr, Wi, ldx, r0);
      r0 += 8;
    } else {
      lower_block_chunk<R, 4>(Lr, Li, np, b0, b1, Wr, Wi, ldx, r0);
      r0 += 4;
    }
  }
}
LS_CLONES void lower_block_multi_d(const double* Lr, const double* Li, long np, long b0, long b1, double* Wr,
                                   double* Wi, long ldx) {
  lower_block_multi_t<double>(Lr, Li, np, b0, b1, Wr, Wi, ldx);
}
LS_CLONES void lower_block_multi_f(const float* Lr, const float* Li, long np, long b0, long b1, float* Wr, float* Wi,
                                   long ldx) {
  lower_block_multi_t<float>(Lr, Li, np, b0, b1, Wr, Wi, ldx);
}
inline void lower_block_multi(const double* Lr, const double* Li, long np, long b0, long b1, double* Wr, double* Wi,
                              long ldx) {
  lower_block_multi_d(Lr, Li, np, b0, b1, Wr, Wi, ldx);
}
inline void lower_block_multi(const float* Lr, const float* Li, long np, long b0, long b1, float* Wr, float* Wi,
                              long ldx) {
  lower_block_multi_f(Lr, Li, np, b0, b1, Wr, Wi, ldx);
}

// W[i][r] = (W[i][r] - sum_{k in (i, b1)} U[i][k] W[k][r]) / U[i][i], i from b1-1 down to b0,
// row i held in local accumulators as above
template <typename R, int RB>
LS_INLINE void upper_block_chunk(const R* __restrict__ Ur, const R* __restrict__ Ui, long np, long b0, long b1,
                                 R* __restrict__ Wr, R* __restrict__ Wi, long ldx, long r0) {
  for (long i = b1 - 1; i >= b0; --i) {
    R yr[RB], yi[RB];
#pragma omp simd
    for (int r = 0; r < RB; ++r) {
      yr[r] = Wr[i * ldx + r0 + r];
      yi[r] = Wi[i * ldx + r0 + r];
    }
    for (long k = i + 1; k < b1; ++k) {
      const R ar = Ur[i * np + k], ai = Ui[i * np + k];
      const R* xr = Wr + k * ldx + r0;
      const R* xi = Wi + k * ldx + r0;
#pragma omp simd
      for (int r = 0; r < RB; ++r) {
        yr[r] -= ar * xr[r] - ai * xi[r];
        yi[r] -= ar * xi[r] + ai * xr[r];
      }
    }
    const R ur = Ur[i * np + i], ui = Ui[i * np + i];
    const R den = ur * ur + ui * ui;
    const R qr = ur / den, qi = -ui / den;      // 1 / u
#pragma omp simd
    for (int r = 0; r < RB; ++r) {
      Wr[i * ldx + r0 + r] = yr[r] * qr - yi[r] * qi;
      Wi[i * ldx + r0 + r] = yr[r] * qi + yi[r] * qr;
    }
  }
}
template <typename R>
LS_INLINE void upper_block_multi_t(const R* __restrict__ Ur, const R* __restrict__ Ui, long np, long b0, long b1,
                                   R* __restrict__ Wr, R* __restrict__ Wi, long ldx) {
  for (long r0 = 0; r0 < ldx;) {
    if (ldx - r0 >= 16) {
      upper_block_chunk<R, 16>(Ur, Ui, np, b0, b1, Wr, Wi, ldx, r0);
      r0 += 16;
    } else if (ldx - r0 >= 8) {
      upper_block_chunk<R, 8>(Ur, Ui, np, b0, b1, Wr, Wi, ldx, r0);
      r0 += 8;
    } else {
      upper_block_chunk<R, 4>(Ur, Ui, np, b0, b1, Wr, Wi, ldx, r0);
      r0 += 4;
    }
  }
}
LS_CLONES void upper_block_multi_d(const double* Ur, const double* Ui, long np, long b0, long b1, double* Wr,
                                   double* Wi, long ldx) {
  upper_block_multi_t<double>(Ur, Ui, np, b0, b1, Wr, Wi, ldx);
}
LS_CLONES void upper_block_multi_f(const float* Ur, const float* Ui, long np, long b0, long b1, float* Wr, float* Wi,
                                   long ldx) {
  upper_block_multi_t<float>(Ur, Ui, np, b0, b1, Wr, Wi, ldx);
}
inline void upper_block_multi(const double* Ur, const double* Ui, long np, long b0, long b1, double* Wr, double* Wi,
                              long ldx) {
  upper_block_multi_d(Ur, Ui, np, b0, b1, Wr, Wi, ldx);
}
inline void upper_block_multi(const float* Ur, const float* Ui, long np, long b0, long b1, float* Wr, float* Wi,
                              long ldx) {
  upper_block_multi_f(Ur, Ui, np, b0, b1, Wr, Wi, ldx);
}

// ---- factorisation -----------------------------------------------------------------

// Partial LU of the nf x nf front: eliminate the first np pivots, choosing
// each pivot by magnitude among the remaining pivot rows; the trailing
// (nf-np) x (nf-np) block becomes the Schur complement.
template <typename R>
void partial_lu(R* Fr, R* Fi, long nf, long np, int* ipiv, double* flops) {
  for (long kb = 0; kb < np; kb += kNB) {
    const long ke = std::min(np, kb + kNB);
    for (long k = kb; k < ke; ++k) {
      long p = k;
      R best = -1;
      for (long i = k; i < np; ++i) {
        const R v = Fr[i * nf + k] * Fr[i * nf + k] + Fi[i * nf + k] * Fi[i * nf + k];
        if (v > best) {
          best = v;
          p = i;
        }
      }
      ipiv[k] = (int)p;
      if (p != k) {
        std::swap_ranges(Fr + k * nf, Fr + (k + 1) * nf, Fr + p * nf);
        std::swap_ranges(Fi + k * nf, Fi + (k + 1) * nf, Fi + p * nf);
      }
      R pr = Fr[k * nf + k], pi = Fi[k * nf + k];
      R den = pr * pr + pi * pi;
      if (den == 0) {   // exactly singular pivot block: perturb (FGMRES absorbs it)
        pr = std::sqrt(std::numeric_limits<R>::min());
        pi = 0;
        Fr[k * nf + k] = pr;
        den = pr * pr;
      }
      const R ir = pr / den, ii = -pi / den;
      // column k of L and the rank-1 update of the panel columns (k, ke);
      // rows are independent, so a tall front splits them into tasks
      auto panel_rows = [&](long i0, long i1) {
        const R* kr = Fr + k * nf;
        const R* ki = Fi + k * nf;
        for (long i = i0; i < i1; ++i) {
          const R xr = Fr[i * nf + k], xi = Fi[i * nf + k];
          const R lr = xr * ir - xi * ii, li = xr * ii + xi * ir;
          Fr[i * nf + k] = lr;
          Fi[i * nf + k] = li;
          R* rr = Fr + i * nf;
          R* ri = Fi + i * nf;
          for (long j = k + 1; j < ke; ++j) {
            rr[j] -= lr * kr[j] - li * ki[j];
            ri[j] -= lr * ki[j] + li * kr[j];
          }
        }
      };
      const long tall = nf - k - 1;
      if (tall * (ke - k) > kPanelTask) {
        constexpr long PR = 256;
#pragma omp taskloop grainsize(1)
        for (long i0 = k + 1; i0 < nf; i0 += PR) panel_rows(i0, std::min(nf, i0 + PR));
      } else {
        panel_rows(k + 1, nf);
      }
    }
    // block row: unit-lower solve for columns [ke, nf) of rows [kb, ke)
    for (long k = kb; k < ke; ++k)
      for (long i = k + 1; i < ke; ++i) {
        const R lr = Fr[i * nf + k], li = Fi[i * nf + k];
        R* rr = Fr + i * nf;
        R* ri = Fi + i * nf;
        const R* kr = Fr + k * nf;
        const R* ki = Fi + k * nf;
        for (long j = ke; j < nf; ++j) {
          rr[j] -= lr * kr[j] - li * ki[j];
          ri[j] -= lr * ki[j] + li * kr[j];
        }
      }
    // trailing update, rows split into tasks when the front is large
    const long rows = nf - ke;
    const double work = (double)rows * (double)rows * (double)(ke - kb);
    *flops += 8.0 * work;
    if (work > 2e6) {
      // 64-row tasks: each 256-column block of the panel rows stays in L2
      // while 16 row quads use it
      constexpr long TR = 64;
#pragma omp taskloop grainsize(1)
      for (long i0 = ke; i0 < nf; i0 += TR) gemm_rows(Fr, Fi, nf, i0, std::min(nf, i0 + TR), ke, nf, kb, ke);
    } else {
      gemm_rows(Fr, Fi, nf, ke, nf, ke, nf, kb, ke);
    }
  }
}

}  // namespace

struct HostSolver {
  int n = 0;
  int dims[3] = {0, 0, 0};
  int nc = 3;                  // unknowns per point
  long npts = 0;
  bool fp32 = false;
  std::vector<Geom> geo;
  int root = -1;
  std::vector<Vals<double>> v64;
  std::vector<Vals<float>> v32;
  size_t bytes = 0;
  double flops = 0.0;
};

namespace {

template <typename R>
std::vector<Vals<R>>& vals_of(HostSolver& hs);
template <>
std::vector<Vals<double>>& vals_of<double>(HostSolver& hs) {
  return hs.v64;
}
template <>
std::vector<Vals<float>>& vals_of<float>(HostSolver& hs) {
  return hs.v32;
}

template <typename R>
void factor_node(HostSolver& hs, int id, const std::complex<double>* rows, std::atomic<double>* flops) {
  const Geom& nd = hs.geo[id];
  std::vector<Vals<R>>& V = vals_of<R>(hs);
  Vals<R>& v = V[id];
  const int* dm = hs.dims;
  const int nc = hs.nc;
  const long np = nd.np, nb = nd.nb, nf = np + nb;
  std::vector<R> Fr((size_t)nf * nf, R(0)), Fi((size_t)nf * nf, R(0));
  auto add_point_rows = [&](int pi, int li, bool pivot_row) {
    const int i3 = pi % dm[2], i2 = (pi / dm[2]) % dm[1], i1 = pi / (dm[1] * dm[2]);
    for (int s1 = -1; s1 <= 1; ++s1)
      for (int s2 = -1; s2 <= 1; ++s2)
        for (int s3 = -1; s3 <= 1; ++s3) {
          const int j1 = i1 + s1, j2 = i2 + s2, j3 = i3 + s3;
          if (j1 < 0 || j1 >= dm[0] || j2 < 0 || j2 >= dm[1] || j3 < 0 || j3 >= dm[2]) continue;
          const int pj = (j1 * dm[1] + j2) * dm[2] + j3;
          const int lj = pivot_row ? front_pos(nd, pj) : pos_in(nd.piv, pj);
          if (lj < 0) continue;
          const int slot = 9 * (s1 + 1) + 3 * (s2 + 1) + (s3 + 1);
          for (int r = 0; r < nc; ++r)
            for (int c = 0; c < nc; ++c) {
              const std::complex<double> val = rows[(size_t)pi * (nc * 27 * nc) + (r * 27 + slot) * nc + c];
              const size_t o = (size_t)(nc * li + r) * nf + (nc * lj + c);
              Fr[o] += (R)val.real();
              Fi[o] += (R)val.imag();
            }
        }
  };
  for (size_t a = 0; a < nd.piv.size(); ++a) add_point_rows(nd.piv[a], (int)a, true);
  for (size_t a = 0; a < nd.bnd.size(); ++a) add_point_rows(nd.bnd[a], (int)(nd.piv.size() + a), false);
  // extend-add of the children's update matrices
  for (int c : nd.child) {
    if (c < 0) continue;
    const Geom& cg = hs.geo[c];
    Vals<R>& cv = V[c];
    std::vector<int> map(cg.nb);
    for (size_t a = 0; a < cg.bnd.size(); ++a) {
      const int fp = front_pos(nd, cg.bnd[a]);
      for (int q = 0; q < hs.nc; ++q) map[hs.nc * a + q] = hs.nc * fp + q;
    }
    for (int r = 0; r < cg.nb; ++r)
      for (int s = 0; s < cg.nb; ++s) {
        const size_t o = (size_t)map[r] * nf + map[s];
        Fr[o] += cv.updr[(size_t)r * cg.nb + s];
        Fi[o] += cv.updi[(size_t)r * cg.nb + s];
      }
    std::vector<R>().swap(cv.updr);
    std::vector<R>().swap(cv.updi);
  }
  v.ipiv.resize(np);
  double fl = 0.0;
  partial_lu(Fr.data(), Fi.data(), nf, np, v.ipiv.data(), &fl);
  double prev = flops->load();
  while (!flops->compare_exchange_weak(prev, prev + fl)) {
  }
  v.l11r.resize(np * np);
  v.l11i.resize(np * np);
  v.u12r.resize(np * nb);
  v.u12i.resize(np * nb);
  v.l21r.resize(nb * np);
  v.l21i.resize(nb * np);
  v.updr.resize(nb * nb);
  v.updi.resize(nb * nb);
  // the root has no boundary (nb = 0): its U12, L21 and update blocks are
  // empty vectors, which are never indexed
  for (long i = 0; i < np; ++i) {
    std::memcpy(v.l11r.data() + i * np, Fr.data() + i * nf, np * sizeof(R));
    std::memcpy(v.l11i.data() + i * np, Fi.data() + i * nf, np * sizeof(R));
    if (nb > 0) {
      std::memcpy(v.u12r.data() + i * nb, Fr.data() + i * nf + np, nb * sizeof(R));
      std::memcpy(v.u12i.data() + i * nb, Fi.data() + i * nf + np, nb * sizeof(R));
    }
  }
  for (long i = 0; i < nb; ++i) {
    std::memcpy(v.l21r.data() + i * np, Fr.data() + (np + i) * nf, np * sizeof(R));
    std::memcpy(v.l21i.data() + i * np, Fi.data() + (np + i) * nf, np * sizeof(R));
    std::memcpy(v.updr.data() + i * nb, Fr.data() + (np + i) * nf + np, nb * sizeof(R));
    std::memcpy(v.updi.data() + i * nb, Fi.data() + (np + i) * nf + np, nb * sizeof(R));
  }
}

template <typename R>
void factor_rec(HostSolver& hs, int id, const std::complex<double>* rows, std::atomic<double>* flops) {
  for (int c : hs.geo[id].child) {
    if (c < 0) continue;
#pragma omp task firstprivate(c) shared(hs) if (hs.geo[c].piv.size() > 16)
    factor_rec<R>(hs, c, rows, flops);
  }
#pragma omp taskwait
  factor_node<R>(hs, id, rows, flops);
}

// ---- solves, one right-hand side at a time ------------------------------------------
// Vectors are kept right-hand-side major ([rhs][dof], real and imaginary
// parts apart) so that every inner product with a factor row is a contiguous
// SIMD dot product.  Per node and rhs: w (nf) = [b at pivots; 0] + children's
// update vectors; z1 = L11^-1 P w1 is kept, u = w2 - L21 z1 goes to the parent.
// Backward: x1 = U11^-1 (z1 - U12 x_B).
template <typename R>
struct SolveWork {
  std::vector<std::vector<R>> ur, ui;   // per node: update vectors
};

constexpr long kRowTask = 64;          // rows per task in the large matrix-vector products
constexpr double kParWork = 4e5;       // complex MACs above which a product is split into tasks

// y[i] -= sum_k A[i][k] x[k] for rows [0, m) of a row-major m x len block (lda), one rhs
template <typename R>
void gemv_sub(const R* Ar, const R* Ai, long lda, long m, long len, const R* xr, const R* xi, R* yr, R* yi) {
  auto rows = [&](long i0, long i1) {
    for (long i = i0; i < i1; ++i) {
      R dr, di;
      cdot(Ar + i * lda, Ai + i * lda, xr, xi, len, &dr, &di);
      yr[i] -= dr;
      yi[i] -= di;
    }
  };
  if ((double)m * (double)len > kParWork) {
#pragma omp taskloop grainsize(1)
    for (long i0 = 0; i0 < m; i0 += kRowTask) rows(i0, std::min(m, i0 + kRowTask));
  } else {
    rows(0, m);
  }
}

// unit-lower solve L x = b in place (rows of L row-major, lda = np), blocked so
// the off-diagonal block products run as tasks
template <typename R>
void lower_unit_solve(const R* Lr, const R* Li, long np, R* xr, R* xi) {
  constexpr long BS = 256;
  for (long b0 = 0; b0 < np; b0 += BS) {
    const long b1 = std::min(np, b0 + BS);
    if (b0 > 0) gemv_sub(Lr + b0 * np, Li + b0 * np, np, b1 - b0, b0, xr, xi, xr + b0, xi + b0);
    for (long i = b0; i < b1; ++i) {
      R dr, di;
      cdot(Lr + i * np + b0, Li + i * np + b0, xr + b0, xi + b0, i - b0, &dr, &di);
      xr[i] -= dr;
      xi[i] -= di;
    }
  }
}

// upper solve U x = b in place (diagonal included)
template <typename R>
void upper_solve(const R* Ur, const R* Ui, long np, R* xr, R* xi) {
  constexpr long BS = 256;
  for (long b1 = np; b1 > 0; b1 -= BS) {
    const long b0 = std::max(0L, b1 - BS);
    if (b1 < np)
      gemv_sub(Ur + b0 * np + b1, Ui + b0 * np + b1, np, b1 - b0, np - b1, xr + b1, xi + b1, xr + b0, xi + b0);
    for (long i = b1 - 1; i >= b0; --i) {
      R dr, di;
      cdot(Ur + i * np + i + 1, Ui + i * np + i + 1, xr + i + 1, xi + i + 1, b1 - i - 1, &dr, &di);
      const R vr = xr[i] - dr, vi = xi[i] - di;
      const R ur = Ur[i * np + i], ui = Ui[i * np + i];
      const R den = ur * ur + ui * ui;
      xr[i] = (vr * ur + vi * ui) / den;
      xi[i] = (vi * ur - vr * ui) / den;
    }
  }
}

template <typename R>
void fwd_node(HostSolver& hs, int id, int nrhs, const R* Br, const R* Bi, R* Zr, R* Zi, SolveWork<R>& W, long ldb) {
  const Geom& nd = hs.geo[id];
  const Vals<R>& v = vals_of<R>(hs)[id];
  const long np = nd.np, nb = nd.nb, nf = np + nb;
  std::vector<R> wr((size_t)nf * nrhs, R(0)), wi((size_t)nf * nrhs, R(0));   // [rhs][dof]
  for (int r = 0; r < nrhs; ++r)
    for (size_t a = 0; a < nd.piv.size(); ++a)
      for (int q = 0; q < hs.nc; ++q) {
        const long g = (long)hs.nc * nd.piv[a] + q;
        wr[r * nf + hs.nc * a + q] = Br[r * ldb + g];
        wi[r * nf + hs.nc * a + q] = Bi[r * ldb + g];
      }
  for (int c : nd.child) {
    if (c < 0) continue;
    const Geom& ch = hs.geo[c];
    std::vector<int> map(ch.nb);
    for (size_t a = 0; a < ch.bnd.size(); ++a) {
      const int fp = front_pos(nd, ch.bnd[a]);
      for (int q = 0; q < hs.nc; ++q) map[hs.nc * a + q] = hs.nc * fp + q;
    }
    for (int r = 0; r < nrhs; ++r)
      for (int e = 0; e < ch.nb; ++e) {
        wr[r * nf + map[e]] += W.ur[c][(size_t)r * ch.nb + e];
        wi[r * nf + map[e]] += W.ui[c][(size_t)r * ch.nb + e];
      }
    std::vector<R>().swap(W.ur[c]);
    std::vector<R>().swap(W.ui[c]);
  }
  for (int r = 0; r < nrhs; ++r) {
    R* xr = &wr[(size_t)r * nf];
    R* xi = &wi[(size_t)r * nf];
    for (long k = 0; k < np; ++k) {
      const long p = v.ipiv[k];
      if (p != k) {
        std::swap(xr[k], xr[p]);
        std::swap(xi[k], xi[p]);
      }
    }
    lower_unit_solve(v.l11r.data(), v.l11i.data(), np, xr, xi);
    if (nb) gemv_sub(v.l21r.data(), v.l21i.data(), np, nb, np, xr, xi, xr + np, xi + np);
  }
  for (int r = 0; r < nrhs; ++r)
    for (size_t a = 0; a < nd.piv.size(); ++a)
      for (int q = 0; q < hs.nc; ++q) {
        const long g = (long)hs.nc * nd.piv[a] + q;
        Zr[r * ldb + g] = wr[r * nf + hs.nc * a + q];
        Zi[r * ldb + g] = wi[r * nf + hs.nc * a + q];
      }
  W.ur[id].resize((size_t)nrhs * nb);
  W.ui[id].resize((size_t)nrhs * nb);
  if (nb > 0)   // the root has no update vector
    for (int r = 0; r < nrhs; ++r) {
      std::memcpy(W.ur[id].data() + (size_t)r * nb, wr.data() + (size_t)r * nf + np, nb * sizeof(R));
      std::memcpy(W.ui[id].data() + (size_t)r * nb, wi.data() + (size_t)r * nf + np, nb * sizeof(R));
    }
}

template <typename R>
void fwd_rec(HostSolver& hs, int id, int nrhs, const R* Br, const R* Bi, R* Zr, R* Zi, SolveWork<R>& W, long ldb) {
  for (int c : hs.geo[id].child) {
    if (c < 0) continue;
#pragma omp task firstprivate(c) shared(hs, W) if (hs.geo[c].piv.size() > 64)
    fwd_rec<R>(hs, c, nrhs, Br, Bi, Zr, Zi, W, ldb);
  }
#pragma omp taskwait
  fwd_node<R>(hs, id, nrhs, Br, Bi, Zr, Zi, W, ldb);
}

template <typename R>
void bwd_node(HostSolver& hs, int id, int nrhs, R* Xr, R* Xi, long ldb) {
  const Geom& nd = hs.geo[id];
  const Vals<R>& v = vals_of<R>(hs)[id];
  const long np = nd.np, nb = nd.nb;
  std::vector<R> xr((size_t)np), xi((size_t)np), yr((size_t)nb), yi((size_t)nb);
  for (int r = 0; r < nrhs; ++r) {
    R* Rr = Xr + r * ldb;
    R* Ri = Xi + r * ldb;
    for (size_t a = 0; a < nd.piv.size(); ++a)
      for (int q = 0; q < hs.nc; ++q) {
        xr[hs.nc * a + q] = Rr[(long)hs.nc * nd.piv[a] + q];
        xi[hs.nc * a + q] = Ri[(long)hs.nc * nd.piv[a] + q];
      }
    for (size_t a = 0; a < nd.bnd.size(); ++a)
      for (int q = 0; q < hs.nc; ++q) {
        yr[hs.nc * a + q] = Rr[(long)hs.nc * nd.bnd[a] + q];
        yi[hs.nc * a + q] = Ri[(long)hs.nc * nd.bnd[a] + q];
      }
    if (nb) gemv_sub(v.u12r.data(), v.u12i.data(), nb, np, nb, yr.data(), yi.data(), xr.data(), xi.data());
    upper_solve(v.l11r.data(), v.l11i.data(), np, xr.data(), xi.data());
    for (size_t a = 0; a < nd.piv.size(); ++a)
      for (int q = 0; q < hs.nc; ++q) {
        Rr[(long)hs.nc * nd.piv[a] + q] = xr[hs.nc * a + q];
        Ri[(long)hs.nc * nd.piv[a] + q] = xi[hs.nc * a + q];
      }
  }
}

template <typename R>
void bwd_rec(HostSolver& hs, int id, int nrhs, R* Xr, R* Xi, long ldb) {
  bwd_node<R>(hs, id, nrhs, Xr, Xi, ldb);
  for (int c : hs.geo[id].child) {
    if (c < 0) continue;
#pragma omp task firstprivate(c) shared(hs) if (hs.geo[c].piv.size() > 64)
    bwd_rec<R>(hs, c, nrhs, Xr, Xi, ldb);
  }
#pragma omp taskwait
}

// ---- solves, block vectors ----------------------------------------------------------

// Y (m rows) -= A X, split into row tasks when large
template <typename R>
void gemm_sub(const R* Ar, const R* Ai, long lda, long m, long K, const R* Xr, const R* Xi, long ldx, R* Yr, R* Yi) {
  if (m <= 0 || K <= 0) return;
  if ((double)m * (double)K * (double)ldx > 4.0 * kParWork) {
    constexpr long RT = 8;
#pragma omp taskloop grainsize(1)
    for (long i0 = 0; i0 < m; i0 += RT) gemm_sub_rows(Ar, Ai, lda, i0, std::min(m, i0 + RT), K, Xr, Xi, ldx, Yr, Yi);
  } else {
    gemm_sub_rows(Ar, Ai, lda, 0, m, K, Xr, Xi, ldx, Yr, Yi);
  }
}

template <typename R>
void lower_unit_solve_multi(const R* Lr, const R* Li, long np, R* Wr, R* Wi, long ldx) {
  constexpr long BS = 128;
  for (long b0 = 0; b0 < np; b0 += BS) {
    const long b1 = std::min(np, b0 + BS);
    if (b0 > 0) gemm_sub(Lr + b0 * np, Li + b0 * np, np, b1 - b0, b0, Wr, Wi, ldx, Wr + b0 * ldx, Wi + b0 * ldx);
    lower_block_multi(Lr, Li, np, b0, b1, Wr, Wi, ldx);
  }
}

template <typename R>
void upper_solve_multi(const R* Ur, const R* Ui, long np, R* Wr, R* Wi, long ldx) {
  constexpr long BS = 128;
  for (long b1 = np; b1 > 0; b1 -= BS) {
    const long b0 = std::max(0L, b1 - BS);
    if (b1 < np)
      gemm_sub(Ur + b0 * np + b1, Ui + b0 * np + b1, np, b1 - b0, np - b1, Wr + b1 * ldx, Wi + b1 * ldx, ldx,
               Wr + b0 * ldx, Wi + b0 * ldx);
    upper_block_multi(Ur, Ui, np, b0, b1, Wr, Wi, ldx);
  }
}

// B, Z, X: block vectors over all 3 n^3 unknowns, [3 p + c][ldx]
template <typename R>
void fwd_node_multi(HostSolver& hs, int id, long ldx, const R* Br, const R* Bi, R* Zr, R* Zi, SolveWork<R>& W) {
  const Geom& nd = hs.geo[id];
  const Vals<R>& v = vals_of<R>(hs)[id];
  const long np = nd.np, nb = nd.nb, nf = np + nb;
  std::vector<R> wr((size_t)nf * ldx, R(0)), wi((size_t)nf * ldx, R(0));
  for (size_t a = 0; a < nd.piv.size(); ++a)
    for (int q = 0; q < hs.nc; ++q) {
      const long g = (long)hs.nc * nd.piv[a] + q;
      std::memcpy(&wr[(hs.nc * a + q) * ldx], Br + g * ldx, ldx * sizeof(R));
      std::memcpy(&wi[(hs.nc * a + q) * ldx], Bi + g * ldx, ldx * sizeof(R));
    }
  for (int c : nd.child) {
    if (c < 0) continue;
    const Geom& ch = hs.geo[c];
    for (size_t a = 0; a < ch.bnd.size(); ++a) {
      const long fp = front_pos(nd, ch.bnd[a]);
      for (int q = 0; q < hs.nc; ++q) {
        const R* ur = &W.ur[c][(hs.nc * a + q) * ldx];
        const R* ui = &W.ui[c][(hs.nc * a + q) * ldx];
        R* xr = &wr[(hs.nc * fp + q) * ldx];
        R* xi = &wi[(hs.nc * fp + q) * ldx];
        for (long r = 0; r < ldx; ++r) {
          xr[r] += ur[r];
          xi[r] += ui[r];
        }
      }
    }
    std::vector<R>().swap(W.ur[c]);
    std::vector<R>().swap(W.ui[c]);
  }
  for (long k = 0; k < np; ++k) {
    const long p = v.ipiv[k];
    if (p != k)
      for (long r = 0; r < ldx; ++r) {
        std::swap(wr[k * ldx + r], wr[p * ldx + r]);
        std::swap(wi[k * ldx + r], wi[p * ldx + r]);
      }
  }
  lower_unit_solve_multi(v.l11r.data(), v.l11i.data(), np, wr.data(), wi.data(), ldx);
  if (nb)
    gemm_sub(v.l21r.data(), v.l21i.data(), np, nb, np, wr.data(), wi.data(), ldx, wr.data() + np * ldx,
             wi.data() + np * ldx);
  for (size_t a = 0; a < nd.piv.size(); ++a)
    for (int q = 0; q < hs.nc; ++q) {
      const long g = (long)hs.nc * nd.piv[a] + q;
      std::memcpy(Zr + g * ldx, &wr[(hs.nc * a + q) * ldx], ldx * sizeof(R));
      std::memcpy(Zi + g * ldx, &wi[(hs.nc * a + q) * ldx], ldx * sizeof(R));
    }
  W.ur[id].assign(wr.begin() + np * ldx, wr.end());
  W.ui[id].assign(wi.begin() + np * ldx, wi.end());
}

template <typename R>
void fwd_rec_multi(HostSolver& hs, int id, long ldx, const R* Br, const R* Bi, R* Zr, R* Zi, SolveWork<R>& W) {
  for (int c : hs.geo[id].child) {
    if (c < 0) continue;
#pragma omp task firstprivate(c) shared(hs, W) if (hs.geo[c].piv.size() > 64)
    fwd_rec_multi<R>(hs, c, ldx, Br, Bi, Zr, Zi, W);
  }
#pragma omp taskwait
  fwd_node_multi<R>(hs, id, ldx, Br, Bi, Zr, Zi, W);
}

template <typename R>
void bwd_node_multi(HostSolver& hs, int id, long ldx, R* Xr, R* Xi) {
  const Geom& nd = hs.geo[id];
  const Vals<R>& v = vals_of<R>(hs)[id];
  const long np = nd.np, nb = nd.nb;
  std::vector<R> xr((size_t)np * ldx), xi((size_t)np * ldx), yr((size_t)nb * ldx), yi((size_t)nb * ldx);
  for (size_t a = 0; a < nd.piv.size(); ++a)
    for (int q = 0; q < hs.nc; ++q) {
      const long g = (long)hs.nc * nd.piv[a] + q;
      std::memcpy(&xr[(hs.nc * a + q) * ldx], Xr + g * ldx, ldx * sizeof(R));
      std::memcpy(&xi[(hs.nc * a + q) * ldx], Xi + g * ldx, ldx * sizeof(R));
    }
  for (size_t a = 0; a < nd.bnd.size(); ++a)
    for (int q = 0; q < hs.nc; ++q) {
      const long g = (long)hs.nc * nd.bnd[a] + q;
      std::memcpy(&yr[(hs.nc * a + q) * ldx], Xr + g * ldx, ldx * sizeof(R));
      std::memcpy(&yi[(hs.nc * a + q) * ldx], Xi + g * ldx, ldx * sizeof(R));
    }
  if (nb) gemm_sub(v.u12r.data(), v.u12i.data(), nb, np, nb, yr.data(), yi.data(), ldx, xr.data(), xi.data());
  upper_solve_multi(v.l11r.data(), v.l11i.data(), np, xr.data(), xi.data(), ldx);
  for (size_t a = 0; a < nd.piv.size(); ++a)
    for (int q = 0; q < hs.nc; ++q) {
      const long g = (long)hs.nc * nd.piv[a] + q;
      std::memcpy(Xr + g * ldx, &xr[(hs.nc * a + q) * ldx], ldx * sizeof(R));
      std::memcpy(Xi + g * ldx, &xi[(hs.nc * a + q) * ldx], ldx * sizeof(R));
    }
}

template <typename R>
void bwd_rec_multi(HostSolver& hs, int id, long ldx, R* Xr, R* Xi) {
  bwd_node_multi<R>(hs, id, ldx, Xr, Xi);
  for (int c : hs.geo[id].child) {
    if (c < 0) continue;
#pragma omp task firstprivate(c) shared(hs) if (hs.geo[c].piv.size() > 64)
    bwd_rec_multi<R>(hs, c, ldx, Xr, Xi);
  }
#pragma omp taskwait
}

// Right-hand sides per block solve: a multiple of 4 (the micro-kernel width);
// larger batches are solved in blocks of this many.
constexpr int kMultiBlock = 32;
constexpr int kMultiMin = 3;         // from this many right-hand sides on, the block solve

template <typename R>
void solve_multi(HostSolver* hs, std::complex<double>* b, int nrhs) {
  const long n3 = hs->npts;
  const int nc = hs->nc;
  const long ldb = nc * n3;
  for (int r0 = 0; r0 < nrhs; r0 += kMultiBlock) {
    const int nr = std::min(kMultiBlock, nrhs - r0);
    const long ldx = (nr + 3) / 4 * 4;
    std::vector<R> Br((size_t)ldb * ldx, R(0)), Bi((size_t)ldb * ldx, R(0));
    std::vector<R> Zr((size_t)ldb * ldx, R(0)), Zi((size_t)ldb * ldx, R(0));
    std::complex<double>* bb = b + (size_t)r0 * ldb;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < n3; ++p)
      for (int c = 0; c < nc; ++c)
        for (int r = 0; r < nr; ++r) {
          const std::complex<double> v = bb[(size_t)r * ldb + c * n3 + p];
          Br[(nc * p + c) * ldx + r] = (R)v.real();
          Bi[(nc * p + c) * ldx + r] = (R)v.imag();
        }
    SolveWork<R> W;
    W.ur.resize(hs->geo.size());
    W.ui.resize(hs->geo.size());
#pragma omp parallel
{
  FlushDenormals fd;
#pragma omp single
  fwd_rec_multi<R>(*hs, hs->root, ldx, Br.data(), Bi.data(), Zr.data(), Zi.data(), W);
}
#pragma omp parallel
{
  FlushDenormals fd;
#pragma omp single
  bwd_rec_multi<R>(*hs, hs->root, ldx, Zr.data(), Zi.data());
}
#pragma omp parallel for schedule(static)
    for (long p = 0; p < n3; ++p)
      for (int c = 0; c < nc; ++c)
        for (int r = 0; r < nr; ++r)
          bb[(size_t)r * ldb + c * n3 + p] =
              std::complex<double>(Zr[(nc * p + c) * ldx + r], Zi[(nc * p + c) * ldx + r]);
  }
}

template <typename R>
void solve_single(HostSolver* hs, std::complex<double>* b, int nrhs) {
  const long n3 = hs->npts;
  const int nc = hs->nc;
  const long ldb = nc * n3;
  std::vector<R> Br((size_t)nrhs * ldb), Bi((size_t)nrhs * ldb);
  for (int r = 0; r < nrhs; ++r)
    for (int c = 0; c < nc; ++c)
      for (long p = 0; p < n3; ++p) {
        const std::complex<double> v = b[(size_t)r * ldb + c * n3 + p];
        Br[r * ldb + nc * p + c] = (R)v.real();
        Bi[r * ldb + nc * p + c] = (R)v.imag();
      }
  std::vector<R> Zr((size_t)nrhs * ldb, R(0)), Zi((size_t)nrhs * ldb, R(0));
  SolveWork<R> W;
  W.ur.resize(hs->geo.size());
  W.ui.resize(hs->geo.size());
#pragma omp parallel
{
  FlushDenormals fd;
#pragma omp single
  fwd_rec<R>(*hs, hs->root, nrhs, Br.data(), Bi.data(), Zr.data(), Zi.data(), W, ldb);
}
#pragma omp parallel
{
  FlushDenormals fd;
#pragma omp single
  bwd_rec<R>(*hs, hs->root, nrhs, Zr.data(), Zi.data(), ldb);
}
  for (int r = 0; r < nrhs; ++r)
    for (int c = 0; c < nc; ++c)
      for (long p = 0; p < n3; ++p)
        b[(size_t)r * ldb + c * n3 + p] = std::complex<double>(Zr[r * ldb + nc * p + c], Zi[r * ldb + nc * p + c]);
}

}  // namespace

ls_status host_factor(int n, const std::complex<double>* rows, size_t mem_cap, bool fp32, HostSolver** out) {
  const int dims[3] = {n, n, n};
  return host_factor_grid(dims, 3, rows, mem_cap, fp32, out);
}

ls_status host_factor_grid(const int dims[3], int nc, const std::complex<double>* rows, size_t mem_cap, bool fp32,
                           HostSolver** out) {
  if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || nc < 1 || nc > 3 || !rows || !out) return LS_EINVAL;
  std::unique_ptr<HostSolver> hs(new HostSolver());
  hs->n = dims[0];
  for (int d = 0; d < 3; ++d) hs->dims[d] = dims[d];
  hs->nc = nc;
  hs->npts = (long)dims[0] * dims[1] * dims[2];
  hs->fp32 = fp32;
  {
    NdTree t = nd_build_grid(dims, nc);
    hs->geo = std::move(t.nodes);
    hs->root = t.root;
  }
  const size_t cbytes = fp32 ? 8 : 16;
  size_t need = 0;
  for (const Geom& nd : hs->geo) need += cbytes * ((size_t)nd.np * nd.np + 2ull * nd.np * nd.nb);
  hs->bytes = need;
  if (mem_cap && need > mem_cap) return LS_EHOST;
  std::atomic<double> flops(0.0);
  if (fp32) {
    hs->v32.resize(hs->geo.size());
#pragma omp parallel
{
  FlushDenormals fd;
#pragma omp single
  factor_rec<float>(*hs, hs->root, rows, &flops);
}
  } else {
    hs->v64.resize(hs->geo.size());
#pragma omp parallel
{
  FlushDenormals fd;
#pragma omp single
  factor_rec<double>(*hs, hs->root, rows, &flops);
}
  }
  hs->flops = flops.load();
  *out = hs.release();
  return LS_OK;
}

ls_status host_solve(HostSolver* hs, std::complex<double>* b, int nrhs) {
  if (!hs || !b || nrhs < 1) return LS_EINVAL;
  if (hs->fp32) {
    if (nrhs >= kMultiMin)
      solve_multi<float>(hs, b, nrhs);
    else
      solve_single<float>(hs, b, nrhs);
  } else {
    if (nrhs >= kMultiMin)
      solve_multi<double>(hs, b, nrhs);
    else
      solve_single<double>(hs, b, nrhs);
  }
  return LS_OK;
}

size_t host_factor_bytes(const HostSolver* hs) { return hs ? hs->bytes : 0; }
double host_factor_flops(const HostSolver* hs) { return hs ? hs->flops : 0.0; }
bool host_factor_is_fp32(const HostSolver* hs) { return hs && hs->fp32; }
void host_free(HostSolver* hs) { delete hs; }

}  // namespace ls
