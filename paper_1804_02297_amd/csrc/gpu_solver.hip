// GPU multifrontal LU of the sparsified system S and its block solves.
//
// Paper: the assembled local rows form a sparse system that is factored by
// nested dissection and used as the preconditioner (end of Section 3.1;
// costs in Section 3.3).  The dissection is the host solver's (nd_tree.h);
// here every front lives in HBM and a whole level of the tree is processed
// by each launch (grid.y or grid.z runs over the level's fronts).
//
// Factorisation of a level:
//   zero the fronts; assemble S's entries; extend-add the children's update
//   blocks (child 0, then child 1: their targets overlap); then for each
//   48-column step kb of the pivot block:
//     diag_kernel   LU of the 48 x 48 diagonal tile in LDS, pivots searched
//                   among the tile's rows; the tile's L^-1 and U^-1
//     panel_kernel  L below the tile (l U = f) and U right of it (L u = P f),
//                   by substitution
//     schur_kernel  F -= L U on the trailing block, complex product on
//                   MFMA (v_mfma_*_16x16x4, FP32 or FP64)
//   and copy the pivot rows and the boundary rows' pivot columns out.
// Pivoting inside 48-row tiles (a multiple of the three unknowns of a
// point) reproduces the host solver's partial pivoting over the whole pivot
// block to rounding on the tested media: the pivots of S sit in each
// point's own 3 x 3 diagonal block.
//
// Tile permutations are not applied to the L part left of the tile: the
// forward solve applies a tile's permutation to its rows right before the
// tile is solved, after every earlier tile has updated them.
//
// Solves (many right-hand sides): vectors in elimination order (each
// node's pivots contiguous), right-hand side fastest, real and imaginary
// parts in separate planes.  Forward by levels from the leaves: add the
// children's update vectors, then per tile z = L^-1 P x and a right-looking
// update of the rows below (pivot rows in place, boundary rows into the
// node's update vector).  Backward from the root: subtract U12 x_boundary,
// then per tile (last first) x = U^-1 z and the update of the rows above.
#include "gpu_solver.h"
#include "gpu_symbolic.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <limits>
#include <functional>
#include <memory>
#include <new>
#include <system_error>
#include <thread>
#include <utility>
#include <vector>

#include "nd_tree.h"

namespace ls {

namespace {

constexpr int kRB = 64;    // rows or columns per workgroup in the panel and solve kernels
constexpr int kSR = 64;    // right-hand sides per workgroup in the solve kernels
constexpr int kKC = 32;    // boundary columns per LDS chunk of the U12 product
constexpr int kKS = 512;   // boundary columns per workgroup of the U12 product (split over workgroups)


// ---- MFMA operand conventions -------------------------------------------------------
// v_mfma_{f32,f64}_16x16x4 (wave64): A lane l holds A[l % 16][l / 16], B lane l holds
// B[l / 16][l % 16].  The 16 x 16 result sits in 4 registers per lane: the f32 form
// holds D[4 (l / 16) + r][l % 16] in register r, the f64 form D[4 r + l / 16][l % 16].
template <typename R>
struct Mma;
template <>
struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

// ---- factorisation kernels ------------------------------------------------------------

template <typename R>
__global__ void zero_kernel(R* __restrict__ a, long cnt) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (long)gridDim.x * blockDim.x) a[i] = R(0);
}

// S's entries into the fronts of a level; each entry of S belongs to exactly
// one front position, so plain additions do not collide.
template <typename R, int NC>
__global__ __launch_bounds__(256) void assemble_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                       int nlvl, const int* __restrict__ ib,
                                                       const C<double>* __restrict__ rows, R* __restrict__ buf) {
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    const int npp = d.np / NC, nbp = d.nb / NC;
    const long nf = d.nf;
    R* Fr = buf + d.f;
    R* Fi = Fr + nf * nf;
    const long work = (long)(npp + nbp) * 27;
    for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < work; w += (long)gridDim.x * blockDim.x) {
      const int a = (int)(w / 27), slot = (int)(w % 27);
      int pt, lj;
      if (a < npp) {
        pt = ib[d.e0 + NC * a];                         // perm (at offset 0): component 0 of point a
        lj = ib[d.am + 27L * a + slot];
      } else {
        pt = ib[d.bp + (a - npp)];
        lj = ib[d.ab + 27L * (a - npp) + slot];
      }
      if (lj < 0) continue;
#pragma unroll
      for (int r = 0; r < NC; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const C<double> v = rows[(((long)pt * NC + r) * 27 + slot) * NC + c];
          const long o = ((long)NC * a + r) * nf + (long)NC * lj + c;
          Fr[o] += (R)v.re;
          Fi[o] += (R)v.im;
        }
    }
  }
}

// F_parent += child's update block (rows and columns mapped through the child's
// boundary-to-parent positions), for child `slot` of every front of a level.
template <typename R, int NC>
__global__ __launch_bounds__(256) void extend_add_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                         int nlvl, int slot, const int* __restrict__ ib,
                                                         const R* __restrict__ cbuf, R* __restrict__ buf) {
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    // the child index read from global memory: indexing the copy's child[]
    // with the runtime slot would put the whole FrontDev copy on the stack
    const int cid = fr[lvl[q]].child[slot];
    if (cid < 0) continue;
    const FrontDev d = fr[lvl[q]];
    const FrontDev c = fr[cid];
    const long nf = d.nf, cnf = c.nf;
    const int cnb = c.nb;
    R* Fr = buf + d.f;
    R* Fi = Fr + nf * nf;
    const R* Cr = cbuf + c.f;
    const R* Ci = Cr + cnf * cnf;
    for (int r = blockIdx.x; r < cnb; r += gridDim.x) {
      const long pr = (long)NC * ib[c.xm + r / NC] + r % NC;
      const R* sr = Cr + (c.np + r) * cnf + c.np;
      const R* si = Ci + (c.np + r) * cnf + c.np;
      R* dr = Fr + pr * nf;
      R* di = Fi + pr * nf;
      for (int s = threadIdx.x; s < cnb; s += blockDim.x) {
        const int ps = NC * ib[c.xm + s / NC] + s % NC;
        dr[ps] += sr[s];
        di[ps] += si[s];
      }
    }
  }
}

// LU with partial pivoting of the diagonal tile [kb, kb + tw)^2 of every front
// of a level (one workgroup per front), then the tile's L^-1 (unit lower) and
// U^-1 (upper), stored for the panel kernel and the solves.
template <typename R>
__global__ __launch_bounds__(256) void diag_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl, int nlvl,
                                                   int kb, R* __restrict__ buf, R* __restrict__ fac,
                                                   int* __restrict__ ib) {
  __shared__ R Dr[kT][kT + 1], Di[kT][kT + 1];
  __shared__ R Xr[kT][kT + 1], Xi[kT][kT + 1];
  __shared__ int perm[kT];
  __shared__ int piv;
  const int tid = threadIdx.x;
  for (int q = blockIdx.x; q < nlvl; q += gridDim.x) {
    const FrontDev d = fr[lvl[q]];
    if (kb >= d.np) continue;
    const int tw = min(kT, d.np - kb);
    const long nf = d.nf;
    R* Fr = buf + d.f;
    R* Fi = Fr + nf * nf;
    for (int o = tid; o < tw * tw; o += blockDim.x) {
      const int i = o / tw, c = o % tw;
      Dr[i][c] = Fr[(kb + i) * nf + kb + c];
      Di[i][c] = Fi[(kb + i) * nf + kb + c];
    }
    if (tid < tw) perm[tid] = tid;
    __syncthreads();
    for (int j = 0; j < tw; ++j) {
      if (tid < 64) {
        R v = R(-1);
        int idx = tid;
        if (tid >= j && tid < tw) v = Dr[tid][j] * Dr[tid][j] + Di[tid][j] * Di[tid][j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const R ov = __shfl_xor(v, off);
          const int oi = __shfl_xor(idx, off);
          if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
          }
        }
        if (tid == 0) piv = idx;
      }
      __syncthreads();
      const int p = piv;
      if (p != j) {
        for (int c = tid; c < tw; c += blockDim.x) {
          R t = Dr[j][c];
          Dr[j][c] = Dr[p][c];
          Dr[p][c] = t;
          t = Di[j][c];
          Di[j][c] = Di[p][c];
          Di[p][c] = t;
        }
        if (tid == 0) {
          const int t = perm[j];
          perm[j] = perm[p];
          perm[p] = t;
        }
      }
      __syncthreads();
      if (tid == 0 && Dr[j][j] == R(0) && Di[j][j] == R(0))
        Dr[j][j] = sqrt(std::numeric_limits<R>::min());   // exactly singular tile: perturb (FGMRES absorbs it)
      __syncthreads();
      const R pr = Dr[j][j], pi = Di[j][j];
      const R den = pr * pr + pi * pi;
      const R ir = pr / den, ii = -pi / den;
      for (int i = j + 1 + tid; i < tw; i += blockDim.x) {
        const R xr = Dr[i][j], xi = Di[i][j];
        Dr[i][j] = xr * ir - xi * ii;
        Di[i][j] = xr * ii + xi * ir;
      }
      __syncthreads();
      const int m = tw - j - 1;
      for (int o = tid; o < m * m; o += blockDim.x) {
        const int i = j + 1 + o / m, c = j + 1 + o % m;
        const R lr = Dr[i][j], li = Di[i][j], ur = Dr[j][c], ui = Di[j][c];
        Dr[i][c] -= lr * ur - li * ui;
        Di[i][c] -= lr * ui + li * ur;
      }
      __syncthreads();
    }
    for (int o = tid; o < tw * tw; o += blockDim.x) {
      const int i = o / tw, c = o % tw;
      Fr[(kb + i) * nf + kb + c] = Dr[i][c];
      Fi[(kb + i) * nf + kb + c] = Di[i][c];
    }
    if (tid < tw) ib[d.pv + kb + tid] = perm[tid];
    R* T = fac + d.t + (long)(kb / kT) * 4 * kTileElems;
    // L^-1, one column per thread: X[r][c] = -sum_{c <= k < r} L[r][k] X[k][c]
    for (int c = tid; c < tw; c += blockDim.x) {
      for (int r = 0; r < tw; ++r) {
        if (r < c) {
          Xr[r][c] = R(0);
          Xi[r][c] = R(0);
        } else if (r == c) {
          Xr[r][c] = R(1);
          Xi[r][c] = R(0);
        } else {
          R sr = R(0), si = R(0);
          for (int k = c; k < r; ++k) {
            sr += Dr[r][k] * Xr[k][c] - Di[r][k] * Xi[k][c];
            si += Dr[r][k] * Xi[k][c] + Di[r][k] * Xr[k][c];
          }
          Xr[r][c] = -sr;
          Xi[r][c] = -si;
        }
      }
    }
    __syncthreads();
    for (int o = tid; o < tw * tw; o += blockDim.x) {
      const int i = o / tw, c = o % tw;
      T[i * kT + c] = Xr[i][c];
      T[kTileElems + i * kT + c] = Xi[i][c];
    }
    __syncthreads();
    // U^-1, one column per thread: X[c][c] = 1 / U[c][c],
    // X[r][c] = -(sum_{r < k <= c} U[r][k] X[k][c]) / U[r][r]
    for (int c = tid; c < tw; c += blockDim.x) {
      for (int r = tw - 1; r > c; --r) {
        Xr[r][c] = R(0);
        Xi[r][c] = R(0);
      }
      for (int r = c; r >= 0; --r) {
        R nr, ni;
        if (r == c) {
          nr = R(1);
          ni = R(0);
        } else {
          R sr = R(0), si = R(0);
          for (int k = r + 1; k <= c; ++k) {
            sr += Dr[r][k] * Xr[k][c] - Di[r][k] * Xi[k][c];
            si += Dr[r][k] * Xi[k][c] + Di[r][k] * Xr[k][c];
          }
          nr = -sr;
          ni = -si;
        }
        const R ur = Dr[r][r], ui = Di[r][r];
        const R dd = ur * ur + ui * ui;
        const R vr = ur / dd, vi = -ui / dd;
        Xr[r][c] = nr * vr - ni * vi;
        Xi[r][c] = nr * vi + ni * vr;
      }
    }
    __syncthreads();
    for (int o = tid; o < tw * tw; o += blockDim.x) {
      const int i = o / tw, c = o % tw;
      T[2 * kTileElems + i * kT + c] = Xr[i][c];
      T[3 * kTileElems + i * kT + c] = Xi[i][c];
    }
    __syncthreads();
  }
}

// Rows (columns) per workgroup of the panel kernel: one per thread, each held
// in a row of LDS.
template <typename R>
struct PanelCfg {
  static constexpr int PR = sizeof(R) == 4 ? 256 : 128;
};

// Workgroups [0, half): the L part below the tile by substitution, l U = f
// for PR rows (U the tile's upper factor).  Workgroups [half, 2 half): the U
// part right of it, L u = P f for PR columns (L the tile's unit lower factor,
// P its row permutation).  Substitution rather than the tile's explicit
// inverse keeps the panel backward stable.
template <typename R>
__global__ __launch_bounds__(256) void panel_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                    int nlvl, int kb, int half, R* __restrict__ buf,
                                                    const int* __restrict__ ib) {
  constexpr int PR = PanelCfg<R>::PR;
  __shared__ R Tr[kT][kT + 1], Ti[kT][kT + 1];   // the factored diagonal tile
  __shared__ R Br[PR][kT + 1], Bi[PR][kT + 1];   // one row (or column) per thread
  const int tid = threadIdx.x;
  const bool lrole = (int)blockIdx.x < half;
  const long blk = lrole ? blockIdx.x : blockIdx.x - half;
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    if (kb >= d.np) continue;
    const int tw = min(kT, d.np - kb);
    const long ke = kb + tw, nf = d.nf;
    const long x0 = ke + blk * PR;
    if (x0 >= nf) continue;
    const int cnt = (int)min((long)PR, nf - x0);
    R* Fr = buf + d.f;
    R* Fi = Fr + nf * nf;
    for (int o = tid; o < tw * tw; o += blockDim.x) {
      const int i = o / tw, c = o % tw;
      Tr[i][c] = Fr[(kb + i) * nf + kb + c];
      Ti[i][c] = Fi[(kb + i) * nf + kb + c];
    }
    if (lrole) {
      for (int o = tid; o < cnt * tw; o += blockDim.x) {
        const int i = o / tw, k = o % tw;
        Br[i][k] = Fr[(x0 + i) * nf + kb + k];
        Bi[i][k] = Fi[(x0 + i) * nf + kb + k];
      }
    } else {
      for (int o = tid; o < cnt * tw; o += blockDim.x) {
        const int k = o / cnt, j = o % cnt;
        const long src = (kb + ib[d.pv + kb + k]) * nf + x0 + j;
        Br[j][k] = Fr[src];
        Bi[j][k] = Fi[src];
      }
    }
    __syncthreads();
    if (tid < cnt) {
      R* br = Br[tid];
      R* bi = Bi[tid];
      if (lrole) {
        for (int j = 0; j < tw; ++j) {   // l_j = f_j / U_jj; f_c -= l_j U_jc for c > j
          const R ur = Tr[j][j], ui = Ti[j][j];
          const R den = ur * ur + ui * ui;
          const R xr = br[j], xi = bi[j];
          const R lr = (xr * ur + xi * ui) / den, li = (xi * ur - xr * ui) / den;
          br[j] = lr;
          bi[j] = li;
          for (int c = j + 1; c < tw; ++c) {
            br[c] -= lr * Tr[j][c] - li * Ti[j][c];
            bi[c] -= lr * Ti[j][c] + li * Tr[j][c];
          }
        }
        for (int c = 0; c < tw; ++c) {
          Fr[(x0 + tid) * nf + kb + c] = br[c];
          Fi[(x0 + tid) * nf + kb + c] = bi[c];
        }
      } else {
        for (int k = 0; k < tw; ++k) {   // u_r -= L_rk u_k for r > k (unit diagonal)
          const R ukr = br[k], uki = bi[k];
          for (int r = k + 1; r < tw; ++r) {
            br[r] -= Tr[r][k] * ukr - Ti[r][k] * uki;
            bi[r] -= Tr[r][k] * uki + Ti[r][k] * ukr;
          }
        }
        for (int r = 0; r < tw; ++r) {
          Fr[(kb + r) * nf + x0 + tid] = br[r];
          Fi[(kb + r) * nf + x0 + tid] = bi[r];
        }
      }
    }
    __syncthreads();
  }
}

// 64 x 64 complex tile product acc += A B on MFMA: A [64][lda] (rows x K) and
// B [K][ldb] in LDS, K a multiple of 4; wave (wm, wn) owns a 32 x 32 quarter.
template <typename R>
__device__ __forceinline__ void cmma64(const R* Ar, const R* Ai, int lda, const R* Br, const R* Bi, int ldb, int K,
                                       int wm, int wn, int lane, typename Mma<R>::v4 (&cr)[2][2],
                                       typename Mma<R>::v4 (&ci)[2][2]) {
  for (int k4 = 0; k4 < K; k4 += 4) {
    const int kr = k4 + (lane >> 4);
    R ar[2], ai[2], br[2], bi[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      ar[a] = Ar[(wm + 16 * a + (lane & 15)) * lda + kr];
      ai[a] = Ai[(wm + 16 * a + (lane & 15)) * lda + kr];
      br[a] = Br[kr * ldb + wn + 16 * a + (lane & 15)];
      bi[a] = Bi[kr * ldb + wn + 16 * a + (lane & 15)];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cr[a][b] = Mma<R>::op(ar[a], br[b], cr[a][b]);
        cr[a][b] = Mma<R>::op(-ai[a], bi[b], cr[a][b]);
        ci[a][b] = Mma<R>::op(ar[a], bi[b], ci[a][b]);
        ci[a][b] = Mma<R>::op(ai[a], br[b], ci[a][b]);
      }
  }
}

// The same 64 x 64 complex product for the solve kernels, accumulated in a
// form chosen by precision: FP32 takes three real products per complex
// multiply-add (ArBr, AiBi and (Ar + Ai)(Br + Bi); re = ArBr - AiBi, im = the
// third minus the other two), three quarters of the MFMAs; FP64 keeps the
// four products of cmma64 (and its rounding).
template <typename R, int NBW = 2>   // NBW: 16-column B tiles per wave
struct CAcc {
  typedef typename Mma<R>::v4 v4;
  static constexpr bool G3 = sizeof(R) == 4;
  static_assert(G3 || NBW == 2, "the four-product form is cmma64's 2 x 2 tiles");
  v4 p[3][2][NBW];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) p[q][a][b] = v4{R(0), R(0), R(0), R(0)};
  }
  __device__ __forceinline__ void mma(const R* Ar, const R* Ai, int lda, const R* Br, const R* Bi, int ldb, int K,
                                      int wm, int wn, int lane) {
    if constexpr (!G3) {
      cmma64<R>(Ar, Ai, lda, Br, Bi, ldb, K, wm, wn, lane, p[0], p[1]);
    } else {
      // two k steps at a time: a full unroll hoists every LDS load of the
      // chunk and leaves no registers for a second wave per SIMD
#pragma unroll 2
      for (int k4 = 0; k4 < K; k4 += 4) {
        const int kr = k4 + (lane >> 4);
        R ar[2], ai[2], br[NBW], bi[NBW];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          ar[a] = Ar[(wm + 16 * a + (lane & 15)) * lda + kr];
          ai[a] = Ai[(wm + 16 * a + (lane & 15)) * lda + kr];
        }
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
          br[b] = Br[kr * ldb + wn + 16 * b + (lane & 15)];
          bi[b] = Bi[kr * ldb + wn + 16 * b + (lane & 15)];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < NBW; ++b) {
            p[0][a][b] = Mma<R>::op(ar[a], br[b], p[0][a][b]);
            p[1][a][b] = Mma<R>::op(ai[a], bi[b], p[1][a][b]);
            p[2][a][b] = Mma<R>::op(ar[a] + ai[a], br[b] + bi[b], p[2][a][b]);
          }
      }
    }
  }
  __device__ __forceinline__ void result(v4 (&cr)[2][NBW], v4 (&ci)[2][NBW]) const {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        if constexpr (G3) {
          cr[a][b] = p[0][a][b] - p[1][a][b];
          ci[a][b] = p[2][a][b] - p[0][a][b] - p[1][a][b];
        } else {
          cr[a][b] = p[0][a][b];
          ci[a][b] = p[1][a][b];
        }
      }
  }
};

// Schur updates F[rows][cols] -= F[rows][K] F[K][cols] on a 64 x 64 tile per
// workgroup (four waves of 32 x 32, the complex product as CAcc forms it:
// three real MFMA products in FP32, four in FP64).  With the 48-column step kb inside the outer block starting at
// kb0 (obe = min(kb0 + kOB, np)):
//   mode 0: rows [ke, nf), cols [ke, obe), K = the step's columns
//   mode 1: rows [ke, obe), cols [obe, nf), K = the step's columns
//   mode 2: rows [obe, nf), cols [obe, nf), K = [kb0, obe)   (once per block)
// Modes 0 and 1 keep the block's own columns and rows current for the next
// step; the rest of the trailing matrix is read by nothing inside the block,
// so its update waits and is applied once with K up to kOB.  Registers are
// capped for two waves per SIMD: uncapped, the FP64 kernel took 214 VGPRs and
// 64 AGPRs (one wave); capped it fits 220 VGPRs without spills.  The FP32
// one keeps three waves (capped for four it spills 28 VGPRs and runs slower).
template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void schur_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                    int nlvl, int kb, int kb0, int mode, R* __restrict__ buf) {
  typedef typename Mma<R>::v4 v4;
  __shared__ R Ar[64][17], Ai[64][17];
  __shared__ R Br[16][65], Bi[16][65];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  for (int q = blockIdx.z; q < nlvl; q += gridDim.z) {
    const FrontDev d = fr[lvl[q]];
    const long nf = d.nf, obe = min((long)kb0 + kOB, (long)d.np);
    long r0, r1, c0, c1, k0, k1;
    if (mode == 2) {
      if (kb0 >= d.np) continue;
      r0 = c0 = obe;
      r1 = c1 = nf;
      k0 = kb0;
      k1 = obe;
    } else {
      if (kb >= d.np) continue;
      k0 = kb;
      k1 = min((long)kb + kT, (long)d.np);
      r0 = c0 = k1;
      r1 = mode == 0 ? nf : obe;
      if (mode == 1) c0 = obe;
      c1 = mode == 0 ? obe : nf;
    }
    const long i0 = r0 + 64L * blockIdx.y, j0 = c0 + 64L * blockIdx.x;
    if (i0 >= r1 || j0 >= c1) continue;
    const int tw = (int)(k1 - k0);
    const long kb_ = k0;
    R* Fr = buf + d.f;
    R* Fi = Fr + nf * nf;
    CAcc<R> acc;
    acc.zero();
    // the next 16-deep K chunk is loaded into registers while the MFMAs
    // consume the current one from LDS
    R par[4], pai[4], pbr[4], pbi[4];
    auto fetch = [&](int kc) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = tid + 256 * u;
        const int ii = o >> 4, kk = o & 15;
        const bool ok = i0 + ii < r1 && kc + kk < tw;
        const long src = (i0 + ii) * nf + kb_ + kc + kk;
        par[u] = ok ? Fr[src] : R(0);
        pai[u] = ok ? Fi[src] : R(0);
        const int kr = o >> 6, jj = o & 63;
        const bool okb = kc + kr < tw && j0 + jj < c1;
        const long srcb = (kb_ + kc + kr) * nf + j0 + jj;
        pbr[u] = okb ? Fr[srcb] : R(0);
        pbi[u] = okb ? Fi[srcb] : R(0);
      }
    };
    fetch(0);
    for (int kc = 0; kc < tw; kc += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = tid + 256 * u;
        Ar[o >> 4][o & 15] = par[u];
        Ai[o >> 4][o & 15] = pai[u];
        Br[o >> 6][o & 63] = pbr[u];
        Bi[o >> 6][o & 63] = pbi[u];
      }
      __syncthreads();
      if (kc + 16 < tw) fetch(kc + 16);
      acc.mma(&Ar[0][0], &Ai[0][0], 17, &Br[0][0], &Bi[0][0], 65, 16, wm, wn, lane);
      __syncthreads();
    }
    v4 cr[2][2], ci[2][2];
    acc.result(cr, ci);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long gi = i0 + wm + 16 * a + Mma<R>::row(lane, r);
          const long gj = j0 + wn + 16 * b + (lane & 15);
          if (gi < r1 && gj < c1) {
            Fr[gi * nf + gj] -= cr[a][b][r];
            Fi[gi * nf + gj] -= ci[a][b][r];
          }
        }
  }
}

// pivot rows and the boundary rows' pivot columns into the factor
template <typename R>
__global__ __launch_bounds__(256) void copyout_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                      int nlvl, const R* __restrict__ buf, R* __restrict__ fac) {
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    const long nf = d.nf, np = d.np, nb = d.nb;
    const R* Fr = buf + d.f;
    const R* Fi = Fr + nf * nf;
    const long c1 = np * nf, c2 = nb * np;
    for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < c1; w += (long)gridDim.x * blockDim.x) {
      fac[d.p + w] = Fr[w];
      fac[d.p + c1 + w] = Fi[w];
    }
    for (long i = blockIdx.x; i < nb; i += gridDim.x)
      for (long j = threadIdx.x; j < np; j += blockDim.x) {
        fac[d.l + i * np + j] = Fr[(np + i) * nf + j];
        fac[d.l + c2 + i * np + j] = Fi[(np + i) * nf + j];
      }
  }
}

// ---- solve kernels --------------------------------------------------------------------

// b (complex128 [nrhs][N]) -> X ([N][nrhs] in elimination order, split planes);
// four unknowns per workgroup pass, the right-hand sides across 64 lanes
// Lanes of a 256-thread workgroup given to one row's right-hand sides (the
// smallest power of two >= nrhs, at most 64); the workgroup covers 256 / lanes
// rows per pass.  One rhs: a row per thread.
__host__ __device__ inline int rhs_lanes(int nrhs) {
  int l = 1;
  while (l < nrhs && l < 64) l *= 2;
  return l;
}

template <typename R>
__global__ __launch_bounds__(256) void sol_in_kernel(const C<double>* __restrict__ b, long N, int nrhs,
                                                     const int* __restrict__ perm, R* __restrict__ Xr,
                                                     R* __restrict__ Xi) {
  const int lanes = rhs_lanes(nrhs), rpp = 256 / lanes;
  for (long e = (long)blockIdx.x * rpp + threadIdx.x / lanes; e < N; e += (long)gridDim.x * rpp) {
    const long pe = perm[e];
    for (int r = threadIdx.x % lanes; r < nrhs; r += lanes) {
      const C<double> v = b[r * N + pe];
      Xr[e * nrhs + r] = (R)v.re;
      Xi[e * nrhs + r] = (R)v.im;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void sol_out_kernel(C<double>* __restrict__ b, long N, int nrhs,
                                                      const int* __restrict__ perm, const R* __restrict__ Xr,
                                                      const R* __restrict__ Xi) {
  const int lanes = rhs_lanes(nrhs), rpp = 256 / lanes;
  for (long e = (long)blockIdx.x * rpp + threadIdx.x / lanes; e < N; e += (long)gridDim.x * rpp) {
    const long pe = perm[e];
    for (int r = threadIdx.x % lanes; r < nrhs; r += lanes)
      b[r * N + pe] = cmk((double)Xr[e * nrhs + r], (double)Xi[e * nrhs + r]);
  }
}

// The same two copies as tiled transposes through LDS, for many right-hand
// sides: a workgroup takes 64 natural unknowns p and 64 rhs r, reads b[r][p]
// along p and writes row ipm[p] of X along r, so both sides are whole runs
// (the per-row kernels above read or write 64 separate lines per row).
// ipm is the inverse of the elimination order: ipm[ib[e]] = e.
constexpr int kTP = 64;
constexpr int kSolTileRhs = 16;    // from this many rhs on the copies take the tiled kernels
__global__ void inv_perm_kernel(const int* __restrict__ perm, long N, int* __restrict__ ipm) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x)
    ipm[perm[e]] = (int)e;
}

template <typename R>
__global__ __launch_bounds__(256) void sol_in_tile_kernel(const C<double>* __restrict__ b, long N, int nrhs,
                                                          const int* __restrict__ ipm, R* __restrict__ Xr,
                                                          R* __restrict__ Xi) {
  __shared__ R tr[kTP][kTP + 1], ti[kTP][kTP + 1];   // [p][r]
  const long p0 = (long)blockIdx.x * kTP;
  const int r0 = blockIdx.y * kTP;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int rr = wv; rr < kTP; rr += 4) {
    const int r = r0 + rr;
    const long p = p0 + lane;
    C<double> v = cmk(0.0, 0.0);
    if (r < nrhs && p < N) v = b[(long)r * N + p];
    tr[lane][rr] = (R)v.re;
    ti[lane][rr] = (R)v.im;
  }
  __syncthreads();
  for (int pp = wv; pp < kTP; pp += 4) {
    const long p = p0 + pp;
    const int r = r0 + lane;
    if (p < N && r < nrhs) {
      const long e = ipm[p];
      Xr[e * nrhs + r] = tr[pp][lane];
      Xi[e * nrhs + r] = ti[pp][lane];
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void sol_out_tile_kernel(C<double>* __restrict__ b, long N, int nrhs,
                                                           const int* __restrict__ ipm, const R* __restrict__ Xr,
                                                           const R* __restrict__ Xi) {
  __shared__ R tr[kTP][kTP + 1], ti[kTP][kTP + 1];   // [p][r]
  const long p0 = (long)blockIdx.x * kTP;
  const int r0 = blockIdx.y * kTP;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int pp = wv; pp < kTP; pp += 4) {
    const long p = p0 + pp;
    const int r = r0 + lane;
    R vr = R(0), vi = R(0);
    if (p < N && r < nrhs) {
      const long e = ipm[p];
      vr = Xr[e * nrhs + r];
      vi = Xi[e * nrhs + r];
    }
    tr[pp][lane] = vr;
    ti[pp][lane] = vi;
  }
  __syncthreads();
  for (int rr = wv; rr < kTP; rr += 4) {
    const int r = r0 + rr;
    const long p = p0 + lane;
    if (r < nrhs && p < N) b[(long)r * N + p] = cmk((double)tr[lane][rr], (double)ti[lane][rr]);
  }
}

// children's update vectors into the pivot rows (x) or the update vector (u)
// of every front of a level, for child `slot`; 256 / rhs_lanes(nrhs) rows per workgroup pass
template <typename R, int NC>
__global__ __launch_bounds__(256) void fwd_child_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                        int nlvl, int slot, const int* __restrict__ ib, int nrhs,
                                                        R* __restrict__ Xr, R* __restrict__ Xi, R* __restrict__ Ur,
                                                        R* __restrict__ Ui) {
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    // the child index read from global memory: indexing the copy's child[]
    // with the runtime slot would put the whole FrontDev copy on the stack
    const int cid = fr[lvl[q]].child[slot];
    if (cid < 0) continue;
    const FrontDev d = fr[lvl[q]];
    const FrontDev c = fr[cid];
    const int lanes = rhs_lanes(nrhs), rpp = 256 / lanes;
    for (int rr = blockIdx.x * rpp + threadIdx.x / lanes; rr < c.nb; rr += gridDim.x * rpp) {
      const int pos = NC * ib[c.xm + rr / NC] + rr % NC;
      const bool piv = pos < d.np;
      const long src = (c.u + rr) * nrhs;
      const long dst = piv ? (long)(d.e0 + pos) * nrhs : (d.u + pos - d.np) * nrhs;
      R* Tr = piv ? Xr : Ur;
      R* Ti = piv ? Xi : Ui;
      for (int r = threadIdx.x % lanes; r < nrhs; r += lanes) {
        Tr[dst + r] += Ur[src + r];
        Ti[dst + r] += Ui[src + r];
      }
    }
  }
}

// acc[rt] (rows 16 rt.., rt < 3; the 16 columns col0..col0+15) = A B for a
// 48 x 48 block A read from global memory (A(i, k) = Ag[i * lda + k] for
// i < arows and k < acols, zero elsewhere) and B rows of an LDS array
// (B(k, c) = Bs[bidx(k) * ldb + c] for k < acols, zero elsewhere).
template <typename R>
__device__ __forceinline__ void mma48_gl(const R* __restrict__ Agr, const R* __restrict__ Agi, long lda, int arows,
                                         int acols, const R* Bsr, const R* Bsi, int ldb, const int* bperm, int brow0,
                                         int col0, int lane, typename Mma<R>::v4 (&yr)[3],
                                         typename Mma<R>::v4 (&yi)[3]) {
  typedef typename Mma<R>::v4 v4;
#pragma unroll
  for (int rt = 0; rt < 3; ++rt) {
    yr[rt] = v4{R(0), R(0), R(0), R(0)};
    yi[rt] = v4{R(0), R(0), R(0), R(0)};
  }
  const int c = col0 + (lane & 15);
#pragma unroll 4
  for (int k4 = 0; k4 < kT; k4 += 4) {
    const int k = k4 + (lane >> 4);
    R br = R(0), bi = R(0);
    if (k < acols) {
      const int row = brow0 + (bperm ? bperm[k] : k);
      br = Bsr[row * ldb + c];
      bi = Bsi[row * ldb + c];
    }
#pragma unroll
    for (int rt = 0; rt < 3; ++rt) {
      const int i = 16 * rt + (lane & 15);
      const bool ok = i < arows && k < acols;
      const R ar = ok ? Agr[i * lda + k] : R(0);
      const R ai = ok ? Agi[i * lda + k] : R(0);
      yr[rt] = Mma<R>::op(ar, br, yr[rt]);
      yr[rt] = Mma<R>::op(-ai, bi, yr[rt]);
      yi[rt] = Mma<R>::op(ar, bi, yi[rt]);
      yi[rt] = Mma<R>::op(ai, br, yi[rt]);
    }
  }
}

constexpr int kLX = kSR + 1;                 // row stride of right-hand-side blocks in LDS
constexpr int kLL = kT + 1;                  // row stride of a 64 x 48 factor block in LDS
template <typename R>
struct SolveCfg {
  static constexpr int RZ = sizeof(R) == 4 ? 64 : 32;   // rhs per super-tile workgroup (LDS: 192 x RZ)
};

// Selective inversion of each super-block [kb0, kb0 + sw) of a front's pivot
// block, at factor time (the front still in its level buffer F):
//   FWD: M with z_block = M x_block for the forward tile procedure (for each
//        48-row tile t: x_t <- L_t^-1 P_t x_t, then x_t' -= L[t'][t] x_t for
//        the later tiles t' of the block);
//   BWD: H = U_block^-1 (tiles from last to first: x_t <- U_t^-1 x_t, then
//        x_t' -= U[t'][t] x_t for the earlier tiles).
// Each workgroup runs the procedure on RZ columns of the identity in LDS
// (grid.y: super-blocks, grid.z: column chunks), products on MFMA.
template <typename R, bool FWD>
__global__ __launch_bounds__(256) void sb_inverse_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                         int nlvl, const R* __restrict__ buf, R* __restrict__ fac,
                                                         const int* __restrict__ ib) {
  typedef typename Mma<R>::v4 v4;
  constexpr int RZ = SolveCfg<R>::RZ, LD = RZ + 1;
  __shared__ R Sr[kSB * LD], Si[kSB * LD];
  __shared__ int perm[kT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool active = wave < RZ / 16;
  for (int q = blockIdx.x; q < nlvl; q += gridDim.x) {
    const FrontDev d = fr[lvl[q]];
    const long nf = d.nf;
    const R* Fr = buf + d.f;
    const R* Fi = Fr + nf * nf;
    for (int sb = blockIdx.y; (long)sb * kSB < d.np; sb += gridDim.y) {
      const int kb0 = sb * kSB;
      const int sw = min(kSB, d.np - kb0);
      const int c0 = blockIdx.z * RZ;
      if (c0 >= sw) continue;
      for (int o = tid; o < kSB * RZ; o += blockDim.x) {
        const int k = o / RZ, r = o % RZ;
        Sr[k * LD + r] = (k == c0 + r && k < sw) ? R(1) : R(0);
        Si[k * LD + r] = R(0);
      }
      __syncthreads();
      const int nt = (sw + kT - 1) / kT;
      for (int s = 0; s < nt; ++s) {
        const int t0 = FWD ? s * kT : (nt - 1 - s) * kT;
        const int tw = min(kT, sw - t0);
        const long kb = kb0 + t0;
        if (FWD && tid < tw) perm[tid] = ib[d.pv + kb + tid];
        __syncthreads();
        if (active) {   // x_t <- L_t^-1 P_t x_t  or  U_t^-1 x_t, in place
          v4 yr[3], yi[3];
          const R* T = fac + d.t + (kb / kT) * 4 * kTileElems + (FWD ? 0 : 2 * kTileElems);
          mma48_gl<R>(T, T + kTileElems, kT, tw, tw, Sr, Si, LD, FWD ? perm : nullptr, t0, 16 * wave, lane, yr, yi);
#pragma unroll
          for (int rt = 0; rt < 3; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = 16 * rt + Mma<R>::row(lane, r);
              if (i < tw) {
                Sr[(t0 + i) * LD + 16 * wave + (lane & 15)] = yr[rt][r];
                Si[(t0 + i) * LD + 16 * wave + (lane & 15)] = yi[rt][r];
              }
            }
        }
        __syncthreads();
        if (active) {   // the other tiles of the block: x_t' -= F[t'][t] x_t
          const int ua = FWD ? t0 + kT : 0, ue = FWD ? sw : t0;
          for (int u0 = ua; u0 < ue; u0 += kT) {
            const int uw = min(kT, sw - u0);
            v4 yr[3], yi[3];
            const long a0 = (kb0 + u0) * nf + kb;
            mma48_gl<R>(Fr + a0, Fi + a0, nf, uw, tw, Sr, Si, LD, nullptr, t0, 16 * wave, lane, yr, yi);
#pragma unroll
            for (int rt = 0; rt < 3; ++rt)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = 16 * rt + Mma<R>::row(lane, r);
                if (i < uw) {
                  Sr[(u0 + i) * LD + 16 * wave + (lane & 15)] -= yr[rt][r];
                  Si[(u0 + i) * LD + 16 * wave + (lane & 15)] -= yi[rt][r];
                }
              }
          }
        }
        __syncthreads();
      }
      R* Mr = fac + (FWD ? d.m : d.h) + (long)sb * 2 * kSB * kSB;
      R* Mi = Mr + kSB * kSB;
      for (int o = tid; o < sw * RZ; o += blockDim.x) {
        const int k = o / RZ, r = o % RZ;
        if (c0 + r < sw) {
          Mr[k * kSB + c0 + r] = Sr[k * LD + r];
          Mi[k * kSB + c0 + r] = Si[k * LD + r];
        }
      }
      __syncthreads();
    }
  }
}

// The factor entries outside a super-block that multiply its unknowns, folded
// with the block's map: LU = 0: Lhat[i][block] = L[i][block] M for the rows
// below the block (pivot rows after it and boundary rows); LU = 1:
// Uhat[i][block] = U[i][block] H for the pivot rows above it.  Read from the
// front F, written into the factor; 64 x 64 output tile per workgroup (grid.y:
// super-block x three column tiles), K = the block width in chunks of 48.
template <typename R, int LU>
__global__ __launch_bounds__(256) void hat_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                  int nlvl, const R* __restrict__ buf, R* __restrict__ fac) {
  typedef typename Mma<R>::v4 v4;
  __shared__ R Ar_[kRB * kLL], Ai_[kRB * kLL];
  __shared__ R Br_[kT * kLX], Bi_[kT * kLX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  constexpr int NCT = kSB / 64;
  for (int q = blockIdx.z; q < nlvl; q += gridDim.z) {
    const FrontDev d = fr[lvl[q]];
    const long nf = d.nf, np = d.np;
    const R* Fr = buf + d.f;
    const R* Fi = Fr + nf * nf;
    for (int y = blockIdx.y; (long)(y / NCT) * kSB < np; y += gridDim.y) {
      const int sb = y / NCT, ct = y % NCT;
      const long kb0 = (long)sb * kSB;
      const int sw = (int)min((long)kSB, np - kb0);
      const int j0 = ct * 64;
      if (j0 >= sw) continue;
      const long r0 = LU == 0 ? kb0 + sw : 0, r1 = LU == 0 ? nf : kb0;
      const long i0 = r0 + (long)blockIdx.x * kRB;
      if (i0 >= r1) continue;
      const int cnt = (int)min((long)kRB, r1 - i0);
      const R* Br = fac + (LU == 0 ? d.m : d.h) + (long)sb * 2 * kSB * kSB;
      const R* Bi = Br + kSB * kSB;
      v4 cr[2][2], ci[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cr[a][b] = v4{R(0), R(0), R(0), R(0)};
          ci[a][b] = v4{R(0), R(0), R(0), R(0)};
        }
      for (int kc = 0; kc < sw; kc += kT) {
        const int kw = min(kT, sw - kc);
        {  // all loads issued before the LDS stores
          constexpr int NU = (kRB * kT) / 256;
          R ld0_[NU], ld1_[NU];
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const int o = tid + 256 * u;
            const int i = o / kT, k = o % kT;
            const bool ok = i < cnt && k < kw;
            const long src = (i0 + i) * nf + kb0 + kc + k;
            ld0_[u] = ok ? Fr[src] : R(0);
            ld1_[u] = ok ? Fi[src] : R(0);
          }
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const int o = tid + 256 * u;
            const int i = o / kT, k = o % kT;
            Ar_[i * kLL + k] = ld0_[u];
            Ai_[i * kLL + k] = ld1_[u];
          }
        }
        {  // all loads issued before the LDS stores
          constexpr int NU = (kT * 64) / 256;
          R ld0_[NU], ld1_[NU];
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const int o = tid + 256 * u;
            const int k = o / 64, c = o % 64;
            const bool ok = k < kw && j0 + c < sw;
            ld0_[u] = ok ? Br[(kc + k) * kSB + j0 + c] : R(0);
            ld1_[u] = ok ? Bi[(kc + k) * kSB + j0 + c] : R(0);
          }
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const int o = tid + 256 * u;
            const int k = o / 64, c = o % 64;
            Br_[k * kLX + c] = ld0_[u];
            Bi_[k * kLX + c] = ld1_[u];
          }
        }
        __syncthreads();
        cmma64<R>(Ar_, Ai_, kLL, Br_, Bi_, kLX, kT, wm, wn, lane, cr, ci);
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = wm + 16 * a + Mma<R>::row(lane, r), col = wn + 16 * b + (lane & 15);
            if (row < cnt && j0 + col < sw) {
              const long gi = i0 + row, gc = kb0 + j0 + col;
              if (gi < np) {
                fac[d.p + gi * nf + gc] = cr[a][b][r];
                fac[d.p + np * nf + gi * nf + gc] = ci[a][b][r];
              } else {
                fac[d.l + (gi - np) * np + gc] = cr[a][b][r];
                fac[d.l + (long)d.nb * np + (gi - np) * np + gc] = ci[a][b][r];
              }
            }
          }
    }
  }
}

// Forward solve step of super-block [kb0, kb0 + sw) of every front of a
// level.  Workgroups [0, 3): z_block (64 rows each) = M x_block, written to Z.
// The others: 64 rows i below the block: x_i -= Lhat[i][block] x_block (pivot
// rows in X, boundary rows in the node's update vector).  Both read only the
// block's x rows, which no workgroup writes.  SR rhs per workgroup (64, or
// 32 in FP32 launches of few workgroups).
template <typename R, int SR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 1, 8))) void fwd_sb_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                     int nlvl, int kb0, const R* __restrict__ fac, int nrhs,
                                                     R* __restrict__ Xr, R* __restrict__ Xi, R* __restrict__ Zr,
                                                     R* __restrict__ Zi, R* __restrict__ Ur, R* __restrict__ Ui) {
  typedef typename Mma<R>::v4 v4;
  constexpr int LX = SR + 1, NBW = SR / 32;
  constexpr int NZB = kSB / kRB;
  __shared__ R Ar_[kRB * kLL], Ai_[kRB * kLL];
  __shared__ R Br_[kT * LX], Bi_[kT * LX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * (SR / 2);
  const int r0 = blockIdx.z * SR;
  const int nr = min(SR, nrhs - r0);
  const bool zrole = (int)blockIdx.x < NZB;
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    if (kb0 >= d.np) continue;
    const int sw = min(kSB, d.np - kb0);
    const long nf = d.nf, np = d.np;
    long i0;
    int cnt;
    if (zrole) {
      i0 = (long)blockIdx.x * kRB;                       // rows of the block
      if (i0 >= sw) continue;
      cnt = (int)min((long)kRB, sw - i0);
    } else {
      i0 = kb0 + sw + (long)(blockIdx.x - NZB) * kRB;    // rows below it
      if (i0 >= nf) continue;
      cnt = (int)min((long)kRB, nf - i0);
    }
    const R* Mr = fac + d.m + (long)(kb0 / kSB) * 2 * kSB * kSB;
    const R* Mi = Mr + kSB * kSB;
    CAcc<R, NBW> acc;
    acc.zero();
    // the next K chunk is loaded into registers while the MFMAs consume the current one
    constexpr int NUA = (kRB * kT) / 256, NUB = (kT * SR) / 256;
    R pa0[NUA], pa1[NUA], pb0[NUB], pb1[NUB];
    auto fetch = [&](int kc) {
      // addresses formed per chunk from an opaque thread index, not kept live
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int kw = min(kT, sw - kc);
#pragma unroll
      for (int u = 0; u < NUA; ++u) {
        const int o = tid + 256 * u;
        const int i = o / kT, k = o % kT;
        R vr = R(0), vi = R(0);
        if (i < cnt && k < kw) {
          if (zrole) {
            vr = Mr[(i0 + i) * kSB + kc + k];
            vi = Mi[(i0 + i) * kSB + kc + k];
          } else {
            const long gi = i0 + i, col = kb0 + kc + k;
            if (gi < np) {
              vr = fac[d.p + gi * nf + col];
              vi = fac[d.p + np * nf + gi * nf + col];
            } else {
              vr = fac[d.l + (gi - np) * np + col];
              vi = fac[d.l + (long)d.nb * np + (gi - np) * np + col];
            }
          }
        }
        pa0[u] = vr;
        pa1[u] = vi;
      }
#pragma unroll
      for (int u = 0; u < NUB; ++u) {
        const int o = tid + 256 * u;
        const int k = o / SR, r = o % SR;
        R vr = R(0), vi = R(0);
        if (k < kw && r < nr) {
          vr = Xr[(d.e0 + kb0 + kc + k) * (long)nrhs + r0 + r];
          vi = Xi[(d.e0 + kb0 + kc + k) * (long)nrhs + r0 + r];
        }
        pb0[u] = vr;
        pb1[u] = vi;
      }
    };
    fetch(0);
    for (int kc = 0; kc < sw; kc += kT) {
#pragma unroll
      for (int u = 0; u < NUA; ++u) {
        const int o = tid + 256 * u;
        Ar_[(o / kT) * kLL + o % kT] = pa0[u];
        Ai_[(o / kT) * kLL + o % kT] = pa1[u];
      }
#pragma unroll
      for (int u = 0; u < NUB; ++u) {
        const int o = tid + 256 * u;
        Br_[(o / SR) * LX + o % SR] = pb0[u];
        Bi_[(o / SR) * LX + o % SR] = pb1[u];
      }
      __syncthreads();
      if (kc + kT < sw) fetch(kc + kT);
      acc.mma(Ar_, Ai_, kLL, Br_, Bi_, LX, kT, wm, wn, lane);
      __syncthreads();
    }
    v4 cr[2][NBW], ci[2][NBW];
    acc.result(cr, ci);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wm + 16 * a + Mma<R>::row(lane, r), col = wn + 16 * b + (lane & 15);
          if (row < cnt && col < nr) {
            if (zrole) {
              Zr[(d.e0 + kb0 + i0 + row) * nrhs + r0 + col] = cr[a][b][r];
              Zi[(d.e0 + kb0 + i0 + row) * nrhs + r0 + col] = ci[a][b][r];
            } else {
              const long gi = i0 + row;
              const long dst = gi < np ? (d.e0 + gi) * nrhs + r0 + col : (d.u + gi - np) * nrhs + r0 + col;
              R* Tr = gi < np ? Xr : Ur;
              R* Ti = gi < np ? Xi : Ui;
              Tr[dst] -= cr[a][b][r];
              Ti[dst] -= ci[a][b][r];
            }
          }
        }
  }
}

// z_i -= sum_j U12[i][j] x_bnd(j) for 64 pivot rows and kKS boundary columns
// per workgroup (grid.z = column split + splits * rhs chunk).  A node with
// one split subtracts in place; with more, each split writes its partial sum
// and u12_reduce_kernel adds them in split order.
template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1, 8))) void bwd_u12_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                      int nlvl, int nks_max, long np_max,
                                                      const R* __restrict__ fac, const int* __restrict__ ib, int nrhs,
                                                      const R* __restrict__ Xr, const R* __restrict__ Xi,
                                                      R* __restrict__ Zr, R* __restrict__ Zi, R* __restrict__ Pr,
                                                      R* __restrict__ Pi) {
  typedef typename Mma<R>::v4 v4;
  constexpr int LA = kKC + 1;
  __shared__ R Ar_[kRB * LA], Ai_[kRB * LA];   // U12 block [64][kKC]
  __shared__ R Br_[kKC * kLX], Bi_[kKC * kLX]; // gathered x_bnd [kKC][kSR]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int ks = blockIdx.z % nks_max;
  const int r0 = (blockIdx.z / nks_max) * kSR;
  const int nr = min(kSR, nrhs - r0);
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    const long np = d.np, nf = d.nf, nb = d.nb;
    const int nks = (int)((nb + kKS - 1) / kKS);
    if (ks >= nks) continue;
    const long i0 = (long)blockIdx.x * kRB;
    if (i0 >= np) continue;
    const int cnt = (int)min((long)kRB, np - i0);
    const long j0 = (long)ks * kKS, j1 = min(nb, j0 + kKS);
    CAcc<R> acc;
    acc.zero();
    // the next chunk is loaded into registers while the MFMAs consume the current one
    constexpr int NUA = (kRB * kKC) / 256, NUB = (kKC * kSR) / 256;
    R pa0[NUA], pa1[NUA], pb0[NUB], pb1[NUB];
    auto fetch = [&](long jc) {
      // addresses formed per chunk from an opaque thread index, not kept live
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int nj = (int)min((long)kKC, j1 - jc);
#pragma unroll
      for (int u = 0; u < NUA; ++u) {
        const int o = tid + 256 * u;
        const int i = o / kKC, j = o % kKC;
        R vr = R(0), vi = R(0);
        if (i < cnt && j < nj) {
          vr = fac[d.p + (i0 + i) * nf + np + jc + j];
          vi = fac[d.p + np * nf + (i0 + i) * nf + np + jc + j];
        }
        pa0[u] = vr;
        pa1[u] = vi;
      }
#pragma unroll
      for (int u = 0; u < NUB; ++u) {
        const int o = tid + 256 * u;
        const int j = o / kSR, r = o % kSR;
        R vr = R(0), vi = R(0);
        if (j < nj && r < nr) {
          const long e = ib[d.bm + jc + j];
          vr = Xr[e * nrhs + r0 + r];
          vi = Xi[e * nrhs + r0 + r];
        }
        pb0[u] = vr;
        pb1[u] = vi;
      }
    };
    fetch(j0);
    for (long jc = j0; jc < j1; jc += kKC) {
#pragma unroll
      for (int u = 0; u < NUA; ++u) {
        const int o = tid + 256 * u;
        Ar_[(o / kKC) * LA + o % kKC] = pa0[u];
        Ai_[(o / kKC) * LA + o % kKC] = pa1[u];
      }
#pragma unroll
      for (int u = 0; u < NUB; ++u) {
        const int o = tid + 256 * u;
        Br_[(o / kSR) * kLX + o % kSR] = pb0[u];
        Bi_[(o / kSR) * kLX + o % kSR] = pb1[u];
      }
      __syncthreads();
      if (jc + kKC < j1) fetch(jc + kKC);
      acc.mma(Ar_, Ai_, LA, Br_, Bi_, kLX, kKC, wm, wn, lane);
      __syncthreads();
    }
    v4 cr[2][2], ci[2][2];
    acc.result(cr, ci);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wm + 16 * a + Mma<R>::row(lane, r), col = wn + 16 * b + (lane & 15);
          if (row < cnt && col < nr) {
            if (nks == 1) {
              Zr[(d.e0 + i0 + row) * nrhs + r0 + col] -= cr[a][b][r];
              Zi[(d.e0 + i0 + row) * nrhs + r0 + col] -= ci[a][b][r];
            } else {
              const long o = (((long)q * nks_max + ks) * np_max + i0 + row) * nrhs + r0 + col;
              Pr[o] = cr[a][b][r];
              Pi[o] = ci[a][b][r];
            }
          }
        }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void u12_reduce_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                         int nlvl, int nks_max, long np_max, int nrhs,
                                                         const R* __restrict__ Pr, const R* __restrict__ Pi,
                                                         R* __restrict__ Zr, R* __restrict__ Zi) {
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    const int nks = (int)((d.nb + kKS - 1) / kKS);
    if (nks < 2) continue;
    for (long i = (long)blockIdx.x * 4 + (threadIdx.x >> 6); i < d.np; i += (long)gridDim.x * 4)
      for (int r = threadIdx.x & 63; r < nrhs; r += 64) {
        R sr = R(0), si = R(0);
        for (int ks = 0; ks < nks; ++ks) {
          const long o = (((long)q * nks_max + ks) * np_max + i) * nrhs + r;
          sr += Pr[o];
          si += Pi[o];
        }
        Zr[(d.e0 + i) * nrhs + r] -= sr;
        Zi[(d.e0 + i) * nrhs + r] -= si;
      }
  }
}

// Backward solve step of super-block [kb0, kb0 + sw).  Workgroups [0, 3):
// x_block (64 rows each) = H y_block, written to X.  The others: 64 rows
// i < kb0: y_i -= Uhat[i][block] y_block.  Both read only the block's y rows.
// SR rhs per workgroup, as in fwd_sb_kernel.
template <typename R, int SR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? (SR == 32 ? 4 : 3) : 1, 8))) void bwd_sb_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                     int nlvl, int kb0, const R* __restrict__ fac, int nrhs,
                                                     R* __restrict__ Xr, R* __restrict__ Xi, R* __restrict__ Zr,
                                                     R* __restrict__ Zi) {
  typedef typename Mma<R>::v4 v4;
  constexpr int LX = SR + 1, NBW = SR / 32;
  constexpr int NZB = kSB / kRB;
  __shared__ R Ar_[kRB * kLL], Ai_[kRB * kLL];
  __shared__ R Br_[kT * LX], Bi_[kT * LX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * (SR / 2);
  const int r0 = blockIdx.z * SR;
  const int nr = min(SR, nrhs - r0);
  const bool xrole = (int)blockIdx.x < NZB;
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    if (kb0 >= d.np) continue;
    const int sw = min(kSB, d.np - kb0);
    const long nf = d.nf, np = d.np;
    long i0;
    int cnt;
    if (xrole) {
      i0 = (long)blockIdx.x * kRB;
      if (i0 >= sw) continue;
      cnt = (int)min((long)kRB, sw - i0);
    } else {
      i0 = (long)(blockIdx.x - NZB) * kRB;
      if (i0 >= kb0) continue;
      cnt = (int)min((long)kRB, kb0 - i0);
    }
    const R* Hr = fac + d.h + (long)(kb0 / kSB) * 2 * kSB * kSB;
    const R* Hi = Hr + kSB * kSB;
    CAcc<R, NBW> acc;
    acc.zero();
    // the next K chunk is loaded into registers while the MFMAs consume the current one
    constexpr int NUA = (kRB * kT) / 256, NUB = (kT * SR) / 256;
    R pa0[NUA], pa1[NUA], pb0[NUB], pb1[NUB];
    auto fetch = [&](int kc) {
      // addresses formed per chunk from an opaque thread index, not kept live
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int kw = min(kT, sw - kc);
#pragma unroll
      for (int u = 0; u < NUA; ++u) {
        const int o = tid + 256 * u;
        const int i = o / kT, k = o % kT;
        R vr = R(0), vi = R(0);
        if (i < cnt && k < kw) {
          if (xrole) {
            vr = Hr[(i0 + i) * kSB + kc + k];
            vi = Hi[(i0 + i) * kSB + kc + k];
          } else {
            vr = fac[d.p + (i0 + i) * nf + kb0 + kc + k];
            vi = fac[d.p + np * nf + (i0 + i) * nf + kb0 + kc + k];
          }
        }
        pa0[u] = vr;
        pa1[u] = vi;
      }
#pragma unroll
      for (int u = 0; u < NUB; ++u) {
        const int o = tid + 256 * u;
        const int k = o / SR, r = o % SR;
        R vr = R(0), vi = R(0);
        if (k < kw && r < nr) {
          vr = Zr[(d.e0 + kb0 + kc + k) * (long)nrhs + r0 + r];
          vi = Zi[(d.e0 + kb0 + kc + k) * (long)nrhs + r0 + r];
        }
        pb0[u] = vr;
        pb1[u] = vi;
      }
    };
    fetch(0);
    for (int kc = 0; kc < sw; kc += kT) {
#pragma unroll
      for (int u = 0; u < NUA; ++u) {
        const int o = tid + 256 * u;
        Ar_[(o / kT) * kLL + o % kT] = pa0[u];
        Ai_[(o / kT) * kLL + o % kT] = pa1[u];
      }
#pragma unroll
      for (int u = 0; u < NUB; ++u) {
        const int o = tid + 256 * u;
        Br_[(o / SR) * LX + o % SR] = pb0[u];
        Bi_[(o / SR) * LX + o % SR] = pb1[u];
      }
      __syncthreads();
      if (kc + kT < sw) fetch(kc + kT);
      acc.mma(Ar_, Ai_, kLL, Br_, Bi_, LX, kT, wm, wn, lane);
      __syncthreads();
    }
    v4 cr[2][NBW], ci[2][NBW];
    acc.result(cr, ci);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wm + 16 * a + Mma<R>::row(lane, r), col = wn + 16 * b + (lane & 15);
          if (row < cnt && col < nr) {
            if (xrole) {
              Xr[(d.e0 + kb0 + i0 + row) * nrhs + r0 + col] = cr[a][b][r];
              Xi[(d.e0 + kb0 + i0 + row) * nrhs + r0 + col] = ci[a][b][r];
            } else {
              Zr[(d.e0 + i0 + row) * nrhs + r0 + col] -= cr[a][b][r];
              Zi[(d.e0 + i0 + row) * nrhs + r0 + col] -= ci[a][b][r];
            }
          }
        }
  }
}

// Few right-hand sides (at most kGemvRhs): the products of fwd_sb_kernel
// (FWD) and bwd_sb_kernel as matrix-vector products, kGemvLanes lanes per
// row with the block's vector in LDS (the 64-rhs MFMA tiles would compute mostly zero
// columns).  Same grid and the same rows read and written as those kernels.
constexpr int kGemvRhs = 4;
constexpr int kGemvLanes = 16;   // lanes per row: four rows per wave, 128-byte row segments per load
constexpr int kGemvRows = 256 / kGemvLanes;   // rows per workgroup (one pass): more workgroups per front
template <typename R, bool FWD>
__global__ __launch_bounds__(256) void sb_gemv_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                      int nlvl, int kb0, const R* __restrict__ fac, int nrhs,
                                                      R* __restrict__ Xr, R* __restrict__ Xi, R* __restrict__ Zr,
                                                      R* __restrict__ Zi, R* __restrict__ Ur, R* __restrict__ Ui) {
  constexpr int NZB = kSB / kGemvRows;
  __shared__ R vr_[kSB * kGemvRhs], vi_[kSB * kGemvRhs];
  const int tid = threadIdx.x, sub = tid % kGemvLanes;
  const bool brole = (int)blockIdx.x < NZB;      // rows of the block (M or H) or rows outside it
  // the block's vector: x rows (forward) or y rows (backward) of the block
  const R* Vr = FWD ? Xr : Zr;
  const R* Vi = FWD ? Xi : Zi;
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    if (kb0 >= d.np) continue;
    const int sw = min(kSB, d.np - kb0);
    const long nf = d.nf, np = d.np;
    long i0;
    int cnt;
    if (brole) {
      i0 = (long)blockIdx.x * kGemvRows;
      if (i0 >= sw) continue;
      cnt = (int)min((long)kGemvRows, sw - i0);
    } else if (FWD) {
      i0 = kb0 + sw + (long)(blockIdx.x - NZB) * kGemvRows;   // rows below the block
      if (i0 >= nf) continue;
      cnt = (int)min((long)kGemvRows, nf - i0);
    } else {
      i0 = (long)(blockIdx.x - NZB) * kGemvRows;              // rows above the block
      if (i0 >= kb0) continue;
      cnt = (int)min((long)kGemvRows, kb0 - i0);
    }
    for (int e = tid; e < sw * nrhs; e += 256) {
      const int k = e / nrhs, r = e % nrhs;
      vr_[k * kGemvRhs + r] = Vr[(d.e0 + kb0 + k) * (long)nrhs + r];
      vi_[k * kGemvRhs + r] = Vi[(d.e0 + kb0 + k) * (long)nrhs + r];
    }
    __syncthreads();
    const R* Br = fac + (FWD ? d.m : d.h) + (long)(kb0 / kSB) * 2 * kSB * kSB;   // M (forward) or H
    const R* Bi = Br + kSB * kSB;
    for (int row = tid / kGemvLanes; row < cnt; row += 256 / kGemvLanes) {
      const long gi = i0 + row;
      const R* ar;
      const R* ai;
      if (brole) {
        ar = Br + gi * kSB;
        ai = Bi + gi * kSB;
      } else if (!FWD || gi < np) {
        ar = fac + d.p + gi * nf + kb0;
        ai = fac + d.p + np * nf + gi * nf + kb0;
      } else {
        ar = fac + d.l + (gi - np) * np + kb0;
        ai = fac + d.l + (long)d.nb * np + (gi - np) * np + kb0;
      }
      R sr[kGemvRhs], si[kGemvRhs];
#pragma unroll
      for (int r = 0; r < kGemvRhs; ++r) sr[r] = si[r] = R(0);
      for (int k = sub; k < sw; k += kGemvLanes) {
        const R a = ar[k], b = ai[k];
#pragma unroll
        for (int r = 0; r < kGemvRhs; ++r) {
          if (r < nrhs) {
            const R xr = vr_[k * kGemvRhs + r], xi = vi_[k * kGemvRhs + r];
            sr[r] += a * xr - b * xi;
            si[r] += a * xi + b * xr;
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kGemvRhs; ++r)
        if (r < nrhs)
#pragma unroll
          for (int off = kGemvLanes / 2; off > 0; off >>= 1) {
            sr[r] += __shfl_xor(sr[r], off);
            si[r] += __shfl_xor(si[r], off);
          }
      if (sub < nrhs) {
        R vr = sr[0], vi = si[0];
#pragma unroll
        for (int r = 1; r < kGemvRhs; ++r)
          if (sub == r) {
            vr = sr[r];
            vi = si[r];
          }
        const int r = sub;
        if (brole) {
          // z (forward) or x (backward) rows of the block
          R* Or = FWD ? Zr : Xr;
          R* Oi = FWD ? Zi : Xi;
          Or[(d.e0 + kb0 + gi) * nrhs + r] = vr;
          Oi[(d.e0 + kb0 + gi) * nrhs + r] = vi;
        } else if (FWD) {
          const long dst = gi < np ? (d.e0 + gi) * nrhs + r : (d.u + gi - np) * nrhs + r;
          R* Tr = gi < np ? Xr : Ur;
          R* Ti = gi < np ? Xi : Ui;
          Tr[dst] -= vr;
          Ti[dst] -= vi;
        } else {
          Zr[(d.e0 + gi) * nrhs + r] -= vr;
          Zi[(d.e0 + gi) * nrhs + r] -= vi;
        }
      }
    }
    __syncthreads();   // the vector is restaged for the next front
  }
}

// Few right-hand sides: bwd_u12_kernel as matrix-vector products,
// kGemvLanes lanes per pivot row over the split's kKS boundary columns (gathered x in LDS); the
// same outputs (in place with one split, else the split's partial sums).
template <typename R>
__global__ __launch_bounds__(256) void u12_gemv_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ lvl,
                                                       int nlvl, int nks_max, long np_max,
                                                       const R* __restrict__ fac, const int* __restrict__ ib, int nrhs,
                                                       const R* __restrict__ Xr, const R* __restrict__ Xi,
                                                       R* __restrict__ Zr, R* __restrict__ Zi, R* __restrict__ Pr,
                                                       R* __restrict__ Pi) {
  __shared__ R vr_[kKS * kGemvRhs], vi_[kKS * kGemvRhs];
  const int tid = threadIdx.x, sub = tid % kGemvLanes;
  const int ks = blockIdx.z;
  for (int q = blockIdx.y; q < nlvl; q += gridDim.y) {
    const FrontDev d = fr[lvl[q]];
    const long np = d.np, nf = d.nf, nb = d.nb;
    const int nks = (int)((nb + kKS - 1) / kKS);
    if (ks >= nks) continue;
    const long i0 = (long)blockIdx.x * kGemvRows;
    if (i0 >= np) continue;
    const int cnt = (int)min((long)kGemvRows, np - i0);
    const long j0 = (long)ks * kKS;
    const int nj = (int)min((long)kKS, nb - j0);
    for (int e = tid; e < nj * nrhs; e += 256) {
      const int j = e / nrhs, r = e % nrhs;
      const long x = ib[d.bm + j0 + j];
      vr_[j * kGemvRhs + r] = Xr[x * nrhs + r];
      vi_[j * kGemvRhs + r] = Xi[x * nrhs + r];
    }
    __syncthreads();
    for (int row = tid / kGemvLanes; row < cnt; row += 256 / kGemvLanes) {
      const long gi = i0 + row;
      const R* ar = fac + d.p + gi * nf + np + j0;
      const R* ai = fac + d.p + np * nf + gi * nf + np + j0;
      R sr[kGemvRhs], si[kGemvRhs];
#pragma unroll
      for (int r = 0; r < kGemvRhs; ++r) sr[r] = si[r] = R(0);
      for (int j = sub; j < nj; j += kGemvLanes) {
        const R a = ar[j], b = ai[j];
#pragma unroll
        for (int r = 0; r < kGemvRhs; ++r) {
          if (r < nrhs) {
            const R xr = vr_[j * kGemvRhs + r], xi = vi_[j * kGemvRhs + r];
            sr[r] += a * xr - b * xi;
            si[r] += a * xi + b * xr;
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kGemvRhs; ++r)
        if (r < nrhs)
#pragma unroll
          for (int off = kGemvLanes / 2; off > 0; off >>= 1) {
            sr[r] += __shfl_xor(sr[r], off);
            si[r] += __shfl_xor(si[r], off);
          }
      if (sub < nrhs) {
        R vr = sr[0], vi = si[0];
#pragma unroll
        for (int r = 1; r < kGemvRhs; ++r)
          if (sub == r) {
            vr = sr[r];
            vi = si[r];
          }
        if (nks == 1) {
          Zr[(d.e0 + gi) * nrhs + sub] -= vr;
          Zi[(d.e0 + gi) * nrhs + sub] -= vi;
        } else {
          const long o = (((long)q * nks_max + ks) * np_max + gi) * nrhs + sub;
          Pr[o] = vr;
          Pi[o] = vi;
        }
      }
    }
    __syncthreads();   // the gathered vector is restaged for the next front
  }
}

inline unsigned grid_for(long work, long per = 256, long cap = 65535) {
  long g = (work + per - 1) / per;
  return (unsigned)std::max(1L, std::min(g, cap));
}

}  // namespace

struct GpuSolver {
  int n = 0;
  int dims[3] = {0, 0, 0};             // grid extents (n, n, n) in 3-D, (n, n, 1) in 2-D
  int nc = 3;                          // unknowns per point (field components)
  long npts = 0;
  bool fp32 = false;
  long N = 0;                          // nc * npts unknowns
  std::vector<FrontDev> fh;            // per node (host copy)
  std::vector<std::vector<int>> levels;   // node ids per depth
  std::vector<long> lvl_off;           // offset of each level's list in lvl_d
  std::vector<int> lvl_np, lvl_nf;     // largest np / nf per level
  std::vector<size_t> lvl_elems;       // level buffer elements (R) per level
  DevBuf fd, lvl_d, ib, fac;
  DevBuf ipm;                          // inverse of the final elimination order (natural -> position)
  long u_rows = 0;                     // sum of nb over the nodes
  DevBuf X, Z, U;                      // solve work, sized for cap_rhs
  DevBuf P;                            // split-K partial sums of the U12 products
  int cap_rhs = 0;
  size_t bytes = 0;
  double flops = 0.0;
};

namespace {

template <typename R>
ls_status factor_numeric(GpuSolver& g, const C<double>* rows, hipStream_t s) {
  const int L = (int)g.levels.size();
  size_t cap[2] = {0, 0};
  for (int dep = 0; dep < L; ++dep) cap[dep & 1] = std::max(cap[dep & 1], g.lvl_elems[dep]);
  DevBuf lb[2];
  LS_TRY(lb[0].alloc(cap[0] * sizeof(R)));
  LS_TRY(lb[1].alloc(cap[1] * sizeof(R)));
  const FrontDev* fr = g.fd.as<FrontDev>();
  int* ib = g.ib.as<int>();
  R* fac = g.fac.as<R>();
  for (int dep = L - 1; dep >= 0; --dep) {
    const int nl = (int)g.levels[dep].size();
    const int* lvl = g.lvl_d.as<int>() + g.lvl_off[dep];
    R* buf = lb[dep & 1].as<R>();
    const R* cbuf = lb[(dep + 1) & 1].as<R>();
    const unsigned gy = (unsigned)std::min(nl, 65535);
    const long mnf = g.lvl_nf[dep], mnp = g.lvl_np[dep];
    hipLaunchKernelGGL(zero_kernel<R>, dim3(grid_for((long)g.lvl_elems[dep], 256, 1 << 20)), dim3(256), 0, s, buf,
                       (long)g.lvl_elems[dep]);
    if (g.nc == 3)
      hipLaunchKernelGGL((assemble_kernel<R, 3>), dim3(grid_for(mnf / 3 * 27), gy), dim3(256), 0, s, fr, lvl, nl, ib,
                         rows, buf);
    else
      hipLaunchKernelGGL((assemble_kernel<R, 2>), dim3(grid_for(mnf / 2 * 27), gy), dim3(256), 0, s, fr, lvl, nl, ib,
                         rows, buf);
    if (dep + 1 < L)
      for (int slot = 0; slot < 2; ++slot) {
        long mcnb = 0;
        for (int id : g.levels[dep])
          if (g.fh[id].child[slot] >= 0) mcnb = std::max(mcnb, (long)g.fh[g.fh[id].child[slot]].nb);
        if (mcnb == 0) continue;
        if (g.nc == 3)
          hipLaunchKernelGGL((extend_add_kernel<R, 3>), dim3((unsigned)std::min(mcnb, 8192L), std::min(gy, 64u)),
                             dim3(256), 0, s, fr, lvl, nl, slot, ib, cbuf, buf);
        else
          hipLaunchKernelGGL((extend_add_kernel<R, 2>), dim3((unsigned)std::min(mcnb, 8192L), std::min(gy, 64u)),
                             dim3(256), 0, s, fr, lvl, nl, slot, ib, cbuf, buf);
      }
    for (long kb0 = 0; kb0 < mnp; kb0 += kOB) {
      const long kbe = std::min(mnp, kb0 + kOB);
      for (long kb = kb0; kb < kbe; kb += kT) {
        hipLaunchKernelGGL(diag_kernel<R>, dim3(gy), dim3(256), 0, s, fr, lvl, nl, (int)kb, buf, fac, ib);
        const long rest = mnf - kb - 1;           // rows right of / below the tile, at most
        const int half = (int)std::max(1L, (rest + PanelCfg<R>::PR - 1) / PanelCfg<R>::PR);
        hipLaunchKernelGGL(panel_kernel<R>, dim3(2 * half, gy), dim3(256), 0, s, fr, lvl, nl, (int)kb, half, buf,
                           (const int*)ib);
        const unsigned tall = (unsigned)std::max(1L, (rest + 63) / 64);
        const unsigned blk = (unsigned)std::max(1L, (kbe - kb - 1 + 63) / 64);   // block columns left
        if (kb + kT < kbe) {
          hipLaunchKernelGGL(schur_kernel<R>, dim3(blk, tall, gy), dim3(256), 0, s, fr, lvl, nl, (int)kb,
                             (int)kb0, 0, buf);
          hipLaunchKernelGGL(schur_kernel<R>, dim3(tall, blk, gy), dim3(256), 0, s, fr, lvl, nl, (int)kb,
                             (int)kb0, 1, buf);
        }
      }
      const unsigned t64 = (unsigned)std::max(1L, (mnf - kb0 - 1 + 63) / 64);
      hipLaunchKernelGGL(schur_kernel<R>, dim3(t64, t64, gy), dim3(256), 0, s, fr, lvl, nl, (int)kb0, (int)kb0, 2,
                         buf);
    }
    hipLaunchKernelGGL(copyout_kernel<R>, dim3(grid_for(mnf * mnf, 256, 8192), std::min(gy, 64u)), dim3(256), 0, s,
                       fr, lvl, nl, (const R*)buf, fac);
    // selective inversion of the super-blocks, then the folded L and U entries
    const unsigned nsb = (unsigned)((mnp + kSB - 1) / kSB);
    const unsigned ncc = (unsigned)(kSB / SolveCfg<R>::RZ);
    hipLaunchKernelGGL((sb_inverse_kernel<R, true>), dim3(gy, nsb, ncc), dim3(256), 0, s, fr, lvl, nl,
                       (const R*)buf, fac, (const int*)ib);
    hipLaunchKernelGGL((sb_inverse_kernel<R, false>), dim3(gy, nsb, ncc), dim3(256), 0, s, fr, lvl, nl,
                       (const R*)buf, fac, (const int*)ib);
    const unsigned hy = std::min(65535u, nsb * (unsigned)(kSB / 64));
    const unsigned hx = (unsigned)std::max(1L, (mnf + kRB - 1) / kRB);
    hipLaunchKernelGGL((hat_kernel<R, 0>), dim3(hx, hy, gy), dim3(256), 0, s, fr, lvl, nl, (const R*)buf, fac);
    hipLaunchKernelGGL((hat_kernel<R, 1>), dim3(hx, hy, gy), dim3(256), 0, s, fr, lvl, nl, (const R*)buf, fac);
    LS_HIP(hipGetLastError());
  }
  // the elimination order is final once the pivots are chosen
  hipLaunchKernelGGL(inv_perm_kernel, dim3(grid_for(g.N, 256, 1 << 16)), dim3(256), 0, s, (const int*)ib, g.N,
                     g.ipm.as<int>());
  LS_HIP(hipGetLastError());
  LS_HIP(hipStreamSynchronize(s));
  return LS_OK;
}

// FP32 super-block launches with fewer than this many 64-rhs workgroups (the
// few large fronts at the top of the tree) take 32-rhs tiles on twice the
// workgroups; the factor blocks are then read once per 32 rhs.
constexpr long kSplitWg = 512;

template <typename R>
void launch_sb(bool fwd, unsigned gx, unsigned gy, int nrhs, hipStream_t s, const FrontDev* fr, const int* lvl,
               int nl, int kb0, const R* fac, R* Xr, R* Xi, R* Zr, R* Zi, R* Ur, R* Ui) {
  const unsigned gz = (unsigned)((nrhs + kSR - 1) / kSR);
  if constexpr (sizeof(R) == 4) {
    if ((long)gx * gy * gz < kSplitWg) {
      const unsigned gz2 = (unsigned)((nrhs + 31) / 32);
      if (fwd)
        hipLaunchKernelGGL((fwd_sb_kernel<R, 32>), dim3(gx, gy, gz2), dim3(256), 0, s, fr, lvl, nl, kb0, fac, nrhs,
                           Xr, Xi, Zr, Zi, Ur, Ui);
      else
        hipLaunchKernelGGL((bwd_sb_kernel<R, 32>), dim3(gx, gy, gz2), dim3(256), 0, s, fr, lvl, nl, kb0, fac, nrhs,
                           Xr, Xi, Zr, Zi);
      return;
    }
  }
  if (fwd)
    hipLaunchKernelGGL((fwd_sb_kernel<R, kSR>), dim3(gx, gy, gz), dim3(256), 0, s, fr, lvl, nl, kb0, fac, nrhs, Xr,
                       Xi, Zr, Zi, Ur, Ui);
  else
    hipLaunchKernelGGL((bwd_sb_kernel<R, kSR>), dim3(gx, gy, gz), dim3(256), 0, s, fr, lvl, nl, kb0, fac, nrhs, Xr,
                       Xi, Zr, Zi);
}

template <typename R>
ls_status solve_numeric(GpuSolver& g, const C<double>* b, C<double>* xo, int nrhs, hipStream_t s) {
  const int L = (int)g.levels.size();
  // split-K partial sums of the U12 products: levels whose widest boundary
  // needs more than one split
  std::vector<int> nks(L, 1);
  size_t pelems = 1;
  for (int dep = 0; dep < L; ++dep) {
    for (int id : g.levels[dep]) nks[dep] = std::max(nks[dep], (int)((g.fh[id].nb + kKS - 1) / kKS));
    if (nks[dep] > 1)
      pelems = std::max(pelems, (size_t)g.levels[dep].size() * nks[dep] * (size_t)g.lvl_np[dep] * nrhs);
  }
  if (g.cap_rhs < nrhs) {
    LS_TRY(g.X.alloc(2 * (size_t)g.N * nrhs * sizeof(R)));
    LS_TRY(g.Z.alloc(2 * (size_t)g.N * nrhs * sizeof(R)));
    LS_TRY(g.U.alloc(2 * (size_t)std::max(1L, g.u_rows) * nrhs * sizeof(R)));
    g.cap_rhs = nrhs;
  }
  if (g.P.bytes < 2 * pelems * sizeof(R)) LS_TRY(g.P.alloc(2 * pelems * sizeof(R)));
  R* Pr = g.P.as<R>();
  R* Pi = Pr + pelems;
  const long N = g.N;
  R* Xr = g.X.as<R>();
  R* Xi = Xr + N * nrhs;
  R* Zr = g.Z.as<R>();
  R* Zi = Zr + N * nrhs;
  R* Ur = g.U.as<R>();
  R* Ui = Ur + std::max(1L, g.u_rows) * nrhs;
  const FrontDev* fr = g.fd.as<FrontDev>();
  const int* ib = g.ib.as<int>();
  const R* fac = g.fac.as<R>();
  const unsigned gz = (unsigned)((nrhs + kSR - 1) / kSR);
  const int rpp = 256 / rhs_lanes(nrhs);     // rows per workgroup pass of the gather kernels
  if (nrhs >= kSolTileRhs)
    hipLaunchKernelGGL(sol_in_tile_kernel<R>, dim3((unsigned)((N + kTP - 1) / kTP), (unsigned)((nrhs + kTP - 1) / kTP)),
                       dim3(256), 0, s, b, N, nrhs, (const int*)g.ipm.as<int>(), Xr, Xi);
  else
    hipLaunchKernelGGL(sol_in_kernel<R>, dim3(grid_for(N, rpp, 65535)), dim3(256), 0, s, b, N, nrhs, ib, Xr, Xi);
  hipLaunchKernelGGL(zero_kernel<R>, dim3(grid_for(2 * std::max(1L, g.u_rows) * nrhs, 256, 1 << 16)), dim3(256), 0,
                     s, Ur, 2 * std::max(1L, g.u_rows) * nrhs);
  for (int dep = L - 1; dep >= 0; --dep) {
    const int nl = (int)g.levels[dep].size();
    const int* lvl = g.lvl_d.as<int>() + g.lvl_off[dep];
    const unsigned gy = (unsigned)std::min(nl, 65535);
    const long mnf = g.lvl_nf[dep], mnp = g.lvl_np[dep];
    if (dep + 1 < L)
      for (int slot = 0; slot < 2; ++slot) {
        long mcnb = 0;
        for (int id : g.levels[dep])
          if (g.fh[id].child[slot] >= 0) mcnb = std::max(mcnb, (long)g.fh[g.fh[id].child[slot]].nb);
        if (mcnb == 0) continue;
        // one front per workgroup row (a front loop would chain descriptor loads)
        const long gxc = std::max(1L, std::min((mcnb + rpp - 1) / rpp, std::max(1L, 65536L / nl)));
        if (g.nc == 3)
          hipLaunchKernelGGL((fwd_child_kernel<R, 3>), dim3((unsigned)gxc, gy), dim3(256), 0, s, fr, lvl, nl, slot,
                             ib, nrhs, Xr, Xi, Ur, Ui);
        else
          hipLaunchKernelGGL((fwd_child_kernel<R, 2>), dim3((unsigned)gxc, gy), dim3(256), 0, s, fr, lvl, nl, slot,
                             ib, nrhs, Xr, Xi, Ur, Ui);
      }
    for (long kb0 = 0; kb0 < mnp; kb0 += kSB) {
      const unsigned gx = (unsigned)(kSB / kRB + std::max(0L, (mnf - kb0 - 1 + kRB - 1) / kRB));
      if (nrhs <= kGemvRhs) {
        const unsigned gxg =
            (unsigned)(kSB / kGemvRows + std::max(0L, (mnf - kb0 - 1 + kGemvRows - 1) / kGemvRows));
        hipLaunchKernelGGL((sb_gemv_kernel<R, true>), dim3(gxg, gy), dim3(256), 0, s, fr, lvl, nl, (int)kb0, fac,
                           nrhs, Xr, Xi, Zr, Zi, Ur, Ui);
      }
      else
        launch_sb<R>(true, gx, gy, nrhs, s, fr, lvl, nl, (int)kb0, fac, Xr, Xi, Zr, Zi, Ur, Ui);
    }
  }
  for (int dep = 0; dep < L; ++dep) {
    const int nl = (int)g.levels[dep].size();
    const int* lvl = g.lvl_d.as<int>() + g.lvl_off[dep];
    const unsigned gy = (unsigned)std::min(nl, 65535);
    const long mnp = g.lvl_np[dep];
    const unsigned gu = (unsigned)std::max(1L, (mnp + kRB - 1) / kRB);
    if (nrhs <= kGemvRhs)
      hipLaunchKernelGGL(u12_gemv_kernel<R>, dim3((unsigned)std::max(1L, (mnp + kGemvRows - 1) / kGemvRows), gy,
                                                  nks[dep]),
                         dim3(256), 0, s, fr, lvl, nl, nks[dep], mnp, fac, ib, nrhs, (const R*)Xr, (const R*)Xi, Zr,
                         Zi, Pr, Pi);
    else
      hipLaunchKernelGGL(bwd_u12_kernel<R>, dim3(gu, gy, gz * nks[dep]), dim3(256), 0, s, fr, lvl, nl, nks[dep],
                         mnp, fac, ib, nrhs, (const R*)Xr, (const R*)Xi, Zr, Zi, Pr, Pi);
    if (nks[dep] > 1)
      hipLaunchKernelGGL(u12_reduce_kernel<R>, dim3(grid_for(mnp, 4, 4096), gy), dim3(256), 0, s, fr, lvl, nl,
                         nks[dep], mnp, nrhs, (const R*)Pr, (const R*)Pi, Zr, Zi);
    for (long kb0 = ((mnp - 1) / kSB) * kSB; kb0 >= 0; kb0 -= kSB) {
      const unsigned gx = (unsigned)(kSB / kRB + (kb0 + kRB - 1) / kRB);
      if (nrhs <= kGemvRhs) {
        const unsigned gxg = (unsigned)(kSB / kGemvRows + (kb0 + kGemvRows - 1) / kGemvRows);
        hipLaunchKernelGGL((sb_gemv_kernel<R, false>), dim3(gxg, gy), dim3(256), 0, s, fr, lvl, nl, (int)kb0, fac,
                           nrhs, Xr, Xi, Zr, Zi, Ur, Ui);
      }
      else
        launch_sb<R>(false, gx, gy, nrhs, s, fr, lvl, nl, (int)kb0, fac, Xr, Xi, Zr, Zi, Ur, Ui);
    }
  }
  if (nrhs >= kSolTileRhs)
    hipLaunchKernelGGL(sol_out_tile_kernel<R>, dim3((unsigned)((N + kTP - 1) / kTP), (unsigned)((nrhs + kTP - 1) / kTP)),
                       dim3(256), 0, s, xo, N, nrhs, (const int*)g.ipm.as<int>(), (const R*)Xr, (const R*)Xi);
  else
    hipLaunchKernelGGL(sol_out_kernel<R>, dim3(grid_for(N, rpp, 65535)), dim3(256), 0, s, xo, N, nrhs, ib,
                       (const R*)Xr, (const R*)Xi);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

}  // namespace

ls_status gpu_factor(int n, const C<double>* rows_dev, bool fp32, hipStream_t s, GpuSolver** out) {
  const int dims[3] = {n, n, n};
  return gpu_factor_grid(dims, 3, rows_dev, fp32, s, out);
}

ls_status gpu_factor_grid(const int dims[3], int nc, const C<double>* rows_dev, bool fp32, hipStream_t s,
                          GpuSolver** out) {
  if (!out) return LS_EINVAL;
  *out = nullptr;
  if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || (nc != 2 && nc != 3) || !rows_dev) return LS_EINVAL;
  std::unique_ptr<GpuSolver> g(new GpuSolver());
  g->n = dims[0];
  for (int d = 0; d < 3; ++d) g->dims[d] = dims[d];
  g->nc = nc;
  g->npts = (long)dims[0] * dims[1] * dims[2];
  g->fp32 = fp32;
  GpuSymbolic sym;
  LS_TRY(gpu_symbolic(dims, nc, sym));
  g->N = sym.N;
  g->fh = std::move(sym.fh);
  g->levels = std::move(sym.levels);
  g->lvl_off = std::move(sym.lvl_off);
  g->lvl_np = std::move(sym.lvl_np);
  g->lvl_nf = std::move(sym.lvl_nf);
  g->lvl_elems = std::move(sym.lvl_elems);
  g->u_rows = sym.u_rows;
  g->flops = sym.flops;
  const long fac_elems = sym.fac_elems;
  const IntMap& ibh = sym.ibh;
  const size_t rs = fp32 ? sizeof(float) : sizeof(double);
  LS_TRY(g->fac.alloc((size_t)fac_elems * rs));
  LS_TRY(g->ib.alloc(ibh.size() * sizeof(int)));
  LS_TRY(g->ipm.alloc((size_t)std::max(1L, g->N) * sizeof(int)));
  LS_TRY(g->fd.alloc(g->fh.size() * sizeof(FrontDev)));
  std::vector<int> lv;
  for (const auto& l : g->levels) lv.insert(lv.end(), l.begin(), l.end());
  LS_TRY(g->lvl_d.alloc(lv.size() * sizeof(int)));
  LS_HIP(hipMemcpyAsync(g->ib.p, ibh.data(), ibh.size() * sizeof(int), hipMemcpyHostToDevice, s));
  LS_HIP(hipMemcpyAsync(g->fd.p, g->fh.data(), g->fh.size() * sizeof(FrontDev), hipMemcpyHostToDevice, s));
  LS_HIP(hipMemcpyAsync(g->lvl_d.p, lv.data(), lv.size() * sizeof(int), hipMemcpyHostToDevice, s));
  g->bytes = (size_t)fac_elems * rs;
  if (fp32)
    LS_TRY(factor_numeric<float>(*g, rows_dev, s));
  else
    LS_TRY(factor_numeric<double>(*g, rows_dev, s));
  *out = g.release();
  return LS_OK;
}

ls_status gpu_solve(GpuSolver* gs, const C<double>* b_dev, C<double>* x_dev, int nrhs, hipStream_t s) {
  if (!gs || !b_dev || !x_dev || nrhs < 1) return LS_EINVAL;
  return gs->fp32 ? solve_numeric<float>(*gs, b_dev, x_dev, nrhs, s)
                  : solve_numeric<double>(*gs, b_dev, x_dev, nrhs, s);
}

size_t gpu_factor_bytes(const GpuSolver* gs) { return gs ? gs->bytes : 0; }
double gpu_factor_flops(const GpuSolver* gs) { return gs ? gs->flops : 0.0; }
bool gpu_factor_is_fp32(const GpuSolver* gs) { return gs && gs->fp32; }
void gpu_free(GpuSolver* gs) { delete gs; }

}  // namespace ls
