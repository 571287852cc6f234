// Kernels and launch helpers of the FFT apply (the five passes, the paper's
// form, the plan set-up transforms), shared by the translation units that
// instantiate the apply for each transform length P.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <utility>

#include "common.h"

namespace ls {

enum ColMode { COL_P1 = 0, COL_FWD = 1, COL_INV = 2, COL_P5 = 3 };

// ---- factor tables ----------------------------------------------------------
struct Fac {
  int n1, n2;
};
constexpr Fac col_factors(int P) {
  switch (P) {
    case 8: return {2, 4};
    case 12: return {3, 4};
    case 16: return {4, 4};
    case 24: return {4, 6};
    case 32: return {4, 8};
    case 48: return {6, 8};
    case 64: return {8, 8};
    case 96: return {8, 12};
    case 128: return {8, 16};
    case 192: return {12, 16};
    case 256: return {16, 16};
    case 384: return {16, 24};
    case 512: return {16, 32};
    case 768: return {24, 32};
    default: return {0, 0};
  }
}
// Pass 3 uses the same factorisation (its 3x3 multiply runs out of LDS slots).
template <typename R>
constexpr Fac row_factors(int P) {
  return col_factors(P);
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// lanes per job of pass 3 (see kmul_kernel)
constexpr int job_lanes(int tpl) { return (tpl > 16 && tpl <= 32) ? 32 : tpl; }
// Lines per workgroup of the strided passes: a LS_COL_RUN_BYTES run per row
// (one or two 128-byte cache lines), LDS <= 64 KB.
#ifndef LS_COL_RUN_BYTES
#define LS_COL_RUN_BYTES 256
#endif
// Every pass uses full runs (with non-temporal loads and stores, halving the
// run of any one pass at 128^3 was 1-11 % slower, and the dim-2 inverse
// gained 2 % from full runs).  The tile is capped at 64 KB of LDS, except
// in the dim-1 passes (modes 0 and 3, whose rows lie n^2 apart) which may
// use 96 KB so that P = 384 keeps full runs (192^3: 0.29 ms faster over the
// two passes; the dim-2 forward is slower with 96 KB).
template <typename R>
constexpr int col_tile(int P, int mode) {
  int t = LS_COL_RUN_BYTES / (2 * (int)sizeof(R));
  const long cap = (mode == 0 || mode == 3) ? 98304 : 65536;
  while (t > 8 && (long)P * t * 2 * (long)sizeof(R) > cap) t /= 2;
  return t;
}

// ---- strided-dimension four-step FFT ----------------------------------------
// Lines are contiguous (index `line` in [0, L)); the transform runs along rows
// with stride L.  Block = T lines x TPL threads; work item blk = batch * ntiles +
// tile.  An ordinary launch has one workgroup per item (blk = blockIdx.x); a
// PERSIST launch has the workgroups the device holds at once, which take
// blk = blockIdx.x, blockIdx.x + gridDim.x, ... < nblk.  The two are
// separate instantiations so that the ordinary one keeps its registers (in a
// loop the compiler holds the twiddles and addresses across items).
template <typename R, typename IO, int P, int N1, int N2, int T, int MODE, bool PAD, bool PERSIST = false>
__global__ __launch_bounds__(T * cmax(N1, N2)) void col_fft_kernel(
    const void* __restrict__ in_, void* __restrict__ out_, const C<R>* __restrict__ mfac,
    const C<R>* __restrict__ tw, int rows_in, int rows_out, long L, long in_bstride,
    long out_bstride, int ntiles, long nblk, R scale) {
  constexpr int DIR = (MODE == COL_P1 || MODE == COL_FWD) ? -1 : 1;
  // PAD: a forward pass reads at most P/2 rows, an inverse pass keeps at most P/2
  constexpr int KIN = (PAD && DIR < 0) ? (N2 + 1) / 2 : N2;
  constexpr int QOUT = (PAD && DIR > 0) ? (N1 + 1) / 2 : N1;
  __shared__ C<R> ex[N1 * N2 * T];
  auto item = [&](long blk, int tid) {
    const int t = tid % T;
    const int j = tid / T;
    const long batch = blk / ntiles;
    const int tile = (int)(blk % ntiles);
    const long line = (long)tile * T + t;
    const bool live = line < L;

    // the identity term of the last pass is loaded with the transform's input
    // rather than after the transform (its latency would otherwise end every
    // workgroup)
    C<IO> xid[QOUT];
    if (MODE == COL_P5) {
      const C<IO>* x = reinterpret_cast<const C<IO>*>(mfac);
#pragma unroll
      for (int q1 = 0; q1 < QOUT; ++q1) {
        const int row = j + N2 * q1;
        xid[q1] = (x && live && j < N2 && row < rows_out)
                      ? ld_stream(x + batch * out_bstride + (long)row * L + line)
                      : cmk<IO>(0, 0);
      }
    }

    if (j < N1) {
      C<R> v[N2];
#pragma unroll
      for (int k = 0; k < KIN; ++k) {
        const int row = j + N1 * k;
        C<R> z = cmk<R>(0, 0);
        if (live && row < rows_in) {
          const long off = batch * in_bstride + (long)row * L + line;
          if (MODE == COL_P1) {
            C<IO> xv = ld_stream(reinterpret_cast<const C<IO>*>(in_) + off);
            z = ccast<R>(xv) * mfac[(long)row * L + line];
          } else {
            z = ld_stream(reinterpret_cast<const C<R>*>(in_) + off);
          }
        }
        v[k] = z;
      }
      DftZ<N2, DIR, R, KIN>::run(v);
#pragma unroll
      for (int q = 0; q < N2; ++q) {
        C<R> w = tw[j * q];
        if (DIR > 0) w = cconj(w);
        ex[(j * N2 + q) * T + t] = (j * q == 0) ? v[q] : v[q] * w;
      }
    }
    __syncthreads();
    if (j < N2) {
      C<R> w[N1];
#pragma unroll
      for (int jj = 0; jj < N1; ++jj) w[jj] = ex[(jj * N2 + j) * T + t];
      Dft<N1, DIR, R>::run(w);
      if (live) {
#pragma unroll
        for (int q1 = 0; q1 < QOUT; ++q1) {
          const int row = j + N2 * q1;
          if (row < rows_out) {
            const long off = batch * out_bstride + (long)row * L + line;
            if (MODE == COL_P5) {
              C<IO>* y = reinterpret_cast<C<IO>*>(out_);
              const C<IO> xv = xid[q1];                                // identity term, or zero
              st_stream(y + off, cmk<IO>(xv.re + (IO)(w[q1].re * scale), xv.im + (IO)(w[q1].im * scale)));
            } else {
              st_stream(reinterpret_cast<C<R>*>(out_) + off, w[q1]);
            }
          }
        }
      }
    }
  };
  if constexpr (PERSIST) {
    for (long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
      if (blk != blockIdx.x) __syncthreads();     // the previous item's reads of ex are done
      // the thread index made opaque per item: the index arithmetic, twiddle
      // loads and addresses derived from it are then formed inside the loop
      // instead of being held in registers across items
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      item(blk, tid);
    }
  } else {
    item(blockIdx.x, threadIdx.x);
  }
}

// ---- pass 3: contiguous-dimension FFT, 3x3 Khat multiply, inverse -----------
// X: [B][3][P][P][n] (q1, q2, i3).  Kh: octant [H][H][6][H], components
// (xx, yy, zz, xy, xz, yz), already divided by P^3.
//
// A team is 4 jobs x JL threads: the up-to-four lines (+-f1, +-f2) of one
// right-hand side, JL = TPL (the larger factor of P) or, for 16 < TPL <= 32,
// 32 so that a job is half a wavefront (TPL = 24 at P = 384: 8 idle lanes per
// job, as the 96-lane team already had in its second wave).  A workgroup
// holds W teams that share one octant line of Khat in LDS and take
// right-hand sides b = team, team + W, ...  When no job straddles two
// wavefronts (JL = 16 or 32) its exchanges need only wavefront-level
// ordering (LDS operations of one wave complete in order), so jobs never
// wait for each other; otherwise W = 1 and the exchange uses a workgroup
// barrier.
// The three components of a line stay in registers from the forward
// transform through the 3x3 multiply into the inverse transform; the LDS
// exchange buffer holds one component at a time.
__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

template <typename R, int P, int N1, int N2, int W, bool PERSIST = false>
__global__ __launch_bounds__(W * 4 * job_lanes(cmax(N1, N2))) void kmul_kernel(C<R>* __restrict__ X,
                                                                               const C<R>* __restrict__ Kh,
                                                                               const C<R>* __restrict__ tw,
                                                                               int n, int B) {
  constexpr int H = P / 2 + 1;
  constexpr int JL = job_lanes(cmax(N1, N2));
  constexpr int TEAM = 4 * JL;
  constexpr bool WAVE_TEAM = (JL == 16 || JL == 32);   // no job straddles two waves
  static_assert(WAVE_TEAM || W == 1, "multi-team workgroups need jobs inside wavefronts");
  constexpr int EXS = N1 * N2 + N2;          // padded exchange stride of one job
  // Frequencies q3 = j + N2 a: with N1 even, a < N1/2 gives q3 < P/2 and
  // a >= N1/2 gives q3 >= P/2 (mirrored, f3 = P - q3), both known at compile
  // time.  The odd components of a mirrored line change sign (xy: q1 or q2
  // mirrored, xz: q1 or q3, yz: q2 or q3); the q1 and q2 signs of each of the
  // four lines are folded into its own copy of the odd components in LDS,
  // and the q3 sign into the multiply's operand modifiers, so the symbol
  // multiply has no sign arithmetic left.  With the fused multiply-adds of
  // the 3x3 product this cut the FP32 pass at 128^3, 8 rhs, from 1.023 to
  // 0.804 ms (2954 instead of 3405 VALU instructions per rhs and lane); the
  // same code with the signs applied by multiplies took 0.817 ms, and
  // without the load prefetch 0.866 ms.  The larger LDS footprint (35 KB per
  // two-team workgroup) caps the kernel at two waves per SIMD, as its
  // registers already did.
  constexpr bool SPLIT3 = (N1 % 2 == 0);
  constexpr bool SIGNED = SPLIT3;
  __shared__ C<R> ke[3 * H];                    // xx, yy, zz
  __shared__ C<R> ko[(SIGNED ? 4 : 1) * 3 * H]; // xy, xz, yz (per line when SIGNED)
  __shared__ C<R> twl[P];
  __shared__ C<R> ex[W * 4 * EXS];
  // a PERSIST launch (gridDim.x < H^2) takes octant lines grid-stride
  auto item = [&](int oline, int tid) {
    const int f1 = oline / H;
    const int f2 = oline % H;
    const int team = tid / TEAM;
    const int lt = tid % TEAM;
    const int job = lt / JL;
    const int j = lt % JL;                      // lanes j >= max(N1, N2) stay idle
    const int s1 = job & 1, s2 = job >> 1;
    const bool edge1 = (f1 == 0) || (2 * f1 == P);
    const bool edge2 = (f2 == 0) || (2 * f2 == P);
    const bool active = !((s1 && edge1) || (s2 && edge2));
    const int q1 = s1 ? P - f1 : f1;
    const int q2 = s2 ? P - f2 : f2;
    const long plane = (long)P * P * n;         // one component of one rhs
    const long lineoff = ((long)q1 * P + q2) * n;

    const C<R>* kg = Kh + ((long)f1 * H + f2) * 6 * H;
    for (int e = tid; e < 3 * H; e += W * TEAM) {
      ke[e] = kg[e];
      const C<R> o = kg[3 * H + e];
      if constexpr (SIGNED) {
        const int comp = e / H;                 // 0 xy, 1 xz, 2 yz
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const bool m1 = l & 1, m2 = l >> 1;
          const bool neg = (comp == 0) ? (m1 != m2) : (comp == 1 ? m1 : m2);
          ko[l * 3 * H + e] = neg ? cmk<R>(-o.re, -o.im) : o;
        }
      } else {
        ko[e] = o;
      }
    }
    for (int e = tid; e < P; e += W * TEAM) twl[e] = tw[e];
    // sign flips of the odd components for a mirrored line (runtime path only)
    const R sxy = (s1 != s2) ? (R)-1 : (R)1;   // xy odd in q1 and q2
    const R sx = s1 ? (R)-1 : (R)1;            // xz odd in q1 (and q3)
    const R sy = s2 ? (R)-1 : (R)1;            // yz odd in q2 (and q3)
    __syncthreads();

    C<R>* myex = ex + (team * 4 + job) * EXS;
    const C<R>* kol = ko + (SIGNED ? job * 3 * H : 0);
    auto tsync = [&]() {
      if (WAVE_TEAM)
        wave_lds_sync();
      else
        __syncthreads();
    };

    constexpr int KIN = (N2 + 1) / 2;     // t = j + N1 k < n <= P/2
    for (int b = team; b < B; b += W) {
      C<R>* base = X + (long)b * 3 * plane + lineoff;
      // FP32 at P = 256: all loads of the three components are issued before
      // any arithmetic.  Without the prefetch registers the kernel fits more
      // waves per SIMD, which wins elsewhere (P = 128, 16 rhs: 0.33 against
      // 0.41 ms, three waves; P = 384: 5.6 against 10.4 ms, two waves instead
      // of one); at P = 256 it still fits only two, and the prefetch wins (1.05
      // against 1.12 ms).  FP64 has no registers to spare for it.
      constexpr bool PREFETCH = sizeof(R) == 4 && P == 256;
      C<R> pre[3][KIN];
      if (PREFETCH && active && j < N1) {
        if (2 * n == P) {     // every t = j + N1 k < P/2 is a grid point: no bounds, no zero fill
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < KIN; ++k) pre[c][k] = ld_stream(base + c * plane + j + N1 * k);
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < KIN; ++k) {
              const int tt = j + N1 * k;
              pre[c][k] = (tt < n) ? ld_stream(base + c * plane + tt) : cmk<R>(0, 0);
            }
        }
      }
      C<R> u[3][N1];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // forward step 1: thread j < N1 owns t = j + N1 k
        if (active && j < N1) {
          C<R> v[N2];
#pragma unroll
          for (int k = 0; k < KIN; ++k) {
            const int tt = j + N1 * k;
            v[k] = PREFETCH ? pre[c][k] : ((tt < n) ? ld_stream(base + c * plane + tt) : cmk<R>(0, 0));
          }
          DftZ<N2, -1, R, KIN>::run(v);
          // twl[0] = 1 exactly, so lane j = 0 needs no exception
#pragma unroll
          for (int q = 0; q < N2; ++q) myex[q * (N1 + 1) + j] = (q == 0) ? v[q] : v[q] * twl[j * q];
        }
        tsync();
        // forward step 3: thread q2 = j < N2 gets X[j + N2 a], a in [0, N1)
        if (active && j < N2) {
#pragma unroll
          for (int a = 0; a < N1; ++a) u[c][a] = myex[j * (N1 + 1) + a];
          Dft<N1, -1, R>::run(u[c]);
        }
        tsync();
      }
      if (active && j < N2) {
#pragma unroll
        for (int a = 0; a < N1; ++a) {
          C<R> kxx, kyy, kzz, kxy, kxz, kyz;
          if constexpr (SPLIT3) {
            const bool hi = 2 * a >= N1;                       // q3 >= P/2
            const int f3 = hi ? P - N2 * a - j : N2 * a + j;
            kxx = ke[f3];
            kyy = ke[H + f3];
            kzz = ke[2 * H + f3];
            kxy = kol[f3];
            kxz = kol[H + f3];
            kyz = kol[2 * H + f3];
            if (!SIGNED) {
              kxy = cscale(kxy, sxy);
              kxz = cscale(kxz, sx);
              kyz = cscale(kyz, sy);
            }
            if (hi) {
              kxz = cmk<R>(-kxz.re, -kxz.im);
              kyz = cmk<R>(-kyz.re, -kyz.im);
            }
          } else {
            const int q3 = j + N2 * a;
            const bool fl3 = 2 * q3 > P;
            const int f3 = fl3 ? P - q3 : q3;
            const R s3 = fl3 ? (R)-1 : (R)1;
            kxx = ke[f3];
            kyy = ke[H + f3];
            kzz = ke[2 * H + f3];
            kxy = cscale(ko[f3], sxy);
            kxz = cscale(ko[H + f3], sx * s3);
            kyz = cscale(ko[2 * H + f3], sy * s3);
          }
          // one multiply and five fused multiply-adds per real part
          const C<R> ux = u[0][a], uy = u[1][a], uz = u[2][a];
          u[0][a] = cfma(kxz, uz, cfma(kxy, uy, kxx * ux));
          u[1][a] = cfma(kyz, uz, cfma(kyy, uy, kxy * ux));
          u[2][a] = cfma(kzz, uz, cfma(kyz, uy, kxz * ux));
          if ((a & 3) == 3) asm volatile("" ::: "memory");   // bound the LDS prefetch depth
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // inverse step 1': thread q2 = j < N2 transforms its N1 values
        if (active && j < N2) {
          Dft<N1, 1, R>::run(u[c]);
#pragma unroll
          for (int t2 = 0; t2 < N1; ++t2)
            myex[j * (N1 + 1) + t2] = (t2 == 0) ? u[c][t2] : u[c][t2] * cconj(twl[j * t2]);
        }
        tsync();
        // inverse step 3': thread t2 = j < N1 produces t = j + N1 t1
        if (active && j < N1) {
          C<R> v[N2];
#pragma unroll
          for (int q = 0; q < N2; ++q) v[q] = myex[q * (N1 + 1) + j];
          Dft<N2, 1, R>::run(v);
#pragma unroll
          for (int t1 = 0; t1 < (N2 + 1) / 2; ++t1) {
            const int tt = j + N1 * t1;
            if (tt < n) st_stream(base + c * plane + tt, v[t1]);
          }
        }
        tsync();
      }
    }
  };
  if constexpr (PERSIST) {
    for (int oline = blockIdx.x; oline < H * H; oline += gridDim.x) {
      if (oline != blockIdx.x) __syncthreads();   // the previous line's LDS reads are done
      item(oline, threadIdx.x);
    }
  } else {
    item(blockIdx.x, threadIdx.x);
  }
}

// ---- pass 3 with two lanes per transform column (FP64, P = 256 = 16 x 16) ----
// The same transform as kmul_kernel, with each length-16 DFT of the four-step
// split between two adjacent lanes by one radix-2 step, so a lane holds 8
// values per component instead of 16 (96 instead of 192 VGPRs in FP64) and
// the kernel fits two waves per SIMD instead of one:
//   forward step 1 (column j, 8 nonzero inputs k < 8 since n <= P/2):
//     V[j][2q'+h] = DFT8_k(x_k W16^{kh})[q']               (no lane exchange)
//   forward step 3 (row q):
//     X[q + 16(2s'+h)] = DFT8_j'((V[j'] + (-1)^h V[j'+8]) W16^{j'h})[s']
//   inverse step 1' (row q, lane h holds s = 2s'+h):
//     E / O = IDFT8 of the even / odd s, y[t'+8m] = E[t'] + (-1)^m W16^{-t'} O[t'];
//     the pair swaps its 8 values once (DPP) and lane h keeps t2 = t' + 8h
//   inverse step 3' (column t2, outputs t1 = 2t1'+h < 8):
//     DFT8^-1_q'((Y[q'] + (-1)^h Y[q'+8]) W16^{-q'h})[t1']
// A job (one line) is 32 lanes, a team (the four mirrored lines) two
// wavefronts; exchanges stay inside a job's half wavefront.  In FP32 the
// extra radix-2 work outweighs the occupancy (both fit two waves), so the
// FP32 path keeps kmul_kernel.
__device__ __forceinline__ int dpp_pair(int x) {
  // quad_perm [1, 0, 3, 2]: the adjacent lane's value
  return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ float pair_swap(float x) { return __int_as_float(dpp_pair(__float_as_int(x))); }
__device__ __forceinline__ double pair_swap(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_pair((int)(b & 0xffffffffLL)), hi = dpp_pair((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename R, int W, bool PERSIST = false>
__global__ __launch_bounds__(W * 128) void kmul2_kernel(C<R>* __restrict__ X, const C<R>* __restrict__ Kh,
                                                         const C<R>* __restrict__ tw, int n, int B) {
  constexpr int P = 256, N = 16, H = P / 2 + 1;
  constexpr int EXS = N * (N + 1);            // padded exchange of one job
  __shared__ C<R> kl[6 * H];
  __shared__ C<R> twl[P];
  __shared__ C<R> ex[W * 4 * EXS];
  // a PERSIST launch (gridDim.x < H^2) takes octant lines grid-stride
  auto item = [&](int oline, int tid) {
    const int f1 = oline / H;
    const int f2 = oline % H;
    const int team = tid / 128;
    const int lt = tid % 128;
    const int job = lt / 32;
    const int col = (lt % 32) >> 1;             // column / row index of the current step
    const int h = lt & 1;                       // which half of the radix-2 split
    const int s1 = job & 1, s2 = job >> 1;
    const bool edge1 = (f1 == 0) || (2 * f1 == P);
    const bool edge2 = (f2 == 0) || (2 * f2 == P);
    const bool active = !((s1 && edge1) || (s2 && edge2));
    const int q1 = s1 ? P - f1 : f1;
    const int q2 = s2 ? P - f2 : f2;
    const long plane = (long)P * P * n;
    const long lineoff = ((long)q1 * P + q2) * n;

    const C<R>* kg = Kh + ((long)f1 * H + f2) * 6 * H;
    for (int e = tid; e < 6 * H; e += W * 128) kl[e] = kg[e];
    for (int e = tid; e < P; e += W * 128) twl[e] = tw[e];
    const R sxy = (s1 != s2) ? (R)-1 : (R)1;
    const R sx = s1 ? (R)-1 : (R)1;
    const R sy = s2 ? (R)-1 : (R)1;
    const R sg = h ? (R)-1 : (R)1;              // (-1)^h
    __syncthreads();

    C<R>* myex = ex + (team * 4 + job) * EXS;
    // z W16^{k h} (forward) and z W16^{-k h} (inverse): multiply by the
    // compile-time constant, then select, so no per-lane twiddle registers
    auto hf = [&](C<R> z, int k) { const C<R> w = z * ctw<R, 16, -1>(k); return h ? w : z; };
    auto hi = [&](C<R> z, int k) { const C<R> w = z * ctw<R, 16, 1>(k); return h ? w : z; };

    for (int b = team; b < B; b += W) {
      C<R>* base = X + (long)b * 3 * plane + lineoff;
      C<R> u[3][8];                             // frequencies col + 16 h + 32 s'
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (active) {
          C<R> v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int tt = col + N * k;
            const C<R> x = (tt < n) ? ld_stream(base + c * plane + tt) : cmk<R>(0, 0);
            v[k] = (k == 0) ? x : hf(x, k);
          }
          Dft<8, -1, R>::run(v);
#pragma unroll
          for (int qq = 0; qq < 8; ++qq) {
            const int q = 2 * qq + h;
            myex[q * (N + 1) + col] = (col * q == 0) ? v[qq] : v[qq] * twl[col * q];
          }
        }
        wave_lds_sync();
        if (active) {
          C<R> y[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const C<R> a = myex[col * (N + 1) + j], bb = myex[col * (N + 1) + j + 8];
            const C<R> d = cmk(a.re + sg * bb.re, a.im + sg * bb.im);
            y[j] = (j == 0) ? d : hf(d, j);
          }
          Dft<8, -1, R>::run(y);
#pragma unroll
          for (int ss = 0; ss < 8; ++ss) u[c][ss] = y[ss];
        }
        wave_lds_sync();
      }
      if (active) {
#pragma unroll
        for (int ss = 0; ss < 8; ++ss) {
          const int q3 = col + N * h + 2 * N * ss;
          const bool fl3 = 2 * q3 > P;
          const int f3 = fl3 ? P - q3 : q3;
          const R s3 = fl3 ? (R)-1 : (R)1;
          const C<R> kxx = kl[0 * H + f3], kyy = kl[1 * H + f3], kzz = kl[2 * H + f3];
          const C<R> kxy = cscale(kl[3 * H + f3], sxy);
          const C<R> kxz = cscale(kl[4 * H + f3], sx * s3);
          const C<R> kyz = cscale(kl[5 * H + f3], sy * s3);
          const C<R> ux = u[0][ss], uy = u[1][ss], uz = u[2][ss];
          u[0][ss] = kxx * ux + kxy * uy + kxz * uz;
          u[1][ss] = kxy * ux + kyy * uy + kyz * uz;
          u[2][ss] = kxz * ux + kyz * uy + kzz * uz;
          if ((ss & 3) == 3) asm volatile("" ::: "memory");   // bound the LDS prefetch depth
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (active) {
          C<R> z[8];
#pragma unroll
          for (int ss = 0; ss < 8; ++ss) z[ss] = u[c][ss];
          Dft<8, 1, R>::run(z);
#pragma unroll
          for (int t = 1; t < 8; ++t) z[t] = hi(z[t], t);
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const C<R> pz = cmk(pair_swap(z[t].re), pair_swap(z[t].im));
            const C<R> e = h ? pz : z[t], o = h ? z[t] : pz;
            const C<R> y = cmk(e.re + sg * o.re, e.im + sg * o.im);
            const int t2 = t + 8 * h;
            myex[col * (N + 1) + t2] = (col * t2 == 0) ? y : y * cconj(twl[col * t2]);
          }
        }
        wave_lds_sync();
        if (active) {
          C<R> v[8];
#pragma unroll
          for (int qq = 0; qq < 8; ++qq) {
            const C<R> a = myex[qq * (N + 1) + col], bb = myex[(qq + 8) * (N + 1) + col];
            const C<R> d = cmk(a.re + sg * bb.re, a.im + sg * bb.im);
            v[qq] = (qq == 0) ? d : hi(d, qq);
          }
          Dft<8, 1, R>::run(v);
#pragma unroll
          for (int t1 = 0; t1 < 4; ++t1) {
            const int tt = col + N * (2 * t1 + h);
            if (tt < n) st_stream(base + c * plane + tt, v[t1]);
          }
        }
        wave_lds_sync();
      }
    }
  };
  if constexpr (PERSIST) {
    for (int oline = blockIdx.x; oline < H * H; oline += gridDim.x) {
      if (oline != blockIdx.x) __syncthreads();   // the previous line's LDS reads are done
      item(oline, threadIdx.x);
    }
  } else {
    item(blockIdx.x, threadIdx.x);
  }
}

// ---- plain row FFT along the contiguous dimension (plan set-up only) --------
// X: nlines lines of length P, transformed in place (forward).
template <typename R, int P, int N1, int N2>
__global__ __launch_bounds__(4 * cmax(N1, N2)) void rowfft_kernel(C<R>* __restrict__ X,
                                                                  const C<R>* __restrict__ tw,
                                                                  long nlines) {
  constexpr int TPL = cmax(N1, N2);
  constexpr int EXS = N1 * N2 + N2;
  __shared__ C<R> ex[4 * EXS];
  const int job = threadIdx.x / TPL;
  const int j = threadIdx.x % TPL;
  const long line = (long)blockIdx.x * 4 + job;
  const bool live = line < nlines;
  C<R>* base = X + line * P;
  C<R>* myex = ex + job * EXS;
  if (live && j < N1) {
    C<R> v[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) v[k] = base[j + N1 * k];
    Dft<N2, -1, R>::run(v);
#pragma unroll
    for (int q = 0; q < N2; ++q) myex[q * (N1 + 1) + j] = (j * q == 0) ? v[q] : v[q] * tw[j * q];
  }
  __syncthreads();
  if (live && j < N2) {
    C<R> w[N1];
#pragma unroll
    for (int jj = 0; jj < N1; ++jj) w[jj] = myex[j * (N1 + 1) + jj];
    Dft<N1, -1, R>::run(w);
#pragma unroll
    for (int a = 0; a < N1; ++a) base[j + N2 * a] = w[a];
  }
}

// w_b = sum_d p^d x_{b,d}  ([B][n^3], the fourth transformed field)
template <typename R, typename IO>
__global__ void pdot_kernel(const C<IO>* __restrict__ x, const C<R>* __restrict__ p, C<R>* __restrict__ w, long n3,
                            int B) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n3 * B) return;
  const long b = id / n3, e = id % n3;
  const C<IO>* xb = x + b * 3 * n3;
  w[id] = p[e] * ccast<R>(xb[e]) + p[n3 + e] * ccast<R>(xb[n3 + e]) + p[2 * n3 + e] * ccast<R>(xb[2 * n3 + e]);
}

// Pass 3 of the paper's form: along dim 3 for each (q1, q2) line, the forward
// transform of the four fields (m x_1, m x_2, m x_3 at fields 3b + c, p.x at
// field 3B + b), v_c = k^2 Ghat u_c + G^c hat w, and the inverse transform of
// the three v_c into fields 3b + c.  k^2 G is even in every coordinate, G^d
// odd in coordinate d: a mirrored line flips the sign of G^1 (q1), G^2 (q2),
// and a frequency past P/2 that of G^3.  One team of four jobs per workgroup.
template <typename R, int P, int N1, int N2>
__global__ __launch_bounds__(4 * cmax(N1, N2)) void kmul34_kernel(C<R>* __restrict__ X,
                                                                  const C<R>* __restrict__ Kp,
                                                                  const C<R>* __restrict__ tw, int n, int B) {
  constexpr int H = P / 2 + 1;
  constexpr int TPL = cmax(N1, N2);
  constexpr int EXS = N1 * N2 + N2;
  __shared__ C<R> kl[4 * H];
  __shared__ C<R> twl[P];
  __shared__ C<R> ex[4 * EXS];
  const int f1 = blockIdx.x / H;
  const int f2 = blockIdx.x % H;
  const int tid = threadIdx.x;
  const int job = tid / TPL;
  const int j = tid % TPL;
  const int s1 = job & 1, s2 = job >> 1;
  const bool edge1 = (f1 == 0) || (2 * f1 == P);
  const bool edge2 = (f2 == 0) || (2 * f2 == P);
  const bool active = !((s1 && edge1) || (s2 && edge2));
  const int q1 = s1 ? P - f1 : f1;
  const int q2 = s2 ? P - f2 : f2;
  const long plane = (long)P * P * n;
  const long lineoff = ((long)q1 * P + q2) * n;
  const C<R>* kg = Kp + ((long)f1 * H + f2) * 4 * H;
  for (int e = tid; e < 4 * H; e += blockDim.x) kl[e] = kg[e];
  for (int e = tid; e < P; e += blockDim.x) twl[e] = tw[e];
  const R sx = s1 ? (R)-1 : (R)1;
  const R sy = s2 ? (R)-1 : (R)1;
  __syncthreads();
  C<R>* myex = ex + job * EXS;
  constexpr int KIN = (N2 + 1) / 2;
  for (int b = 0; b < B; ++b) {
    C<R>* base[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) base[c] = X + ((long)b * 3 + c) * plane + lineoff;
    base[3] = X + ((long)B * 3 + b) * plane + lineoff;
    C<R> u[4][N1];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (active && j < N1) {
        C<R> v[N2];
#pragma unroll
        for (int k = 0; k < KIN; ++k) {
          const int tt = j + N1 * k;
          v[k] = (tt < n) ? base[c][tt] : cmk<R>(0, 0);
        }
        DftZ<N2, -1, R, KIN>::run(v);
#pragma unroll
        for (int q = 0; q < N2; ++q) myex[q * (N1 + 1) + j] = (j * q == 0) ? v[q] : v[q] * twl[j * q];
      }
      __syncthreads();
      if (active && j < N2) {
#pragma unroll
        for (int a = 0; a < N1; ++a) u[c][a] = myex[j * (N1 + 1) + a];
        Dft<N1, -1, R>::run(u[c]);
      }
      __syncthreads();
    }
    if (active && j < N2) {
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const int q3 = j + N2 * a;
        const bool fl3 = 2 * q3 > P;
        const int f3 = fl3 ? P - q3 : q3;
        const R s3 = fl3 ? (R)-1 : (R)1;
        const C<R> g0 = kl[f3];
        const C<R> g1 = cscale(kl[H + f3], sx), g2 = cscale(kl[2 * H + f3], sy), g3 = cscale(kl[3 * H + f3], s3);
        const C<R> w = u[3][a];
        u[0][a] = g0 * u[0][a] + g1 * w;
        u[1][a] = g0 * u[1][a] + g2 * w;
        u[2][a] = g0 * u[2][a] + g3 * w;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (active && j < N2) {
        Dft<N1, 1, R>::run(u[c]);
#pragma unroll
        for (int t2 = 0; t2 < N1; ++t2)
          myex[j * (N1 + 1) + t2] = (j * t2 == 0) ? u[c][t2] : u[c][t2] * cconj(twl[j * t2]);
      }
      __syncthreads();
      if (active && j < N1) {
        C<R> v[N2];
#pragma unroll
        for (int q = 0; q < N2; ++q) v[q] = myex[q * (N1 + 1) + j];
        Dft<N2, 1, R>::run(v);
#pragma unroll
        for (int t1 = 0; t1 < (N2 + 1) / 2; ++t1) {
          const int tt = j + N1 * t1;
          if (tt < n) base[c][tt] = v[t1];
        }
      }
      __syncthreads();
    }
  }
}

// ---- launch helpers -----------------------------------------------------------
// Workgroups of `kern` (with `threads` threads) that the current device holds at
// once: the grid of a persistent launch.  Occupancy is queried once per kernel
// and device and kept in a fixed table (no allocation, so that the apply that
// allocates nothing can use persistent launches too); a full table just
// queries again.
inline long resident_workgroups(const void* kern, int threads) {
  struct Slot {
    const void* kern;
    int dev;
    long value;
  };
  static constexpr int kSlots = 256;
  static Slot table[kSlots];
  static int used = 0;
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < used; ++i)
    if (table[i].kern == kern && table[i].dev == dev) return table[i].value;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const long r = (long)std::max(per_cu, 1) * std::max(cus, 1);
  if (used < kSlots) table[used++] = Slot{kern, dev, r};
  return r;
}

// HALF: rows are read and written in runs of half the default length (T / 2
// lines).  persist: a grid of the resident workgroups only (at least one work
// item each), which then stride over the work items.
template <typename R, typename IO, int P, int MODE, bool PAD = true, bool HALF = false>
static ls_status launch_col(const void* in, void* out, const void* aux, const C<R>* tw, int rows_in,
                            int rows_out, long L, long in_bs, long out_bs, long nbatch, R scale,
                            hipStream_t s, bool persist = false) {
  constexpr Fac f = col_factors(P);
  constexpr int T0 = col_tile<R>(P, MODE);
  constexpr int T = (HALF && T0 >= 16) ? T0 / 2 : T0;
  constexpr int threads = T * cmax(f.n1, f.n2);
  const auto kern = persist ? col_fft_kernel<R, IO, P, f.n1, f.n2, T, MODE, PAD, true>
                            : col_fft_kernel<R, IO, P, f.n1, f.n2, T, MODE, PAD, false>;
  const long ntiles = (L + T - 1) / T;
  const long blocks = nbatch * ntiles;
  if (blocks <= 0) return LS_OK;
  if (ntiles > 0x7fffffffL) return LS_EINVAL;
  long grid = blocks;
  if (persist) {
    const long r = resident_workgroups(reinterpret_cast<const void*>(kern), threads);
    if (r <= 0) return LS_EHIP;
    grid = std::min(grid, r);
  }
  if (grid > 0x7fffffffL) return LS_EINVAL;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), 0, s, in, out, reinterpret_cast<const C<R>*>(aux),
                     tw, rows_in, rows_out, L, in_bs, out_bs, (int)ntiles, blocks, scale);
  return hipGetLastError() == hipSuccess ? LS_OK : LS_EHIP;
}

// launch_col with the run length chosen at run time (half runs only where the
// default run holds at least 16 lines and P >= 64; elsewhere the default)
template <typename R, typename IO, int P, int MODE>
static ls_status launch_col_rt(bool half, bool persist, const void* in, void* out, const void* aux, const C<R>* tw,
                               int rows_in, int rows_out, long L, long in_bs, long out_bs, long nbatch, R scale,
                               hipStream_t s) {
  if constexpr (P >= 64 && col_tile<R>(P, MODE) >= 16) {
    if (half)
      return launch_col<R, IO, P, MODE, true, true>(in, out, aux, tw, rows_in, rows_out, L, in_bs, out_bs, nbatch,
                                                    scale, s, persist);
  }
  return launch_col<R, IO, P, MODE, true, false>(in, out, aux, tw, rows_in, rows_out, L, in_bs, out_bs, nbatch,
                                                 scale, s, persist);
}

template <typename R, int P, int W>
static ls_status launch_kmul_w(C<R>* X, const C<R>* Kh, const C<R>* tw, int n, int B, bool persist, hipStream_t s) {
  constexpr Fac f = row_factors<R>(P);
  constexpr int H = P / 2 + 1;
  constexpr int threads = W * 4 * job_lanes(cmax(f.n1, f.n2));
  const auto kern = persist ? kmul_kernel<R, P, f.n1, f.n2, W, true> : kmul_kernel<R, P, f.n1, f.n2, W, false>;
  long grid = (long)H * H;
  if (persist) {
    const long r = resident_workgroups(reinterpret_cast<const void*>(kern), threads);
    if (r <= 0) return LS_EHIP;
    grid = std::min(grid, r);
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), 0, s, X, Kh, tw, n, B);
  return hipGetLastError() == hipSuccess ? LS_OK : LS_EHIP;
}

// Teams per workgroup (wt; 0 = default 2).  Measured at 128^3 with 8
// right-hand sides: two teams (1.04 ms) beat one (1.07 ms), four (1.04 ms)
// and eight (1.30 ms): small workgroups let several workgroups per CU sit in
// different phases (loads, arithmetic, stores), which one large workgroup
// cannot.  The autotuner may pick another count per plan.
template <typename R, int P>
static ls_status launch_kmul(C<R>* X, const C<R>* Kh, const C<R>* tw, int n, int B, int wt, bool persist,
                            hipStream_t s) {
  constexpr Fac f = row_factors<R>(P);
  constexpr int TPL = cmax(f.n1, f.n2);
  if constexpr (P == 256 && sizeof(R) == 8) {
    // FP64: paired lanes; teams are two wavefronts, one or two per workgroup
    constexpr int H = P / 2 + 1;
    const bool two = wt >= 2 && B >= 2;
    const auto kern = two ? (persist ? kmul2_kernel<R, 2, true> : kmul2_kernel<R, 2, false>)
                          : (persist ? kmul2_kernel<R, 1, true> : kmul2_kernel<R, 1, false>);
    const int threads = two ? 256 : 128;
    long grid = (long)H * H;
    if (persist) {
      const long r = resident_workgroups(reinterpret_cast<const void*>(kern), threads);
      if (r <= 0) return LS_EHIP;
      grid = std::min(grid, r);
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), 0, s, X, Kh, tw, n, B);
    return hipGetLastError() == hipSuccess ? LS_OK : LS_EHIP;
  }
  if (wt <= 0) wt = 2;
  if constexpr (4 * TPL == 64) {
    if (wt >= 4 && B >= 4) return launch_kmul_w<R, P, 4>(X, Kh, tw, n, B, persist, s);
    if (wt >= 2 && B >= 2) return launch_kmul_w<R, P, 2>(X, Kh, tw, n, B, persist, s);
  } else if constexpr (job_lanes(TPL) == 32) {
    if (wt >= 2 && B >= 2) return launch_kmul_w<R, P, 2>(X, Kh, tw, n, B, persist, s);
  }
  return launch_kmul_w<R, P, 1>(X, Kh, tw, n, B, persist, s);
}

template <typename R, int P>
static ls_status launch_rowfft(C<R>* X, const C<R>* tw, long nlines, hipStream_t s) {
  constexpr Fac f = col_factors(P);
  const long blocks = (nlines + 3) / 4;
  hipLaunchKernelGGL((rowfft_kernel<R, P, f.n1, f.n2>), dim3((unsigned)blocks),
                     dim3(4 * cmax(f.n1, f.n2)), 0, s, X, tw, nlines);
  return hipGetLastError() == hipSuccess ? LS_OK : LS_EHIP;
}

// Full forward 3-D FFT of a P^3 FP64 array (plan set-up), scratch of P^3.
template <int P>
static ls_status fft3d_f64(C<double>* E, C<double>* scratch, const C<double>* tw, hipStream_t s) {
  const long P2 = (long)P * P;
  // dim 1: lines = P^2 (dims 2,3), rows = dim 1
  LS_TRY((launch_col<double, double, P, COL_FWD, false>(E, scratch, nullptr, tw, P, P, P2, 0, 0, 1, 1.0, s)));
  // dim 2: batch over dim 1, lines = P (dim 3)
  LS_TRY((launch_col<double, double, P, COL_FWD, false>(scratch, E, nullptr, tw, P, P, P, P2, P2, P, 1.0, s)));
  // dim 3: contiguous
  LS_TRY((launch_rowfft<double, P>(E, tw, P2, s)));
  return LS_OK;
}

template <typename R, typename IO, int P>
static ls_status run_passes(ApplyPlan& ap, const void* x, void* y, int nrhs, const C<R>* m,
                            const C<R>* kh, const C<R>* tw, bool minus_conv, const ApplyTune& tn, hipStream_t s,
                            hipEvent_t* ev, void* work) {
  const int n = ap.n;
  const long n2 = (long)n * n, n3 = n2 * n;
  C<R>* X1 = work ? static_cast<C<R>*>(work) : ap.work.as<C<R>>();   // [B][3][P][n^2]  (also Y1)
  C<R>* X2 = X1 + (long)nrhs * 3 * P * n2;                 // [B][3][P][P][n]
  const long nb = (long)nrhs * 3;
#define LS_MARK(i) \
  if (ev) LS_HIP(hipEventRecord(ev[i], s))
  LS_MARK(0);
  const bool pe = (tn.persist & 1) != 0, pe3 = (tn.persist & 2) != 0;
  // pass 1: along dim 1, lines = n^2
  LS_TRY((launch_col_rt<R, IO, P, COL_P1>(tn.half_runs & 1, pe, x, X1, m, tw, n, P, n2, n3, (long)P * n2, nb, (R)1,
                                          s)));
  LS_MARK(1);
  // pass 2: along dim 2, batch (b, c, q1), lines = n
  LS_TRY((launch_col_rt<R, R, P, COL_FWD>(tn.half_runs & 2, pe, X1, X2, nullptr, tw, n, P, n, n2, (long)P * n,
                                          nb * P, (R)1, s)));
  LS_MARK(2);
  // pass 3: along dim 3 with the 3x3 multiply
  LS_TRY((launch_kmul<R, P>(X2, kh, tw, n, nrhs, tn.kmul_w, pe3, s)));
  LS_MARK(3);
  // pass 4: inverse along dim 2
  LS_TRY((launch_col_rt<R, R, P, COL_INV>(tn.half_runs & 4, pe, X2, X1, nullptr, tw, P, n, n, (long)P * n, n2,
                                          nb * P, (R)1, s)));
  LS_MARK(4);
  // pass 5: inverse along dim 1, y = x + v
  if (minus_conv)   // y = -K*(m x)
    LS_TRY((launch_col_rt<R, IO, P, COL_P5>(tn.half_runs & 8, pe, X1, y, nullptr, tw, P, n, n2, (long)P * n2, n3,
                                            nb, (R)-1, s)));
  else
    LS_TRY((launch_col_rt<R, IO, P, COL_P5>(tn.half_runs & 8, pe, X1, y, x, tw, P, n, n2, (long)P * n2, n3, nb,
                                            (R)1, s)));
  LS_MARK(5);
#undef LS_MARK
  return LS_OK;
}

// The paper's form: passes 1 and 2 on the three fields m x_d and on p.x, the
// 3x4 multiply in pass 3, passes 4 and 5 on the three results as in the
// dyadic form.  work34: X1 [4B][P][n^2], X2 [4B][P][P][n], W [B][n^3].
template <typename R, typename IO, int P>
static ls_status run_passes34(ApplyPlan& ap, const void* x, void* y, int nrhs, const C<R>* m, const C<R>* p,
                              const C<R>* kp, const C<R>* tw, bool minus_conv, hipStream_t s, hipEvent_t* ev) {
  const int n = ap.n;
  const long n2 = (long)n * n, n3 = n2 * n;
  C<R>* X1 = ap.work34.as<C<R>>();
  C<R>* X2 = X1 + (long)nrhs * 4 * P * n2;
  C<R>* W = X2 + (long)nrhs * 4 * P * P * n;
  const long nb = (long)nrhs * 3;
#define LS_MARK(i) \
  if (ev) LS_HIP(hipEventRecord(ev[i], s))
  LS_MARK(0);
  hipLaunchKernelGGL((pdot_kernel<R, IO>), dim3((unsigned)((n3 * nrhs + 255) / 256)), dim3(256), 0, s,
                     static_cast<const C<IO>*>(x), p, W, n3, nrhs);
  LS_HIP(hipGetLastError());
  LS_TRY((launch_col<R, IO, P, COL_P1>(x, X1, m, tw, n, P, n2, n3, (long)P * n2, nb, (R)1, s)));
  LS_TRY((launch_col<R, R, P, COL_FWD>(W, X1 + nb * P * n2, nullptr, tw, n, P, n2, n3, (long)P * n2, nrhs, (R)1,
                                       s)));
  LS_MARK(1);
  LS_TRY((launch_col<R, R, P, COL_FWD>(X1, X2, nullptr, tw, n, P, n, n2, (long)P * n, 4L * nrhs * P, (R)1, s)));
  LS_MARK(2);
  {
    constexpr Fac f = row_factors<R>(P);
    constexpr int H = P / 2 + 1;
    hipLaunchKernelGGL((kmul34_kernel<R, P, f.n1, f.n2>), dim3(H * H), dim3(4 * cmax(f.n1, f.n2)), 0, s, X2, kp, tw,
                       n, nrhs);
    LS_HIP(hipGetLastError());
  }
  LS_MARK(3);
  LS_TRY((launch_col<R, R, P, COL_INV>(X2, X1, nullptr, tw, P, n, n, (long)P * n, n2, nb * P, (R)1, s)));
  LS_MARK(4);
  if (minus_conv)
    LS_TRY((launch_col<R, IO, P, COL_P5>(X1, y, nullptr, tw, P, n, n2, (long)P * n2, n3, nb, (R)-1, s)));
  else
    LS_TRY((launch_col<R, IO, P, COL_P5>(X1, y, x, tw, P, n, n2, (long)P * n2, n3, nb, (R)1, s)));
  LS_MARK(5);
#undef LS_MARK
  return LS_OK;
}

template <int P>
ls_status apply_dispatch(ApplyPlan& ap, const void* x, void* y, int nrhs, ls_prec prec,
                                bool minus_conv, hipStream_t s, hipEvent_t* ev, void* work) {
  const ApplyTune& tn = ap.tune[prec];
  if (ap.form == 1) {
    if (work) return LS_ESTATE;                 // the paper's form keeps its own workspace
    switch (prec) {
      case LS_C128:
        return run_passes34<double, double, P>(ap, x, y, nrhs, ap.m64.as<C<double>>(), ap.p64.as<C<double>>(),
                                               ap.kp64.as<C<double>>(), ap.tw64.as<C<double>>(), minus_conv, s, ev);
      case LS_C64:
        return run_passes34<float, float, P>(ap, x, y, nrhs, ap.m32.as<C<float>>(), ap.p32.as<C<float>>(),
                                             ap.kp32.as<C<float>>(), ap.tw32.as<C<float>>(), minus_conv, s, ev);
      case LS_MIXED:
        return run_passes34<float, double, P>(ap, x, y, nrhs, ap.m32.as<C<float>>(), ap.p32.as<C<float>>(),
                                              ap.kp32.as<C<float>>(), ap.tw32.as<C<float>>(), minus_conv, s, ev);
    }
    return LS_EINVAL;
  }
  switch (prec) {
    case LS_C128:
      return run_passes<double, double, P>(ap, x, y, nrhs, ap.m64.as<C<double>>(), ap.kh64.as<C<double>>(),
                                           ap.tw64.as<C<double>>(), minus_conv, tn, s, ev, work);
    case LS_C64:
      return run_passes<float, float, P>(ap, x, y, nrhs, ap.m32.as<C<float>>(), ap.kh32.as<C<float>>(),
                                         ap.tw32.as<C<float>>(), minus_conv, tn, s, ev, work);
    case LS_MIXED:
      return run_passes<float, double, P>(ap, x, y, nrhs, ap.m32.as<C<float>>(), ap.kh32.as<C<float>>(),
                                          ap.tw32.as<C<float>>(), minus_conv, tn, s, ev, work);
  }
  return LS_EINVAL;
}

// Instantiated for each supported P in the fft_inst_*.hip units.
#define LS_FOR_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384)
#define X(SZ) \
  extern template ls_status apply_dispatch<SZ>(ApplyPlan&, const void*, void*, int, ls_prec, bool, hipStream_t, \
                                               hipEvent_t*, void*);
LS_FOR_SIZES(X)
#undef X

}  // namespace ls
