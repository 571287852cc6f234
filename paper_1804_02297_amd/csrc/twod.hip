// The 2-D variant: the scattered-field equation on the n x n grid of the
// unit square with the 2-D Helmholtz kernel (Section 2 notes that the
// equation holds in 2-D with that kernel; Section 3.3 gives its costs and
// Section 4 its examples).  Two field components, the paper's own form:
//
//   y_d = x_d + k^2 G * (m x_d) + G^d * (p . x),   d = 1, 2,
//
// G(x) = (i/4) H_0^(1)(k|x|), G^d = dG/dx_d, weights h^2 G(x_i - x_j); the
// self weight of G is its integral over the disc of area h^2, that of G^d is
// 0; p^d = (central difference of m, zero off the grid) / (1 - m).
//
// Apply: three kernels over HBM, every FFT of length P (the padded length,
// P >= 2n - 1, even, 2^a 3^b) held in LDS.
//   pass A  rows:    u_f = (m x_1, m x_2, p.x) per row, zero-padded, FFT
//                    along i2; [rhs][3][n][P] in HBM;
//   pass B  columns: per workgroup one rhs and a few adjacent columns: FFT
//                    of the three fields along i1, the 2x3 symbol multiply
//                    in registers, two inverse FFTs, rows i1 < n kept;
//                    [rhs][2][n][P];
//   pass C  rows:    inverse FFT along i2, the first n kept, + x.
// The symbol (k^2 Ghat, Ghat^1, Ghat^2) / P^2 is stored on the quadrant
// [H][H][3], H = P/2 + 1: k^2 Ghat is even in both frequencies, Ghat^1 is
// odd in q1 and even in q2, Ghat^2 the reverse.  The paper's lengths
// (P = 256, 486, 972, 1944) have the passes compiled for them; forward
// transforms skip their zero upper half, inverse ones the unused half of
// their output.
#include "twod.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <stdexcept>
#include <vector>

#include "gpu_solver.h"
#include "host_solver.h"

namespace ls {

namespace {

constexpr int kT2 = 256;                 // threads per workgroup of the 2-D row and plan kernels
constexpr int kTB = 512;                 // threads per workgroup of the column pass (fewer registers each)
constexpr size_t kLds2 = 65536;          // LDS bytes a 2-D FFT workgroup may use
constexpr size_t kLdsTarget = 32768;     // LDS bytes aimed for (five workgroups per CU)

double wall_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---- FFT of runtime length P = 2^a 3^b in LDS (Stockham, radices 8, 4, 2, 9, 3) ----
// The radices are packed three bits per stage (0: 4, 1: 2, 2: 3, 3: 8, 4: 9),
// first stage lowest.  Large radices first: fewer stages, fewer barriers.
__host__ __device__ constexpr Radices factor_radices(int P) {
  Radices r{};
  int m = P, st = 0;
  const int rad[5] = {8, 4, 2, 9, 3};
  const unsigned codes[5] = {3, 0, 1, 4, 2};
  for (int q = 0; q < 5; ++q)
    while (m % rad[q] == 0) {
      r.code |= (unsigned long long)codes[q] << (3 * st);
      ++st;
      m /= rad[q];
    }
  r.nst = (m == 1 && st <= 21) ? st : -1;
  return r;
}

// The same stages in reverse order (an even radix last when P is even): the
// inverse transforms, whose last stage then stores only the lower half.
__host__ __device__ constexpr Radices reverse_radices(Radices r) {
  Radices o{};
  o.nst = r.nst;
  for (int st = 0; st < r.nst; ++st) {
    const unsigned long long c = (r.code >> (3 * st)) & 7ull;
    o.code |= c << (3 * (r.nst - 1 - st));
  }
  return o;
}

// Twiddles W^t = exp(-2 pi i t / P) from two short tables held in LDS:
// W^t = hi[t / 64] lo[t % 64] (one extra rounding against a full table).
constexpr int kTwLo = 64;
template <typename R>
struct Tw {
  const C<R>* lo;   // W^t, t < 64
  const C<R>* hi;   // W^(64 t), t < P / 64 + 1
  __device__ __forceinline__ C<R> operator()(int t) const { return hi[t >> 6] * lo[t & (kTwLo - 1)]; }
};
__host__ __device__ constexpr int tw_entries(int P) { return kTwLo + P / kTwLo + 1; }

// Fill the two twiddle tables (lo then hi) at t[0 .. tw_entries(P)) from the full table tw_g.
template <typename R>
__device__ Tw<R> load_twiddles(C<R>* t, const C<R>* __restrict__ tw_g, int P) {
  const int nhi = P / kTwLo + 1;
  for (int e = threadIdx.x; e < kTwLo + nhi; e += blockDim.x) {
    const long idx = e < kTwLo ? e : (long)(e - kTwLo) * kTwLo;
    t[e] = tw_g[idx % P];
  }
  return Tw<R>{t, t + kTwLo};
}

// One radix-RR butterfly of a Stockham stage.  FIRST: the first stage (all
// twiddles 1).  ZIN: inputs r >= RR/2 are zero (the first stage of a
// transform whose upper half is zero padding) and are not read.  HOUT: only
// outputs r < RR/2 are stored (the last stage of a transform of which only
// the lower half is used).
template <typename R, int DIR, int RR, bool FIRST, bool ZIN, bool HOUT>
__device__ __forceinline__ void stage_bfly(const C<R>* __restrict__ src, C<R>* __restrict__ dst, int j, int Ns,
                                           int NR, int tstep, int es, const Tw<R>& tw) {
  constexpr int NIN = ZIN ? RR / 2 : RR;
  constexpr int NOUT = HOUT ? RR / 2 : RR;
  const int k = FIRST ? 0 : j % Ns;
  C<R> v[RR];
#pragma unroll
  for (int r = 0; r < NIN; ++r) v[r] = src[(j + r * NR) * es];
  if (!FIRST) {
    // one table lookup per butterfly: W^(r k tstep) = (W^(k tstep))^r by recurrence
    C<R> w1 = tw(k * tstep);
    if (DIR > 0) w1 = cconj(w1);
    C<R> w = w1;
#pragma unroll
    for (int r = 1; r < NIN; ++r) {
      v[r] = v[r] * w;
      if (r + 1 < NIN) w = w * w1;
    }
  }
  DftZ<RR, DIR, R, NIN>::run(v);
  const int d0 = (j - k) * RR + k;
#pragma unroll
  for (int r = 0; r < NOUT; ++r) dst[(d0 + r * Ns) * es] = v[r];
}

template <typename R, int DIR, int RR, bool ZIN, bool HOUT>
__device__ __forceinline__ void stage_pick(const C<R>* s, C<R>* d, int j, int Ns, int NR, int tstep, int es,
                                           const Tw<R>& tw, bool first, bool last) {
  // pruning applies to even radices only (the first radix of a forward order, the last of a reversed one)
  constexpr bool EV = RR % 2 == 0;
  if (first) {
    if (ZIN && EV) stage_bfly<R, DIR, RR, true, EV && ZIN, false>(s, d, j, Ns, NR, tstep, es, tw);
    else if (last && HOUT && EV) stage_bfly<R, DIR, RR, true, false, EV && HOUT>(s, d, j, Ns, NR, tstep, es, tw);
    else stage_bfly<R, DIR, RR, true, false, false>(s, d, j, Ns, NR, tstep, es, tw);
  } else if (last && HOUT && EV) {
    stage_bfly<R, DIR, RR, false, false, EV && HOUT>(s, d, j, Ns, NR, tstep, es, tw);
  } else {
    stage_bfly<R, DIR, RR, false, false, false>(s, d, j, Ns, NR, tstep, es, tw);
  }
}

// nb transforms of length P held in LDS: element e of transform t at
// a[t * bs + e * es].  b is scratch of the same extent.  BFAST: consecutive
// threads take consecutive transforms (columns), else consecutive elements.
// ZIN: the upper half of every input is zero (never read).  HOUT: only the
// lower half of every output is used (the upper half is left unspecified).
// Returns the buffer that holds the result.  Ends with a barrier.
template <typename R, int DIR, bool BFAST, bool ZIN = false, bool HOUT = false, int NT = kT2>
__device__ __forceinline__ C<R>* lds_fft(C<R>* a, C<R>* b, int P, Radices rd, int nb, int es, int bs,
                                         const Tw<R>& tw) {
  int Ns = 1;
#pragma unroll
  for (int st = 0; st < rd.nst; ++st) {
    const unsigned code = (unsigned)(rd.code >> (3 * st)) & 7u;
    const int RR = code == 0 ? 4 : (code == 1 ? 2 : (code == 2 ? 3 : (code == 3 ? 8 : 9)));
    const int NR = P / RR;
    const int tstep = P / (RR * Ns);
    const int total = nb * NR;
    const bool first = st == 0, last = st + 1 == rd.nst;
    for (int w = threadIdx.x; w < total; w += NT) {
      const int t = BFAST ? w % nb : w / NR;
      const int j = BFAST ? w / nb : w % NR;
      const C<R>* s = a + t * bs;
      C<R>* d = b + t * bs;
      switch (code) {
        case 0: stage_pick<R, DIR, 4, ZIN, HOUT>(s, d, j, Ns, NR, tstep, es, tw, first, last); break;
        case 1: stage_pick<R, DIR, 2, ZIN, HOUT>(s, d, j, Ns, NR, tstep, es, tw, first, last); break;
        case 2: stage_pick<R, DIR, 3, ZIN, HOUT>(s, d, j, Ns, NR, tstep, es, tw, first, last); break;
        case 3: stage_pick<R, DIR, 8, ZIN, HOUT>(s, d, j, Ns, NR, tstep, es, tw, first, last); break;
        default: stage_pick<R, DIR, 9, ZIN, HOUT>(s, d, j, Ns, NR, tstep, es, tw, first, last); break;
      }
    }
    __syncthreads();
    C<R>* t = a;
    a = b;
    b = t;
    Ns *= RR;
  }
  return a;
}

// The same transforms for a compile-time length P (the paper's lengths): the
// stages are unrolled at compile time, so each stage's radix, span and
// twiddle step are constants and the index arithmetic has no runtime
// division and no switch over the radix.  REV: the reversed stage order.
template <int P, bool REV>
struct CtStages {
  static constexpr Radices rd = REV ? reverse_radices(factor_radices(P)) : factor_radices(P);
  static constexpr int nst = rd.nst;
  static constexpr int radix(int st) {
    const unsigned c = (unsigned)(rd.code >> (3 * st)) & 7u;
    return c == 0 ? 4 : (c == 1 ? 2 : (c == 2 ? 3 : (c == 3 ? 8 : 9)));
  }
  static constexpr int span(int st) {   // product of the radices of the stages before st
    int v = 1;
    for (int q = 0; q < st; ++q) v *= radix(q);
    return v;
  }
};

template <typename R, int DIR, bool BFAST, bool ZIN, bool HOUT, int NT, int P, bool REV>
__device__ __forceinline__ C<R>* lds_fft_ct(C<R>* a, C<R>* b, int nb, int es, int bs, const Tw<R>& tw) {
  using S = CtStages<P, REV>;
  static_assert(S::nst > 1, "a compile-time length has at least two stages");
  static_for<0, S::nst>([&](auto sc) {
    constexpr int st = decltype(sc)::value;
    constexpr int RR = S::radix(st);
    constexpr int Ns = S::span(st);
    constexpr int NR = P / RR;
    constexpr int tstep = P / (RR * Ns);
    constexpr bool EV = RR % 2 == 0;
    constexpr bool first = st == 0, last = st + 1 == S::nst;
    const int total = nb * NR;
    for (int w = threadIdx.x; w < total; w += NT) {
      const int t = BFAST ? w % nb : w / NR;
      const int j = BFAST ? w / nb : w % NR;
      stage_bfly<R, DIR, RR, first, first && ZIN && EV, last && HOUT && EV>(a + t * bs, b + t * bs, j, Ns, NR,
                                                                              tstep, es, tw);
    }
    __syncthreads();
    C<R>* tmp = a;
    a = b;
    b = tmp;
  });
  return a;
}

// Work index of a block: consecutive indices stay on one XCD (blocks are
// dispatched round-robin over the 8 XCDs), so blocks that share rows or
// symbol lines share that XCD's L2.
__device__ __forceinline__ int xcd_work_index(int bid, int nblk) {
  const int xcd = bid & 7, slot = bid >> 3;
  const int q = nblk >> 3, r = nblk & 7;
  return xcd * q + min(xcd, r) + slot;
}

// ---- weights and symbol (FP64, once per plan) ----
__device__ void weights_at(int r1, int r2, double k, double h, C<double>* w) {
  if (r1 == 0 && r2 == 0) {
    const double a = h * 0.56418958354775628694807945156;   // h / sqrt(pi)
    const double c = 1.5707963267948966192313216916398 * a / k;
    // k^2 [(i pi a / (2k)) H_1(k a) - 1/k^2]
    w[0] = cmk<double>((-c * y1(k * a) - 1.0 / (k * k)) * k * k, c * j1(k * a) * k * k);
    w[1] = cmk<double>(0.0, 0.0);
    w[2] = cmk<double>(0.0, 0.0);
    return;
  }
  const double x1 = h * r1, x2 = h * r2;
  const double R = sqrt(x1 * x1 + x2 * x2);
  const double z = k * R, h2 = h * h;
  // k^2 h^2 (i/4)(J0 + i Y0);  h^2 dG/dR x_d / R with dG/dR = (k/4)(Y1 - i J1)
  w[0] = cmk<double>(-0.25 * y0(z) * h2 * k * k, 0.25 * j0(z) * h2 * k * k);
  const double g1r = 0.25 * k * y1(z) * h2 / R, g1i = -0.25 * k * j1(z) * h2 / R;
  w[1] = cmk<double>(g1r * x1, g1i * x1);
  w[2] = cmk<double>(g1r * x2, g1i * x2);
}

// emb[c][s1][s2]: circulant embedding of (k^2 G, G^1, G^2) weights, offset r = s mod P.
__global__ void embed_kernel(C<double>* __restrict__ emb, int n, int P, double k, double h) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)P * P) return;
  const int s1 = (int)(idx / P), s2 = (int)(idx % P);
  const int r1 = s1 <= n - 1 ? s1 : (s1 >= P - (n - 1) ? s1 - P : P);
  const int r2 = s2 <= n - 1 ? s2 : (s2 >= P - (n - 1) ? s2 - P : P);
  C<double> w[3] = {cmk(0.0, 0.0), cmk(0.0, 0.0), cmk(0.0, 0.0)};
  if (r1 != P && r2 != P) weights_at(r1, r2, k, h, w);
  const long PP = (long)P * P;
  for (int c = 0; c < 3; ++c) emb[c * PP + idx] = w[c];
}

// In-place FFT of `rows` contiguous rows of length P, nb rows per block.
template <typename R, int DIR>
__global__ __launch_bounds__(kT2) void fft_rows_kernel(C<R>* __restrict__ data, int rows, int P, Radices rd, int nb,
                                                       const C<R>* __restrict__ tw) {
  extern __shared__ unsigned char lds_raw[];
  C<R>* a = reinterpret_cast<C<R>*>(lds_raw);
  C<R>* b = a + (size_t)nb * P;
  const Tw<R> tws = load_twiddles(b + (size_t)nb * P, tw, P);
  const long r0 = (long)blockIdx.x * nb;
  for (int e = threadIdx.x; e < nb * P; e += blockDim.x) {
    const long r = r0 + e / P;
    a[e] = r < rows ? data[r * P + e % P] : cmk<R>(0, 0);
  }
  __syncthreads();
  C<R>* x = lds_fft<R, DIR, false>(a, b, P, rd, nb, 1, P, tws);
  for (int e = threadIdx.x; e < nb * P; e += blockDim.x) {
    const long r = r0 + e / P;
    if (r < rows) data[r * P + e % P] = x[e];
  }
}

// In-place FFT along the first index of planes [planes][P][P], nb columns per block.
template <typename R, int DIR>
__global__ __launch_bounds__(kT2) void fft_cols_kernel(C<R>* __restrict__ data, int P, Radices rd, int nb,
                                                       const C<R>* __restrict__ tw) {
  extern __shared__ unsigned char lds_raw[];
  C<R>* a = reinterpret_cast<C<R>*>(lds_raw);
  C<R>* b = a + (size_t)nb * P;
  const Tw<R> tws = load_twiddles(b + (size_t)nb * P, tw, P);
  const int ncb = P / nb;
  const int plane = blockIdx.x / ncb, q0 = (blockIdx.x % ncb) * nb;
  C<R>* base = data + (size_t)plane * P * P + q0;
  for (int e = threadIdx.x; e < nb * P; e += blockDim.x) a[e] = base[(size_t)(e / nb) * P + e % nb];
  __syncthreads();
  C<R>* x = lds_fft<R, DIR, true>(a, b, P, rd, nb, nb, 1, tws);
  for (int e = threadIdx.x; e < nb * P; e += blockDim.x) base[(size_t)(e / nb) * P + e % nb] = x[e];
}

// Quadrant of the transformed embedding / P^2: sym[a1][a2][c].
// The quadrant twice: [a1][a2][3] (the register column pass) and column-major
// [3][a2][a1] (the LDS column pass, whose workgroups walk one column's a1).
__global__ void quadrant_kernel(const C<double>* __restrict__ emb, C<double>* __restrict__ s64,
                                C<float>* __restrict__ s32, C<double>* __restrict__ c64,
                                C<float>* __restrict__ c32, int P, int H) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)H * H) return;
  const int a1 = (int)(idx / H), a2 = (int)(idx % H);
  const double sc = 1.0 / ((double)P * P);
  for (int c = 0; c < 3; ++c) {
    const C<double> v = cscale(emb[(size_t)c * P * P + (size_t)a1 * P + a2], sc);
    s64[idx * 3 + c] = v;
    s32[idx * 3 + c] = ccast<float>(v);
    const size_t t = ((size_t)c * H + a2) * H + a1;
    c64[t] = v;
    c32[t] = ccast<float>(v);
  }
}

// p^d = (central difference of m over 2h, m = 0 off the grid) / (1 - m), [2][n][n].
__global__ void gradient_kernel(const C<double>* __restrict__ m, C<double>* __restrict__ p64,
                                C<float>* __restrict__ p32, C<float>* __restrict__ m32, int n, double h) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nn = (long)n * n;
  if (idx >= nn) return;
  const int i1 = (int)(idx / n), i2 = (int)(idx % n);
  const C<double> z = cmk(0.0, 0.0);
  const C<double> e1 = i1 + 1 < n ? m[idx + n] : z, w1 = i1 > 0 ? m[idx - n] : z;
  const C<double> e2 = i2 + 1 < n ? m[idx + 1] : z, w2 = i2 > 0 ? m[idx - 1] : z;
  const C<double> one_m = cmk(1.0 - m[idx].re, -m[idx].im);
  // 1 / (1 - m)
  const double den = one_m.re * one_m.re + one_m.im * one_m.im;
  const C<double> inv = cmk(one_m.re / den, -one_m.im / den);
  const double s = 0.5 / h;
  const C<double> p1 = cscale(e1 - w1, s) * inv, p2 = cscale(e2 - w2, s) * inv;
  p64[idx] = p1;
  p64[nn + idx] = p2;
  p32[idx] = ccast<float>(p1);
  p32[nn + idx] = ccast<float>(p2);
  m32[idx] = ccast<float>(m[idx]);
}

// ---- the apply ----
template <typename T>
__device__ __forceinline__ C<T> ld_c(const void* p, long i) { return reinterpret_cast<const C<T>*>(p)[i]; }

// pass A: block w -> (rhs b, row block rb); the three fields of its rows in
// turn, from x, m and p loaded once into registers.
template <typename R, typename IO, int PT, int NBT>
__global__ __launch_bounds__(kT2) void pass_a_kernel(const void* __restrict__ x, const C<R>* __restrict__ m,
                                                      const C<R>* __restrict__ p, C<R>* __restrict__ T, int n, int P_,
                                                      Radices rd_, int nb_, int nrb, int nwork,
                                                      const C<R>* __restrict__ tw) {
  // PT, NBT > 0: the length and batch fixed at compile time (constant divisions, unrolled stages)
  const int P = PT > 0 ? PT : P_, nb = NBT > 0 ? NBT : nb_;
  const Radices rd = PT > 0 ? factor_radices(PT) : rd_;
  extern __shared__ unsigned char lds_raw[];
  C<R>* a = reinterpret_cast<C<R>*>(lds_raw);
  C<R>* bb = a + (size_t)nb * P;
  const Tw<R> tws = load_twiddles(bb + (size_t)nb * P, tw, P);
  const int w = xcd_work_index(blockIdx.x, nwork);
  const int rb = w % nrb, b = w / nrb;
  const long nn = (long)n * n;
  const long xb = (long)b * 2 * nn;
  // only the lower half of each row is read by the pruned first stage (n <= P/2);
  // nb P / 2 <= UA kT2: nb P is at most what two buffers of kLdsTarget hold, or
  // one row of the largest P when a single row exceeds that
  constexpr size_t kHalfMax = std::max<size_t>(kLdsTarget / (2 * sizeof(C<R>)), kMaxP2) / 2;
  constexpr int UA = (int)((kHalfMax + kT2 - 1) / kT2);
  const int Ph = P / 2;
  C<R> rx0[UA], rx1[UA], rm[UA], rp0[UA], rp1[UA];
#pragma unroll
  for (int u = 0; u < UA; ++u) {
    const int e = threadIdx.x + kT2 * u;
    const int t = e / Ph, j = e % Ph;
    const int i1 = rb * nb + t;
    const C<R> z = cmk<R>(0, 0);
    rx0[u] = rx1[u] = rm[u] = rp0[u] = rp1[u] = z;
    if (e < nb * Ph && i1 < n && j < n) {
      const long o = (long)i1 * n + j;
      rx0[u] = ccast<R>(ld_c<IO>(x, xb + o));
      rx1[u] = ccast<R>(ld_c<IO>(x, xb + nn + o));
      rm[u] = m[o];
      rp0[u] = p[o];
      rp1[u] = p[nn + o];
    }
  }
#pragma unroll 1
  for (int f = 0; f < 3; ++f) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const int e = threadIdx.x + kT2 * u;
      if (e < nb * Ph) {
        const C<R> v = f == 0 ? rm[u] * rx0[u] : (f == 1 ? rm[u] * rx1[u] : rp0[u] * rx0[u] + rp1[u] * rx1[u]);
        a[(e / Ph) * P + e % Ph] = v;
      }
    }
    __syncthreads();
    const C<R>* X;
    if constexpr (PT > 0) X = lds_fft_ct<R, -1, false, true, false, kT2, PT, false>(a, bb, nb, 1, P, tws);
    else X = lds_fft<R, -1, false, true, false>(a, bb, P, rd, nb, 1, P, tws);
    C<R>* out = T + ((size_t)(b * 3 + f) * n) * P;
    for (int e = threadIdx.x; e < nb * P; e += kT2) {
      const int i1 = rb * nb + e / P;
      if (i1 < n) out[(size_t)i1 * P + e % P] = X[e];
    }
    __syncthreads();   // X may be the buffer the next field is written to
  }
}

// pass B: block -> (rhs, block of nb adjacent columns), NTH threads.
// Registers capped for four waves per SIMD (two workgroups of 512 threads and
// 62 KiB LDS, or one of 1024 threads and 125 KiB, per CU).  symc: the
// symbol quadrant column-major ([3][a2][a1]), so the rows of a column block
// read whole lines of it.
template <typename R, int EMAX, int PT, int NBT, int NTH = kTB>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4, 8))) void pass_b_kernel(
    const C<R>* __restrict__ T, C<R>* __restrict__ T2, const C<R>* __restrict__ symc, int n, int P_, int H,
    Radices rd_, int nb_, int nrhs, const C<R>* __restrict__ tw) {
  const int P = PT > 0 ? PT : P_, nb = NBT > 0 ? NBT : nb_;
  const Radices rd = PT > 0 ? factor_radices(PT) : rd_;
  extern __shared__ unsigned char lds_raw[];
  C<R>* a = reinterpret_cast<C<R>*>(lds_raw);
  C<R>* bb = a + (size_t)nb * P;
  const Tw<R> tws = load_twiddles(bb + (size_t)nb * P, tw, P);
  const int ncb = P / nb;
  // block -> (rhs, column block), the rhs fastest: the blocks of one column
  // block (same symbol lines) and of its neighbours (same 128-byte lines of
  // the intermediate) run together on one XCD and share its L2
  const int w = xcd_work_index(blockIdx.x, ncb * nrhs);
  const int b = w % nrhs;
  const int q0 = (w / nrhs) * nb;
  const int tot = nb * P;
  // symbol at the element e of the column block: q1 = e / nb, q2 = q0 + e % nb, read
  // from the quadrant at use (the same columns' blocks of the other rhs read the
  // same lines beside it on the XCD)
  auto symv = [&](int e, int c) -> C<R> {
    const int q1 = e / nb, q2 = q0 + e % nb;
    const bool f1 = q1 > P / 2, f2 = q2 > P / 2;
    const int a1 = f1 ? P - q1 : q1, a2 = f2 ? P - q2 : q2;
    const C<R> v = symc[((size_t)c * H + a2) * H + a1];
    const bool neg = (c == 1 && f1) || (c == 2 && f2);
    return neg ? cmk<R>(-v.re, -v.im) : v;
  };
  C<R> o0[EMAX], o1[EMAX];
  // the next field's column is loaded into registers while the current one
  // is transformed (rows below P/2 only: the rest is never read)
  constexpr int UL = (EMAX + 1) / 2;
  C<R> pf[UL];
  auto fetch = [&](int f) {
    const C<R>* in = T + ((size_t)(b * 3 + f) * n) * P + q0;
#pragma unroll
    for (int u = 0; u < UL; ++u) {
      const int e = threadIdx.x + NTH * u;
      C<R> v = cmk<R>(0, 0);
      if (e < tot / 2 && e / nb < n) v = in[(size_t)(e / nb) * P + e % nb];
      pf[u] = v;
    }
  };
  // FP32: the symbol component a field is multiplied by is loaded before the
  // field's transform, so its latency is hidden behind the transform (FP64
  // has no registers to spare for it and loads at use)
  constexpr bool SPRE = sizeof(R) == 4;
  C<R> sv[SPRE ? EMAX : 1];
  auto load_sym = [&](int c) {
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int u = 0; u < EMAX; ++u) {
      const int e = tid + NTH * u;
      sv[u] = e < tot ? symv(e, c) : cmk<R>(0, 0);
    }
  };
  fetch(0);
  if constexpr (SPRE) load_sym(0);    // fields 0 and 1 take component 0
#pragma unroll 1
  for (int f = 0; f < 3; ++f) {
#pragma unroll
    for (int u = 0; u < UL; ++u) {
      const int e = threadIdx.x + NTH * u;
      if (e < tot / 2) a[e] = pf[u];
    }
    __syncthreads();
    if (f < 2) fetch(f + 1);
    if constexpr (SPRE)
      if (f == 2) load_sym(1);
    const C<R>* X;
    if constexpr (PT > 0) X = lds_fft_ct<R, -1, true, true, false, NTH, PT, false>(a, bb, nb, nb, 1, tws);
    else X = lds_fft<R, -1, true, true, false, NTH>(a, bb, P, rd, nb, nb, 1, tws);
    // the symbol addresses are formed per field from an opaque thread index
    // rather than kept across the loop (they would not fit beside the
    // accumulators without spilling)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int u = 0; u < EMAX; ++u) {
      const int e = tid + NTH * u;
      if (e < tot) {
        const C<R> v = X[e];
        C<R> s01;
        if constexpr (SPRE) s01 = sv[u];
        else s01 = symv(e, f == 2 ? 1 : 0);
        if (f == 0) {
          o0[u] = s01 * v;
        } else if (f == 1) {
          o1[u] = s01 * v;
        } else {
          o0[u] = cfma(s01, v, o0[u]);
          o1[u] = cfma(symv(e, 2), v, o1[u]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll 1
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int u = 0; u < EMAX; ++u) {
      const int e = threadIdx.x + NTH * u;
      if (e < tot) {   // two stores, not a select between the arrays (that puts them on the stack)
        if (d == 0) a[e] = o0[u];
        else a[e] = o1[u];
      }
    }
    __syncthreads();
    const C<R>* X;
    if constexpr (PT > 0) X = lds_fft_ct<R, 1, true, false, true, NTH, PT, true>(a, bb, nb, nb, 1, tws);
    else X = lds_fft<R, 1, true, false, true, NTH>(a, bb, P, reverse_radices(rd), nb, nb, 1, tws);
    C<R>* out = T2 + ((size_t)(b * 2 + d) * n) * P + q0;
    for (int e = threadIdx.x; e < tot; e += NTH) {
      const int i1 = e / nb;
      if (i1 < n) out[(size_t)i1 * P + e % nb] = X[e];
    }
    __syncthreads();
  }
}

// pass B held in registers (FP32 at the paper's lengths P = 972 and 486).
// Each column transform of length P = N1 N2 is a four-step FFT: N1 threads
// each take a length-N2 DFT of the rows t = j + N1 k (only rows below P/2
// hold data), a twiddle by W_P^{j q}, one LDS exchange, then N2 threads each
// take a length-N1 DFT; the inverse runs the same steps backwards.  A
// workgroup owns NB adjacent columns of one rhs (consecutive lanes take
// consecutive columns, so every row access is a run of NB values) and keeps
// one exchange buffer of NB P values in LDS, with the twiddle table.
// The two steps run on different waves: "row" waves (the length-N2 DFTs,
// HBM loads and stores) and "frequency" waves (the length-N1 DFTs and the
// symbol multiply), so each holds only its own values.  The fields are
// transformed in the order p.x, m x_1, m x_2: the spectrum of p.x is kept in
// LDS, and each of the other two is multiplied by the symbol together with
// it and inverse-transformed at once, so no output accumulator lives across
// the three forward transforms.
// Measured at 8 rhs: P = 972 (n = 479) 0.135 against 0.167 ms for the LDS
// kernel, P = 486 (n = 239) 0.030 against 0.042 ms.  At P = 1944 (36 x 54,
// four columns per workgroup, 229 VGPRs, 140 KB of LDS: one workgroup of
// seven waves per CU) it took 0.82 against 0.76 ms, so that length keeps the
// LDS kernel.
template <int P>
struct ColRegCfg {
  static constexpr int N1 = P == 972 ? 27 : (P == 486 ? 18 : 0);
  static constexpr int N2 = P / (N1 > 0 ? N1 : 1);
  static constexpr int NB = P == 972 ? 8 : 16;          // columns per workgroup
  static constexpr int RPW = 64 / NB;                   // DFT indices per wavefront
  static constexpr int RA = (N1 + RPW - 1) / RPW * RPW; // row-wave threads per column
  static constexpr int RB = (N2 + RPW - 1) / RPW * RPW; // frequency-wave threads per column
  static constexpr int THREADS = NB * (RA + RB);
  static constexpr int EXS = P + 8;                     // exchange stride of one column (complex)
};

template <int P>
__global__ __launch_bounds__(ColRegCfg<P>::THREADS) void pass_b_reg_kernel(
    const C<float>* __restrict__ T, C<float>* __restrict__ T2, const C<float>* __restrict__ sym, int n, int H,
    int nrhs, const C<float>* __restrict__ tw) {
  using Cfg = ColRegCfg<P>;
  constexpr int N1 = Cfg::N1, N2 = Cfg::N2, NB = Cfg::NB, EXS = Cfg::EXS, RA = Cfg::RA;
  constexpr int KIN = (P / 2 + N1 - 1) / N1;       // rows t = j + N1 k < P/2
  constexpr int KOUT = (P / 2 + N1 - 1) / N1;      // outputs t = j + N1 t1 < P/2
  __shared__ C<float> ex[NB * EXS];
  __shared__ C<float> x2l[NB * P];         // spectrum of p.x, [column][a][j]
  __shared__ C<float> twl[P];
  for (int e = threadIdx.x; e < P; e += blockDim.x) twl[e] = tw[e];
  const int ncb = (P + NB - 1) / NB;       // the last block may hang over the last column
  const int w = xcd_work_index(blockIdx.x, ncb * nrhs);
  const int b = w % nrhs;
  const int q0 = (w / nrhs) * NB;
  const int c = threadIdx.x % NB;          // column within the block
  const int r = threadIdx.x / NB;          // wave-uniform role: r < RA row waves
  const bool live = q0 + c < P;            // columns past the last are computed on zeros, never stored
  const int q2 = live ? q0 + c : 0;
  C<float>* myex = ex + (size_t)c * EXS;
  __syncthreads();
  if (r < RA) {
    // row waves: forward step 1 of the three fields, inverse step 3' of the two outputs
#pragma unroll 1
    for (int f = 0; f < 3; ++f) {
      const int fld = f == 0 ? 2 : f - 1;
      // the row offsets are recomputed per field rather than kept live
      // across the loop (27 of them would not fit beside the transform)
      int j = r, col = q2;
      asm volatile("" : "+v"(j), "+v"(col));
      if (j < N1) {
        // a uniform base and 32-bit element offsets (the field is < 2^31 bytes)
        const C<float>* in = T + ((size_t)(b * 3 + fld) * n) * P;
        C<float> v[N2];
#pragma unroll
        for (int k = 0; k < KIN; ++k) {
          const int t = j + N1 * k;
          v[k] = (live && t < n) ? ld_stream(in + (col + t * P)) : cmk<float>(0.f, 0.f);
        }
        DftZ<N2, -1, float, KIN>::run(v);
#pragma unroll
        for (int q = 0; q < N2; ++q) myex[q * N1 + j] = (q == 0) ? v[q] : v[q] * twl[j * q];
      }
      __syncthreads();   // exchange written
      __syncthreads();   // exchange read by the frequency waves
      if (f == 0) continue;
      __syncthreads();   // inverse exchange written
      if (j < N1) {
        C<float> v[N2];
#pragma unroll
        for (int q = 0; q < N2; ++q) v[q] = myex[q * N1 + j];
        Dft<N2, 1, float>::run(v);
        C<float>* out = T2 + ((size_t)(b * 2 + fld) * n) * P;
#pragma unroll
        for (int t1 = 0; t1 < KOUT; ++t1) {
          const int t = j + N1 * t1;
          if (live && t < n) st_stream(out + (col + t * P), v[t1]);
        }
      }
      __syncthreads();   // inverse exchange read
    }
  } else {
    // frequency waves: forward step 3, the symbol multiply, inverse step 1'
    const bool f2 = 2 * q2 > P;
    C<float>* x2 = x2l + (size_t)c * P + (r - RA);   // this thread's frequencies, stride N2 (read back by itself only)
#pragma unroll 1
    for (int f = 0; f < 3; ++f) {
      const int d = f - 1;
      // symbol offsets are recomputed per output rather than kept live across the loop
      int j = r - RA, a2 = f2 ? P - q2 : q2;
      asm volatile("" : "+v"(j), "+v"(a2));
      __syncthreads();   // exchange written
      C<float> u[N1];
      if (j < N2) {
#pragma unroll
        for (int a = 0; a < N1; ++a) u[a] = myex[j * N1 + a];
        Dft<N1, -1, float>::run(u);
      }
      __syncthreads();   // exchange read
      if (f == 0) {
        if (j < N2)
#pragma unroll
          for (int a = 0; a < N1; ++a) x2[a * N2] = u[a];
        continue;
      }
      if (j < N2) {
#pragma unroll
        for (int a = 0; a < N1; ++a) {
          const int q1 = j + N2 * a;
          const bool f1 = 2 * q1 > P;
          const int a1 = f1 ? P - q1 : q1;
          const int so = (a1 * H + a2) * 3;
          const C<float> s0 = sym[so];
          C<float> sd = sym[so + 1 + d];
          if (d == 0 ? f1 : f2) sd = cmk<float>(-sd.re, -sd.im);   // G^1 odd in q1, G^2 odd in q2
          u[a] = cfma(sd, x2[a * N2], s0 * u[a]);
        }
        Dft<N1, 1, float>::run(u);
#pragma unroll
        for (int t2 = 0; t2 < N1; ++t2) myex[j * N1 + t2] = (t2 == 0) ? u[t2] : u[t2] * cconj(twl[j * t2]);
      }
      __syncthreads();   // inverse exchange written
      __syncthreads();   // inverse exchange read
    }
  }
}

// pass C: block w -> (rhs b, component d, row block rb); y = x + v (or -v).
template <typename R, typename IO, int PT, int NBT>
__global__ __launch_bounds__(kT2) void pass_c_kernel(const C<R>* __restrict__ T2, const void* __restrict__ x,
                                                      void* __restrict__ y, int n, int P_, Radices rd_, int nb_, int nrb,
                                                      int nwork, int minus_conv, const C<R>* __restrict__ tw) {
  const int P = PT > 0 ? PT : P_, nb = NBT > 0 ? NBT : nb_;
  const Radices rd = PT > 0 ? factor_radices(PT) : rd_;
  extern __shared__ unsigned char lds_raw[];
  C<R>* a = reinterpret_cast<C<R>*>(lds_raw);
  C<R>* bb = a + (size_t)nb * P;
  const Tw<R> tws = load_twiddles(bb + (size_t)nb * P, tw, P);
  const int w = xcd_work_index(blockIdx.x, nwork);
  const int rb = w % nrb, d = (w / nrb) % 2, b = w / (2 * nrb);
  const C<R>* in = T2 + ((size_t)(b * 2 + d) * n) * P;
  for (int e = threadIdx.x; e < nb * P; e += kT2) {
    const int i1 = rb * nb + e / P;
    a[e] = i1 < n ? in[(size_t)i1 * P + e % P] : cmk<R>(0, 0);
  }
  __syncthreads();
  const C<R>* X;
  if constexpr (PT > 0) X = lds_fft_ct<R, 1, false, false, true, kT2, PT, true>(a, bb, nb, 1, P, tws);
  else X = lds_fft<R, 1, false, false, true>(a, bb, P, reverse_radices(rd), nb, 1, P, tws);
  const long nn = (long)n * n;
  const long base = ((long)b * 2 + d) * nn;
  C<IO>* yo = reinterpret_cast<C<IO>*>(y);
  for (int e = threadIdx.x; e < nb * n; e += kT2) {
    const int t = e / n, j = e % n;
    const int i1 = rb * nb + t;
    if (i1 < n) {
      const long o = base + (long)i1 * n + j;
      const C<R> v = X[t * P + j];
      C<IO> r;
      if (minus_conv) {
        r = cmk<IO>(-(IO)v.re, -(IO)v.im);
      } else {
        const C<IO> xv = ld_c<IO>(x, o);
        r = cmk<IO>(xv.re + (IO)v.re, xv.im + (IO)v.im);
      }
      yo[o] = r;
    }
  }
}


// ---- stencils (Sections 3.1 and 3.2 in two dimensions) ----
// Per dimension a point is lo (i_d = 1), in, or hi (i_d = n); class 3 c1 + c2
// (4 = interior).  tau_d = {0, 1}, {-1, 0, 1}, {-1, 0}; the enlarged
// complement ranges are {0 .. n-1}, {-(n-2) .. n-2}, {-(n-1) .. 0} minus
// the 3 x 3 block about 0.  tau is listed with the second offset fastest;
// Gram rows are (t, c) -> 2 t + c.
__host__ __device__ inline int tau_lo(int c) { return c == 0 ? 0 : -1; }
__host__ __device__ inline int tau_len(int c) { return c == 1 ? 3 : 2; }
__host__ __device__ inline int rng_lo(int c, int n) { return c == 0 ? 0 : (c == 1 ? -(n - 2) : -(n - 1)); }
__host__ __device__ inline int rng_len(int c, int n) { return c == 1 ? 2 * n - 3 : n; }
__host__ __device__ inline int dim_class(int i, int n) { return i == 0 ? 0 : (i == n - 1 ? 2 : 1); }

// W[f][r1 + n - 1][r2 + n - 1] = (k^2 G, G^1, G^2) weights, r in [-(n-1), n-1]^2
__global__ void wtable_kernel(C<double>* __restrict__ W, int n, double k, double h) {
  const int L = 2 * n - 1;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)L * L) return;
  C<double> w[3];
  weights_at((int)(idx / L) - (n - 1), (int)(idx % L) - (n - 1), k, h, w);
  for (int f = 0; f < 3; ++f) W[(long)f * L * L + idx] = w[f];
}

constexpr int kGramCols = 128;          // complement columns staged in LDS per step
constexpr int kGramBlocks = 256;        // workgroups per class

// partial[kappa][block][rho][sigma] = sum over this block's columns j of
//   delta_{c c'} k^2G(a - j) conj(k^2G(b - j)) + G^c(a - j) conj(G^c'(b - j)),  rho = 2 t_a + c
__global__ __launch_bounds__(256) void gram2_kernel(const C<double>* __restrict__ W, C<double>* __restrict__ partial,
                                                    int n) {
  __shared__ C<double> V[9][3][kGramCols];
  const int kappa = blockIdx.y, c1 = kappa / 3, c2 = kappa % 3;
  const int T1 = tau_len(c1), T2 = tau_len(c2), T = T1 * T2, D = 2 * T;
  const int L = 2 * n - 1;
  const long LL = (long)L * L;
  const int R1 = rng_len(c1, n), R2 = rng_len(c2, n), o1 = rng_lo(c1, n), o2 = rng_lo(c2, n);
  const long ncols = (long)R1 * R2;
  C<double> acc[2] = {cmk(0.0, 0.0), cmk(0.0, 0.0)};
  for (long j0 = (long)blockIdx.x * kGramCols; j0 < ncols; j0 += (long)gridDim.x * kGramCols) {
    for (int e = threadIdx.x; e < T * kGramCols; e += kT2) {
      const int t = e / kGramCols, col = e % kGramCols;
      const long j = j0 + col;
      C<double> v0 = cmk(0.0, 0.0), v1 = v0, v2 = v0;
      if (j < ncols) {
        const int jj1 = o1 + (int)(j / R2), jj2 = o2 + (int)(j % R2);
        if (abs(jj1) > 1 || abs(jj2) > 1) {
          const int a1 = tau_lo(c1) + t / T2, a2 = tau_lo(c2) + t % T2;
          const long o = (long)(a1 - jj1 + n - 1) * L + (a2 - jj2 + n - 1);
          v0 = W[o];
          v1 = W[LL + o];
          v2 = W[2 * LL + o];
        }
      }
      V[t][0][col] = v0;
      V[t][1][col] = v1;
      V[t][2][col] = v2;
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < D * D) {
        const int rho = e / D, sig = e % D;
        const int ta = rho / 2, ca = rho % 2, tb = sig / 2, cb = sig % 2;
        C<double> sum = acc[q];
        for (int col = 0; col < kGramCols; ++col) {
          if (ca == cb) sum = cfma(V[ta][0][col], cconj(V[tb][0][col]), sum);
          sum = cfma(V[ta][1 + ca][col], cconj(V[tb][1 + cb][col]), sum);
        }
        acc[q] = sum;
      }
    }
    __syncthreads();
  }
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + 256 * q;
    if (e < 324) partial[((size_t)kappa * gridDim.x + blockIdx.x) * 324 + e] = e < D * D ? acc[q] : cmk(0.0, 0.0);
  }
}

// gram[kappa][e] = sum over blocks in order (a fixed order: the same result every run)
__global__ void gram2_reduce_kernel(const C<double>* __restrict__ partial, C<double>* __restrict__ gram, int nblk) {
  const int kappa = blockIdx.x, e = threadIdx.x;
  if (e >= 324) return;
  C<double> s = cmk(0.0, 0.0);
  for (int b = 0; b < nblk; ++b) s = s + partial[((size_t)kappa * nblk + b) * 324 + e];
  gram[kappa * 324 + e] = s;
}

// Rows of S in the 27-slot form of the sparse factors ([point][2 rows][27
// slots][2 comps], slot 9 (s1+1) + 3 (s2+1) + 1):
//   S = conj(alpha[2t+c][r]) + conj(beta[3t+c][r]) m_j + conj(beta[3t+2][r]) p^c_j,  j = i + tau[t]
__global__ void rows2_kernel(const C<double>* __restrict__ alpha, const C<double>* __restrict__ beta,
                             const C<double>* __restrict__ m, const C<double>* __restrict__ p,
                             C<double>* __restrict__ S, int n) {
  const long nn = (long)n * n;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const int i1 = (int)(idx / n), i2 = (int)(idx % n);
  const int c1 = dim_class(i1, n), c2 = dim_class(i2, n), kappa = 3 * c1 + c2, T2 = tau_len(c2);
  const C<double>* al = alpha + (size_t)kappa * 36;
  const C<double>* be = beta + (size_t)kappa * 54;
  C<double>* sr = S + idx * 108;
  for (int e = 0; e < 108; ++e) sr[e] = cmk(0.0, 0.0);
  for (int s1 = -1; s1 <= 1; ++s1)
    for (int s2 = -1; s2 <= 1; ++s2) {
      const int t1 = s1 - tau_lo(c1), t2 = s2 - tau_lo(c2);
      if (t1 < 0 || t1 >= tau_len(c1) || t2 < 0 || t2 >= T2) continue;
      const int t = t1 * T2 + t2;
      const long j = idx + (long)s1 * n + s2;
      const int slot27 = 9 * (s1 + 1) + 3 * (s2 + 1) + 1;
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
          const C<double> qa = cconj(al[(2 * t + c) * 2 + r]);
          sr[(r * 27 + slot27) * 2 + c] =
              qa + cconj(be[(3 * t + c) * 2 + r]) * m[j] + cconj(be[(3 * t + 2) * 2 + r]) * p[c * nn + j];
        }
    }
}

// w = Q v for nrhs fields [rhs][2][n][n].  Q's rows depend only on the
// point's class: Q[(r, i), (c, i + a)] = conj(alpha[2t + c][r]), a = tau[t];
// the nine class stencils sit in LDS.
__global__ __launch_bounds__(256) void qapply2_kernel(const C<double>* __restrict__ alpha,
                                                      const C<double>* __restrict__ v, C<double>* __restrict__ w,
                                                      int n, int nrhs) {
  __shared__ C<double> al[9 * 36];
  for (int e = threadIdx.x; e < 9 * 36; e += blockDim.x) al[e] = alpha[e];
  __syncthreads();
  const long nn = (long)n * n;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * nrhs) return;
  const long b = idx / nn, i = idx % nn;
  const int i1 = (int)(i / n), i2 = (int)(i % n);
  const int c1 = dim_class(i1, n), c2 = dim_class(i2, n), T2 = tau_len(c2);
  const C<double>* ak = al + (3 * c1 + c2) * 36;
  const C<double>* vb = v + b * 2 * nn;
  C<double> acc[2] = {cmk(0.0, 0.0), cmk(0.0, 0.0)};
  for (int s1 = -1; s1 <= 1; ++s1)
    for (int s2 = -1; s2 <= 1; ++s2) {
      const int t1 = s1 - tau_lo(c1), t2 = s2 - tau_lo(c2);
      if (t1 < 0 || t1 >= tau_len(c1) || t2 < 0 || t2 >= T2) continue;
      const int t = t1 * T2 + t2;
      const long j = i + (long)s1 * n + s2;
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) acc[r] = cfma(cconj(ak[(2 * t + c) * 2 + r]), vb[c * nn + j], acc[r]);
    }
  w[b * 2 * nn + i] = acc[0];
  w[b * 2 * nn + nn + i] = acc[1];
}

// Eigenvectors of a Hermitian matrix (row-major, dim D) by cyclic Jacobi rotations, ascending.
void herm_eig(int D, std::vector<std::complex<double>> A, std::vector<double>& ev,
              std::vector<std::complex<double>>& V) {
  using cd = std::complex<double>;
  V.assign((size_t)D * D, cd(0.0));
  for (int i = 0; i < D; ++i) V[i * D + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        tot += std::norm(A[i * D + j]);
        if (i != j) off += std::norm(A[i * D + j]);
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < D - 1; ++p)
      for (int q = p + 1; q < D; ++q) {
        const cd apq = A[p * D + q];
        const double ab = std::abs(apq);
        if (ab == 0.0) continue;
        const double app = A[p * D + p].real(), aqq = A[q * D + q].real();
        // rotate to zero A[p][q]: with e = apq / |apq|, a real Jacobi rotation on (p, q)
        const cd e = apq / ab;
        const double theta = 0.5 * std::atan2(2.0 * ab, aqq - app);
        const double c = std::cos(theta), sn = std::sin(theta);
        // columns: new_p = c col_p - s conj(e) col_q ; new_q = s e col_p + c col_q
        for (int i = 0; i < D; ++i) {
          const cd aip = A[i * D + p], aiq = A[i * D + q];
          A[i * D + p] = c * aip - sn * std::conj(e) * aiq;
          A[i * D + q] = sn * e * aip + c * aiq;
        }
        for (int j = 0; j < D; ++j) {
          const cd apj = A[p * D + j], aqj = A[q * D + j];
          A[p * D + j] = c * apj - sn * e * aqj;
          A[q * D + j] = sn * std::conj(e) * apj + c * aqj;
        }
        for (int i = 0; i < D; ++i) {
          const cd vip = V[i * D + p], viq = V[i * D + q];
          V[i * D + p] = c * vip - sn * std::conj(e) * viq;
          V[i * D + q] = sn * e * vip + c * viq;
        }
      }
  }
  std::vector<int> ord(D);
  for (int i = 0; i < D; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return A[a * D + a].real() < A[b * D + b].real(); });
  std::vector<cd> Vs((size_t)D * D);
  ev.resize(D);
  for (int k = 0; k < D; ++k) {
    ev[k] = A[ord[k] * D + ord[k]].real();
    for (int i = 0; i < D; ++i) Vs[i * D + k] = V[i * D + ord[k]];
  }
  V.swap(Vs);
}

template <typename R>
__host__ __device__ constexpr int batch_for(int P, size_t budget = kLdsTarget) {
  const size_t per = 2 * (size_t)P * sizeof(C<R>);
  const size_t avail = (budget - tw_entries(kMaxP2) * sizeof(C<R>)) / per;
  int nb = avail > 16 ? 16 : (avail < 1 ? 1 : (int)avail);
  // a power of two that divides P (the column blocks tile P exactly)
  int b = 1;
  while (b * 2 <= nb && P % (b * 2) == 0) b *= 2;
  return b;
}

template <typename R>
size_t lds_bytes(int P, int nb) { return (2 * (size_t)nb * P + tw_entries(P)) * sizeof(C<R>); }

template <typename R, typename IO, int PT>
ls_status run_apply_p(Plan2& pl, const void* x, void* y, int nrhs, bool minus_conv, hipStream_t s,
                      hipEvent_t* ev) {
  constexpr int NBA = PT > 0 ? batch_for<R>(PT) : 0;
  constexpr int NBB = PT > 0 ? batch_for<R>(PT, kLds2) : 0;
  const int n = pl.n, P = pl.P;
  const C<R>* m = (const C<R>*)(std::is_same<R, double>::value ? pl.m64.p : pl.m32.p);
  const C<R>* p = (const C<R>*)(std::is_same<R, double>::value ? pl.p64.p : pl.p32.p);
  const C<R>* sym = (const C<R>*)(std::is_same<R, double>::value ? pl.sym64.p : pl.sym32.p);
  const C<R>* symc = (const C<R>*)(std::is_same<R, double>::value ? pl.symc64.p : pl.symc32.p);
  const C<R>* tw = (const C<R>*)(std::is_same<R, double>::value ? pl.tw64.p : pl.tw32.p);
  C<R>* T = pl.work.as<C<R>>();
  C<R>* T2 = T + (size_t)pl.max_rhs * 3 * n * P;
  const int nb = batch_for<R>(P);
  const size_t lds = lds_bytes<R>(P, nb);
  const int nrb = (n + nb - 1) / nb;
  // column pass: more adjacent columns per block (wider row segments per load)
  const int nbc = batch_for<R>(P, kLds2);
  const size_t ldsc = lds_bytes<R>(P, nbc);
  for (int r0 = 0; r0 < nrhs; r0 += pl.max_rhs) {
    const int nr = std::min(pl.max_rhs, nrhs - r0);
    const size_t off = (size_t)r0 * 2 * n * n * sizeof(C<IO>);
    const void* xr = (const unsigned char*)x + off;
    void* yr = (unsigned char*)y + off;
    const int wa = nr * nrb;
    if (ev) LS_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL((pass_a_kernel<R, IO, PT, NBA>), dim3(wa), dim3(kT2), lds, s, xr, m, p, T, n, P, pl.rd, nb, nrb, wa,
                       tw);
    LS_HIP(hipGetLastError());
    constexpr int EMAX = (int)(kLds2 / (2 * sizeof(C<R>)) / kTB);
    if (ev) LS_HIP(hipEventRecord(ev[1], s));
    if constexpr (std::is_same<R, float>::value && PT > 0 && ColRegCfg<(PT > 0 ? PT : 1)>::N1 > 0) {
      using Cfg = ColRegCfg<PT>;
      hipLaunchKernelGGL((pass_b_reg_kernel<PT>), dim3(((PT + Cfg::NB - 1) / Cfg::NB) * nr), dim3(Cfg::THREADS), 0, s, T,
                         T2, sym, n, pl.H, nr, tw);
    } else if constexpr (std::is_same<R, float>::value && PT == 1944) {
      // four columns (32-byte row runs) per workgroup of 1024 threads, one
      // workgroup per CU (125 KiB of LDS): half the partial-line reads of
      // two columns per 512-thread workgroup, at the same four waves per SIMD
      constexpr int NBW = 4, NTW = 1024, EMW = (NBW * PT + NTW - 1) / NTW;
      const auto kern = pass_b_kernel<R, EMW, PT, NBW, NTW>;
      const size_t ldsw = lds_bytes<R>(PT, NBW);
      static std::once_flag attr_once;
      std::call_once(attr_once, [&]() {
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsw);
      });
      hipLaunchKernelGGL(kern, dim3((PT / NBW) * nr), dim3(NTW), ldsw, s, T, T2, symc, n, P, pl.H, pl.rd, NBW, nr,
                         tw);
    } else {
      hipLaunchKernelGGL((pass_b_kernel<R, EMAX, PT, NBB>), dim3((P / nbc) * nr), dim3(kTB), ldsc, s, T, T2, symc, n,
                         P, pl.H, pl.rd, nbc, nr, tw);
    }
    LS_HIP(hipGetLastError());
    const int wc = nr * 2 * nrb;
    if (ev) LS_HIP(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL((pass_c_kernel<R, IO, PT, NBA>), dim3(wc), dim3(kT2), lds, s, T2, xr, yr, n, P, pl.rd, nb, nrb, wc,
                       minus_conv ? 1 : 0, tw);
    LS_HIP(hipGetLastError());
    if (ev) LS_HIP(hipEventRecord(ev[3], s));
  }
  return LS_OK;
}

// The paper's 2-D grids (n = 119, 239, 479, 959) use P = 256, 486, 972, 1944:
// kernels compiled for those lengths; any other length takes the runtime path.
template <typename R, typename IO>
ls_status run_apply(Plan2& pl, const void* x, void* y, int nrhs, bool minus_conv, hipStream_t s,
                    hipEvent_t* ev = nullptr) {
  switch (pl.P) {
    case 256: return run_apply_p<R, IO, 256>(pl, x, y, nrhs, minus_conv, s, ev);
    case 486: return run_apply_p<R, IO, 486>(pl, x, y, nrhs, minus_conv, s, ev);
    case 972: return run_apply_p<R, IO, 972>(pl, x, y, nrhs, minus_conv, s, ev);
    case 1944: return run_apply_p<R, IO, 1944>(pl, x, y, nrhs, minus_conv, s, ev);
    default: return run_apply_p<R, IO, 0>(pl, x, y, nrhs, minus_conv, s, ev);
  }
}

}  // namespace

int fft_size_2d(int n) {
  for (int P = 2 * n - 1; P <= 4096; ++P) {
    if (P % 2) continue;
    int m = P;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    if (m == 1) return P;
  }
  return 0;
}

ls_status plan2_init(Plan2& pl, int n, double k, int max_rhs, const void* m_dev, hipStream_t s) {
  if (n < 3 || !(k > 0.0) || max_rhs < 1 || !m_dev) return LS_EINVAL;
  const int P = fft_size_2d(n);
  if (P == 0 || P > kMaxP2) return LS_EINVAL;
  pl.n = n;
  pl.P = P;
  pl.H = P / 2 + 1;
  pl.k = k;
  pl.h = 1.0 / (n + 1);
  pl.max_rhs = max_rhs;
  Radices rd = factor_radices(P);
  if (rd.nst < 0) return LS_EINVAL;
  pl.rd = rd;
  const long nn = (long)n * n;
  LS_TRY(pl.m64.alloc(nn * sizeof(C<double>)));
  LS_TRY(pl.m32.alloc(nn * sizeof(C<float>)));
  LS_TRY(pl.p64.alloc(2 * nn * sizeof(C<double>)));
  LS_TRY(pl.p32.alloc(2 * nn * sizeof(C<float>)));
  LS_TRY(pl.sym64.alloc((size_t)pl.H * pl.H * 3 * sizeof(C<double>)));
  LS_TRY(pl.sym32.alloc((size_t)pl.H * pl.H * 3 * sizeof(C<float>)));
  LS_TRY(pl.symc64.alloc((size_t)pl.H * pl.H * 3 * sizeof(C<double>)));
  LS_TRY(pl.symc32.alloc((size_t)pl.H * pl.H * 3 * sizeof(C<float>)));
  LS_TRY(pl.tw64.alloc(P * sizeof(C<double>)));
  LS_TRY(pl.tw32.alloc(P * sizeof(C<float>)));
  // workspace: three transformed fields and two products per rhs, in FP64 (FP32 uses half)
  LS_TRY(pl.work.alloc((size_t)max_rhs * 5 * n * P * sizeof(C<double>)));
  std::vector<C<double>> t64(P);
  std::vector<C<float>> t32(P);
  for (int t = 0; t < P; ++t) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * t / P;
    t64[t] = cmk((double)cosl(ang), (double)sinl(ang));
    t32[t] = cmk((float)cosl(ang), (float)sinl(ang));
  }
  LS_HIP(hipMemcpyAsync(pl.tw64.p, t64.data(), P * sizeof(C<double>), hipMemcpyHostToDevice, s));
  LS_HIP(hipMemcpyAsync(pl.tw32.p, t32.data(), P * sizeof(C<float>), hipMemcpyHostToDevice, s));
  LS_HIP(hipMemcpyAsync(pl.m64.p, m_dev, nn * sizeof(C<double>), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(gradient_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, pl.m64.as<C<double>>(),
                     pl.p64.as<C<double>>(), pl.p32.as<C<float>>(), pl.m32.as<C<float>>(), n, pl.h);
  LS_HIP(hipGetLastError());
  // symbol: embed, FFT rows then columns of the three planes in FP64, keep the quadrant / P^2
  DevBuf emb;
  const size_t PP = (size_t)P * P;
  LS_TRY(emb.alloc(3 * PP * sizeof(C<double>)));
  hipLaunchKernelGGL(embed_kernel, dim3((unsigned)((PP + 255) / 256)), dim3(256), 0, s, emb.as<C<double>>(), n, P,
                     k, pl.h);
  LS_HIP(hipGetLastError());
  const int nb = batch_for<double>(P);
  const size_t lds = lds_bytes<double>(P, nb);
  hipLaunchKernelGGL((fft_rows_kernel<double, -1>), dim3((unsigned)((3 * P + nb - 1) / nb)), dim3(kT2), lds, s,
                     emb.as<C<double>>(), 3 * P, P, rd, nb, pl.tw64.as<C<double>>());
  LS_HIP(hipGetLastError());
  hipLaunchKernelGGL((fft_cols_kernel<double, -1>), dim3((unsigned)(3 * (P / nb))), dim3(kT2), lds, s,
                     emb.as<C<double>>(), P, rd, nb, pl.tw64.as<C<double>>());
  LS_HIP(hipGetLastError());
  const long HH = (long)pl.H * pl.H;
  hipLaunchKernelGGL(quadrant_kernel, dim3((unsigned)((HH + 255) / 256)), dim3(256), 0, s, emb.as<C<double>>(),
                     pl.sym64.as<C<double>>(), pl.sym32.as<C<float>>(), pl.symc64.as<C<double>>(),
                     pl.symc32.as<C<float>>(), P, pl.H);
  LS_HIP(hipGetLastError());
  LS_HIP(hipStreamSynchronize(s));   // emb is released on return
  return LS_OK;
}


void plan2_drop_factor(Plan2& pl) {
  if (pl.hs) host_free(pl.hs);
  if (pl.gs) gpu_free(pl.gs);
  pl.hs = nullptr;
  pl.gs = nullptr;
}

ls_status plan2_fit(Plan2& pl, hipStream_t s) {
  const int n = pl.n;
  if (n < 4) return LS_EINVAL;   // the interior class needs a non-empty complement
  const int L = 2 * n - 1;
  const long LL = (long)L * L;
  DevBuf W, partial, gram;
  LS_TRY(W.alloc(3 * LL * sizeof(C<double>)));
  LS_TRY(partial.alloc((size_t)9 * kGramBlocks * 324 * sizeof(C<double>)));
  LS_TRY(gram.alloc((size_t)9 * 324 * sizeof(C<double>)));
  hipLaunchKernelGGL(wtable_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, s, W.as<C<double>>(), n, pl.k,
                     pl.h);
  LS_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram2_kernel, dim3(kGramBlocks, 9), dim3(256), 0, s, W.as<C<double>>(),
                     partial.as<C<double>>(), n);
  LS_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram2_reduce_kernel, dim3(9), dim3(324), 0, s, partial.as<C<double>>(), gram.as<C<double>>(),
                     kGramBlocks);
  LS_HIP(hipGetLastError());
  using cd = std::complex<double>;
  std::vector<cd> G(9 * 324), Wc(3 * 25);
  LS_HIP(hipMemcpyAsync(G.data(), gram.p, G.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
  // the weights at offsets in [-2, 2]^2 (the local block B)
  for (int f = 0; f < 3; ++f)
    for (int d1 = -2; d1 <= 2; ++d1)
      LS_HIP(hipMemcpyAsync(&Wc[(f * 5 + d1 + 2) * 5], W.as<C<double>>() + f * LL + (long)(d1 + n - 1) * L + (n - 3),
                            5 * sizeof(cd), hipMemcpyDeviceToHost, s));
  LS_HIP(hipStreamSynchronize(s));
  auto wloc = [&](int f, int d1, int d2) { return Wc[(f * 5 + d1 + 2) * 5 + d2 + 2]; };
  pl.alpha.assign(9 * 36, cd(0.0));
  pl.beta.assign(9 * 54, cd(0.0));
  pl.eig.assign(9 * 18, 0.0);
  for (int kappa = 0; kappa < 9; ++kappa) {
    const int c1 = kappa / 3, c2 = kappa % 3, T2 = tau_len(c2), T = tau_len(c1) * T2, D = 2 * T;
    std::vector<cd> A((size_t)D * D);
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) A[i * D + j] = 0.5 * (G[kappa * 324 + i * D + j] + std::conj(G[kappa * 324 + j * D + i]));
    std::vector<double> ev;
    std::vector<cd> V;
    herm_eig(D, A, ev, V);
    for (int i = 0; i < D; ++i) pl.eig[kappa * 18 + i] = ev[i];
    for (int i = 0; i < D; ++i)
      for (int r = 0; r < 2; ++r) pl.alpha[kappa * 36 + i * 2 + r] = V[i * D + r];
    // beta[(b, f)][r] = sum_{(a, c)} conj(B[(a, c)][(b, f)]) alpha[(a, c)][r],
    // B[(a, c)][(b, f)] = delta_{f c} k^2 G(a - b) + delta_{f 2} G^c(a - b)
    for (int tb = 0; tb < T; ++tb)
      for (int f = 0; f < 3; ++f)
        for (int r = 0; r < 2; ++r) {
          cd acc = 0.0;
          for (int ta = 0; ta < T; ++ta) {
            const int d1 = ta / T2 - tb / T2, d2 = ta % T2 - tb % T2;
            for (int c = 0; c < 2; ++c) {
              cd B = 0.0;
              if (f == c) B = wloc(0, d1, d2);
              else if (f == 2) B = wloc(1 + c, d1, d2);
              acc += std::conj(B) * pl.alpha[kappa * 36 + (2 * ta + c) * 2 + r];
            }
          }
          pl.beta[kappa * 54 + (3 * tb + f) * 2 + r] = acc;
        }
  }
  // rows
  const long nn = (long)n * n;
  DevBuf dbe;
  LS_TRY(pl.alpha_dev.alloc(pl.alpha.size() * sizeof(cd)));
  LS_TRY(dbe.alloc(pl.beta.size() * sizeof(cd)));
  LS_TRY(pl.srows.alloc((size_t)nn * 108 * sizeof(cd)));
  LS_HIP(hipMemcpyAsync(pl.alpha_dev.p, pl.alpha.data(), pl.alpha_dev.bytes, hipMemcpyHostToDevice, s));
  LS_HIP(hipMemcpyAsync(dbe.p, pl.beta.data(), dbe.bytes, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(rows2_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s,
                     pl.alpha_dev.as<C<double>>(), dbe.as<C<double>>(), pl.m64.as<C<double>>(),
                     pl.p64.as<C<double>>(), pl.srows.as<C<double>>(), n);
  LS_HIP(hipGetLastError());
  LS_HIP(hipStreamSynchronize(s));
  pl.fitted = true;
  plan2_drop_factor(pl);
  return LS_OK;
}

ls_status plan2_factor(Plan2& pl, bool fp32, hipStream_t s) {
  if (!pl.fitted) return LS_ESTATE;
  plan2_drop_factor(pl);
  std::vector<std::complex<double>> rows(pl.srows.bytes / sizeof(std::complex<double>));
  LS_HIP(hipMemcpyAsync(rows.data(), pl.srows.p, pl.srows.bytes, hipMemcpyDeviceToHost, s));
  LS_HIP(hipStreamSynchronize(s));
  const int dims[3] = {pl.n, pl.n, 1};
  return host_factor_grid(dims, 2, rows.data(), 0, fp32, &pl.hs);
}

ls_status plan2_factor_gpu(Plan2& pl, bool fp32, hipStream_t s) {
  if (!pl.fitted) return LS_ESTATE;
  plan2_drop_factor(pl);
  const int dims[3] = {pl.n, pl.n, 1};
  LS_TRY(gpu_factor_grid(dims, 2, pl.srows.as<C<double>>(), fp32, s, &pl.gs));
  LS_HIP(hipStreamSynchronize(s));
  return LS_OK;
}

// z = S^-1 Q v for the listed fields (in place), S^-1 on host cores.
ls_status plan2_precond(Plan2& pl, const std::vector<int>& lb, const std::function<C<double>*(int)>& ptr,
                        hipStream_t s, double* t_host) {
  if (!pl.hs && !pl.gs) return LS_ESTATE;
  const long len = 2L * pl.n * pl.n;
  const size_t vb = (size_t)len * sizeof(C<double>);
  const int nb = (int)lb.size();
  const long nn = (long)pl.n * pl.n;
  if (pl.gs) {   // GPU factor: Q v into a contiguous block, S^-1 in HBM
    if (t_host) *t_host = 0.0;
    if (pl.pbuf.bytes < (size_t)nb * vb) LS_TRY(pl.pbuf.alloc((size_t)nb * vb));
    C<double>* blk = pl.pbuf.as<C<double>>();
    for (int q = 0; q < nb; ++q) {
      hipLaunchKernelGGL(qapply2_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s,
                         pl.alpha_dev.as<C<double>>(), ptr(lb[q]), blk + (size_t)q * len, pl.n, 1);
      LS_HIP(hipGetLastError());
    }
    LS_TRY(gpu_solve(pl.gs, blk, blk, nb, s));
    for (int q = 0; q < nb; ++q)
      LS_HIP(hipMemcpyAsync(ptr(lb[q]), blk + (size_t)q * len, vb, hipMemcpyDeviceToDevice, s));
    return LS_OK;
  }
  if (pl.pbuf.bytes < vb) LS_TRY(pl.pbuf.alloc(vb));
  std::vector<std::complex<double>> hb((size_t)nb * len);
  for (int q = 0; q < nb; ++q) {
    hipLaunchKernelGGL(qapply2_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s,
                       pl.alpha_dev.as<C<double>>(), ptr(lb[q]), pl.pbuf.as<C<double>>(), pl.n, 1);
    LS_HIP(hipGetLastError());
    LS_HIP(hipMemcpyAsync(hb.data() + (size_t)q * len, pl.pbuf.p, vb, hipMemcpyDeviceToHost, s));
  }
  LS_HIP(hipStreamSynchronize(s));
  const double t0 = wall_seconds();
  LS_TRY(host_solve(pl.hs, hb.data(), nb));
  if (t_host) *t_host = wall_seconds() - t0;
  for (int q = 0; q < nb; ++q)
    LS_HIP(hipMemcpyAsync(ptr(lb[q]), hb.data() + (size_t)q * len, vb, hipMemcpyHostToDevice, s));
  LS_HIP(hipStreamSynchronize(s));
  return LS_OK;
}

ls_status plan2_solve(Plan2& pl, const void* g, void* x, int nrhs, double tol, int restart, int maxit, ls_prec prec,
                      ls_solve_info* info, hipStream_t s) {
  if (!g || !x || nrhs < 1 || !info || restart < 1 || maxit < 1 || !(tol > 0.0)) return LS_EINVAL;
  if (prec != LS_C128 && prec != LS_MIXED) return LS_EINVAL;
  if (!pl.hs && !pl.gs) return LS_ESTATE;
  pl.gctx.len = 2L * pl.n * pl.n;
  GmresOps ops;
  Plan2* P = &pl;
  ops.apply = [P](const C<double>* xx, C<double>* yy, int nb, ls_prec pr, hipStream_t st) {
    return plan2_apply(*P, xx, yy, nb, pr, st, false);
  };
  ops.precond_batch = [P](const std::vector<int>& lb, const std::function<C<double>*(int)>& ptr, hipStream_t st,
                          double* th) { return plan2_precond(*P, lb, ptr, st, th); };
  const double t0 = wall_seconds();
  const ls_status st = gmres_solve(pl.gctx, ops, static_cast<const C<double>*>(g), static_cast<C<double>*>(x), nrhs,
                                   tol, restart, maxit, prec, info, s);
  const double tt = wall_seconds() - t0;
  for (int b = 0; b < nrhs; ++b) info[b].t_gpu = tt / nrhs - info[b].t_host;
  return st;
}

ls_status plan2_apply(Plan2& pl, const void* x, void* y, int nrhs, ls_prec prec, hipStream_t s, bool minus_conv,
                      hipEvent_t* ev) {
  if (nrhs < 1 || !x || !y) return LS_EINVAL;
  switch (prec) {
    case LS_C128: return run_apply<double, double>(pl, x, y, nrhs, minus_conv, s, ev);
    case LS_C64: return run_apply<float, float>(pl, x, y, nrhs, minus_conv, s, ev);
    case LS_MIXED: return run_apply<float, double>(pl, x, y, nrhs, minus_conv, s, ev);
  }
  return LS_EINVAL;
}

}  // namespace ls

// ---- C ABI ----
struct ls2_plan {
  ls::Plan2 pl;
};

namespace ls {
Plan2::~Plan2() {
  if (hs) host_free(hs);
  if (gs) gpu_free(gs);
}
}  // namespace ls

// Host allocations inside an entry point (the symbolic phase of the factor,
// host staging) may throw; no exception crosses the C boundary.
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

extern "C" {

ls_status ls2_plan_create(int n, double k, int max_rhs, const void* m_dev, void* hip_stream, ls2_plan** out) {
  return guarded([&]() -> ls_status {
    if (!out) return LS_EINVAL;
    *out = nullptr;
    ls2_plan* p = new (std::nothrow) ls2_plan;
    if (!p) return LS_ENOMEM;
    const ls_status st = ls::plan2_init(p->pl, n, k, max_rhs, m_dev, (hipStream_t)hip_stream);
    if (st != LS_OK) {
      delete p;
      return st;
    }
    *out = p;
    return LS_OK;
  });
}

ls_status ls2_apply(ls2_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    return ls::plan2_apply(plan->pl, x_dev, y_dev, nrhs, prec, (hipStream_t)hip_stream, false);
  });
}

ls_status ls2_rhs_from_incident(ls2_plan* plan, const void* Ei_dev, void* g_dev, int nrhs, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    return ls::plan2_apply(plan->pl, Ei_dev, g_dev, nrhs, LS_C128, (hipStream_t)hip_stream, true);
  });
}

int ls2_plan_fft_size(const ls2_plan* plan) { return plan ? plan->pl.P : 0; }

ls_status ls2_apply_timed(ls2_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec, void* hip_stream,
                          double* pass_ms) {
  return guarded([&]() -> ls_status {
    if (!plan || !pass_ms || nrhs > plan->pl.max_rhs) return LS_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t ev[4];
    for (int i = 0; i < 4; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
        return LS_EHIP;
      }
    ls_status st = ls::plan2_apply(plan->pl, x_dev, y_dev, nrhs, prec, s, false, ev);
    if (st == LS_OK && hipEventSynchronize(ev[3]) != hipSuccess) st = LS_EHIP;
    for (int i = 0; i < 3 && st == LS_OK; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) st = LS_EHIP;
      pass_ms[i] = ms;
    }
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
    return st;
  });
}

ls_status ls2_stencil_fit(ls2_plan* plan, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    return ls::plan2_fit(plan->pl, (hipStream_t)hip_stream);
  });
}

ls_status ls2_get_stencils(const ls2_plan* plan, void* alpha_host, void* beta_host, double* eig_host) {
  return guarded([&]() -> ls_status {
    if (!plan || !alpha_host || !beta_host || !eig_host) return LS_EINVAL;
    if (!plan->pl.fitted) return LS_ESTATE;
    std::memcpy(alpha_host, plan->pl.alpha.data(), plan->pl.alpha.size() * sizeof(std::complex<double>));
    std::memcpy(beta_host, plan->pl.beta.data(), plan->pl.beta.size() * sizeof(std::complex<double>));
    std::memcpy(eig_host, plan->pl.eig.data(), plan->pl.eig.size() * sizeof(double));
    return LS_OK;
  });
}

ls_status ls2_factor(ls2_plan* plan, ls_prec factor_prec, double* seconds_out) {
  return guarded([&]() -> ls_status {
    if (!plan || (factor_prec != LS_C128 && factor_prec != LS_C64)) return LS_EINVAL;
    const double t0 = ls::wall_seconds();
    const ls_status st = ls::plan2_factor(plan->pl, factor_prec == LS_C64, nullptr);
    if (seconds_out) *seconds_out = ls::wall_seconds() - t0;
    return st;
  });
}

ls_status ls2_factor_gpu(ls2_plan* plan, ls_prec factor_prec, void* hip_stream, double* seconds_out) {
  return guarded([&]() -> ls_status {
    if (!plan || (factor_prec != LS_C128 && factor_prec != LS_C64)) return LS_EINVAL;
    const double t0 = ls::wall_seconds();
    const ls_status st = ls::plan2_factor_gpu(plan->pl, factor_prec == LS_C64, (hipStream_t)hip_stream);
    if (seconds_out) *seconds_out = ls::wall_seconds() - t0;
    return st;
  });
}

ls_status ls2_precond_apply(ls2_plan* plan, const void* v_dev, void* z_dev, int nrhs, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan || !v_dev || !z_dev || nrhs < 1) return LS_EINVAL;
    const long len = 2L * plan->pl.n * plan->pl.n;
    hipStream_t s = (hipStream_t)hip_stream;
    if (v_dev != z_dev)
      LS_HIP(hipMemcpyAsync(z_dev, v_dev, (size_t)nrhs * len * sizeof(ls::C<double>), hipMemcpyDeviceToDevice, s));
    std::vector<int> lb(nrhs);
    for (int b = 0; b < nrhs; ++b) lb[b] = b;
    ls::C<double>* z = static_cast<ls::C<double>*>(z_dev);
    return ls::plan2_precond(plan->pl, lb, [&](int b) { return z + (long)b * len; }, s, nullptr);
  });
}

ls_status ls2_gmres_solve(ls2_plan* plan, const void* g_dev, void* x_dev, int nrhs, double tol, int restart,
                          int maxit, ls_prec apply_prec, ls_solve_info* info, void* hip_stream) {
  return guarded([&]() -> ls_status {
    if (!plan) return LS_EINVAL;
    return ls::plan2_solve(plan->pl, g_dev, x_dev, nrhs, tol, restart, maxit, apply_prec, info,
                           (hipStream_t)hip_stream);
  });
}

void ls2_plan_destroy(ls2_plan* plan) { delete plan; }

}  // extern "C"
