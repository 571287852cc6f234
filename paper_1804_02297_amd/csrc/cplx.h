// Complex arithmetic and in-register small DFTs for the gfx950 FFT kernels.
//
// The small DFTs are unrolled completely at compile time: a length-N DFT on
// an array held in VGPRs, decimation in time over its first factor (4, 2 or
// 3), with the internal twiddles W_N^k = exp(-+2 pi i k / N) folded in as
// compile-time constants.  Those constants come from a constexpr Taylor
// series evaluated on an argument reduced to |phi| <= pi/4 with exact
// integer arithmetic, so every constant is correctly rounded to about one
// ulp of double.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace ls {

template <typename R>
struct alignas(2 * sizeof(R)) C {
  R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ C<R> cmk(R a, R b) {
  C<R> z;
  z.re = a;
  z.im = b;
  return z;
}
template <typename R>
__host__ __device__ __forceinline__ C<R> operator+(C<R> a, C<R> b) { return cmk(a.re + b.re, a.im + b.im); }
template <typename R>
__host__ __device__ __forceinline__ C<R> operator-(C<R> a, C<R> b) { return cmk(a.re - b.re, a.im - b.im); }
template <typename R>
__host__ __device__ __forceinline__ C<R> operator*(C<R> a, C<R> b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ __forceinline__ C<R> cscale(C<R> a, R s) { return cmk(a.re * s, a.im * s); }
template <typename R>
__host__ __device__ __forceinline__ C<R> cconj(C<R> a) { return cmk(a.re, -a.im); }
// a * (-i) and a * (+i)
template <typename R>
__host__ __device__ __forceinline__ C<R> mul_mi(C<R> a) { return cmk(a.im, -a.re); }
template <typename R>
__host__ __device__ __forceinline__ C<R> mul_pi(C<R> a) { return cmk(-a.im, a.re); }
// fused a + b*c
template <typename R>
__host__ __device__ __forceinline__ C<R> cfma(C<R> b, C<R> c, C<R> a) {
  return cmk(a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re);
}

template <typename To, typename Ti>
__host__ __device__ __forceinline__ C<To> ccast(C<Ti> a) { return cmk((To)a.re, (To)a.im); }

// Streaming global loads and stores (non-temporal: data read or written once
// per pass is not kept in the caches).
#ifndef LS_NT
#define LS_NT 1
#endif
template <typename R>
__device__ __forceinline__ C<R> ld_stream(const C<R>* p) {
  if constexpr (LS_NT) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return cmk<R>(v.x, v.y);
  } else {
    return *p;
  }
}
template <typename R>
__device__ __forceinline__ void st_stream(C<R>* p, C<R> z) {
  if constexpr (LS_NT) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 v = {z.re, z.im};
    __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
  } else {
    *p = z;
  }
}

// ---- compile-time twiddles -------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_sin_small(double x) {  // |x| <= pi/4
  double t = x, s = x;
  for (int i = 1; i < 14; ++i) {
    t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
constexpr double ct_cos_small(double x) {
  double t = 1.0, s = 1.0;
  for (int i = 1; i < 14; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}
// cos / sin of 2 pi k / N, exact quadrant reduction on integers.
constexpr double ct_cos2pi(long k, long N) {
  k %= N;
  if (k < 0) k += N;
  long q = (4 * k + N / 2) / N;            // nearest quarter turn
  long r = 4 * k - q * N;                  // |r| <= N/2
  double phi = (kPi / 2.0) * (double)r / (double)N;
  double c = ct_cos_small(phi), s = ct_sin_small(phi);
  switch (q & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
  }
}
constexpr double ct_sin2pi(long k, long N) {
  k %= N;
  if (k < 0) k += N;
  long q = (4 * k + N / 2) / N;
  long r = 4 * k - q * N;
  double phi = (kPi / 2.0) * (double)r / (double)N;
  double c = ct_cos_small(phi), s = ct_sin_small(phi);
  switch (q & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
  }
}

// W_N^k for direction DIR (-1: forward exp(-2 pi i k/N), +1: inverse).
template <typename R, int N, int DIR>
__device__ __forceinline__ C<R> ctw(int k) {
  return cmk<R>((R)ct_cos2pi(k, N), (R)(DIR * ct_sin2pi(k, N)));
}

// a * W_N^k with k a compile-time constant after unrolling: the quarter turns
// are sign swaps (free as operand modifiers), the rest a complex multiply by
// the constant.  An IEEE multiply by 0 or -1 cannot be folded by the
// compiler, so these cases are spelt out.
template <typename R, int N, int DIR>
__device__ __forceinline__ C<R> twmul(C<R> a, int k) {
  k %= N;
  if (k == 0) return a;
  if (2 * k == N) return cmk<R>(-a.re, -a.im);
  if (4 * k == N) return (DIR < 0) ? mul_mi(a) : mul_pi(a);
  if (4 * k == 3 * N) return (DIR < 0) ? mul_pi(a) : mul_mi(a);
  return a * ctw<R, N, DIR>(k);
}

// ---- in-register DFTs --------------------------------------------------------
template <int N>
struct FirstFactor {
  static constexpr int value = (N % 4 == 0 && N > 8) ? 4 : (N % 2 == 0 ? 2 : (N % 3 == 0 ? 3 : N));
};

template <int N, int DIR, typename R>
struct Dft;

template <int DIR, typename R>
struct Dft<1, DIR, R> {
  static __device__ __forceinline__ void run(C<R>*) {}
};

template <int DIR, typename R>
struct Dft<2, DIR, R> {
  static __device__ __forceinline__ void run(C<R>* v) {
    C<R> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <int DIR, typename R>
struct Dft<3, DIR, R> {
  static __device__ __forceinline__ void run(C<R>* v) {
    // X0 = a+b+c; X1,2 = a - (b+c)/2 -+ i DIR... with s = sin(2pi/3)
    const R s = (R)(0.86602540378443864676372317075293618);
    C<R> a = v[0], b = v[1], c = v[2];
    C<R> t = b + c;
    C<R> d = b - c;
    C<R> m = cmk<R>(a.re - (R)0.5 * t.re, a.im - (R)0.5 * t.im);
    // DIR = -1: X1 = m - i s d ; X2 = m + i s d
    C<R> isd = cmk<R>(-s * d.im, s * d.re);  // i s d
    v[0] = a + t;
    if (DIR < 0) {
      v[1] = m - isd;
      v[2] = m + isd;
    } else {
      v[1] = m + isd;
      v[2] = m - isd;
    }
  }
};

template <int DIR, typename R>
struct Dft<4, DIR, R> {
  static __device__ __forceinline__ void run(C<R>* v) {
    C<R> a0 = v[0] + v[2], a1 = v[0] - v[2];
    C<R> b0 = v[1] + v[3], b1 = v[1] - v[3];
    C<R> jb1 = (DIR < 0) ? mul_mi(b1) : mul_pi(b1);
    v[0] = a0 + b0;
    v[2] = a0 - b0;
    v[1] = a1 + jb1;
    v[3] = a1 - jb1;
  }
};

// Generic: N = F * M, input index f + F m, output index q + M s.
template <int N, int DIR, typename R>
struct Dft {
  static __device__ __forceinline__ void run(C<R>* v) {
    constexpr int F = FirstFactor<N>::value;
    constexpr int M = N / F;
    static_assert(F * M == N && F > 1 && M > 1, "unsupported DFT length");
    C<R> sub[F][M];
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int m = 0; m < M; ++m) sub[f][m] = v[f + F * m];
#pragma unroll
    for (int f = 0; f < F; ++f) Dft<M, DIR, R>::run(sub[f]);
#pragma unroll
    for (int q = 0; q < M; ++q) {
      C<R> t[F];
#pragma unroll
      for (int f = 0; f < F; ++f) t[f] = twmul<R, N, DIR>(sub[f][q], f * q);
      Dft<F, DIR, R>::run(t);
#pragma unroll
      for (int s = 0; s < F; ++s) v[q + M * s] = t[s];
    }
  }
};

// Length 16 (4 x 4): the four sub-transforms of inputs f + 4m, then per output
// column q a radix-4 butterfly over f of sub[f][q] W^(fq).  The twiddles are
// folded into fused multiply-adds: W^(fq) s is written as a real scale times
// s + t rot(s) or t s + rot(s) (t = tan(pi/8), rot = multiplication by the
// direction's quarter turn), and the columns q = 1, 3 pair terms whose
// scales are both cos(pi/8), q = 1, 2, 3 terms with scale cos(pi/4), so each
// scale is applied once in the final multiply-adds.  144 real operations for
// the full transform instead of 160 with the twiddles multiplied out.
template <int DIR, typename R>
__device__ __forceinline__ C<R> qrot(C<R> a) {   // a * W^4 = a * (DIR i)
  return (DIR < 0) ? mul_mi(a) : mul_pi(a);
}
// c * x + a, c a real constant
template <typename R>
__device__ __forceinline__ C<R> rfma(R c, C<R> x, C<R> a) {
  return cmk<R>(c * x.re + a.re, c * x.im + a.im);
}
template <int DIR, typename R>
__device__ __forceinline__ void dft16_finish(const C<R> (&sub)[4][4], C<R>* v) {
  constexpr R Cp8 = (R)0.92387953251128675612818318939678829;   // cos(pi/8)
  constexpr R Tp8 = (R)0.41421356237309504880168872420969808;   // tan(pi/8)
  constexpr R Cp4 = (R)0.70710678118654752440084436210484903;   // cos(pi/4)
  // q = 0: no twiddles
  {
    const C<R> a0 = sub[0][0] + sub[2][0], a1 = sub[0][0] - sub[2][0];
    const C<R> b0 = sub[1][0] + sub[3][0], b1 = qrot<DIR>(sub[1][0] - sub[3][0]);
    v[0] = a0 + b0;
    v[8] = a0 - b0;
    v[4] = a1 + b1;
    v[12] = a1 - b1;
  }
  // s + t rot(s) and t s + rot(s)
  auto zt = [](C<R> s) { return s + cscale(qrot<DIR>(s), Tp8); };
  auto yt = [](C<R> s) { return cscale(s, Tp8) + qrot<DIR>(s); };
  // q = 1: W^1 s1 = Cp8 z(s1), W^2 s2 = Cp4 (s2 + rot s2), W^3 s3 = Cp8 y(s3)
  {
    const C<R> p2 = sub[2][1] + qrot<DIR>(sub[2][1]);
    const C<R> a0 = rfma(Cp4, p2, sub[0][1]), a1 = rfma(-Cp4, p2, sub[0][1]);
    const C<R> z1 = zt(sub[1][1]), y3 = yt(sub[3][1]);
    const C<R> e = z1 + y3, d = qrot<DIR>(z1 - y3);
    v[1] = rfma(Cp8, e, a0);
    v[9] = rfma(-Cp8, e, a0);
    v[5] = rfma(Cp8, d, a1);
    v[13] = rfma(-Cp8, d, a1);
  }
  // q = 2: W^2 s1 = Cp4 (s1 + rot s1), W^4 s2 = rot s2, W^6 s3 = Cp4 (rot s3 - s3)
  {
    const C<R> r2 = qrot<DIR>(sub[2][2]);
    const C<R> a0 = sub[0][2] + r2, a1 = sub[0][2] - r2;
    const C<R> u = sub[1][2] - sub[3][2], w = sub[1][2] + sub[3][2];
    const C<R> e = u + qrot<DIR>(w);                 // (s1 + rot s1) + (rot s3 - s3)
    const C<R> d = qrot<DIR>(w + qrot<DIR>(u));      // rot of (s1 + rot s1) - (rot s3 - s3)
    v[2] = rfma(Cp4, e, a0);
    v[10] = rfma(-Cp4, e, a0);
    v[6] = rfma(Cp4, d, a1);
    v[14] = rfma(-Cp4, d, a1);
  }
  // q = 3: W^3 s1 = Cp8 y(s1), W^6 s2 = Cp4 (rot s2 - s2), W^9 s3 = -Cp8 z(s3)
  {
    const C<R> p2 = qrot<DIR>(sub[2][3]) - sub[2][3];
    const C<R> a0 = rfma(Cp4, p2, sub[0][3]), a1 = rfma(-Cp4, p2, sub[0][3]);
    const C<R> y1 = yt(sub[1][3]), z3 = zt(sub[3][3]);
    const C<R> e = y1 - z3, d = qrot<DIR>(y1 + z3);
    v[3] = rfma(Cp8, e, a0);
    v[11] = rfma(-Cp8, e, a0);
    v[7] = rfma(Cp8, d, a1);
    v[15] = rfma(-Cp8, d, a1);
  }
}

template <int DIR, typename R>
struct Dft<16, DIR, R> {
  static __device__ __forceinline__ void run(C<R>* v) {
    C<R> sub[4][4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
      for (int m = 0; m < 4; ++m) sub[f][m] = v[f + 4 * m];
      Dft<4, DIR, R>::run(sub[f]);
    }
    dft16_finish<DIR>(sub, v);
  }
};

// ---- DFTs with known-zero inputs ---------------------------------------------
// DftZ<N, DIR, R, NIN>: the same transform when v[k] = 0 for k >= NIN (those
// entries are never read).  The zero-padded halves of the circulant
// embedding make NIN = N/2 in the forward passes; IEEE arithmetic forbids
// the compiler from folding x + 0 and 0 * w itself, so the pruning is spelt
// out here.  Outputs that a caller never reads are removed by dead-code
// elimination, so no output pruning is needed.
template <int I, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (I < E) {
    fn(std::integral_constant<int, I>{});
    static_for<I + 1, E>(fn);
  }
}

template <int N, int DIR, typename R, int NIN>
struct DftZ {
  static __device__ __forceinline__ void run(C<R>* v) {
    if constexpr (NIN >= N) {
      Dft<N, DIR, R>::run(v);
    } else if constexpr (NIN <= 0) {
#pragma unroll
      for (int q = 0; q < N; ++q) v[q] = cmk<R>(0, 0);
    } else if constexpr (NIN == 1) {
#pragma unroll
      for (int q = 1; q < N; ++q) v[q] = v[0];
    } else if constexpr (N == 4 && NIN == 2) {
      const C<R> a = v[0], b = v[1];
      const C<R> jb = (DIR < 0) ? mul_mi(b) : mul_pi(b);
      v[0] = a + b;
      v[1] = a + jb;
      v[2] = a - b;
      v[3] = a - jb;
    } else if constexpr (N <= 4) {
#pragma unroll
      for (int k = NIN; k < N; ++k) v[k] = cmk<R>(0, 0);
      Dft<N, DIR, R>::run(v);
    } else if constexpr (N == 16 && NIN >= 4) {
      C<R> sub[4][4];
      static_for<0, 4>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        constexpr int nin = (NIN > f) ? (NIN - f + 3) / 4 : 0;
#pragma unroll
        for (int m = 0; m < nin; ++m) sub[f][m] = v[f + 4 * m];
        DftZ<4, DIR, R, nin>::run(sub[f]);
      });
      dft16_finish<DIR>(sub, v);
    } else {
      constexpr int F = FirstFactor<N>::value;
      constexpr int M = N / F;
      C<R> sub[F][M];
      static_for<0, F>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        constexpr int nin = (NIN > f) ? (NIN - f + F - 1) / F : 0;
#pragma unroll
        for (int m = 0; m < nin; ++m) sub[f][m] = v[f + F * m];
        DftZ<M, DIR, R, nin>::run(sub[f]);
      });
      constexpr int FIN = NIN < F ? NIN : F;     // sub-transforms that are not all zero
#pragma unroll
      for (int q = 0; q < M; ++q) {
        C<R> t[F];
#pragma unroll
        for (int f = 0; f < FIN; ++f) t[f] = twmul<R, N, DIR>(sub[f][q], f * q);
        DftZ<F, DIR, R, FIN>::run(t);
#pragma unroll
        for (int s = 0; s < F; ++s) v[q + M * s] = t[s];
      }
    }
  }
};

}  // namespace ls
