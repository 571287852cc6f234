// Right-preconditioned flexible GMRES in FP64 on the GPU.
//
// Paper: the sparse solve is the preconditioner of standard GMRES (end of
// Section 3.1; Section 4 uses restart 20 and relative residual 1e-6).  Here
// every Krylov vector, the classical Gram-Schmidt orthogonalisation (two
// passes), the update x += Z y and the true residual are complex128 on the
// GPU; the small Hessenberg least-squares problem (Givens rotations) is on
// the host.  Right-hand sides advance in lockstep: each step applies the
// operator and the preconditioner to the whole batch, and a right-hand side
// that has converged is frozen.
//
// Mixed precision: with LS_MIXED the Krylov operator apply runs its FFTs in
// FP32 while the identity term, all vectors and the residual stay FP64.  An
// Arnoldi cycle then cannot reduce the FP64 residual much below the FP32
// apply accuracy, so a cycle ends once its estimated residual fell by the
// factor `mixed_drop`, and the restart recomputes the true residual with the
// FP64 apply (iterative refinement on top of FGMRES).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "gmres.h"

namespace ls {

namespace {

constexpr int kRed = 256;        // threads per reduction block

// partial[b][blk] = sum over the block's elements of conj(V_q) w for q < nv
// V: nv vectors of length len (stride vstride), w: length len; batched over
// right-hand sides b with strides.
__global__ void multidot_kernel(const C<double>* __restrict__ V, long vstride, int nv,
                                const C<double>* __restrict__ w, long len, int nblk,
                                C<double>* __restrict__ partial) {
  __shared__ double sr[kRed], si[kRed];
  const int q = blockIdx.y;
  const int blk = blockIdx.x;
  const C<double>* v = V + (long)q * vstride;
  double ar = 0.0, ai = 0.0;
  for (long e = (long)blk * kRed + threadIdx.x; e < len; e += (long)nblk * kRed) {
    const C<double> a = v[e], b = w[e];
    ar += a.re * b.re + a.im * b.im;
    ai += a.re * b.im - a.im * b.re;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = kRed / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long)q * nblk + blk] = cmk(sr[0], si[0]);
}

__global__ void sum_partials_kernel(const C<double>* __restrict__ partial, int nblk, int nv,
                                    C<double>* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nv) return;
  double r = 0.0, i = 0.0;
  for (int b = 0; b < nblk; ++b) {
    r += partial[(long)q * nblk + b].re;
    i += partial[(long)q * nblk + b].im;
  }
  out[q] = cmk(r, i);
}

// w -= sum_q V_q h_q
__global__ void subtract_combo_kernel(const C<double>* __restrict__ V, long vstride, int nv,
                                      const C<double>* __restrict__ h, C<double>* __restrict__ w, long len) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  C<double> acc = w[e];
  for (int q = 0; q < nv; ++q) acc = acc - V[(long)q * vstride + e] * h[q];
  w[e] = acc;
}

// x += sum_q Z_q y_q
__global__ void add_combo_kernel(const C<double>* __restrict__ Z, long zstride, int nv,
                                 const C<double>* __restrict__ y, C<double>* __restrict__ x, long len) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  C<double> acc = x[e];
  for (int q = 0; q < nv; ++q) acc = acc + Z[(long)q * zstride + e] * y[q];
  x[e] = acc;
}

__global__ void scale_copy_kernel(const C<double>* __restrict__ a, double s, C<double>* __restrict__ b, long len) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) b[e] = cscale(a[e], s);
}

// r = g - r  (r holds A x on entry)
__global__ void residual_kernel(const C<double>* __restrict__ g, C<double>* __restrict__ r, long len) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) r[e] = g[e] - r[e];
}

inline unsigned blocks_for(long len, int t) { return (unsigned)((len + t - 1) / t); }

// ---- fused Gram-Schmidt passes over a run of right-hand sides ----------------
// The two classical Gram-Schmidt passes and the norm of one Arnoldi step read
// each Krylov vector three times instead of four and the new vector once per
// pass instead of once per Krylov vector, and one launch covers every rhs of
// a contiguous run.  The sums are the same as multidot's, in another order.
constexpr int kOrthBlk = 64;    // blocks per rhs
constexpr int kMaxV = 32;       // Krylov vectors a fused pass handles

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// For rhs b = b0 + blockIdx.y (V_q of rhs b at V + q qstride + b len, w at
// W + b len):
//   SUB = false:            h_q = sum conj(V_q) w, q < nv;
//   SUB = true, NORM = false: w -= sum_q V_q hin_q, then h_q = sum conj(V_q) w;
//   SUB = true, NORM = true:  w -= sum_q V_q hin_q, then h_0 = sum |w|^2.
// Block partial sums go to partial[((b - b0) nblk + blk) kMaxV + q], nblk = gridDim.x.
template <bool SUB, bool NORM>
__global__ __launch_bounds__(256) void orth_pass_kernel(const C<double>* __restrict__ V, long qstride, int nv,
                                                        C<double>* __restrict__ W, long len, int b0,
                                                        const C<double>* __restrict__ hin, long hstride,
                                                        C<double>* __restrict__ partial) {
  __shared__ C<double> hl[kMaxV];
  __shared__ double red[4][2 * kMaxV];
  const int b = b0 + blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  const C<double>* Vb = V + (long)b * len;
  C<double>* w = W + (long)b * len;
  if (SUB && tid < nv) hl[tid] = hin[(long)b * hstride + tid];
  __syncthreads();
  constexpr int NA = NORM ? 1 : kMaxV;
  double ar[NA], ai[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) ar[q] = ai[q] = 0.0;
  for (long e = (long)blk * 256 + tid; e < len; e += (long)gridDim.x * 256) {
    C<double> we = w[e];
    if constexpr (SUB) {
#pragma unroll
      for (int q = 0; q < kMaxV; ++q)
        if (q < nv) we = we - Vb[q * qstride + e] * hl[q];
      w[e] = we;
    }
    if constexpr (NORM) {
      ar[0] += we.re * we.re + we.im * we.im;
    } else {
      // after a subtraction the Krylov values are loaded again (from the
      // cache) rather than kept: nv of them beside the accumulators would not
      // fit the registers
      long e2 = e;
      if constexpr (SUB) asm volatile("" : "+v"(e2));
#pragma unroll
      for (int q = 0; q < kMaxV; ++q)
        if (q < nv) {
          const C<double> v = Vb[q * qstride + e2];
          ar[q] += v.re * we.re + v.im * we.im;
          ai[q] += v.re * we.im - v.im * we.re;
        }
    }
  }
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int q = 0; q < NA; ++q)
    if (q < nv) {
      const double sr = wave_sum(ar[q]), si = wave_sum(ai[q]);
      if (lane == 0) {
        red[wv][2 * q] = sr;
        red[wv][2 * q + 1] = si;
      }
    }
  __syncthreads();
  if (tid < (NORM ? 1 : nv)) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < 4; ++k) {
      sr += red[k][2 * tid];
      si += red[k][2 * tid + 1];
    }
    partial[((long)blockIdx.y * gridDim.x + blk) * kMaxV + tid] = cmk(sr, si);
  }
}

// out[b hstride + q] = the nblk block partials of rhs b = b0 + blockIdx.x added in block order
__global__ void orth_sum_kernel(const C<double>* __restrict__ partial, int nblk, int nv, int b0,
                                C<double>* __restrict__ out, long hstride) {
  const int b = b0 + blockIdx.x, q = threadIdx.x;
  if (q >= nv) return;
  double r = 0.0, i = 0.0;
  for (int k = 0; k < nblk; ++k) {
    const C<double> v = partial[((long)blockIdx.x * nblk + k) * kMaxV + q];
    r += v.re;
    i += v.im;
  }
  out[(long)b * hstride + q] = cmk(r, i);
}

}  // namespace

// sums conj(V_q) . w for q < nv into hout (device), blocking
ls_status multidot(const C<double>* V, long vstride, int nv, const C<double>* w, long len, C<double>* partial,
                   C<double>* hdev, hipStream_t s) {
  const int nblk = 64;
  hipLaunchKernelGGL(multidot_kernel, dim3(nblk, nv), dim3(kRed), 0, s, V, vstride, nv, w, len, nblk, partial);
  LS_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3(blocks_for(nv, 64)), dim3(64), 0, s, partial, nblk, nv, hdev);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status gmres_solve(GmresContext& ctx, const GmresOps& ops, const C<double>* g, C<double>* x, int nrhs,
                      double tol, int restart, int maxit, ls_prec prec, ls_solve_info* info, hipStream_t s) {
  const long len = ctx.len;
  const int m = restart;
  // device workspace: V (m+1) and Z (m) per rhs, temporaries
  const size_t vbytes = (size_t)len * sizeof(C<double>);
  LS_TRY(ctx.V.alloc(vbytes * (size_t)(m + 1) * nrhs));
  LS_TRY(ctx.Z.alloc(vbytes * (size_t)m * nrhs));
  LS_TRY(ctx.W.alloc(vbytes * (size_t)nrhs));
  LS_TRY(ctx.partial.alloc(sizeof(C<double>) *
                           std::max((size_t)64 * (m + 1),
                                    (size_t)kMaxV * kOrthBlk * nrhs)));
  // per rhs: h1, h2 (the two Gram-Schmidt passes) and the norm, m + 1 each
  const size_t hslot = (size_t)3 * (m + 1);
  if (ctx.hdev.bytes < sizeof(C<double>) * hslot * nrhs) LS_TRY(ctx.hdev.alloc(sizeof(C<double>) * hslot * nrhs));
  std::vector<C<double>> hhost(hslot * nrhs);
  C<double>* V = ctx.V.as<C<double>>();
  C<double>* Z = ctx.Z.as<C<double>>();
  C<double>* W = ctx.W.as<C<double>>();
  // vector q of every rhs is contiguous ([q][rhs][len]) so a step can apply the
  // operator to the whole batch in one call
  const long qstride = (long)nrhs * len;
  auto Vp = [&](int b, int q) { return V + q * qstride + (long)b * len; };
  auto Zp = [&](int b, int q) { return Z + q * qstride + (long)b * len; };
  auto Wp = [&](int b) { return W + (long)b * len; };

  // squared norms of nrhs vectors (w(b)) into hslot b, one copy and one wait
  C<double>* hd = ctx.hdev.as<C<double>>();
  auto norms = [&](const std::function<const C<double>*(int)>& w, std::vector<double>& out) -> ls_status {
    for (int b = 0; b < nrhs; ++b)
      LS_TRY(multidot(w(b), len, 1, w(b), len, ctx.partial.as<C<double>>(), hd + (size_t)b * hslot, s));
    LS_HIP(hipMemcpyAsync(hhost.data(), hd, sizeof(C<double>) * hslot * nrhs, hipMemcpyDeviceToHost, s));
    LS_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nrhs; ++b) out[b] = sqrt(fmax(hhost[(size_t)b * hslot].re, 0.0));
    return LS_OK;
  };
  std::vector<double> gnorm(nrhs), rel(nrhs);
  std::vector<int> iters(nrhs, 0), restarts(nrhs, 0);
  std::vector<char> done(nrhs, 0);
  LS_TRY(norms([&](int b) { return g + (long)b * len; }, gnorm));
  for (int b = 0; b < nrhs; ++b) info[b] = ls_solve_info{0, 0, 0.0, 0.0, 0.0};
  LS_HIP(hipMemsetAsync(x, 0, (size_t)nrhs * vbytes, s));
  double t_host = 0.0;
  const double mixed_drop = 1e-4;
  int total = 0;
  while (true) {
    // true residual with the FP64 apply
    LS_TRY(ops.apply(x, W, nrhs, LS_C128, s));
    std::vector<double> beta(nrhs);
    int active = 0;
    for (int b = 0; b < nrhs; ++b) {
      hipLaunchKernelGGL(residual_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, g + (long)b * len, Wp(b), len);
      LS_HIP(hipGetLastError());
    }
    LS_TRY(norms([&](int b) { return (const C<double>*)Wp(b); }, beta));
    for (int b = 0; b < nrhs; ++b) {
      rel[b] = gnorm[b] > 0 ? beta[b] / gnorm[b] : 0.0;
      if (rel[b] <= tol || gnorm[b] == 0.0) done[b] = 1;
      if (!done[b]) ++active;
    }
    if (active == 0 || total >= maxit) break;
    // start a cycle
    std::vector<std::vector<C<double>>> H(nrhs, std::vector<C<double>>((size_t)(m + 1) * m));
    std::vector<std::vector<double>> cs(nrhs, std::vector<double>(m));
    std::vector<std::vector<C<double>>> sn(nrhs, std::vector<C<double>>(m)), e(nrhs, std::vector<C<double>>(m + 1));
    std::vector<char> live(nrhs, 0);
    std::vector<int> jused(nrhs, 0);
    for (int b = 0; b < nrhs; ++b) {
      if (done[b]) continue;
      live[b] = 1;
      hipLaunchKernelGGL(scale_copy_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, Wp(b), 1.0 / beta[b],
                         Vp(b, 0), len);
      LS_HIP(hipGetLastError());
      e[b][0] = cmk(beta[b], 0.0);
    }
    const bool mixed = (prec == LS_MIXED);
    for (int j = 0; j < m && total < maxit; ++j) {
      // gather live rhs: preconditioner and operator on the batch
      std::vector<int> lb;
      for (int b = 0; b < nrhs; ++b)
        if (live[b]) lb.push_back(b);
      if (lb.empty()) break;
      const bool run = lb.back() - lb.front() + 1 == (int)lb.size();   // consecutive rhs: one copy
      if (run)
        LS_HIP(hipMemcpyAsync(Zp(lb.front(), j), Vp(lb.front(), j), vbytes * lb.size(), hipMemcpyDeviceToDevice, s));
      else
        for (int b : lb) LS_HIP(hipMemcpyAsync(Zp(b, j), Vp(b, j), vbytes, hipMemcpyDeviceToDevice, s));
      // preconditioner, in place on Z_j of every live rhs
      {
        double th = 0.0;
        LS_TRY(ops.precond_batch(lb, [&](int b) { return Zp(b, j); }, s, &th));
        t_host += th;
      }
      LS_TRY(ops.apply(Zp(0, j), W, nrhs, mixed ? LS_MIXED : LS_C128, s));
      ++total;
      // classical Gram-Schmidt, two passes, for every live rhs: the
      // coefficients stay on the device for the subtractions; one copy and
      // one wait bring all of them (and the norms) to the host.  Up to kMaxV
      // Krylov vectors the fused passes take each contiguous run of two or
      // more live rhs in one launch per pass; a single rhs keeps the per-vector
      // kernels, whose grids spread one rhs over more blocks (measured 1-5 %
      // faster for the single-rhs solve).
      auto orth_one = [&](int b) -> ls_status {
        C<double>* h1d = hd + (size_t)b * hslot;
        C<double>* h2d = h1d + (m + 1);
        C<double>* hnd = h2d + (m + 1);
        LS_TRY(multidot(Vp(b, 0), qstride, j + 1, Wp(b), len, ctx.partial.as<C<double>>(), h1d, s));
        hipLaunchKernelGGL(subtract_combo_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, Vp(b, 0), qstride,
                           j + 1, (const C<double>*)h1d, Wp(b), len);
        LS_HIP(hipGetLastError());
        LS_TRY(multidot(Vp(b, 0), qstride, j + 1, Wp(b), len, ctx.partial.as<C<double>>(), h2d, s));
        hipLaunchKernelGGL(subtract_combo_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, Vp(b, 0), qstride,
                           j + 1, (const C<double>*)h2d, Wp(b), len);
        LS_HIP(hipGetLastError());
        return multidot(Wp(b), len, 1, Wp(b), len, ctx.partial.as<C<double>>(), hnd, s);
      };
      if (j + 1 <= kMaxV) {
        C<double>* part = ctx.partial.as<C<double>>();
        const int nv = j + 1;
        for (size_t i0 = 0; i0 < lb.size();) {
          size_t i1 = i0 + 1;
          while (i1 < lb.size() && lb[i1] == lb[i1 - 1] + 1) ++i1;
          const int b0 = lb[i0], nb = (int)(i1 - i0), nblk = kOrthBlk;
          if (nb == 1) {
            LS_TRY(orth_one(b0));
            i0 = i1;
            continue;
          }
          const dim3 g(nblk, nb);
          hipLaunchKernelGGL((orth_pass_kernel<false, false>), g, dim3(256), 0, s, V, qstride, nv, W, len, b0,
                             (const C<double>*)nullptr, 0L, part);
          hipLaunchKernelGGL(orth_sum_kernel, dim3(nb), dim3(kMaxV), 0, s, (const C<double>*)part, nblk, nv, b0, hd,
                             (long)hslot);
          hipLaunchKernelGGL((orth_pass_kernel<true, false>), g, dim3(256), 0, s, V, qstride, nv, W, len, b0,
                             (const C<double>*)hd, (long)hslot, part);
          hipLaunchKernelGGL(orth_sum_kernel, dim3(nb), dim3(kMaxV), 0, s, (const C<double>*)part, nblk, nv, b0,
                             hd + (m + 1), (long)hslot);
          hipLaunchKernelGGL((orth_pass_kernel<true, true>), g, dim3(256), 0, s, V, qstride, nv, W, len, b0,
                             (const C<double>*)(hd + (m + 1)), (long)hslot, part);
          hipLaunchKernelGGL(orth_sum_kernel, dim3(nb), dim3(kMaxV), 0, s, (const C<double>*)part, nblk, 1, b0,
                             hd + 2 * (m + 1), (long)hslot);
          LS_HIP(hipGetLastError());
          i0 = i1;
        }
      } else {
        for (int b : lb) LS_TRY(orth_one(b));
      }
      LS_HIP(hipMemcpyAsync(hhost.data(), hd, sizeof(C<double>) * hslot * nrhs, hipMemcpyDeviceToHost, s));
      LS_HIP(hipStreamSynchronize(s));
      for (int b : lb) {
        const C<double>* h1 = hhost.data() + (size_t)b * hslot;
        const C<double>* h2 = h1 + (m + 1);
        const double hn = sqrt(fmax(h2[m + 1].re, 0.0));
        auto& Hb = H[b];
        for (int i = 0; i <= j; ++i) Hb[(size_t)i * m + j] = h1[i] + h2[i];
        Hb[(size_t)(j + 1) * m + j] = cmk(hn, 0.0);
        for (int i = 0; i < j; ++i) {   // earlier rotations
          const C<double> a = Hb[(size_t)i * m + j], c = Hb[(size_t)(i + 1) * m + j];
          Hb[(size_t)i * m + j] = cscale(a, cs[b][i]) + sn[b][i] * c;
          Hb[(size_t)(i + 1) * m + j] = cscale(c, cs[b][i]) - cconj(sn[b][i]) * a;
        }
        const C<double> a = Hb[(size_t)j * m + j], c = Hb[(size_t)(j + 1) * m + j];
        const double aa = sqrt(a.re * a.re + a.im * a.im), cc = sqrt(c.re * c.re + c.im * c.im);
        if (cc == 0.0) {
          cs[b][j] = 1.0;
          sn[b][j] = cmk(0.0, 0.0);
        } else if (aa == 0.0) {
          cs[b][j] = 0.0;
          sn[b][j] = cmk(1.0, 0.0);
        } else {
          const double den = sqrt(aa * aa + cc * cc);
          cs[b][j] = aa / den;
          sn[b][j] = cscale(cmk(a.re / aa, a.im / aa) * cconj(c), 1.0 / den);
        }
        Hb[(size_t)j * m + j] = cscale(a, cs[b][j]) + sn[b][j] * c;
        Hb[(size_t)(j + 1) * m + j] = cmk(0.0, 0.0);
        e[b][j + 1] = cconj(sn[b][j]) * e[b][j];
        e[b][j + 1] = cmk(-e[b][j + 1].re, -e[b][j + 1].im);
        e[b][j] = cscale(e[b][j], cs[b][j]);
        iters[b] += 1;
        jused[b] = j + 1;
        const double est = sqrt(e[b][j + 1].re * e[b][j + 1].re + e[b][j + 1].im * e[b][j + 1].im);
        const bool conv = est <= tol * gnorm[b];
        const bool refine = mixed && est <= mixed_drop * beta[b];
        if (conv || refine || hn == 0.0) {
          live[b] = 0;
        } else if (j + 1 < m) {
          hipLaunchKernelGGL(scale_copy_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, Wp(b), 1.0 / hn,
                             Vp(b, j + 1), len);
          LS_HIP(hipGetLastError());
        }
      }
    }
    // x += Z y for every rhs that ran this cycle
    for (int b = 0; b < nrhs; ++b) {
      const int ju = jused[b];
      if (ju == 0) continue;
      std::vector<C<double>> y(ju);
      for (int i = ju - 1; i >= 0; --i) {
        C<double> acc = e[b][i];
        for (int k2 = i + 1; k2 < ju; ++k2) acc = acc - H[b][(size_t)i * m + k2] * y[k2];
        const C<double> d = H[b][(size_t)i * m + i];
        const double dd = d.re * d.re + d.im * d.im;
        y[i] = dd > 0 ? cscale(acc * cconj(d), 1.0 / dd) : cmk(0.0, 0.0);
      }
      C<double>* yd = hd + (size_t)b * hslot;   // this rhs's own slot: no reuse before the copy lands
      LS_HIP(hipMemcpyAsync(yd, y.data(), ju * sizeof(C<double>), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(add_combo_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, Zp(b, 0), qstride, ju,
                         (const C<double>*)yd, x + (long)b * len, len);
      LS_HIP(hipGetLastError());
      restarts[b] += 1;
    }
  }
  LS_HIP(hipStreamSynchronize(s));
  bool all = true;
  for (int b = 0; b < nrhs; ++b) {
    info[b].iters = iters[b];
    info[b].restarts = restarts[b];
    info[b].rel_resid = rel[b];
    info[b].t_host = t_host / nrhs;
    if (!(rel[b] <= tol)) all = false;
  }
  return all ? LS_OK : LS_ENOCONV;
}

}  // namespace ls
