// Local stencils alpha, beta and the sparse rows S, Q on gfx950.
//
// Paper: Section 3.1 (rows alpha^H E_tau + beta^H diag(m)_tau E_tau = alpha^H g_tau,
// Eq. (11); beta = B^H alpha, Eq. (12); alpha = the three left singular
// vectors of the non-local block M with the smallest singular values) and
// Section 3.2 (the stencils depend only on the position class of a point;
// 27 classes with enlarged complements).  The conjugate transpose is used
// for the paper's transpose (the literal transpose has no SVD solution).
//
//   gram_partial_kernel : split-K symmetric product X X^T of the realified
//                         non-local block X = [Re M; Im M], on FP64 MFMA
//                         (v_mfma_f64_16x16x4); M's columns K(a - j) are
//                         evaluated on the fly from the closed form.
//   gram_sum_kernel     : sums the partial tiles in 16 chunks (coalesced).
//   gram_reduce_kernel  : sums the chunks, forms the complex Gram M M^H.
//   heev_low3_kernel    : three smallest eigenvectors of the Hermitian Gram by
//                         Cholesky + block inverse iteration (8 vectors) +
//                         Rayleigh-Ritz with a cyclic Jacobi on the 8x8 block.
//   beta_kernel         : beta = B^H alpha.
//   assemble_rows_kernel: S rows per point, slots indexed by neighbour offset.
//   qapply_kernel       : z = Q v, a 27-point 3x3-block stencil.
#include "common.h"
#include "kernel_eval.h"
#include "stencil.h"

namespace ls {

// ---- class geometry -----------------------------------------------------------
ClassGeom class_geom(int kappa, int n) {
  ClassGeom g{};
  g.cd[0] = kappa / 9;
  g.cd[1] = (kappa / 3) % 3;
  g.cd[2] = kappa % 3;
  int t1[3], n1[3];
  for (int d = 0; d < 3; ++d) {
    switch (g.cd[d]) {
      case CLS_LO: g.rlo[d] = 0; g.rlen[d] = n; t1[d] = 0; n1[d] = 2; break;
      case CLS_IN: g.rlo[d] = -(n - 2); g.rlen[d] = 2 * n - 3; t1[d] = -1; n1[d] = 3; break;
      default: g.rlo[d] = -(n - 1); g.rlen[d] = n; t1[d] = -1; n1[d] = 2; break;
    }
    g.tlo[d] = t1[d];
    g.tlen[d] = n1[d];
  }
  int c = 0;
  for (int a = 0; a < n1[0]; ++a)
    for (int b = 0; b < n1[1]; ++b)
      for (int e = 0; e < n1[2]; ++e) {
        g.tau[c][0] = t1[0] + a;
        g.tau[c][1] = t1[1] + b;
        g.tau[c][2] = t1[2] + e;
        ++c;
      }
  g.ntau = c;
  g.nbox = (long)g.rlen[0] * g.rlen[1] * g.rlen[2];
  return g;
}

__host__ __device__ inline int class_dim(int i, int n) { return i == 0 ? CLS_LO : (i == n - 1 ? CLS_HI : CLS_IN); }

// ---- Gram: split-K realified symmetric product on FP64 MFMA -------------------
// Operand layout of v_mfma_f64_16x16x4f64 (wave64): A lane l holds A[l % 16][l / 16],
// B lane l holds B[l / 16][l % 16]; the 16x16 result holds D[4 r + l / 16][l % 16]
// in register r of lane l (checked on gfx950 with an in-bounds probe).
constexpr int GJC = 16;            // complement points per chunk
constexpr int GKC = 3 * GJC;       // columns of X per chunk

template <int NT>
__global__ __launch_bounds__(256) void gram_partial_kernel(ClassGeom g, double k, double h,
                                                           long chunks_per_wg, double* __restrict__ partial) {
  constexpr int RP = NT * 16;
  constexpr int LDR = RP + 2;                       // padded LDS row
  constexpr int NTILE = NT * (NT + 1) / 2;
  constexpr int TPW = (NTILE + 3) / 4;
  __shared__ double X[GKC * LDR];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int R = 3 * g.ntau;

  int ti[TPW], tj[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    int tile = wave + 4 * t, I = 0;
    if (tile >= NTILE) tile = -1;
    int rem = tile;
    while (rem >= 0 && rem >= NT - I) {
      rem -= NT - I;
      ++I;
    }
    ti[t] = tile < 0 ? -1 : I;
    tj[t] = tile < 0 ? -1 : I + rem;
  }
  typedef double v4d __attribute__((ext_vector_type(4)));
  v4d acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};

  for (int e = tid; e < GKC * LDR; e += 256) X[e] = 0.0;   // padding rows stay zero
  __syncthreads();

  const long c0 = (long)blockIdx.x * chunks_per_wg;
  for (long ch = c0; ch < c0 + chunks_per_wg; ++ch) {
    const long jbase = ch * GJC;
    if (jbase >= g.nbox) break;
    for (int idx = tid; idx < g.ntau * GJC; idx += 256) {
      const int a = idx / GJC, jj = idx % GJC;
      const long jl = jbase + jj;
      C<double> Kv[6];
      bool valid = jl < g.nbox;
      int j0 = 0, j1 = 0, j2 = 0;
      if (valid) {
        j2 = g.rlo[2] + (int)(jl % g.rlen[2]);
        j1 = g.rlo[1] + (int)((jl / g.rlen[2]) % g.rlen[1]);
        j0 = g.rlo[0] + (int)(jl / ((long)g.rlen[2] * g.rlen[1]));
        const bool in_tau = (j0 >= g.tlo[0] && j0 < g.tlo[0] + g.tlen[0]) &&
                            (j1 >= g.tlo[1] && j1 < g.tlo[1] + g.tlen[1]) &&
                            (j2 >= g.tlo[2] && j2 < g.tlo[2] + g.tlen[2]);
        valid = !in_tau;
      }
      if (valid) {
        dyadic_K(g.tau[a][0] - j0, g.tau[a][1] - j1, g.tau[a][2] - j2, k, h, Kv);
      } else {
#pragma unroll
        for (int q = 0; q < 6; ++q) Kv[q] = cmk(0.0, 0.0);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const C<double> v = Kv[sym_index(c, e)];
          X[(3 * jj + e) * LDR + 3 * a + c] = v.re;
          X[(3 * jj + e) * LDR + R + 3 * a + c] = v.im;
        }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GKC; kk += 4) {
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        if (ti[t] >= 0) {
          const double av = X[kr * LDR + ti[t] * 16 + (lane & 15)];
          const double bv = X[kr * LDR + tj[t] * 16 + (lane & 15)];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  double* out = partial + (long)blockIdx.x * NTILE * 256;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if (ti[t] >= 0) {
      int tile = 0;
      for (int I = 0; I < ti[t]; ++I) tile += NT - I;
      tile += tj[t] - ti[t];
#pragma unroll
      for (int r = 0; r < 4; ++r) out[tile * 256 + (4 * r + (lane >> 4)) * 16 + (lane & 15)] = acc[t][r];
    }
  }
}

// A[x][y] of the realified product from the summed upper tiles.
__device__ inline double gram_real_entry(const double* __restrict__ partial, int nwg, int NT, int x, int y) {
  if (x / 16 > y / 16) {
    const int t = x;
    x = y;
    y = t;
  }
  const int I = x / 16, J = y / 16;
  int tile = 0;
  for (int q = 0; q < I; ++q) tile += NT - q;
  tile += J - I;
  const int NTILE = NT * (NT + 1) / 2;
  const long off = (long)tile * 256 + (x % 16) * 16 + (y % 16);
  double s = 0.0;
  for (int w = 0; w < nwg; ++w) s += partial[(long)w * NTILE * 256 + off];
  return s;
}

// First stage of the tile reduction: part2[c][e] = sum over the workgroups w
// of chunk c of partial[w][e], e < len (len = tiles x 256), kGramChunks
// chunks; the result has the partial layout with kGramChunks "workgroups".
constexpr int kGramChunks = 16;
__global__ void gram_sum_kernel(const double* __restrict__ partial, int nwg, long len, double* __restrict__ part2) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const int per = (nwg + kGramChunks - 1) / kGramChunks;
  const int w0 = blockIdx.y * per, w1 = min(nwg, w0 + per);
  double acc = 0.0;
  for (int w = w0; w < w1; ++w) acc += partial[(long)w * len + e];
  part2[(long)blockIdx.y * len + e] = acc;
}

__global__ void gram_reduce_kernel(const double* __restrict__ partial, int nwg, int NT, int R,
                                   C<double>* __restrict__ G) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= R * R) return;
  const int u = id / R, v = id % R;
  const double re = gram_real_entry(partial, nwg, NT, u, v) + gram_real_entry(partial, nwg, NT, R + u, R + v);
  const double im = gram_real_entry(partial, nwg, NT, R + u, v) - gram_real_entry(partial, nwg, NT, u, R + v);
  G[u * 81 + v] = cmk(re, im);   // row stride 81 for every class
}

// ---- smallest three eigenvectors of a Hermitian positive (semi)definite matrix ----
constexpr int EB = 8;          // block size of the inverse iteration
constexpr int EITER = 20;      // iterations from a cold start

// Cyclic Jacobi on an 8x8 Hermitian matrix (one thread): T -> V^H T V diagonal.
__device__ inline void jacobi8(C<double> (*T)[EB], C<double> (*V)[EB]) {
  for (int i = 0; i < EB; ++i)
    for (int j = 0; j < EB; ++j) V[i][j] = cmk(i == j ? 1.0 : 0.0, 0.0);
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < EB; ++i) {
      dia += T[i][i].re * T[i][i].re;
      for (int j = i + 1; j < EB; ++j) off += T[i][j].re * T[i][j].re + T[i][j].im * T[i][j].im;
    }
    if (off <= 1e-34 * dia) break;
    for (int p = 0; p < EB; ++p)
      for (int q = p + 1; q < EB; ++q) {
        const C<double> apq = T[p][q];
        const double ab = sqrt(apq.re * apq.re + apq.im * apq.im);
        if (ab == 0.0) continue;
        const C<double> ph = cmk(apq.re / ab, apq.im / ab);          // e^{i phi}
        const double app = T[p][p].re, aqq = T[q][q].re;
        const double tau = (aqq - app) / (2.0 * ab);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        // rotation J: columns p, q:  p' = c p - s conj(ph) q ,  q' = s ph p + c q
        for (int i = 0; i < EB; ++i) {
          const C<double> tp = T[i][p], tq = T[i][q];
          T[i][p] = cscale(tp, c) - cscale(cconj(ph) * tq, s);
          T[i][q] = cscale(ph * tp, s) + cscale(tq, c);
        }
        for (int j = 0; j < EB; ++j) {
          const C<double> tp = T[p][j], tq = T[q][j];
          T[p][j] = cscale(tp, c) - cscale(ph * tq, s);
          T[q][j] = cscale(cconj(ph) * tp, s) + cscale(tq, c);
        }
        T[p][q] = cmk(0.0, 0.0);
        T[q][p] = cmk(0.0, 0.0);
        T[p][p].im = 0.0;
        T[q][q].im = 0.0;
        for (int i = 0; i < EB; ++i) {
          const C<double> vp = V[i][p], vq = V[i][q];
          V[i][p] = cscale(vp, c) - cscale(cconj(ph) * vq, s);
          V[i][q] = cscale(ph * vp, s) + cscale(vq, c);
        }
      }
  }
}

// One workgroup (256 threads) per matrix.  G: R x R row-major (R <= 81).
// Writes alpha (R x 3, column-major per vector: alpha[(row) * 3 + v]) and the
// three smallest Ritz values.
__global__ __launch_bounds__(256) void heev_low3_kernel(const C<double>* __restrict__ Gall, const int* __restrict__ Rs,
                                                        long gstride, C<double>* __restrict__ alpha_all,
                                                        long astride, double* __restrict__ evals,
                                                        C<double>* __restrict__ ritz8) {
  constexpr int RMAX = 81;
  __shared__ C<double> L[RMAX * (RMAX + 1) / 2];
  __shared__ C<double> Xb[RMAX][EB];
  __shared__ C<double> Yk[EB];
  __shared__ C<double> T[EB][EB];
  __shared__ C<double> V[EB][EB];
  __shared__ double shift;
  const int mat = blockIdx.x;
  const int R = Rs[mat];
  const C<double>* G = Gall + mat * gstride;
  const int tid = threadIdx.x;
  auto LI = [](int i, int j) { return i * (i + 1) / 2 + j; };

  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < R; ++i) tr += G[i * 81 + i].re;
    shift = 1e-15 * tr;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, j = e % R;
    if (j <= i) {
      C<double> v = G[i * 81 + j];
      if (i == j) v = cmk(v.re + shift, 0.0);
      L[LI(i, j)] = v;
    }
  }
  __syncthreads();
  // Cholesky G + shift I = L L^H, in place
  for (int kk = 0; kk < R; ++kk) {
    if (tid == 0) L[LI(kk, kk)] = cmk(sqrt(fmax(L[LI(kk, kk)].re, 1e-300)), 0.0);
    __syncthreads();
    const double dinv = 1.0 / L[LI(kk, kk)].re;
    for (int i = kk + 1 + tid; i < R; i += 256) L[LI(i, kk)] = cscale(L[LI(i, kk)], dinv);
    __syncthreads();
    const int m = R - kk - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int i = kk + 1 + e / m, j = kk + 1 + e % m;
      if (j <= i) L[LI(i, j)] = L[LI(i, j)] - L[LI(i, kk)] * cconj(L[LI(j, kk)]);
    }
    __syncthreads();
  }
  // deterministic start block
  for (int e = tid; e < R * EB; e += 256) {
    const int i = e / EB, c = e % EB;
    unsigned hsh = (unsigned)(i * 7919 + c * 104729 + 12345);
    hsh ^= hsh >> 13;
    hsh *= 0x5bd1e995u;
    hsh ^= hsh >> 15;
    const double a = ((hsh & 0xffff) / 65536.0) - 0.5, b = (((hsh >> 16) & 0xffff) / 65536.0) - 0.5;
    Xb[i][c] = cmk(a + (i == c ? 1.0 : 0.0), b);
  }
  __syncthreads();
  for (int it = 0; it < EITER; ++it) {
    // forward solve L Y = X (in place)
    for (int kk = 0; kk < R; ++kk) {
      if (tid < EB) Yk[tid] = cscale(Xb[kk][tid], 1.0 / L[LI(kk, kk)].re);
      __syncthreads();
      if (tid < EB) Xb[kk][tid] = Yk[tid];
      for (int e = tid; e < (R - kk - 1) * EB; e += 256) {
        const int i = kk + 1 + e / EB, c = e % EB;
        Xb[i][c] = Xb[i][c] - L[LI(i, kk)] * Yk[c];
      }
      __syncthreads();
    }
    // backward solve L^H Z = Y (in place)
    for (int kk = R - 1; kk >= 0; --kk) {
      if (tid < EB) Yk[tid] = cscale(Xb[kk][tid], 1.0 / L[LI(kk, kk)].re);
      __syncthreads();
      if (tid < EB) Xb[kk][tid] = Yk[tid];
      for (int e = tid; e < kk * EB; e += 256) {
        const int i = e / EB, c = e % EB;
        Xb[i][c] = Xb[i][c] - cconj(L[LI(kk, i)]) * Yk[c];
      }
      __syncthreads();
    }
    // modified Gram-Schmidt, twice
    for (int pass = 0; pass < 2; ++pass) {
      for (int c = 0; c < EB; ++c) {
        if (tid < 64) {
          double nr = 0.0;
          for (int i = tid; i < R; i += 64) nr += Xb[i][c].re * Xb[i][c].re + Xb[i][c].im * Xb[i][c].im;
          for (int o = 32; o > 0; o >>= 1) nr += __shfl_xor(nr, o);
          if (tid == 0) Yk[0] = cmk(1.0 / sqrt(nr), 0.0);
        }
        __syncthreads();
        for (int i = tid; i < R; i += 256) Xb[i][c] = cscale(Xb[i][c], Yk[0].re);
        __syncthreads();
        // project column c out of columns d > c
        const int w = tid >> 6, l = tid & 63;
        for (int d = c + 1 + w; d < EB; d += 4) {
          double pr = 0.0, pi = 0.0;
          for (int i = l; i < R; i += 64) {
            const C<double> a = Xb[i][c], b = Xb[i][d];      // conj(a) b
            pr += a.re * b.re + a.im * b.im;
            pi += a.re * b.im - a.im * b.re;
          }
          for (int o = 32; o > 0; o >>= 1) {
            pr += __shfl_xor(pr, o);
            pi += __shfl_xor(pi, o);
          }
          const C<double> pc = cmk(pr, pi);
          for (int i = l; i < R; i += 64) Xb[i][d] = Xb[i][d] - Xb[i][c] * pc;
        }
        __syncthreads();
      }
    }
  }
  // Rayleigh-Ritz with the unshifted matrix: T = X^H G X
  for (int e = tid; e < EB * EB; e += 256) {
    const int p = e / EB, q = e % EB;
    C<double> s = cmk(0.0, 0.0);
    for (int i = 0; i < R; ++i) {
      C<double> gx = cmk(0.0, 0.0);
      for (int j = 0; j < R; ++j) gx = gx + G[i * 81 + j] * Xb[j][q];
      s = s + cconj(Xb[i][p]) * gx;
    }
    T[p][q] = s;
  }
  __syncthreads();
  if (tid == 0) {
    for (int p = 0; p < EB; ++p)
      for (int q = p + 1; q < EB; ++q) {   // exact Hermitian symmetrisation
        const C<double> a = T[p][q], b = cconj(T[q][p]);
        T[p][q] = cmk(0.5 * (a.re + b.re), 0.5 * (a.im + b.im));
        T[q][p] = cconj(T[p][q]);
      }
    jacobi8(T, V);
    // selection sort of the Ritz values: keep order in Yk as indices
    int idx[EB];
    for (int p = 0; p < EB; ++p) idx[p] = p;
    for (int p = 0; p < EB; ++p)
      for (int q = p + 1; q < EB; ++q)
        if (T[idx[q]][idx[q]].re < T[idx[p]][idx[p]].re) {
          const int t = idx[p];
          idx[p] = idx[q];
          idx[q] = t;
        }
    for (int v = 0; v < EB; ++v) Yk[v] = cmk((double)idx[v], 0.0);
    for (int v = 0; v < 3; ++v) evals[mat * 3 + v] = T[idx[v]][idx[v]].re;
  }
  __syncthreads();
  C<double>* alpha = alpha_all + mat * astride;
  for (int e = tid; e < R * 3; e += 256) {
    const int i = e / 3, v = e % 3;
    const int col = (int)Yk[v].re;
    C<double> s = cmk(0.0, 0.0);
    for (int q = 0; q < EB; ++q) s = s + Xb[i][q] * V[q][col];
    alpha[i * 3 + v] = s;
  }
  // all eight Ritz vectors in ascending order (warm start of the per-point fit)
  C<double>* r8 = ritz8 + (long)mat * 81 * EB;
  for (int e = tid; e < R * EB; e += 256) {
    const int i = e / EB, v = e % EB;
    const int col = (int)Yk[v].re;
    C<double> s = cmk(0.0, 0.0);
    for (int q = 0; q < EB; ++q) s = s + Xb[i][q] * V[q][col];
    r8[i * EB + v] = s;
  }
}

// beta = B^H alpha with B[(a,c),(b,c')] = K_{c c'}(tau_a - tau_b)
__global__ void beta_kernel(const ClassGeom* __restrict__ geoms, double k, double h,
                            const C<double>* __restrict__ alpha_all, C<double>* __restrict__ beta_all,
                            long astride) {
  const ClassGeom& g = geoms[blockIdx.x];
  const C<double>* alpha = alpha_all + blockIdx.x * astride;
  C<double>* beta = beta_all + blockIdx.x * astride;
  const int R = 3 * g.ntau;
  for (int e = threadIdx.x; e < R * 3; e += blockDim.x) {
    const int row = e / 3, v = e % 3;
    const int b = row / 3, cp = row % 3;
    C<double> s = cmk(0.0, 0.0);
    for (int a = 0; a < g.ntau; ++a) {
      C<double> Kv[6];
      dyadic_K(g.tau[a][0] - g.tau[b][0], g.tau[a][1] - g.tau[b][1], g.tau[a][2] - g.tau[b][2], k, h, Kv);
      for (int c = 0; c < 3; ++c) s = s + cconj(Kv[sym_index(c, cp)]) * alpha[(3 * a + c) * 3 + v];
    }
    beta[row * 3 + v] = s;
  }
}

// ---- rows ---------------------------------------------------------------------
// Slot of a neighbour offset s in {-1,0,1}^3: 9 (s1+1) + 3 (s2+1) + (s3+1).
// S[i][r][slot][c] = conj(alpha[(a,c), r]) + conj(beta[(a,c), r]) m_{i+a};
// alpha/beta per class (pstride = 0) or per point (pstride = 81*3).
__global__ void assemble_rows_kernel(int n, const C<double>* __restrict__ m, const ClassGeom* __restrict__ geoms,
                                     const C<double>* __restrict__ alpha, const C<double>* __restrict__ beta,
                                     long cstride, long pstride, C<double>* __restrict__ S) {
  const long n3 = (long)n * n * n;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n3) return;
  const int i3 = (int)(id % n), i2 = (int)((id / n) % n), i1 = (int)(id / ((long)n * n));
  const int kappa = 9 * class_dim(i1, n) + 3 * class_dim(i2, n) + class_dim(i3, n);
  const ClassGeom& g = geoms[kappa];
  const C<double>* al = alpha + (pstride ? id * pstride : kappa * cstride);
  const C<double>* be = beta + (pstride ? id * pstride : kappa * cstride);
  C<double>* out = S + id * 243;
  for (int e = 0; e < 243; ++e) out[e] = cmk(0.0, 0.0);
  for (int a = 0; a < g.ntau; ++a) {
    const int s1 = g.tau[a][0], s2 = g.tau[a][1], s3 = g.tau[a][2];
    const int slot = 9 * (s1 + 1) + 3 * (s2 + 1) + (s3 + 1);
    const C<double> mj = m[((long)(i1 + s1) * n + (i2 + s2)) * n + (i3 + s3)];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const C<double> av = cconj(al[(3 * a + c) * 3 + r]);
        const C<double> bv = cconj(be[(3 * a + c) * 3 + r]);
        out[(r * 27 + slot) * 3 + c] = av + bv * mj;
      }
  }
}

// z = Q v: z_r(i) = sum_{a in tau(i)} sum_c conj(alpha[(a,c), r]) v_c(i + a).  Fields [rhs][3][n^3].
// A thread takes one point and RB right-hand sides, so that each 3 x 3 block
// of the point's coefficients is read once per RB rhs: per-point stencils
// hold 243 coefficients (3.9 KB) for every point, and one thread per (point,
// rhs) read them once per rhs (17 ms for 64 rhs at n = 64 against 2.7 ms
// with the 27 shared class stencils; 5.3 ms with eight rhs per thread).  Per
// (point, rhs, r) the sum runs over (a, c) in the same order for every RB.
template <int RB>
__global__ __launch_bounds__(256) void qapply_kernel(int n, int nrhs, const ClassGeom* __restrict__ geoms,
                                                     const C<double>* __restrict__ alpha, long cstride, long pstride,
                                                     const C<double>* __restrict__ v, C<double>* __restrict__ z) {
  const long n3 = (long)n * n * n;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nchunk = (nrhs + RB - 1) / RB;
  if (id >= n3 * nchunk) return;
  const long p = id % n3;
  const int b0 = (int)(id / n3) * RB;
  const int i3 = (int)(p % n), i2 = (int)((p / n) % n), i1 = (int)(p / ((long)n * n));
  const int kappa = 9 * class_dim(i1, n) + 3 * class_dim(i2, n) + class_dim(i3, n);
  const ClassGeom& g = geoms[kappa];
  const C<double>* al = alpha + (pstride ? p * pstride : kappa * cstride);
  C<double> acc[RB][3];
#pragma unroll
  for (int j = 0; j < RB; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) acc[j][r] = cmk(0.0, 0.0);
  for (int a = 0; a < g.ntau; ++a) {
    const long q = ((long)(i1 + g.tau[a][0]) * n + (i2 + g.tau[a][1])) * n + (i3 + g.tau[a][2]);
    C<double> w[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 3; ++r) w[c][r] = cconj(al[(3 * a + c) * 3 + r]);
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      if (RB > 1 && b0 + j >= nrhs) break;
      const C<double>* vb = v + (long)(b0 + j) * 3 * n3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const C<double> vv = vb[c * n3 + q];
#pragma unroll
        for (int r = 0; r < 3; ++r) acc[j][r] = acc[j][r] + w[c][r] * vv;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    if (RB > 1 && b0 + j >= nrhs) break;
#pragma unroll
    for (int r = 0; r < 3; ++r) z[(long)(b0 + j) * 3 * n3 + r * n3 + p] = acc[j][r];
  }
}

// ---- host driver ------------------------------------------------------------------
template <int NT>
static ls_status launch_gram(const ClassGeom& g, double k, double h, double* partial, int nwg, hipStream_t s) {
  const long nchunks = (g.nbox + GJC - 1) / GJC;
  const long per = (nchunks + nwg - 1) / nwg;
  hipLaunchKernelGGL((gram_partial_kernel<NT>), dim3(nwg), dim3(256), 0, s, g, k, h, per, partial);
  return hipGetLastError() == hipSuccess ? LS_OK : LS_EHIP;
}

ls_status class_fit(StencilData& sd, int n, double k, hipStream_t s) {
  const double h = 1.0 / (n + 1);
  std::vector<ClassGeom> geoms(27);
  std::vector<int> Rs(27);
  for (int kap = 0; kap < 27; ++kap) {
    geoms[kap] = class_geom(kap, n);
    Rs[kap] = 3 * geoms[kap].ntau;
  }
  LS_TRY(sd.geoms.alloc(27 * sizeof(ClassGeom)));
  LS_HIP(hipMemcpyAsync(sd.geoms.p, geoms.data(), 27 * sizeof(ClassGeom), hipMemcpyHostToDevice, s));
  LS_TRY(sd.gram.alloc(27L * 81 * 81 * sizeof(C<double>)));
  LS_TRY(sd.alpha.alloc(27L * 81 * 3 * sizeof(C<double>)));
  LS_TRY(sd.beta.alloc(27L * 81 * 3 * sizeof(C<double>)));
  LS_TRY(sd.evals.alloc(27L * 3 * sizeof(double)));
  LS_TRY(sd.ritz8.alloc(27L * 81 * 8 * sizeof(C<double>)));
  LS_HIP(hipMemsetAsync(sd.ritz8.p, 0, sd.ritz8.bytes, s));
  DevBuf dR;
  LS_TRY(dR.alloc(27 * sizeof(int)));
  LS_HIP(hipMemcpyAsync(dR.p, Rs.data(), 27 * sizeof(int), hipMemcpyHostToDevice, s));
  LS_HIP(hipMemsetAsync(sd.alpha.p, 0, sd.alpha.bytes, s));
  LS_HIP(hipMemsetAsync(sd.beta.p, 0, sd.beta.bytes, s));
  LS_HIP(hipMemsetAsync(sd.gram.p, 0, sd.gram.bytes, s));
  const int nwg_max = 512;
  DevBuf partial, part2;
  LS_TRY(partial.alloc((size_t)nwg_max * 66 * 256 * sizeof(double)));
  LS_TRY(part2.alloc((size_t)kGramChunks * 66 * 256 * sizeof(double)));
  for (int kap = 0; kap < 27; ++kap) {
    const ClassGeom& g = geoms[kap];
    const long nchunks = (g.nbox + GJC - 1) / GJC;
    const int nwg = (int)(nchunks < nwg_max ? nchunks : nwg_max);
    const int NT = (2 * Rs[kap] + 15) / 16;
    ls_status st;
    switch (NT) {
      case 11: st = launch_gram<11>(g, k, h, partial.as<double>(), nwg, s); break;
      case 7: st = launch_gram<7>(g, k, h, partial.as<double>(), nwg, s); break;
      case 5: st = launch_gram<5>(g, k, h, partial.as<double>(), nwg, s); break;
      case 3: st = launch_gram<3>(g, k, h, partial.as<double>(), nwg, s); break;
      default: return LS_EINVAL;
    }
    LS_TRY(st);
    // the per-workgroup count in the launch equals ceil(nchunks / nwg); every
    // workgroup index < nwg wrote its tiles
    const int R = Rs[kap];
    const long len = (long)NT * (NT + 1) / 2 * 256;
    hipLaunchKernelGGL(gram_sum_kernel, dim3((unsigned)((len + 255) / 256), kGramChunks), dim3(256), 0, s,
                       partial.as<double>(), nwg, len, part2.as<double>());
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((R * R + 255) / 256), dim3(256), 0, s, part2.as<double>(),
                       kGramChunks, NT, R, sd.gram.as<C<double>>() + (long)kap * 81 * 81);
    LS_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(heev_low3_kernel, dim3(27), dim3(256), 0, s, sd.gram.as<C<double>>(), dR.as<int>(),
                     81L * 81, sd.alpha.as<C<double>>(), 81L * 3, sd.evals.as<double>(), sd.ritz8.as<C<double>>());
  LS_HIP(hipGetLastError());
  hipLaunchKernelGGL(beta_kernel, dim3(27), dim3(256), 0, s, sd.geoms.as<ClassGeom>(), k, h,
                     sd.alpha.as<C<double>>(), sd.beta.as<C<double>>(), 81L * 3);
  LS_HIP(hipGetLastError());
  LS_HIP(hipStreamSynchronize(s));
  sd.have_class = true;
  return LS_OK;
}

ls_status assemble_rows(StencilData& sd, int n, const C<double>* m, hipStream_t s) {
  const long n3 = (long)n * n * n;
  LS_TRY(sd.rows.alloc((size_t)n3 * 243 * sizeof(C<double>)));
  const bool pp = sd.have_point;
  hipLaunchKernelGGL(assemble_rows_kernel, dim3((unsigned)((n3 + 127) / 128)), dim3(128), 0, s, n, m,
                     sd.geoms.as<ClassGeom>(), pp ? sd.palpha.as<C<double>>() : sd.alpha.as<C<double>>(),
                     pp ? sd.pbeta.as<C<double>>() : sd.beta.as<C<double>>(), 81L * 3, pp ? 81L * 3 : 0L,
                     sd.rows.as<C<double>>());
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status q_apply(const StencilData& sd, int n, const C<double>* v, C<double>* z, int nrhs, hipStream_t s) {
  const long n3 = (long)n * n * n;
  const bool pp = sd.have_point;
  const C<double>* al = pp ? sd.palpha.as<C<double>>() : sd.alpha.as<C<double>>();
  const long ps = pp ? 81L * 3 : 0L;
  // the 27 class stencils stay in cache: one (point, rhs) per thread, eight
  // waves per SIMD (taking eight rhs per thread there measured 3.4 against
  // 2.7 ms for 64 rhs at n = 64)
  if (pp && nrhs >= 8)
    hipLaunchKernelGGL(qapply_kernel<8>, dim3((unsigned)((n3 * ((nrhs + 7) / 8) + 255) / 256)), dim3(256), 0, s, n,
                       nrhs, sd.geoms.as<ClassGeom>(), al, 81L * 3, ps, v, z);
  else if (pp && nrhs >= 4)
    hipLaunchKernelGGL(qapply_kernel<4>, dim3((unsigned)((n3 * ((nrhs + 3) / 4) + 255) / 256)), dim3(256), 0, s, n,
                       nrhs, sd.geoms.as<ClassGeom>(), al, 81L * 3, ps, v, z);
  else
    hipLaunchKernelGGL(qapply_kernel<1>, dim3((unsigned)((n3 * nrhs + 255) / 256)), dim3(256), 0, s, n, nrhs,
                       sd.geoms.as<ClassGeom>(), al, 81L * 3, ps, v, z);
  return hipGetLastError() == hipSuccess ? LS_OK : LS_EHIP;
}

}  // namespace ls
