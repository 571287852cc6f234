// Host-only exercise of the sparse solvers' host code, built with sanitizers
// (AddressSanitizer + UndefinedBehaviorSanitizer, ThreadSanitizer) by
// tests/test_host_sanitizers.py.  Covers the nested dissection (nd_tree.cpp),
// the OpenMP multifrontal factor and its single and block solves
// (host_solver.cpp, complex128 and complex64 factors) and the threaded
// symbolic phase of the GPU factor (gpu_symbolic.cpp), on a 3-D grid with
// three unknowns per point and a 2-D grid with two.
//
// The matrices are seeded random 27-point block stencils with a dominant
// diagonal block, so that every pivot block is well conditioned; each
// solve's residual ||b - S x|| / ||b|| is recomputed from the rows.
// Exit status 0 when every check passes.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "gpu_symbolic.h"
#include "host_solver.h"
#include "nd_tree.h"

using cplx = std::complex<double>;

namespace {

struct Lcg {
  uint64_t s;
  double next() {   // uniform in [-1, 1)
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(s >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
};

// rows [points][nc][27][nc], slots outside the grid left zero
std::vector<cplx> make_rows(const int d[3], int nc, uint64_t seed) {
  const long np = (long)d[0] * d[1] * d[2];
  std::vector<cplx> rows((size_t)np * nc * 27 * nc, cplx(0, 0));
  Lcg g{seed};
  for (long p = 0; p < np; ++p) {
    const int i3 = (int)(p % d[2]), i2 = (int)((p / d[2]) % d[1]), i1 = (int)(p / ((long)d[1] * d[2]));
    for (int s1 = -1; s1 <= 1; ++s1)
      for (int s2 = -1; s2 <= 1; ++s2)
        for (int s3 = -1; s3 <= 1; ++s3) {
          const int j1 = i1 + s1, j2 = i2 + s2, j3 = i3 + s3;
          if (j1 < 0 || j1 >= d[0] || j2 < 0 || j2 >= d[1] || j3 < 0 || j3 >= d[2]) continue;
          const int slot = 9 * (s1 + 1) + 3 * (s2 + 1) + (s3 + 1);
          for (int r = 0; r < nc; ++r)
            for (int c = 0; c < nc; ++c) {
              cplx v(0.1 * g.next(), 0.1 * g.next());
              if (slot == 13 && r == c) v += cplx(4.0, 1.0);
              rows[(size_t)p * nc * 27 * nc + (r * 27 + slot) * nc + c] = v;
            }
        }
  }
  return rows;
}

// y = S x for b-layout vectors [nc][points]
void matvec(const int d[3], int nc, const std::vector<cplx>& rows, const cplx* x, cplx* y) {
  const long np = (long)d[0] * d[1] * d[2];
  for (long p = 0; p < np; ++p) {
    const int i3 = (int)(p % d[2]), i2 = (int)((p / d[2]) % d[1]), i1 = (int)(p / ((long)d[1] * d[2]));
    for (int r = 0; r < nc; ++r) {
      cplx acc(0, 0);
      for (int s1 = -1; s1 <= 1; ++s1)
        for (int s2 = -1; s2 <= 1; ++s2)
          for (int s3 = -1; s3 <= 1; ++s3) {
            const int j1 = i1 + s1, j2 = i2 + s2, j3 = i3 + s3;
            if (j1 < 0 || j1 >= d[0] || j2 < 0 || j2 >= d[1] || j3 < 0 || j3 >= d[2]) continue;
            const long q = ((long)j1 * d[1] + j2) * d[2] + j3;
            const int slot = 9 * (s1 + 1) + 3 * (s2 + 1) + (s3 + 1);
            for (int c = 0; c < nc; ++c) acc += rows[(size_t)p * nc * 27 * nc + (r * 27 + slot) * nc + c] * x[c * np + q];
          }
      y[r * np + p] = acc;
    }
  }
}

int check_solver(const int d[3], int nc, bool fp32, int nrhs, double tol) {
  const long np = (long)d[0] * d[1] * d[2], len = nc * np;
  const std::vector<cplx> rows = make_rows(d, nc, 7 + nrhs);
  ls::HostSolver* hs = nullptr;
  if (ls::host_factor_grid(d, nc, rows.data(), 0, fp32, &hs) != LS_OK) {
    std::printf("factor failed\n");
    return 1;
  }
  Lcg g{99};
  std::vector<cplx> b((size_t)nrhs * len), x;
  for (auto& v : b) v = cplx(g.next(), g.next());
  x = b;
  if (ls::host_solve(hs, x.data(), nrhs) != LS_OK) {
    std::printf("solve failed\n");
    ls::host_free(hs);
    return 1;
  }
  double worst = 0.0;
  std::vector<cplx> y(len);
  for (int r = 0; r < nrhs; ++r) {
    matvec(d, nc, rows, x.data() + (size_t)r * len, y.data());
    double num = 0.0, den = 0.0;
    for (long i = 0; i < len; ++i) {
      num += std::norm(b[(size_t)r * len + i] - y[i]);
      den += std::norm(b[(size_t)r * len + i]);
    }
    worst = std::max(worst, std::sqrt(num / den));
  }
  ls::host_free(hs);
  std::printf("host solver grid %dx%dx%d nc=%d %s nrhs=%d: residual %.2e\n", d[0], d[1], d[2], nc,
              fp32 ? "complex64" : "complex128", nrhs, worst);
  return worst <= tol ? 0 : 1;
}

int check_symbolic(const int d[3], int nc) {
  ls::GpuSymbolic sym;
  if (ls::gpu_symbolic(d, nc, sym) != LS_OK) {
    std::printf("symbolic failed\n");
    return 1;
  }
  // the first N entries are a permutation of the unknowns
  const long N = sym.N;
  std::vector<char> seen(N, 0);
  for (long e = 0; e < N; ++e) {
    const int u = sym.ibh[e];
    if (u < 0 || u >= N || seen[u]) {
      std::printf("elimination order is not a permutation at %ld\n", e);
      return 1;
    }
    seen[u] = 1;
  }
  long piv = 0;
  for (const ls::FrontDev& f : sym.fh) piv += f.np;
  std::printf("symbolic grid %dx%dx%d nc=%d: %zu fronts, %zu levels, %ld factor elements\n", d[0], d[1], d[2], nc,
              sym.fh.size(), sym.levels.size(), sym.fac_elems);
  return (piv == N && sym.fac_elems > 0) ? 0 : 1;
}

}  // namespace

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 9;       // 3-D grid n^3
  const int m = argc > 2 ? std::atoi(argv[2]) : 31;      // 2-D grid m^2
  if (n < 3 || m < 3) return 2;
  const int d3[3] = {n, n, n};
  const int d2[3] = {m, m, 1};
  int bad = 0;
  bad += check_solver(d3, 3, false, 1, 1e-12);
  bad += check_solver(d3, 3, false, 8, 1e-12);
  bad += check_solver(d3, 3, true, 1, 1e-5);
  bad += check_solver(d3, 3, true, 8, 1e-5);
  bad += check_solver(d2, 2, false, 4, 1e-12);
  bad += check_symbolic(d3, 3);
  bad += check_symbolic(d2, 2);
  const int d3b[3] = {12, 10, 7};
  bad += check_symbolic(d3b, 3);
  std::printf(bad ? "FAILED %d\n" : "ALL OK\n", bad);
  return bad ? 1 : 0;
}
