// The 2-D variant of the method: plan, apply, stencils and preconditioner.
#pragma once

#include <complex>
#include <vector>

#include "../../include/ls2d.h"
#include "common.h"
#include "gmres.h"

namespace ls {

struct HostSolver;
struct GpuSolver;

constexpr int kMaxP2 = 1944;       // largest padded FFT length of the 2-D apply (n <= 972)

struct Radices {                   // FFT stages: three bits each (0: radix 4, 1: 2, 2: 3, 3: 8, 4: 9)
  unsigned long long code = 0;
  int nst = 0;
};

struct Plan2 {
  int n = 0, P = 0, H = 0, max_rhs = 1;
  double k = 0.0, h = 0.0;
  Radices rd;
  DevBuf m64, m32;                 // contrast [n][n]
  DevBuf p64, p32;                 // p^d, [2][n][n]
  DevBuf sym64, sym32;             // symbol quadrant / P^2, [H][H][3]
  DevBuf symc64, symc32;           // the same column-major, [3][H (q2)][H (q1)]
  DevBuf tw64, tw32;               // exp(-2 pi i t / P)
  DevBuf work;                     // pass intermediates, max_rhs x 5 x n x P
  // stencils (class fit) and the sparse system
  bool fitted = false;
  std::vector<std::complex<double>> alpha;   // [9][18][2]  (rows 2 t + c of tau, columns r)
  std::vector<std::complex<double>> beta;    // [9][27][2]  (rows 3 t + f)
  std::vector<double> eig;                   // [9][18] Gram eigenvalues, ascending
  DevBuf alpha_dev;                // the class stencils on the device (Q v is formed from them)
  DevBuf srows;                    // S rows [n^2][2 rows][27 slots][2 comps] complex128 (slots s3 = 0 used)
  HostSolver* hs = nullptr;        // factor of S on host cores, or
  GpuSolver* gs = nullptr;         // factor of S in HBM
  GmresContext gctx;
  DevBuf pbuf;                     // preconditioner staging
  ~Plan2();
};

int fft_size_2d(int n);
ls_status plan2_init(Plan2& pl, int n, double k, int max_rhs, const void* m_dev, hipStream_t s);
// ev, when given, holds 4 events recorded around the three passes (nrhs <= max_rhs).
ls_status plan2_apply(Plan2& pl, const void* x, void* y, int nrhs, ls_prec prec, hipStream_t s, bool minus_conv,
                      hipEvent_t* ev = nullptr);

}  // namespace ls
