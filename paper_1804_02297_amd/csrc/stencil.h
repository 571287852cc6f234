// Stencil data owned by a plan, and the class geometry of Section 3.2.
#pragma once

#include "common.h"

namespace ls {

enum { CLS_LO = 0, CLS_IN = 1, CLS_HI = 2 };

// Position class kappa = 9 c1 + 3 c2 + c3 (c_d in {lo, in, hi}); tau in
// lexicographic order with the last dimension fastest; the enlarged
// complement is the box [rlo, rlo + rlen) per dimension minus tau.
struct ClassGeom {
  int cd[3];
  int ntau;
  int tau[27][3];
  int tlo[3], tlen[3];
  int rlo[3], rlen[3];
  long nbox;
};

ClassGeom class_geom(int kappa, int n);

struct StencilData {
  DevBuf geoms;                  // 27 ClassGeom
  DevBuf gram;                   // 27 x 81 x 81 complex128 (class Gram M M^H)
  DevBuf alpha, beta;            // 27 x 81 x 3 complex128 (rows (a, c), column v)
  DevBuf evals;                  // 27 x 3: three smallest eigenvalues of each Gram
  DevBuf ritz8;                  // 27 x 81 x 8: the eight lowest Ritz vectors of each Gram
  DevBuf palpha, pbeta;          // per-point stencils n^3 x 81 x 3 (medium-dependent modes)
  DevBuf peval;                  // n^3 x 3: per-point smallest eigenvalues (0 where unset)
  DevBuf rows;                   // S rows: n^3 x [3 rows][27 slots][3 comps] complex128
  bool have_class = false;
  bool have_point = false;
  bool have_rows = false;
  // outcome of the last learned fit, per grid point (host): 1 the prediction was
  // accepted, 0 the point fell back to the exact fit, -1 a boundary point; the
  // locality ratio of the prediction (0 at boundary points)
  std::vector<int> learned_accept;
  std::vector<double> learned_ratio;
  bool have_learned = false;
};

ls_status class_fit(StencilData& sd, int n, double k, hipStream_t s);
ls_status assemble_rows(StencilData& sd, int n, const C<double>* m, hipStream_t s);
ls_status q_apply(const StencilData& sd, int n, const C<double>* v, C<double>* z, int nrhs, hipStream_t s);

}  // namespace ls
