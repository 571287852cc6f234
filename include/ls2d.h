/*
 * ls2d.h - C ABI of the 2-D variant of the sparsifying-preconditioned solver
 * (the paper notes in Section 2 that the scattered-field equation holds in
 * 2-D with the 2-D Helmholtz kernel; Section 3.3 gives the 2-D costs and
 * Section 4 the 2-D examples).
 *
 * Problem: on the unit square with n points per dimension, h = 1/(n+1),
 * nodes x_i = i h, i in {1..n}^2, the field E has two complex components
 * and the operator is the paper's own form in two dimensions:
 *
 *     (A E)^d_i = E^d_i + k^2 sum_j G_ij m_j E^d_j + sum_j G^d_ij (p . E)_j ,
 *
 * G(x) = (i/4) H_0^(1)(k|x|), G^d = dG/dx_d, G_ij = h^2 G(x_i - x_j) and
 * G^d_ij = h^2 G^d(x_i - x_j) for i != j; the self weight of G is its
 * integral over the disc of area h^2, that of G^d is 0; p^d = (dm/dx_d) /
 * (1 - m) with dm/dx_d by central differences (m = 0 off the grid).
 *
 * Layout of every field: interleaved complex, [rhs][component(2)][i1][i2]
 * with i2 fastest; the contrast m is complex128 [i1][i2].  Field and
 * contrast pointers are DEVICE pointers owned by the caller; nothing is
 * retained after a call except what the plan copies.  Calls are ordered on
 * the HIP stream passed in (NULL = the default stream); calls that do host
 * work synchronise it before they return.  Status codes and precisions are
 * those of ls.h.
 */
#ifndef LS2D_H
#define LS2D_H

#include "ls.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ls2_plan ls2_plan;

/* Create a plan for 3 <= n <= 972 (padded FFT length P <= 1944, the
 * smallest even 2^a 3^b >= 2n - 1), wavenumber k > 0 and at most max_rhs
 * right-hand sides per internal launch set (any nrhs is accepted later).
 * Copies m (complex128 [n][n], device), computes p, samples the weights in
 * FP64 on the GPU and transforms their circulant embedding into the symbol
 * (k^2 Ghat, Ghat^1, Ghat^2), kept in FP64 and rounded to FP32.  Workspace:
 * max_rhs * 5 n P complex128.  LS_EINVAL on a bad argument, LS_ENOMEM when
 * the device allocations fail.  Synchronises. */
ls_status ls2_plan_create(int n, double k, int max_rhs, const void* m_dev, void* hip_stream, ls2_plan** out);

/* y = A x for nrhs fields (the discrete equations above, by zero-padded 2-D
 * FFTs: three forward, the 2x3 symbol multiply, two inverse).  x, y: device
 * [nrhs][2][n][n], complex128 for LS_C128 and LS_MIXED, complex64 for LS_C64;
 * x and y must not overlap.  Stream-ordered, no host sync. */
ls_status ls2_apply(ls2_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec, void* hip_stream);

/* ls2_apply for nrhs <= max_rhs, also returning the GPU time of each pass
 * in pass_ms[0..2] (milliseconds; HIP events recorded on hip_stream between
 * the launches): 0 row FFTs with the m and p scaling, 1 column FFTs + 2x3
 * symbol multiply + inverse column FFTs, 2 inverse row FFTs with the
 * identity term.  Synchronises.  For profiling and the roofline report. */
ls_status ls2_apply_timed(ls2_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec, void* hip_stream,
                          double* pass_ms);

/* g = E^i - A E^i (FP64): the right-hand side of the equation for the
 * scattered field when the incident field E^i is given (complex128
 * [nrhs][2][n][n], device).  Stream-ordered. */
ls_status ls2_rhs_from_incident(ls2_plan* plan, const void* Ei_dev, void* g_dev, int nrhs, void* hip_stream);

/* Class stencils on the GPU (Section 3.1, the optimisation for alpha and the
 * formula for beta; Section 3.2 in two dimensions).  Per dimension a point
 * is lo (i_d = 1), in or hi (i_d = n): 9 classes 3 c1 + c2 (4 = interior)
 * with neighbourhood tau (tau_d = {0,1}, {-1,0,1}, {-1,0}; listed with the
 * second offset fastest) and enlarged complement tau^c (offsets in
 * {0..n-1}, {-(n-2)..n-2}, {-(n-1)..0} per dimension, minus the 3 x 3
 * block about 0).  alpha holds the two eigenvectors with the smallest
 * eigenvalues of the Gram matrix M M^H (= the two left singular vectors of
 * M with the smallest singular values), M = [[k^2 G, 0, G^1], [0, k^2 G,
 * G^2]] over tau x tau^c, rows (t, c) -> 2 t + c; beta = B^H alpha with B
 * the same block over tau x tau, rows (t, f) -> 3 t + f (f = 2: the p.E
 * column).  Every point i gets the two rows alpha^H E_tau + beta^H u_tau,
 * u = (m E^1, m E^2, p.E), and Q = alpha^H.  The conjugate transpose is used
 * for the paper's transpose.  Needs n >= 4 (LS_EINVAL).  Synchronises. */
ls_status ls2_stencil_fit(ls2_plan* plan, void* hip_stream);

/* The class stencils of ls2_stencil_fit, host arrays: alpha complex128
 * [9][18][2], beta complex128 [9][27][2] (rows beyond the class's tau are
 * 0), eig [9][18] the Gram eigenvalues ascending (0 past 2 |tau|).
 * LS_ESTATE before a fit. */
ls_status ls2_get_stencils(const ls2_plan* plan, void* alpha_host, void* beta_host, double* eig_host);

/* Factor the sparse system S (rows of the fit) on host cores by nested
 * dissection (Section 3.1 ends with the sparse system solved by nested
 * dissection; Section 3.3 gives its 2-D cost O(N^{3/2})): line separators,
 * dense fronts, partial pivoting inside each front's pivot block.
 * factor_prec LS_C128 or LS_C64 (the factor kept in complex64).  The time
 * taken is written to *seconds_out when not NULL.  LS_ESTATE before a fit. */
ls_status ls2_factor(ls2_plan* plan, ls_prec factor_prec, double* seconds_out);

/* The same factorisation on the GPU (the multifrontal of ls_factor_gpu on
 * the n x n x 1 grid with two unknowns per point): fronts and factor in
 * HBM, pivots searched inside 48-row diagonal tiles (24 whole points);
 * later preconditioner applies solve on the GPU.  factor_prec LS_C128 or
 * LS_C64.  LS_ESTATE before a fit, LS_ENOMEM when HBM is short.
 * Synchronises hip_stream. */
ls_status ls2_factor_gpu(ls2_plan* plan, ls_prec factor_prec, void* hip_stream, double* seconds_out);

/* z = S^-1 (Q v) for nrhs fields (device, complex128 [nrhs][2][n][n]; z may
 * equal v): Q v on the GPU, S^-1 by the latest factor (on the GPU after
 * ls2_factor_gpu, on host cores over PCIe after ls2_factor).  LS_ESTATE
 * before a factorisation.  Synchronises. */
ls_status ls2_precond_apply(ls2_plan* plan, const void* v_dev, void* z_dev, int nrhs, void* hip_stream);

/* Right-preconditioned FGMRES for A x = g, as ls_gmres_solve (restart,
 * maxit, tol on ||g - A x|| / ||g|| with the FP64 apply, x0 = 0, a lockstep
 * block of nrhs right-hand sides; apply_prec LS_C128 or LS_MIXED).  g, x:
 * device complex128 [nrhs][2][n][n]; info: host array of nrhs records.
 * LS_ESTATE before a factorisation, LS_ENOCONV when maxit is reached. */
ls_status ls2_gmres_solve(ls2_plan* plan, const void* g_dev, void* x_dev, int nrhs, double tol, int restart,
                          int maxit, ls_prec apply_prec, ls_solve_info* info, void* hip_stream);

/* Padded FFT length of the plan. */
int ls2_plan_fft_size(const ls2_plan* plan);

void ls2_plan_destroy(ls2_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* LS2D_H */
