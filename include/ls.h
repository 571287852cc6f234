/*
 * ls.h - C ABI of the MI355X (gfx950) sparsifying-preconditioned solver for the
 * time-harmonic Maxwell volume integral equation (Liu & Ying, "Sparsifying
 * preconditioner for the time-harmonic Maxwell's equations").
 *
 * Problem (Section 2, Eq. (4) and Eq. (5)): on the unit cube with n points per
 * dimension, h = 1/(n+1), nodes x_i = i h, i in {1..n}^3, find the scattered
 * field E (3 complex components per node) with
 *
 *     (A E)_i = E_i + sum_j K(i - j) m_j E_j = g_i ,
 *
 * K(r) = h^3 (k^2 I + grad grad) G(h r) for r != 0, G(x) = exp(ik|x|)/(4 pi |x|),
 * and K(0) = {(2/3)[(1 - ika) e^{ika} - 1] - 1/3} I with a = h (3/(4 pi))^(1/3)
 * (equal-volume-ball self term; the paper's own near-diagonal correction is
 * not specified).  This is the dyadic form of Eq. (4): the same continuum
 * equation, with grad grad G in place of the grad G * (p . E) term.
 *
 * Memory layout of every field: interleaved complex (re, im), index
 * [rhs][component][i1][i2][i3] with i3 fastest; the contrast m is
 * complex128 [i1][i2][i3].  All field and contrast pointers are DEVICE
 * pointers owned by the caller; nothing is retained after a call returns
 * except what a plan copies into its own workspace.  Calls are ordered on the
 * HIP stream passed in (NULL = the default stream); the calls that do host
 * work synchronise that stream before they return.
 *
 * Every call returns an ls_status.  On an error the outputs are unspecified,
 * except LS_ENOCONV, where x holds the last iterate and info is filled.
 */
#ifndef LS_H
#define LS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ls_plan ls_plan;

typedef enum {
  LS_OK = 0,
  LS_EINVAL = -1,   /* bad argument: NULL pointer, n < 3, nrhs < 1 or > max_rhs, ... */
  LS_ENOMEM = -2,   /* device or host allocation failed                              */
  LS_EHIP = -3,     /* a HIP runtime call failed                                     */
  LS_ENOCONV = -4,  /* FGMRES reached maxit before the residual met tol              */
  LS_EHOST = -5,    /* the host factorisation would exceed the plan's memory cap     */
  LS_ESTATE = -6,   /* call out of order (e.g. a solve before ls_stencil_fit)        */
  LS_EIO = -7       /* a weights file could not be read or has the wrong format      */
} ls_status;

/* Arithmetic of the operator apply.  Krylov vectors, orthogonalisation and
 * residual recomputation are always complex128. */
typedef enum {
  LS_C128 = 0,      /* complex128 in, complex128 out, FFTs in FP64                    */
  LS_C64 = 1,       /* complex64 in, complex64 out, FFTs in FP32                      */
  LS_MIXED = 2      /* complex128 in/out, the convolution K*(m x) in FP32; the
                       identity term is added in FP64                                 */
} ls_prec;

typedef struct {
  int n;                 /* grid points per dimension, 3 <= n <= 384                   */
  double k;              /* background wavenumber k > 0                                */
  int max_rhs;           /* largest nrhs any later call will pass (>= 1)              */
  size_t host_mem_cap;   /* bytes the host factorisation may use; 0 = no cap           */
  const char* tune_cache;/* autotuner cache file (JSON), or NULL                       */
} ls_plan_desc;

/* Create a plan: validates the descriptor, copies m (complex128, n^3, device)
 * into the plan, samples the Nystrom weights K(r) in FP64 on the GPU and
 * transforms their circulant embedding (Section 2: the Toeplitz matrices are
 * applied by FFT) into the symbol Khat, kept in FP64 and rounded to FP32.
 * *out receives the plan; destroy it with ls_plan_destroy. */
ls_status ls_plan_create(const ls_plan_desc* desc, const void* m_dev, void* hip_stream,
                         ls_plan** out);

/* Nystrom apply (Eq. (5), Eq. (6)):  y = x + K * (m x)  for nrhs fields.
 * x, y: device [nrhs][3][n][n][n], element type set by prec (complex128 for
 * LS_C128 and LS_MIXED, complex64 for LS_C64).  x == y (in place) is allowed;
 * otherwise x and y must not overlap.  Stream-ordered, no host sync. */
ls_status ls_apply(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                   void* hip_stream);

/* ls_apply, also returning the GPU time of each of the five FFT passes in
 * pass_ms[0..4] (milliseconds, summed over internal rhs chunks), measured with
 * HIP events recorded on hip_stream between the passes: 0 dim-1 forward with
 * the m scaling, 1 dim-2 forward, 2 dim-3 forward + 3x3 symbol multiply +
 * dim-3 inverse, 3 dim-2 inverse, 4 dim-1 inverse with the identity term.
 * Synchronises hip_stream.  For profiling and the roofline report. */
ls_status ls_apply_timed(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                         void* hip_stream, double* pass_ms);

/* Right-hand side of the scattered-field equation (Eq. (4)):
 * g = -K * (m E^i) = E^i - A E^i, complex128, computed with the FP64 apply.
 * Ei, g: device [nrhs][3][n][n][n] complex128. */
ls_status ls_rhs_from_incident(ls_plan* plan, const void* Ei_dev, void* g_dev, int nrhs,
                               void* hip_stream);

/* Padded FFT length P used by the plan (P >= 2n - 1, even, 2^a 3^b). */
int ls_plan_fft_size(const ls_plan* plan);

void ls_plan_destroy(ls_plan* plan);
const char* ls_status_string(ls_status s);

#ifdef __cplusplus
}
#endif
#endif /* LS_H */
