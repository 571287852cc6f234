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
  int n;                 /* grid points per dimension, 3 <= n <= 192 (FFT length <= 384) */
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

/* Launch choices of the batched apply (block right-hand sides; the FFT of
 * Section 2 applied to many incident fields at once).  Results never depend
 * on them: every choice computes the same operations in the same order. */
typedef struct {
  int chunk;                  /* right-hand sides per launch set, 1..max_rhs            */
  int kmul_w;                 /* pass-3 teams per workgroup (1, 2 or 4)                 */
  double ms_per_rhs;          /* measured GPU ms per rhs of the chosen choice           */
  double ms_default_per_rhs;  /* the same for the built-in default (0 on a cache hit)   */
  int from_cache;             /* 1: read from desc.tune_cache, nothing was timed        */
  int n_tried;                /* choices timed                                          */
  int half_runs;              /* bit i: strided pass i (dim-1 forward, dim-2 forward,
                                 dim-2 inverse, dim-1 inverse) reads and writes rows in
                                 128-byte runs (its FFT tile halved) instead of 256     */
  int persist;                /* persistent launches (grids of the resident
                                 workgroups, which stride over the work items):
                                 bit 0 the four strided passes, bit 1 pass 3            */
} ls_tune_info;

/* Autotune the apply of prec for batches of nrhs: look the key (GPU, n, P,
 * form, prec, nrhs, max_rhs) up in the plan's tune_cache file; on a miss time the
 * choices on the plan's operator (scratch fields of nrhs, allocated and freed
 * here): every chunk x team count, then each strided pass with half runs in
 * turn (kept where faster), then persistent launches of the strided passes, of
 * pass 3 and of both; keep the fastest and
 * append it to the cache file (a JSON array, one object per line; rewritten
 * through a temporary file).  The choice then holds
 * for every later apply and solve of that precision.  A cache that cannot be
 * written is not an error.  The choices are those of the dyadic form:
 * LS_ESTATE while the plan's form is LS_FORM_PAPER, whose apply has a single
 * launch choice.  Synchronises hip_stream.  info may be NULL. */
ls_status ls_plan_tune(ls_plan* plan, int nrhs, ls_prec prec, void* hip_stream, ls_tune_info* info);

/* Set the launch choice of prec by hand (chunk 0 / kmul_w 0 = default;
 * half_runs and persist as in ls_tune_info, 0 = default).  LS_EINVAL for
 * chunk > max_rhs, kmul_w not in {0, 1, 2, 4}, half_runs outside 0..15 or
 * persist outside 0..3. */
ls_status ls_plan_set_tune(ls_plan* plan, ls_prec prec, int chunk, int kmul_w, int half_runs, int persist);

/* ls_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result as ls_apply, with the pass intermediates in a
 * fixed 128 MiB device array that the library holds on every GPU it runs
 * on, instead of the plan's workspace.  No allocation of any kind happens in
 * the call.  One rhs needs 3 (P n^2 + P^2 n) complex values of 8 (LS_C64,
 * LS_MIXED) or 16 (LS_C128) bytes, P the plan's FFT length; larger batches
 * run in chunks that fit, and nrhs is not limited by max_rhs.  LS_ENOMEM
 * when one rhs needs more than 128 MiB (e.g. n = 96 in complex128, n = 128
 * in complex64); LS_ESTATE in the paper's form.  All calls on one GPU share
 * the array: calls that overlap in time on the same GPU race and give
 * undefined results.  Stream-ordered, like ls_apply. */
ls_status ls_apply_noalloc(ls_plan* plan, const void* x_dev, void* y_dev, int nrhs, ls_prec prec,
                           void* hip_stream);

/* Right-hand side of the scattered-field equation (Eq. (4)):
 * g = -K * (m E^i) = E^i - A E^i, complex128, computed with the FP64 apply.
 * Ei, g: device [nrhs][3][n][n][n] complex128. */
ls_status ls_rhs_from_incident(ls_plan* plan, const void* Ei_dev, void* g_dev, int nrhs,
                               void* hip_stream);

/* ---- sparsifying preconditioner (Section 3) ------------------------------- */

typedef enum {
  LS_FIT_CLASS = 0,     /* the paper's fit: one stencil per position class     */
  LS_FIT_POINT = 1      /* medium-dependent per-point fit (project extension):
                           interior points minimise sum_j w_j^2 |alpha^H K_{tau,j}|^2
                           with w_j = 1 + |m_{i+j}| / 0.1 on the 5^3 shell around i
                           and w_j = 1 beyond; boundary points keep the class fit */
} ls_fit_mode;

typedef struct {
  int iters;             /* FGMRES iterations (operator applications)          */
  int restarts;          /* Arnoldi cycles                                      */
  double rel_resid;      /* final ||g - A x|| / ||g|| with the FP64 apply      */
  double t_gpu, t_host;  /* seconds: whole solve on the GPU side / host solves  */
} ls_solve_info;

/* Stencil fit and row assembly on the GPU (Section 3.1, Eqs. (10)-(12);
 * Section 3.2).  LS_FIT_CLASS: for each of the 27 position classes (interior,
 * 6 faces, 12 edges, 8 vertices) with neighbourhood tau and enlarged
 * complement tau^c, alpha holds the three eigenvectors of the Gram matrix
 * M M^H, M = [K(a - j)]_{a in tau, j in tau^c}, with the smallest eigenvalues
 * (= the left singular vectors of M with the smallest singular values),
 * beta = B^H alpha with B = [K(a - b)]_{a, b in tau}, and every point i gets
 * the three rows alpha^H E_tau + beta^H diag(m)_tau E_tau of Eq. (11).
 * The conjugate transpose is used for the paper's transpose.  Synchronises. */
ls_status ls_stencil_fit(ls_plan* plan, ls_fit_mode mode, void* hip_stream);

/* Copies of the fit to host memory (for inspection and tests).
 * alpha_host, beta_host: [27][81][3] complex128, row 3 a + c for neighbour a
 * (tau order: lexicographic offsets, last dimension fastest) and component c;
 * a class with |tau| < 27 fills the first 3|tau| rows, the rest are zero.
 * eig_host: [27][3] the three smallest Gram eigenvalues; gram_host:
 * [27][81][81] complex128, the class Gram matrices M M^H (row-major, first
 * 3|tau| rows and columns used).  Any pointer may be NULL.  LS_ESTATE before
 * ls_stencil_fit. */
ls_status ls_get_class_stencils(const ls_plan* plan, void* alpha_host, void* beta_host, double* eig_host,
                                void* gram_host);

/* Per-point stencils after LS_FIT_POINT: alpha_host [n^3][81][3] complex128
 * (interior points: the medium-weighted fit; others: their class stencil in
 * the first 3|tau| rows); eig_host [n^3][3] (the three smallest eigenvalues
 * of each interior point's weighted Gram, zero elsewhere).  Either may be
 * NULL.  LS_ESTATE unless the last fit was LS_FIT_POINT. */
ls_status ls_get_point_stencils(const ls_plan* plan, void* alpha_host, double* eig_host);

/* The assembled rows S to host memory: [n^3][3 rows][27 slots][3 comps]
 * complex128, slot 9 (s1+1) + 3 (s2+1) + (s3+1) for the neighbour at offset
 * s; slots outside the grid are zero.  LS_ESTATE before ls_stencil_fit. */
ls_status ls_get_rows(const ls_plan* plan, void* rows_host);

/* Nested-dissection multifrontal LU of S on the host cores (the paper's
 * sparse direct solve; Section 3.3).  Copies the rows from the GPU.
 * LS_EHOST if the factor would exceed desc->host_mem_cap.  seconds_out may be
 * NULL.  LS_ESTATE before ls_stencil_fit. */
ls_status ls_factor(ls_plan* plan, double* seconds_out);

/* ls_factor with the factor's precision: LS_C128 keeps it in complex128
 * (what ls_factor does); LS_C64 (or LS_MIXED, the same) in complex64, half the
 * host memory and about twice as fast to factor and to solve.  A complex64
 * factor is an inexact S^-1; the flexible GMRES still reaches its tolerance
 * on the FP64 residual, possibly with more iterations.  Errors as ls_factor. */
ls_status ls_factor_prec(ls_plan* plan, ls_prec factor_prec, double* seconds_out);

/* Nested-dissection multifrontal LU of S on the GPU (the paper's sparse
 * direct solve, Section 3.3, with every front in device memory): the same
 * dissection as ls_factor, pivots chosen by magnitude within 48-row tiles of
 * each front's pivot block (a whole number of points' three unknowns; on the
 * tested media this picks the pivots of ls_factor), Schur complements on the
 * matrix cores.  factor_prec LS_C128: complex128 factor; LS_C64 or
 * LS_MIXED: complex64.  Replaces any earlier factor of the plan; from then
 * on ls_precond_apply and ls_gmres_solve apply S^-1 on the GPU.  Device
 * memory: about 8 (complex64) or 16 (complex128) bytes per factor entry, plus
 * two levels of fronts while factoring.  LS_ENOMEM if it does not fit.
 * seconds_out may be NULL.  LS_ESTATE before ls_stencil_fit.  Synchronises. */
ls_status ls_factor_gpu(ls_plan* plan, ls_prec factor_prec, void* hip_stream, double* seconds_out);

/* Preconditioner z = S^-1 (Q v): Q v on the GPU, S^-1 on the host (after
 * ls_factor / ls_factor_prec) or on the GPU (after ls_factor_gpu).
 * v, z: device [nrhs][3][n][n][n] complex128 (may alias).  Synchronises.
 * LS_ESTATE before a factorisation. */
ls_status ls_precond_apply(ls_plan* plan, const void* v_dev, void* z_dev, int nrhs, void* hip_stream);

/* Right-preconditioned FGMRES (restart `restart`, at most `maxit` operator
 * applications per rhs) for A x = g, x0 = 0, until ||g - A x|| <= tol ||g||
 * with the FP64 apply.  apply_prec: LS_C128, or LS_MIXED (FP32 FFTs inside
 * the FP64 Krylov loop, with FP64 true-residual restarts).  g, x: device
 * [nrhs][3][n][n][n] complex128; info: host array of nrhs records.
 * LS_ENOCONV when maxit is reached (x holds the last iterate).  LS_ESTATE
 * before a factorisation (ls_factor, ls_factor_prec or ls_factor_gpu).
 * Synchronises. */
ls_status ls_gmres_solve(ls_plan* plan, const void* g_dev, void* x_dev, int nrhs, double tol, int restart,
                         int maxit, ls_prec apply_prec, ls_solve_info* info, void* hip_stream);

/* ---- learned stencils (project extension) ----------------------------------
 * A network predicts each interior point's medium-dependent stencil from the
 * 5^3 patch of m around it (x = Re, Im of m / 0.3, 250 inputs, last dimension
 * fastest, zero off the grid): 250 -> 256 GELU -> 256 GELU -> 468, GELU(x) =
 * x Phi(x).  The 468 outputs are the 26 off-centre 3x3 blocks [block][c][r]
 * (re, im interleaved) of (alpha~_i - alpha~_class) / 3e-3, alpha~ = alpha
 * (alpha_centre)^-1 (the scale brings the corrections to unit size).
 * Parameters: flat float32 W1[250][256] b1[256] W2[256][256] b2[256]
 * W3[256][468] b3[468] (250324 values, y = x W + b).  Products use BF16
 * operands with FP32 accumulation on MFMA; Adam (0.9, 0.999, 1e-8) updates
 * FP32 masters.  The network lives on the device current at creation. */
typedef struct ls_mlp ls_mlp;

#define LS_MLP_NPARAM 250324

ls_status ls_mlp_create(const float* params_host, ls_mlp** out);
ls_status ls_mlp_get_params(const ls_mlp* mlp, float* params_host);
/* One forward + backward pass on host data: x_host [B][250], t_host [B][468]
 * (float32); y_host [B][468] outputs, grad_host [LS_MLP_NPARAM] the gradient of
 * mean((y - t)^2), loss_out the loss.  Outputs may be NULL.  Synchronises. */
ls_status ls_mlp_forward_backward(ls_mlp* mlp, const float* x_host, const float* t_host, int B, float* y_host,
                                  float* grad_host, double* loss_out, void* hip_stream);
/* The network's inference on host data: x_host [B][250] (float32, rounded to
 * BF16 as the features are), y_host [B][468] outputs.  The same evaluation the
 * learned fit makes (ls_stencil_fit_learned): the three layers fused per tile
 * of rows; it agrees with the forward pass of ls_mlp_forward_backward to FP32
 * rounding (the order of the sums differs).  Synchronises. */
ls_status ls_mlp_forward(ls_mlp* mlp, const float* x_host, int B, float* y_host, void* hip_stream);
/* One Adam step (learning rate lr > 0) with the gradient of the last backward
 * pass; LS_ESTATE before any backward pass (ls_mlp_forward_backward or
 * ls_mlp_train). */
ls_status ls_mlp_adam_step(ls_mlp* mlp, double lr, void* hip_stream);
/* Exact per-point fits (LS_FIT_POINT definition) at the listed interior points
 * (linear indices (i1 n + i2) n + i3) of the plan's medium become training
 * samples: input = the 5^3 patch of m, target = the gauge-fixed stencil
 * alpha (alpha_centre)^-1 minus the interior class's, over a fixed scale.  A
 * point whose centre block has Frobenius condition number above 1e6 (gauge
 * undefined) is skipped; ls_mlp_num_samples tells how many were kept.
 * LS_EINVAL for a boundary point.  Synchronises. */
ls_status ls_mlp_add_samples(ls_mlp* mlp, ls_plan* plan, const int* points_host, int npts, void* hip_stream);
long ls_mlp_num_samples(const ls_mlp* mlp);
/* Copies of the samples: x_host [N][256] float32 (the BF16 features, zero
 * padded), t_host [N][468] float32 targets.  Either may be NULL. */
ls_status ls_mlp_get_samples(const ls_mlp* mlp, float* x_host, float* t_host);
/* `steps` Adam steps on minibatches of `batch` samples (a seeded permutation
 * per epoch); loss_out (may be NULL) receives the loss of every step. */
ls_status ls_mlp_train(ls_mlp* mlp, int steps, int batch, double lr, unsigned seed, double* loss_out,
                       void* hip_stream);
/* Checkpoint: a JSON header line, then float32 parameters, Adam m and v. */
ls_status ls_mlp_save(const ls_mlp* mlp, const char* path);
ls_status ls_mlp_load(const char* path, ls_mlp** out);
void ls_mlp_destroy(ls_mlp* mlp);

/* Learned fit: every interior point gets the network's stencil when its
 * locality tr(Q^H Gram_i Q) (Q an orthonormal basis of it, Gram_i the
 * medium-weighted Gram of LS_FIT_POINT) is below the class stencil's by more
 * than a relative 1e-9;
 * otherwise the exact per-point fit.  Boundary points keep the class fit.
 * n_fallback_out (may be NULL): the number of points that fell back.  Then
 * assembles the rows, like ls_stencil_fit.  Synchronises. */
ls_status ls_stencil_fit_learned(ls_plan* plan, ls_mlp* mlp, int* n_fallback_out, void* hip_stream);

/* Outcome of the last learned fit, per grid point (host arrays of n^3 entries,
 * linear index (i1 n + i2) n + i3): accept_host 1 where the prediction was
 * accepted, 0 where the point fell back to the exact per-point fit, -1 at
 * boundary points (no prediction); ratio_host the locality ratio
 * tr(Q^H Gram_i Q) / tr(alpha_c^H Gram_i alpha_c) of the prediction (0 at
 * boundary points).  Either pointer may be NULL.  LS_ESTATE unless the last
 * fit of the plan was ls_stencil_fit_learned. */
ls_status ls_get_learned_info(const ls_plan* plan, int* accept_host, double* ratio_host);

/* ---- the sparse solver on its own (host or GPU factor) --------------------- */
typedef struct ls_sparse ls_sparse;

/* Factor rows given in the ls_get_rows layout on an n^3 grid; factor_prec as
 * in ls_factor_prec (solves take and return complex128 either way). */
ls_status ls_sparse_factor_host(int n, const void* rows_host, size_t host_mem_cap, ls_prec factor_prec,
                                ls_sparse** out);
/* Solve S x = b in place, b host [nrhs][3][n][n][n] complex128. */
ls_status ls_sparse_solve_host(ls_sparse* sp, void* b_host, int nrhs);
/* The same factorisation on the GPU (as ls_factor_gpu): rows_host in the
 * ls_get_rows layout, copied to the device; 3 <= n <= 192. */
ls_status ls_sparse_factor_gpu(int n, const void* rows_host, ls_prec factor_prec, void* hip_stream, ls_sparse** out);
/* Solve S x = b in place on the GPU, b device [nrhs][3][n][n][n] complex128,
 * stream-ordered.  LS_ESTATE for a host-factored ls_sparse (and
 * ls_sparse_solve_host returns LS_ESTATE for a GPU-factored one). */
ls_status ls_sparse_solve_gpu(ls_sparse* sp, void* b_dev, int nrhs, void* hip_stream);
/* Factor size in bytes and factorisation flop count. */
ls_status ls_sparse_info(const ls_sparse* sp, size_t* bytes, double* flops);
void ls_sparse_destroy(ls_sparse* sp);

/* Measurement helper: a streaming device-to-device copy of `bytes` bytes
 * (dst and src device pointers, 16-byte aligned, not overlapping), the
 * achievable HBM bandwidth against which the apply's passes are read.
 * Stream-ordered; LS_EINVAL for a NULL or misaligned pointer. */
ls_status ls_hbm_copy(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream);

/* Operator form of the plan's apply (ls_apply, ls_apply_timed,
 * ls_rhs_from_incident and the FGMRES solves). */
typedef enum {
  LS_FORM_DYADIC = 0,  /* y = x + K*(m x), K = (k^2 I + grad grad) G (the default) */
  LS_FORM_PAPER = 1    /* the paper's own form (Section 2, the discrete equations):
                          y_d = x_d + k^2 G*(m x_d) + G^d*(p.x), p^d = (dm/dx_d)/(1 - m),
                          G^d = dG/dx_d; self weights: the integral of G over the ball of
                          volume h^3, 0 for G^d; dm/dx_d by central differences with m = 0
                          outside the grid */
} ls_form;

/* Select the operator form.  The first selection of LS_FORM_PAPER builds its
 * symbol (four FP64 FFTs of P^3), p and a workspace of about 4/3 the dyadic
 * one; LS_ENOMEM if that does not fit.  The stencils, S and its factor stay
 * those of the dyadic fit (a preconditioner for either form).  LS_EINVAL for
 * an unknown form.  Stream-ordered. */
ls_status ls_plan_set_form(ls_plan* plan, ls_form form, void* hip_stream);

/* Padded FFT length P used by the plan (P >= 2n - 1, even, 2^a 3^b). */
int ls_plan_fft_size(const ls_plan* plan);

void ls_plan_destroy(ls_plan* plan);
const char* ls_status_string(ls_status s);

#ifdef __cplusplus
}
#endif
#endif /* LS_H */
