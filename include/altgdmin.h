/*
 * altgdmin.h -- C ABI of the MI355X (gfx950) altGDmin library.
 *
 * The library reconstructs a dynamic MRI sequence Z (n x q, n = nx*ny pixels,
 * q frames) as a rank-r product U B from undersampled multi-coil Cartesian
 * k-space, with the alternating GD-minimisation of the paper (Algorithm 2,
 * "auto-altGDmin", Sec. III-B) at a fixed rank r:
 *
 *   init:  gamma = trunc_c * sum |y|^2 / (m q),   m = max_k m_k,
 *          X_0 = [A_k^H (y_k o 1{|y_k| <= sqrt(gamma)}) / sqrt(m_k mbar)]_k,
 *          U_0 = top-r left singular vectors of X_0;
 *   loop:  b_k = (A_k U)^dagger y_k,   x_k = U b_k,
 *          grad = sum_k A_k^H (A_k U b_k - y_k) b_k^H,
 *          eta  = eta_c / ||grad||_2   (first iteration only),
 *          U    = Q of QR(U - eta grad).
 *
 * The measurement operator is the multi-coil model of Sec. II-A:
 *   y_{k,c} = H_k F (s_c o z_k),  A_k = [H_k F D_1; ...; H_k F D_nc],
 * with F the unitary 2D DFT (1/sqrt(n) both ways; natural index order, DC at
 * index 0, no fftshift) and H_k the 0/1 selector of frame k's samples.
 *
 * Conventions
 * -----------
 *  - Complex data are interleaved single precision (float2: re, im).
 *  - Pixel index p = x + nx*y (x, the readout direction, fastest); k-space
 *    index ky*nx + kx likewise.
 *  - U is n x r column-major (U[j*n + p]); B is r x q column-major
 *    (B[k*r + j], so b_k is contiguous); X is n x q column-major.
 *  - Coil maps are nc x n: coils[c*n + p].
 *  - y is the padded "long" form of eq. Ymat: y[(k*nc + c)*m_max + i] for
 *    i < m_k, zero (output) or ignored (input) for m_k <= i < m_max.
 *  - Masks.  ALTGDMIN_MASK_LINES (1D Cartesian, every sampled phase-encode
 *    line complete along kx): mask is int32 [q][m_max/nx], mask[k][l] = ky of
 *    frame k's l-th line for l < m_k/nx; y is ordered [k][c][l][kx].
 *    ALTGDMIN_MASK_INDEX (any Cartesian-grid sampling, e.g. pseudo-radial
 *    spokes rounded onto the grid, Sec. V): mask is int32 [q][m_max],
 *    mask[k][i] = ky*nx + kx for i < m_k; entries must be distinct within a
 *    frame.  m_k is int32 [q], the number of samples per coil in frame k
 *    (a multiple of nx for LINES).
 *
 * Ownership and execution
 * -----------------------
 *  - Every pointer named d_* is device memory owned by the caller.  The
 *    library never allocates or frees device memory and never synchronises
 *    the device except where stated; it keeps host-side state and pointers
 *    into one caller-provided workspace (size from altgdmin_workspace_bytes).
 *  - Inputs bound by altgdmin_set_problem must stay alive and unchanged
 *    until altgdmin_destroy or the next altgdmin_set_problem.
 *  - Every call enqueues asynchronously on the stream given to
 *    altgdmin_set_problem; results are valid once that stream has
 *    synchronised.  Calls that synchronise the stream: altgdmin_get_stats,
 *    altgdmin_last_error, altgdmin_iterate when h_iters_done is non-NULL,
 *    altgdmin_get_eta, altgdmin_kernel_time.
 *  - A context is not thread-safe; separate contexts are independent.
 *
 * Errors
 * ------
 *  Every function returns an altgdmin_status (0 = OK) and never aborts,
 *  prints or throws.  Argument errors are found before any launch
 *  (ALTGDMIN_EINVAL); calls out of order give ALTGDMIN_ESTATE; HIP runtime
 *  errors give ALTGDMIN_EHIP.  Conditions found on the device (a per-frame
 *  Gram or a QR Gram that is not positive definite, a non-finite value) set
 *  a device flag; after that the remaining kernels of the call do nothing,
 *  and the next synchronising call returns ALTGDMIN_ENOTPD or
 *  ALTGDMIN_ENONFINITE (altgdmin_last_error also gives the frame index).
 */
#ifndef ALTGDMIN_H
#define ALTGDMIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ALTGDMIN_OK = 0,
  ALTGDMIN_EINVAL = 1,      /* bad argument (shape, pointer, value)        */
  ALTGDMIN_ESTATE = 2,      /* call out of order (e.g. iterate before init) */
  ALTGDMIN_EHIP = 3,        /* a HIP runtime call failed                    */
  ALTGDMIN_ENOTPD = 4,      /* a Gram matrix was not positive definite      */
  ALTGDMIN_ENONFINITE = 5,  /* a NaN or Inf appeared                         */
  ALTGDMIN_EUNSUPPORTED = 6, /* valid but not supported by this library      */
  ALTGDMIN_ESCRATCH = 7      /* problem too large for the built-in scratch     */
} altgdmin_status;

enum { ALTGDMIN_MASK_LINES = 0, ALTGDMIN_MASK_INDEX = 1 };
enum { ALTGDMIN_FP32 = 0, ALTGDMIN_MIXED = 1 };

/* Problem shape and Algorithm 2's constants.
 *  nx, ny      image size; each a power of two in [8, 512].
 *  nc          coils, 1..64.        q   frames, 1..128.
 *  r           rank, 1..16.
 *  m_max       padded samples per coil per frame (max_k m_k).
 *  mask_kind   ALTGDMIN_MASK_LINES or ALTGDMIN_MASK_INDEX.
 *  precision   ALTGDMIN_FP32 (every step in FP32) or ALTGDMIN_MIXED (the
 *              per-frame r x r Gram/Cholesky and the Gram of U's QR in FP64;
 *              everything else FP32).
 *  trunc_c     truncation constant (paper: 36); <= 0 disables truncation.
 *  eta_c       step-size constant (paper: 0.14).
 *  eta_cap_c   > 0: eta = min(eta_c/||grad_0||, eta_cap_c*n/(mbar*||B_0||^2)),
 *              the conservative rule eta = c/(m ||U_0 B_0||^2) of Sec. III-B
 *              expressed for a unitary F; 0 disables the cap.
 *  eps_exit    > 0: stop when SD(U, U+)/sqrt(r) < eps_exit (paper: 0.01);
 *              <= 0: run the requested number of iterations.
 *  t_max       iteration cap used by altgdmin_iterate when n_iter <= 0.
 *  exit_consec the exit rule fires after this many consecutive iterations
 *              with SD(U, U+)/sqrt(r) < eps_exit (0 or 1: Algorithm 2's rule;
 *              more: the more robust variant suggested in Sec. VI).
 *  r may exceed q for a context used only for the LS step, the operators and
 *  the steps around the loop (e.g. per-frame online tracking); the spectral
 *  initialisation needs r <= q.
 */
typedef struct {
  int32_t nx, ny, nc, q, r, m_max, mask_kind, precision;
  double trunc_c, eta_c, eta_cap_c, eps_exit;
  int32_t t_max;
  int32_t exit_consec;
} altgdmin_params;

/* Per-iteration statistics of the last completed iteration. */
typedef struct {
  int32_t t;            /* iterations completed since init                 */
  int32_t exited;       /* 1 if the exit rule fired                        */
  double f;             /* f(U_{t-1}, B_t) = sum_k ||y_k - A_k U b_k||^2    */
  double sd;            /* SD(U_{t-1}, U_t)                                */
  double grad_norm;     /* ||grad_t||_F                                    */
  double eta;           /* step size in use                                */
  double gamma;         /* truncation threshold gamma (init)               */
  int32_t n_trunc;      /* samples (over every frame and coil) zeroed by the
                           truncation of the last altgdmin_init            */
} altgdmin_stats;

typedef struct altgdmin_ctx altgdmin_ctx;

/* Host-only: validates the shape and constants and creates a context. */
altgdmin_status altgdmin_create(const altgdmin_params* params, altgdmin_ctx** out);

/* Bytes of device workspace this context needs (host-only). */
altgdmin_status altgdmin_workspace_bytes(const altgdmin_ctx* ctx, size_t* bytes);

/* Binds the problem: coil maps s_c (Sec. II-A, D_c = diag(s_c)), masks
 * (H_k), m_k, the measurements y_k = A_k z_k (+ noise) in the padded form
 * (eq. Ymat; may be NULL when only the operators are used), the workspace
 * (>= altgdmin_workspace_bytes, 256-byte aligned) and the stream
 * (hipStream_t; NULL = default stream).  Enqueues the one-time setup: index
 * tables, the per-line inverse DFT along kx of y (LINES), ||y_k||^2, m_k and
 * mbar.  Resets the iteration state. */
altgdmin_status altgdmin_set_problem(altgdmin_ctx* ctx, const void* d_coils, const int32_t* d_mask,
                                     const int32_t* d_m_k, const void* d_y, void* d_workspace,
                                     void* stream);

/* Spectral initialisation (Algorithm 2): truncation, scaled back-projection
 * X_0, U_0 = top-r left singular vectors of X_0 (written to d_U, n x r,
 * orthonormal; unique up to an r x r unitary).  Resets t and eta. */
altgdmin_status altgdmin_init(altgdmin_ctx* ctx, void* d_U);

/* Warm start: d_U = an orthonormal basis of span(d_U0) (QR of a given n x r
 * basis; e.g. the previous mini-batch's U, Algorithm 4, or a learned
 * initialiser).  d_U0 and d_U may alias.  Resets t and eta. */
altgdmin_status altgdmin_init_from(altgdmin_ctx* ctx, const void* d_U0, void* d_U);

/* Input of the learned initialiser: the zero-filled, coil-combined frames
 * A_k^H y_k (no truncation, no 1/sqrt(m_k m) scaling), as 2q real planes
 * d_in[2k] = Re, d_in[2k+1] = Im, each ny x nx with x fastest, all divided
 * by the root mean square of the 2q*n values (FP32, caller-allocated,
 * 2q*n floats).  Requires a bound problem with measurements. */
altgdmin_status altgdmin_cnn_input(altgdmin_ctx* ctx, float* d_in);

/* Initialisation with a learned guess and the spectral fallback: the
 * spectral U_0 (as altgdmin_init) and the CholeskyQR of d_M (n x r, e.g. the
 * network output; a small ridge is added if its Gram is numerically
 * singular) are both scored by f(U) = sum_k (||y_k||^2 - h_k^H G_k^-1 h_k),
 * the cost after the exact LS step (Sec. III-B), and the one with the
 * strictly lower cost is written to d_U.  The step size is set by
 * Algorithm 2's first-iteration rule at the spectral basis (the rule at a
 * good learned basis, whose gradient is small, would overshoot), so with
 * the fallback the run is exactly the plain one.  A guess that cannot be
 * scored (its Gram, or a frame's Gram of A_k QR(M), is not positive
 * definite, or a value is not finite: e.g. an all-zero or NaN network
 * output) counts as infinitely costly: the spectral basis is kept and no
 * error is left set.  No host synchronisation: if d_choice is not NULL, the
 * device int it points to receives 1 when the learned guess was kept, 0
 * otherwise.  Resets t. */
altgdmin_status altgdmin_init_warm(altgdmin_ctx* ctx, const void* d_M, void* d_U, int32_t* d_choice);

/* altgdmin_init_warm with the fallback basis supplied instead of computed:
 * d_Ufb (device, n x r, column-major complex64, orthonormal; typically the
 * output of altgdmin_init on this context) takes the place of the spectral
 * initialisation (Algorithm 2's U_0), and d_U (out, may equal d_Ufb)
 * receives the lower-cost of it and QR(d_M), d_choice as above.  Splitting
 * the warm start this way lets the network's forward pass that produces
 * d_M run on another stream while altgdmin_init runs on the context's; the
 * caller orders d_M's producer before this call.  Errors: EINVAL for a NULL
 * context, guess or basis; ESTATE before altgdmin_set_problem.  Resets t. */
altgdmin_status altgdmin_init_warm_from(altgdmin_ctx* ctx, const void* d_M, const void* d_Ufb, void* d_U,
                                        int32_t* d_choice);

/* n_iter iterations of the alternating loop (Algorithm 2), continuing from
 * d_U (in/out, n x r orthonormal).  d_B (out, r x q) receives B_T computed
 * from U_{T-1}; d_U_prev (out, may be NULL) receives U_{T-1}, so that
 * X_T = U_{T-1} B_T is the reconstruction.  eta is set at the context's
 * first iteration and persists across calls (see altgdmin_set_eta).
 * n_iter <= 0 means t_max.  With eps_exit > 0 the loop stops on the device
 * when the exit rule fires (the remaining launches do nothing).
 * h_iters_done (host, may be NULL) receives the number of iterations done by
 * this call; passing it synchronises the stream (before the call's work, to
 * read the starting count, and after it). */
altgdmin_status altgdmin_iterate(altgdmin_ctx* ctx, int32_t n_iter, void* d_U, void* d_B,
                                 void* d_U_prev, int32_t* h_iters_done);

/* The step size eta (host double).  get synchronises; set makes a resumed
 * run exact (a value <= 0 clears it, so the next iteration sets it). */
altgdmin_status altgdmin_get_eta(altgdmin_ctx* ctx, double* eta);
altgdmin_status altgdmin_set_eta(altgdmin_ctx* ctx, double eta);

/* f(U) = min_B sum_k ||y_k - A_k U b_k||^2 = sum_k (||y_k||^2 - h_k^H G_k^{-1} h_k)
 * for an orthonormal d_U, written as one double to device memory d_f. */
altgdmin_status altgdmin_cost(altgdmin_ctx* ctx, const void* d_U, double* d_f);

/* The LS step and the gradient at a given n x r basis d_U (Algorithm 2):
 * d_B (r x q, may be NULL) receives b_k = (A_k U)^dagger y_k for every frame
 * and d_G (n x r, may be NULL) receives
 * grad = sum_k A_k^H (A_k U b_k - y_k) b_k^H; with d_G NULL only the LS step
 * runs.  Does not change the iteration state (t, eta). */
altgdmin_status altgdmin_gradient(altgdmin_ctx* ctx, const void* d_U, void* d_B, void* d_G);

/* Y = A(X) (eq. Ymat): d_X n x q in, d_Y [q][nc][m_max] out (padding
 * written as 0).  And X = A^H(Y), padding of d_Y ignored. */
altgdmin_status altgdmin_apply_A(altgdmin_ctx* ctx, const void* d_X, void* d_Y);
altgdmin_status altgdmin_apply_AH(altgdmin_ctx* ctx, const void* d_Y, void* d_X);

/* Statistics of the last iteration (synchronises).  When the exit rule is
 * off, the loop only stores the r x r inputs of f, sd and grad_norm; this
 * call forms them first (one small kernel on the context's stream). */
altgdmin_status altgdmin_get_stats(altgdmin_ctx* ctx, altgdmin_stats* stats);

/* The device error flag, if any (synchronises).  *frame receives the frame
 * index of an ENOTPD per-frame Gram, -1 otherwise.  Clears the flag. */
altgdmin_status altgdmin_last_error(altgdmin_ctx* ctx, int32_t* frame);

/* Timing of one kernel class of the loop, for measurement.
 * altgdmin_set_timing(ctx, which) makes the loop record HIP events on the
 * context's stream around every launch of kernel class `which`
 * (0 none, 1 forward transform, 2 per-frame Gram/rhs, 3 batched solve,
 * 4 gradient fold, 5 adjoint transform + coil combine, 6 QR Gram, 7 QR
 * small work, 8 QR update); altgdmin_kernel_time (synchronises) returns the
 * class name, the number of launches timed and their total milliseconds,
 * and resets the counters. */
altgdmin_status altgdmin_set_timing(altgdmin_ctx* ctx, int32_t which);
altgdmin_status altgdmin_kernel_time(altgdmin_ctx* ctx, const char** name, int32_t* launches,
                                     double* total_ms);

/* ---- the steps around the loop: altGDmin-MRI (Algorithms 1 and 3) -------
 * These calls use the measurements bound by altgdmin_set_problem and an
 * auxiliary device workspace d_aux (caller-owned, 256-byte aligned, at least
 * altgdmin_aux_bytes; its contents need not survive between calls).  Image
 * sequences are n x q column-major complex64 (X[k*n + p]); residual
 * measurements use the padded layout of y.  They run on the context's stream
 * and do not change the iteration state of the loop. */
altgdmin_status altgdmin_aux_bytes(const altgdmin_ctx* ctx, size_t* bytes);

/* The mean image (Algorithm 1, step 1): zbar = argmin_z sum_k ||y_k - A_k z||^2
 * by conjugate gradients on the normal equations from z = 0 (the CGLS
 * iterates; the normal operator sum_k A_k^H A_k is applied as
 * sum_c conj(s_c) F^H (cnt o F(s_c z)), cnt the number of frames sampling each
 * k-space location).  Stops after the iteration at which
 * ||A^H(y - A z)|| <= tol ||A^H y||, or after maxit iterations (paper: 1e-3,
 * 10).  d_zbar: n complex64 out.  h_iters (host, may be NULL) receives the
 * iterations done; passing it synchronises.  EINVAL for maxit < 0 or
 * tol < 0. */
altgdmin_status altgdmin_mean(altgdmin_ctx* ctx, double tol, int32_t maxit, void* d_zbar, void* d_aux,
                              int32_t* h_iters);

/* altgdmin_mean without the auxiliary workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments and result as
 * altgdmin_mean (bitwise: the same kernels in the same order); its scratch
 * (three n-vectors, nc*n coil images, reduction partials and scalars) is a
 * 16 MiB array built into the library, one per GPU, kept until the process
 * ends.  Problems whose scratch exceeds it (8 (3 + nc) n bytes plus about
 * 2 KiB; e.g. 256x256 with up to 28 coils) return ALTGDMIN_ESCRATCH before
 * any launch.  Calls allocate nothing.  Every call on one GPU shares that
 * GPU's scratch, so calls that overlap on one GPU (two streams, two threads)
 * race and must be serialised by the caller.  The stream's device must be
 * the current device. */
altgdmin_status altgdmin_mean_noalloc(altgdmin_ctx* ctx, double tol, int32_t maxit, void* d_zbar,
                                      int32_t* h_iters);

/* Residual measurements (Algorithm 1, steps 2a and 3a):
 * d_yres = y - A(zbar 1^T + X), frame by frame, in the padded layout (padding
 * written as 0).  d_zbar (n) and d_X (n x q) may each be NULL (then taken as
 * zero).  d_yres must not alias y. */
altgdmin_status altgdmin_residual(altgdmin_ctx* ctx, const void* d_zbar, const void* d_X, void* d_yres,
                                  void* d_aux);

/* MEC model 1 (Algorithm 3, altGDmin-MRI1): for every frame, `iters` CGLS
 * iterations from e = 0 on min_e ||yres_k - A_k e||^2, a frame stopping early
 * once ||A_k^H(yres_k - A_k e)|| <= tol ||A_k^H yres_k|| (paper: 3
 * iterations, tol 1e-36).  d_yres: padded residual measurements (padding
 * ignored); d_E: n x q complex64 out. */
altgdmin_status altgdmin_mec_cgls(altgdmin_ctx* ctx, const void* d_yres, int32_t iters, double tol, void* d_E,
                                  void* d_aux);

/* MEC model 2 (Algorithm 3, altGDmin-MRI2): ISTA on the temporal DFT of the
 * error.  From E_0 = 0, for t = 0, 1, ...: M_t = F_t(E_t + A^H(yres - A(E_t)))
 * with F_t the unitary DFT along the frames of every pixel;
 * omega = omega_frac * max|M_0| (paper: 0.001); E_{t+1} =
 * F_t^-1(SThr_omega(M_t)) with the complex soft threshold s/|s| (|s| - omega)
 * (0 where |s| <= omega).  Ends after max_iter updates (paper: 10) or after
 * the update that follows an M_t (t >= 1) with
 * ||M_t - M_{t-1}||_F / ||M_{t-1}||_F < tol (paper: 0.0025).  d_E: n x q out.
 * h_iters (may be NULL; synchronises) receives the updates done.  Needs
 * q <= 128. */
altgdmin_status altgdmin_mec_ista(altgdmin_ctx* ctx, const void* d_yres, int32_t max_iter, double omega_frac,
                                  double tol, void* d_E, void* d_aux, int32_t* h_iters);

/* The output of Algorithm 1: d_Z[:, k] = zbar + U b_k + e_k (n x q,
 * complex64), each term optional: d_U (n x r) and d_B (r x q) together or
 * neither, d_zbar (n), d_E (n x q).  d_Z may alias d_E. */
altgdmin_status altgdmin_expand(altgdmin_ctx* ctx, const void* d_U, const void* d_B, const void* d_zbar,
                                const void* d_E, void* d_Z);

/* The spectrum behind the automatic rank (Algorithm 2, parameter setting):
 * the r_cap largest eigenvalues of X_0^H X_0 (the squared singular values of
 * the truncated, scaled back-projection X_0 of the initialisation),
 * descending, into h_sigma2 (host, r_cap doubles; 1 <= r_cap <= min(16, q)).
 * Synchronises. */
altgdmin_status altgdmin_rank_energy(altgdmin_ctx* ctx, int32_t r_cap, double* h_sigma2, void* d_aux);

/* The automatic rank: r_cap = floor(min(n, q, nc min_k m_k) / 10) (at least
 * 1, at most 16), then the smallest r with
 * sum_{j<=r} sigma_j^2 >= (b_percent/100) sum_{j<=r_cap} sigma_j^2 (paper:
 * b = 85).  h_rank (host) receives r, h_rcap (may be NULL) r_cap.
 * Synchronises.  The result is the rank to create the reconstruction's
 * context with. */
altgdmin_status altgdmin_auto_rank(altgdmin_ctx* ctx, double b_percent, int32_t* h_rank, int32_t* h_rcap,
                                   void* d_aux);

/* A static description of status s (one of the altgdmin_status values). */
const char* altgdmin_status_string(altgdmin_status s);

void altgdmin_destroy(altgdmin_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ALTGDMIN_H */
