/*
 * ls.h - C ABI of the MI355X (gfx950) Lippmann-Schwinger (LS) displacement solver.
 *
 * The library evaluates and solves the frequency-domain volume integral equation of
 * Shekhar, Jakobsen, Iversen, Berre and Radu (arXiv 2301.12836) for the particle
 * displacement u in a heterogeneous anisotropic elastic medium:
 *
 *     A u = u0,   A = I - Gconv B,   B = -E^T dC E + w^2 drho            (Eq 19-21)
 *
 * with E the finite-difference Voigt strain of Eq 17-18 (central inside, one-sided
 * first-order on the model boundary), dC the per-cell 6x6 stiffness contrast and drho
 * the density contrast (Eq 2-3, 11-12), Gconv the linear convolution with h^3 times the
 * isotropic background Green's tensor of Eq 7 / Appendix A (the r = 0 cell takes the
 * average over the sphere of volume h^3), evaluated with zero-padded 3-D FFTs, and u0
 * the incident field of a moment tensor source (Eq 13-16): u0 = e^{i w t0} Gconv E^T (M delta_s)/h^3.
 * The system is solved with BiCGSTAB to the relative residual e = ||u0 - A u|| / ||u0||
 * of Eq 22.
 *
 * Conventions shared by every call
 *   - Grid: n[0] = N1 (x), n[1] = N2 (y), n[2] = N3 (z) cells, spacing h (m); cell
 *     (i, j, k) sits at (i h, j h, k h).  Each n[a] must be in [2, 256].
 *   - Field arrays are component-major, x fastest: u[c][N3][N2][N1] for c = x, y, z,
 *     complex interleaved (re, im): "c128" = two doubles, "c64" = two floats.  A batch
 *     of R fields is R such arrays back to back.
 *   - Contrast: dC[21][N3][N2][N1] doubles, the Voigt upper triangle of each cell's 6x6
 *     in row order 11,12,13,14,15,16,22,...,26,33,...,66 (Voigt 1..6 = 11,22,33,23,13,12);
 *     drho[N3][N2][N1] doubles.  Units Pa and kg/m^3.
 *   - Moment tensor: M[6] in Voigt order (M11, M22, M33, M23, M13, M12), N m.
 *   - Every device pointer is caller-owned HIP device memory; the library reads or writes
 *     it on the context's stream and never frees it.  Calls are stream-ordered and return
 *     without synchronising unless stated.  A context is not thread-safe; use one context
 *     per host thread / stream.
 *   - Return codes: LS_OK (0) or a negative LS_ERR_*; ls_last_error() gives a message
 *     (thread-local).  No C++ exception crosses this interface.
 */
#ifndef LS_H
#define LS_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LS_OK = 0,
    LS_ERR_ARG = -1,            /* invalid argument (null pointer, bad size or index)      */
    LS_ERR_OOM = -2,            /* device allocation failed                                */
    LS_ERR_HIP = -3,            /* a HIP runtime call failed                               */
    LS_ERR_BREAKDOWN = -4,      /* BiCGSTAB breakdown (rho, r^H v or t^H t vanished)       */
    LS_ERR_NOT_CONVERGED = -5,  /* maxit reached; the output holds the best iterate found  */
    LS_ERR_NONFINITE = -6,      /* NaN or Inf met in the residual                          */
    LS_ERR_STATE = -7           /* the context was not built for the requested precision   */
};

enum { LS_PREC_C128 = 0, LS_PREC_MIXED = 1 };
enum { LS_GREEN_EXACT = 0, LS_GREEN_PAPER_SUM = 1, LS_GREEN_ANISO = 2 };
enum { LS_PRECOND_NONE = 0, LS_PRECOND_BLOCK_JACOBI = 1 };

typedef struct {
    int n[3];       /* N1, N2, N3 */
    double h;       /* grid spacing (m) */
} ls_grid;

typedef struct {
    int precision;  /* LS_PREC_C128: FP64 operator only; LS_PREC_MIXED: also the FP32 operator */
    int green_mode; /* LS_GREEN_EXACT (default): the closed-form solution of Eq 7;
                       LS_GREEN_PAPER_SUM: the near-field A.4 plus far-field A.5 tensors;
                       LS_GREEN_ANISO: the solution of Eq 7 for the anisotropic C0 itself
                       (see below)                                                          */
    int max_rhs;    /* largest batch of right-hand sides one call may carry (>= 1)         */
    int flags;      /* LS_FLAG_* bits (0: defaults)                                          */
    int taper;      /* absorbing boundary layer thickness in cells (0: off); see below        */
    int bicgstab_l; /* Krylov method: 1 (or 0) Bi-CGSTAB, the paper's solver; 2..4 BiCGSTAB(l)  */
    int precond;    /* LS_PRECOND_NONE (0) or LS_PRECOND_BLOCK_JACOBI; see below               */
    int reserved[1];
} ls_options;

/* ls_options.bicgstab_l = l > 1 solves with BiCGSTAB(l) (Sleijpen and Fokkema 1993): l Bi-CG steps, then a
 * minimal-residual polynomial of degree l over the residuals those steps produced.  l = 1 is Bi-CGSTAB.  At
 * high frequency, where Bi-CGSTAB stagnates (its degree-one minimal-residual steps cannot follow a
 * spectrum spread around the origin), l = 4 often converges at about the same work per matvec.  The
 * cycle's scalars are formed on the host (one round trip per inner product), so these solves are not
 * captured in graphs.  Costs 2 l + 3 field vectors per right-hand side (and as many FP32 ones for
 * mixed precision) instead of 6, allocated at set-up.  ls_info.iters counts Bi-CG steps (2 matvecs each). */

/* ls_options.precond = LS_PRECOND_BLOCK_JACOBI preconditions every Bi-CGSTAB solve of the context on the right
 * with the point-block Jacobi matrix M = blockdiag D(x), D(x) the 3x3 block of A = I - Gconv B (Eq 19-21) that
 * couples the three components at cell x with themselves (the paper's concluding remarks name
 * preconditioning as the next speed-up without fixing one).  Bi-CGSTAB then iterates on A M^-1 with the
 * directions M^-1 p and M^-1 s, so the solution and the stopping rule (Eq 22) are those of the
 * unpreconditioned system; transposed solves use M^T.  The blocks follow from the strain stencil, the
 * contrast and the Green's tensor at offsets within two cells; they are built and inverted in FP64 per
 * frequency at set-up and again by ls_set_contrast.  Costs 9 complex values per cell and frequency (FP64, and
 * FP32 for mixed precision) plus two field vectors per right-hand side and precision.  It cuts iterations
 * where the contrast is strong and varies from cell to cell (a third fewer matvecs at +-30-40 % random
 * contrast) and gains nothing where smooth contrast and propagation over many wavelengths set the count.
 * Needs bicgstab_l = 1 (LS_ERR_ARG otherwise); a singular block fails the set-up with LS_ERR_NONFINITE. */

/* ls_options.taper = d > 0 weights the total contrast (input plus background fold) of every cell within
 * d cells of a face by 1 - exp(-l^2 / (N_a h^2)) (the absorbing boundary of Eq 23-25), at set-up and
 * in ls_set_contrast: l is the distance from the cell centre to the point where the ray from the model
 * centre through it leaves the box (the faces lie half a cell outside the outer cell centres), N_a the
 * number of cells along the axis of the face it crosses.  Gradients (ls_grad_contrast, ls_grad) are
 * taken with respect to the input contrast, so they carry the same weight.  0 <= d <= min(N)/2. */

/* ls_options.green_mode = LS_GREEN_ANISO convolves with the Green's tensor of the background C0 itself
 * instead of folding C0 into an isotropic reference plus contrast (the paper's method admits an arbitrary
 * background, Eq 2-3, 7; Appendix A writes out only the isotropic tensor).  The tensor is evaluated from
 * its plane-wave (unit-sphere) representation: with Gamma(n) the Christoffel matrix, lambda_m, P_m its
 * eigenvalues and eigenprojectors and k_m = w sqrt(rho0 / lambda_m),
 *     G(x) = 1/(8 pi^2 r) int_{n.x = 0} Gamma(n)^{-1} dphi
 *          + i/(8 pi^2) int_{n.x > 0} sum_m P_m k_m / lambda_m e^{i k_m n.x} dS(n),
 * and the zero-offset cell takes the integral over the sphere of volume h^3,
 *     1/(4 pi) int sum_m P_m I(k_m) / lambda_m dS,  I(k) = int_0^R r e^{i k r} dr,  R = (3/(4 pi))^{1/3} h
 * (for an isotropic C0 both equal the LS_GREEN_EXACT table).  Any stiffness is accepted: one with the
 * three coordinate mirror planes (orthorhombic, VTI or isotropic in the grid axes: C14..C16, C24..C26,
 * C34..C36, C45, C46, C56 zero) keeps the octant k-space table, any other (tilted media) uses a table
 * over the half-space k_x <= L1/2 (4 times the memory and table traffic).  Checked at set-up (LS_ERR_ARG
 * otherwise): C0 is positive definite, its quasi-P eigenvalue stays at least 5 % above the quasi-S ones
 * in every direction, and the largest phase w r / v_min over the grid is at most 1600 rad.  Nothing is
 * folded into the contrast.  The table is computed once per frequency at set-up (FP64 quadrature on the
 * device: about 1.3 s per frequency for a tilted background at 128^3). */

/* ls_options.flags:
 *   LS_FLAG_NO_GRAPH  run every BiCGSTAB iteration as separate launches instead of replaying one
 *                     captured hipGraph per iteration (the default when the stream can be captured).
 *   LS_FLAG_AUTOTUNE  at set-up, time the available kernel variants of every FFT pass (register
 *                     four-step and LDS Stockham) at the context's sizes and keep the fastest.  The
 *                     choice is cached, keyed by device, grid, FFT lengths, max_rhs, buffer layout,
 *                     table kind and precision, in the text file that the environment variable
 *                     LS_AUTOTUNE_CACHE names (default $HOME/.cache/lsvie/autotune.txt); a context
 *                     whose key is cached takes the cached choice without timing. */
enum { LS_FLAG_NO_GRAPH = 1, LS_FLAG_AUTOTUNE = 2 };

typedef struct {
    int iters;           /* BiCGSTAB iterations (inner iterations summed for mixed solves)  */
    int matvecs;         /* operator applications, the final true-residual check included  */
    int refinements;     /* outer FP64 refinement steps (mixed precision), else 0          */
    int status;          /* LS_OK or the LS_ERR_* code of this right-hand side              */
    double rel_res;      /* last recursively updated relative residual                     */
    double rel_res_true; /* ||u0 - A u|| / ||u0|| recomputed with the FP64 operator (Eq 22) */
} ls_info;

typedef struct ls_ctx ls_ctx;

/* Build a context for one grid and medium at n_omega angular frequencies (Eq 1-3, 7, 21).
 *   C0[36]  host, row-major 6x6 background stiffness (must be symmetric).  If it is not
 *           isotropic and green_mode is not LS_GREEN_ANISO, the isotropic reference c11 = C33,
 *           c44 = (C44 + C55)/2 is used (the rule of the paper's Model 1) and C0 minus that
 *           reference is added to every cell's contrast.
 *   rho0    background density.
 *   dC      device, [21][N3][N2][N1] doubles (see conventions); drho device, [N3][N2][N1].
 *           Both are copied; the caller may free them after the call returns.
 *   omega   host, n_omega angular frequencies (rad/s, > 0).
 *   opt     may be NULL (c128, exact Green's tensor, max_rhs 1).
 *   stream  a hipStream_t (NULL = the null stream); all work of this context runs on it.
 * Allocates all device memory the context will use (tables, contrast, workspaces).
 * Synchronises the stream before returning.  On error *out is NULL. */
int ls_setup(const ls_grid* grid, const double C0[36], double rho0,
             const double* dC, const double* drho,
             const double* omega, int n_omega, const ls_options* opt,
             void* stream, ls_ctx** out);

/* Release every device allocation of the context (synchronises its stream). NULL is a no-op. */
void ls_destroy(ls_ctx* ctx);

/* Replace the medium's contrast (same layout and background fold as ls_setup) without rebuilding the
 * Green's tables, which depend only on the background and the frequencies.  dC, drho: device, copied.
 * Rebuilds the block-Jacobi preconditioner if the context has one.  Synchronises the stream. */
int ls_set_contrast(ls_ctx* ctx, const double* dC, const double* drho);

/* The inverse diagonal blocks M^-1 of the block-Jacobi preconditioner at frequency omega[i_omega] (see
 * ls_options.precond): minv, device c128 [9][N3][N2][N1] owned by the caller, entry (a, b) of the inverse
 * block of cell p at [3 a + b][p].  LS_ERR_STATE if the context was built without the preconditioner.
 * Asynchronous. */
int ls_precond_blocks(ls_ctx* ctx, int i_omega, void* minv);

/* One LS matvec Au = u - Gconv B u at frequency omega[i_omega] (Eq 19-21), for n_rhs fields
 * (1 <= n_rhs <= max_rhs).  u, Au: device c128 arrays [n_rhs][3][N3][N2][N1]; they must not
 * overlap (LS_ERR_ARG otherwise).  Asynchronous. */
int ls_apply(ls_ctx* ctx, int i_omega, const void* u, void* Au, int n_rhs);

/* For callers that cannot allocate device memory during the call (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): ls_apply with its padded FFT work buffer taken from a
 * fixed 64 MiB device array that the library holds on each GPU it runs on until the process ends, instead
 * of the context's workspace.  Same arguments, result (bitwise equal to ls_apply's) and errors as ls_apply;
 * n_rhs x 3 N3 L2 L1 x 16 bytes (L_a the padded FFT lengths: 50 MB for one 64^3 field) must fit in the
 * 64 MiB, else LS_ERR_ARG.  Allocates nothing and clears nothing (every value of the buffer that is read
 * was written earlier in the same call).  Every call on a GPU uses that GPU's one array, so calls that
 * overlap in time on one GPU (different streams or host threads) race; serialise them.  Asynchronous. */
int ls_apply_noalloc(ls_ctx* ctx, int i_omega, const void* u, void* Au, int n_rhs);

/* The same matvec with the operator, its FFTs and Green's multiply in FP32 (c64 fields; u and Au must
 * not overlap).  Needs a context built with LS_PREC_MIXED, else LS_ERR_STATE.  Asynchronous. */
int ls_apply_c64(ls_ctx* ctx, int i_omega, const void* u, void* Au, int n_rhs);

/* Incident field of a moment tensor M at source cell src[3] = (i, j, k) with rupture time t0
 * (Eq 13-16): b = e^{i w t0} Gconv E^T (M delta_src) / h^3, evaluated cell by cell from the
 * closed-form Green's tensor.  b: device c128 [3][N3][N2][N1].  Asynchronous. */
int ls_rhs_moment(ls_ctx* ctx, int i_omega, const double M[6], const int src[3], double t0, void* b);

/* Incident field of a point force F (N) at cell[3] (Eq 6): b = Gconv (F delta_cell) / h^3.
 * b: device c128 [3][N3][N2][N1].  Asynchronous. */
int ls_rhs_force(ls_ctx* ctx, int i_omega, const double F[3], const int cell[3], void* b);

/* Solve A u = b for n_rhs right-hand sides b (device c128 [n_rhs][3][N3][N2][N1]) with
 * BiCGSTAB (x0 = 0 or the given guess), stopping when the recursive residual reaches tol
 * (Eq 22), then recomputing the true FP64 residual.  With precision LS_PREC_MIXED the
 * context's FP32 operator runs the inner BiCGSTAB inside an FP64 iterative-refinement loop
 * whose residual b - A u uses the FP64 operator; the stopping test is always the FP64 true
 * residual.  All n_rhs systems advance together through batched operator applications.
 *   x0     device c128 like b, or NULL for zero.   u_out device c128 like b.
 *          b and u_out must not overlap; x0 is either u_out itself (an in-place warm start) or
 *          disjoint from it (LS_ERR_ARG otherwise).
 *   info   host array of n_rhs entries (may be NULL).
 *   precision  LS_PREC_C128 or LS_PREC_MIXED (the latter needs a mixed context).
 * Returns LS_OK when every system met tol; LS_ERR_NOT_CONVERGED, LS_ERR_BREAKDOWN or
 * LS_ERR_NONFINITE otherwise (per-system codes in info[].status, u_out holds the best
 * iterate).  Synchronises the stream. */
int ls_solve(ls_ctx* ctx, int i_omega, const void* b, int n_rhs, double tol, int maxit,
             int precision, const void* x0, void* u_out, ls_info* info);

/* ls_solve with each system at its own frequency: system q solves A(omega[i_omega[q]]) u_q = b_q (the
 * paper solves one system per frequency and source, Eq 21-22, and notes that frequencies can be solved
 * simultaneously).  i_omega: host int [n_rhs].  The systems share every operator launch and every
 * Bi-CGSTAB vector kernel; a launch covers only the systems still iterating (converged ones drop out),
 * and every decision (inner tolerance, stopping, refinement) is taken per system, so each result is
 * bitwise the one ls_solve returns for that system alone.  Arguments, buffers and return codes otherwise
 * as ls_solve.  Synchronises the stream. */
int ls_solve_multi(ls_ctx* ctx, const int* i_omega, const void* b, int n_rhs, double tol, int maxit,
                   int precision, const void* x0, void* u_out, ls_info* info);

/* The moment-tensor solve in the form the method states it (Eq 13-16, 21-22): the incident field of M at
 * source cell src with rupture time t0 (ls_rhs_moment, into the context's own buffer), then ls_solve of
 * that one system from the initial guess x0 (device c128 [3][N3][N2][N1] or NULL for zero; it may be
 * u_out itself) to relative residual tol, the solution into u_out.  Same return codes as ls_solve. */
int ls_solve_moment(ls_ctx* ctx, int i_omega, const double M[6], const int src[3], double t0,
                    double tol, int maxit, int precision, const void* x0, void* u_out, ls_info* info);

/* Convenience form for one unit point force: builds b with ls_rhs_force (F delta_cell / h^3,
 * Eq 6), then ls_solve.  Used for reciprocity checks and receiver-side Green's functions. */
int ls_solve_force(ls_ctx* ctx, int i_omega, const double F[3], const int cell[3], double tol, int maxit,
                   int precision, void* u_out, ls_info* info);

/* One moment-tensor solve of a batch: the source M (Voigt 11,22,33,23,13,12) at cell src with rupture
 * time t0, on context ctxs[ctx] at frequency index i_omega; the solution goes to u_out (device c128
 * [3][N3][N2][N1] of that context's grid, owned by the caller). */
typedef struct ls_job {
    int ctx;
    int i_omega;
    double M[6];
    int src[3];
    double t0;
    void* u_out;
} ls_job;

/* Solve every job of a batch over several contexts, whose grids may differ (the paper treats each
 * frequency and source as an independent system, Eq 21-22).  Per context the jobs are ordered by
 * frequency and solved max_rhs at a time as one multi-right-hand-side solve whose systems may sit at
 * different frequencies (ls_solve_multi with the given precision), so device residency stays within
 * what the contexts were built for; contexts are driven concurrently, one host thread and the
 * context's own stream each (contexts must be distinct and are used exclusively for the duration of
 * the call).  The first call on a context
 * allocates two [max_rhs][3][N3][N2][N1] c128 batch buffers that it keeps until ls_destroy.
 * infos: host array of n_jobs entries (may be NULL).  All arguments are checked before any work.
 * Returns LS_OK when every job met tol; a hard error (LS_ERR_HIP, LS_ERR_OOM) of any context stops
 * that context and is returned first; otherwise the first context's LS_ERR_NOT_CONVERGED /
 * LS_ERR_BREAKDOWN / LS_ERR_NONFINITE (every job's u_out and info are still written).
 * Synchronises every context's stream. */
int ls_solve_batch(ls_ctx* const* ctxs, int n_ctx, const ls_job* jobs, int n_jobs, double tol, int maxit,
                   int precision, ls_info* infos);

/* Receiver samples of n_rhs fields: out[r][m][c] = u[r][c][rec_m] for the n_rec cells rec (host int
 * [n_rec][3] = (i, j, k), each inside the grid, else LS_ERR_ARG).  u: device c128 [n_rhs][3][N3][N2][N1];
 * out: device c128 [n_rhs][n_rec][3].  Synchronises the context's stream. */
int ls_sample(ls_ctx* ctx, const void* u, int n_rhs, const int* rec, int n_rec, void* out);

/* Time-domain traces from one-sided spectra (the frequency loop up to Nyquist and inverse transform of the
 * paper's comparisons with finite differences).  With time dependence e^{-i w t} and w_k = 2 pi k / (nt dt),
 *   traces[j][n] = (1/(nt dt)) sum_q c_q Re[S(w_{k_q}) spectra[q][j] e^{-i w_{k_q} n dt}],
 * c_q = 1 for k_q = 0 or 2 k_q = nt, else 2 (the negative frequencies of a real signal); S is the Ricker
 * wavelet of peak frequency fp delayed by ts (Tables 1 and 3), S(w) = (4 sqrt(pi) w^2 / wp^3)
 * e^{-w^2/wp^2} e^{i w ts} with wp = 2 pi fp, or 1 when fp <= 0.  Frequencies not listed count as zero.
 *   spectra: device c128 [n_freq][n_trace];  k: host [n_freq], 0 <= k <= nt/2;
 *   traces: device double [n_trace][nt].  Uses the context's stream; synchronises it. */
int ls_synthesize(ls_ctx* ctx, const void* spectra, const int* k, int n_freq, int n_trace, int nt, double dt,
                  double fp, double ts, double* traces);

/* Voigt engineering strain of n_rhs fields (Eq 17-18): eps device c128 [n_rhs][6][N3][N2][N1], disjoint
 * from u (LS_ERR_ARG otherwise). */
int ls_strain(ls_ctx* ctx, const void* u, void* eps, int n_rhs);

/* Adjoint side of the operator (for gradients of misfits through the solution of Eq 21).
 * Both Gconv (the Green's tensor is symmetric and even) and B are symmetric, so the transpose is
 * A^T = I - B Gconv: the Green's convolution first, then the contrast.  The conjugate transpose is
 * A^H y = conj(A^T conj(y)).
 *
 * ls_apply_T: ATy = A^T y for n_rhs c128 fields (y, ATy must not overlap).  Asynchronous.
 * ls_convolve: out = Gconv f (f a force density on the cells, c128): the zero-padded convolution
 *   with h^3 G of Eq 21 alone.  Asynchronous.
 * ls_solve_T: BiCGSTAB on A^T x = b, with the same contract as ls_solve (FP64 true residual of the
 *   transposed system; mixed precision runs the FP32 transposed operator inside FP64 refinement).
 * ls_grad_contrast: for forward fields u and fields mu (both device c128 [n_rhs][3][N3][N2][N1]),
 *   accumulate into the device arrays g_dC [21][N3][N2][N1] and g_drho [N3][N2][N1] (doubles):
 *     g_dC[JK] += -Re[conj(eps_J(mu)) eps_K(u) + (J != K) conj(eps_K(mu)) eps_J(u)]   (packed J <= K)
 *     g_drho   += w^2 Re[sum_c conj(mu_c) u_c]
 *   summed over the n_rhs pairs.  With r = P u - d the receiver residual of the misfit
 *   J = 1/2 ||P u - d||^2, lambda_bar solving A^T lambda_bar = conj(P^H r) and mu = conj(Gconv
 *   lambda_bar), these are dJ/d(dC) and dJ/d(drho) of one frequency.  Asynchronous. */
int ls_apply_T(ls_ctx* ctx, int i_omega, const void* y, void* ATy, int n_rhs);
int ls_convolve(ls_ctx* ctx, int i_omega, const void* f, void* out, int n_rhs);
int ls_solve_T(ls_ctx* ctx, int i_omega, const void* b, int n_rhs, double tol, int maxit, int precision,
               const void* x0, void* x_out, ls_info* info);
int ls_grad_contrast(ls_ctx* ctx, int i_omega, const void* u, const void* mu, int n_rhs, double* g_dC,
                     double* g_drho);

/* The whole gradient of one frequency from the forward fields u and the adjoint solutions lam_bar
 * (lam_bar solving A^T lam_bar = conj(P^H r), from ls_solve_T), both device c128
 * [n_rhs][3][N3][N2][N1], n_rhs <= max_rhs: forms mu = conj(Gconv lam_bar) in the context's
 * workspace, accumulates g_dC and g_drho as ls_grad_contrast does, and, when g_M is not NULL,
 * writes the moment-tensor gradient of each right-hand side's source (Eq 13-16)
 *     g_M[r][J] = Re[e^{i w t0[r]} conj(eps_J(mu_r)(src_r))] / h^3
 * into the host array g_M [n_rhs][6] (src: host [n_rhs][3] cells inside the grid; t0: host
 * [n_rhs]).  Synchronises the stream when g_M is given, else asynchronous. */
int ls_grad(ls_ctx* ctx, int i_omega, const void* u, const void* lam_bar, int n_rhs, const int* src,
            const double* t0, double* g_dC, double* g_drho, double* g_M);

/* Convergence record of the last ls_solve / ls_solve_moment / ls_solve_force / ls_solve_T on the context:
 * the relative residual ||r|| / ||b|| after each BiCGSTAB iteration of right-hand side rhs (the
 * recursive residual; with LS_PREC_MIXED, each inner iteration's residual scaled by the outer residual
 * it started from, so the values refer to the original system).  Copies up to max_len values into the
 * host array hist and returns how many the record holds (>= 0), or a negative LS_ERR_* code. */
int ls_residual_history(ls_ctx* ctx, int rhs, double* hist, int max_len);

/* Per-kernel timing of the library's own launches.  ls_profile(ctx, 1) starts recording a
 * HIP event pair around every kernel launch on the context's stream (at most 16384 launches;
 * later ones are not recorded); while it is on, Bi-CGSTAB iterations run as separate launches
 * instead of graph replays.  ls_profile(ctx, 0) stops.  ls_profile_read synchronises, then for
 * each kernel family k < n_max writes its name (NUL-terminated, at most 63 chars) into
 * names + 64 k, its launch count into counts[k], the summed event time in milliseconds into
 * ms[k] and, when units is not NULL, the summed right-hand sides the launches covered into
 * units[2 k] and the summed number of distinct Green's tables they read into units[2 k + 1]
 * (the quantities a launch's algorithmic bytes depend on); returns the number of families,
 * and clears the record.  Any of names, counts, ms, units may be NULL. */
int ls_profile(ls_ctx* ctx, int enable);
int ls_profile_read(ls_ctx* ctx, char* names, int* counts, double* ms, long long* units, int n_max);

/* Bytes of device memory the context holds. */
long long ls_device_bytes(const ls_ctx* ctx);

/* The FFT kernel variant each pass uses (0 register four-step, 1 LDS Stockham): variants[5 p + q]
 * for precision p (0 c128, 1 c64) and pass q (0 x forward, 1 y forward, 2 z with the Green's
 * multiply, 3 y inverse, 4 x inverse).  Chosen by timing when built with LS_FLAG_AUTOTUNE. */
int ls_kernel_variants(const ls_ctx* ctx, int* variants);

/* The apply schedule: schedule[p] the right-hand sides per chunk of the x and y passes for precision p (0 c128,
 * 1 c64) at max_rhs right-hand sides (the x and y passes of an operator call run chunk by chunk so that each
 * pass's output is still in the memory-side cache when the next pass reads it), schedule[2 + p] 1 when the
 * strided passes take 256-byte column tiles where the x length allows, 0 for 128-byte ones.  Chosen by timing
 * when built with LS_FLAG_AUTOTUNE, else by the cache size.  schedule: host int [4]. */
int ls_kernel_schedule(const ls_ctx* ctx, int* schedule);

/* Values per cell of the contrast the fused contrast kernel reads (Eq 8, 11-12): 9 when every cell's total
 * contrast (input plus background fold, tapered) vanishes off the orthotropic pattern 11, 12, 13, 22, 23,
 * 33, 44, 55, 66 (isotropic, VTI and orthorhombic media in the grid axes), 21 otherwise; decided at
 * ls_setup and again by ls_set_contrast (LS_CONTRAST_K=21 in the environment keeps 21).  Returns 9 or 21,
 * or LS_ERR_ARG for a null context. */
int ls_contrast_format(const ls_ctx* ctx);

/* Message of the last error on this host thread ("" if none). */
const char* ls_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LS_H */
