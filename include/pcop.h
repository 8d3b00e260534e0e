/*
 * pcop.h -- C ABI of the MI355X solver for the all-at-once KKT system of the
 * parabolic tracking-type optimal-control problem, preconditioned by the
 * epsilon-circulant rotated-block-diagonal (RBD) preconditioner P_eps.
 *
 * Problem (Section 1 of the paper): minimise
 *     1/2 ||y - g||^2 + gamma/2 ||u||^2  over Omega x (0,T),  Omega = (0,1)^d,
 * subject to y_t - div(a grad y) = f + u, y = 0 on the boundary, y(0) = y0.
 * Backward Euler with N = nt steps (tau = T/N) and finite differences on nx
 * interior points per dimension (h = 1/(nx+1), K = -L_h, M = I) give the
 * all-at-once system A x = b of eq. main_system with n = N - 1 time blocks:
 *     A = [[alpha I, T^T], [-T, alpha I]],  T = B_n (x) I + tau I (x) K,
 *     alpha = tau/sqrt(gamma),  x = [sqrt(gamma) y; p],  b = [g; -sqrt(gamma) f]
 * (eq. matrix_A, eq. matrix_T; the blocks of b follow eq. main_system_before).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * m = nx^dim spatial unknowns in lexicographic order, x1 fastest.
 *  * A "vector" is a device array of float64 laid out [batch][2][n][m]:
 *    block 0 holds sqrt(gamma_b) y (or its analogue), block 1 holds p; time
 *    block j = 0..n-1 is level j+1.
 *  * Field arrays g, f are device float64 [batch][n][m] (levels 1..n), y0 is
 *    device float64 [batch][m].
 *  * All device buffers, including the workspace, are allocated and owned by
 *    the caller; the library never allocates or frees device memory.  The
 *    context owns only host state and the layout of the workspace.
 *  * Every call is enqueued on the stream given in pcop_options (0 = the
 *    default stream).  kkt_apply, precond_apply, rhs, unpack and data_grad
 *    only enqueue; pcop_solve synchronises the stream to test convergence.
 *  * Every function returns a pcop_status and never aborts or prints;
 *    arguments are validated before any device work is enqueued.
 *    pcop_last_error() returns a description of the last failure on the
 *    calling thread.
 *  * A context may be used from one host thread at a time.
 */
#ifndef PCOP_H
#define PCOP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcop_ctx_s* pcop_ctx;

typedef enum {
  PCOP_OK = 0,
  PCOP_ERR_INVALID_ARG = 1,  /* rejected before any device work */
  PCOP_ERR_UNSUPPORTED = 2,  /* valid request this build does not implement */
  PCOP_ERR_WORKSPACE = 3,    /* workspace too small or misaligned */
  PCOP_ERR_DEVICE = 4,       /* a HIP runtime call failed */
  PCOP_NOT_CONVERGED = 5     /* outputs valid, tolerance not met within maxit */
} pcop_status;

enum { PCOP_FP64 = 0, PCOP_MIXED = 1 };          /* precision of P_eps^{-1} */
enum { PCOP_DST = 0, PCOP_MG = 1 };              /* spatial solver of Step 2 */
enum { PCOP_RIGHT = 0, PCOP_LEFT = 1, PCOP_FLEXIBLE = 2 };  /* GMRES variant */
enum { PCOP_COEFF_ONE = 0, PCOP_COEFF_HALFGRID = 1 };        /* a(x) */
enum { PCOP_PRECOND_EPS = 0, PCOP_PRECOND_IDEAL = 1 };      /* preconditioner */
enum { PCOP_MASS_IDENTITY = 0, PCOP_MASS_Q1 = 1 };           /* M_m of Section 1 */

/* Problem statement (Section 1; Section 3 for the discretisation).
 *   dim      2 or 3.
 *   nx       interior points per dimension (>= 1; 2^p - 1 for PCOP_MG).
 *   nt       number of backward-Euler steps N (>= 2); n = nt - 1 blocks.
 *            With PCOP_PRECOND_EPS, n <= 2048 (the time FFT runs in LDS;
 *            longer lengths return PCOP_ERR_UNSUPPORTED).
 *   T        final time (> 0).
 *   batch    number of independent systems solved together (>= 1).
 *   gamma    host array [batch] of regularisation parameters (> 0).
 *   eps      epsilon of C_{eps,n} in (0,1] (eq. matrix_C_eps_n); a value
 *            <= 0 selects sqrt(tau).
 *   coeff_kind / coeff
 *            PCOP_COEFF_ONE: a = 1 (coeff must be NULL).
 *            PCOP_COEFF_HALFGRID: coeff is a host array of (2 nx + 1)^dim
 *            values of a(x) sampled at x = k h/2, k = 1..2nx+1 in every
 *            dimension (lexicographic, x1 fastest); these samples contain
 *            a at every face midpoint of every multigrid level.  The values
 *            are copied at pcop_setup.
 *   mass     PCOP_MASS_IDENTITY: finite differences, M_m = I and K_m = -L_h
 *            (5-point / 7-point stencil).  PCOP_MASS_Q1: bilinear (2-D) or
 *            trilinear (3-D) finite elements on the same grid, M_m and K_m
 *            the element mass and stiffness matrices (Section 1 with
 *            M_m != I: eq. matrix_A_before, eq. matrix_A, eq. matrix_P_eps
 *            carry I (x) M_m and C_eps (x) M_m); requires PCOP_COEFF_ONE,
 *            PCOP_DST and PCOP_PRECOND_EPS.  The right-hand side of
 *            pcop_rhs, the maps of pcop_data_grad and the end-level solves
 *            of pcop_post_solve include M_m.
 *            Appended last: zero-initialised callers get finite differences. */
typedef struct {
  int dim;
  int nx;
  int nt;
  double T;
  int batch;
  const double* gamma;
  double eps;
  int coeff_kind;
  const double* coeff;
  int mass;
} pcop_problem;

/* Solver options.
 *   precision  PCOP_FP64, or PCOP_MIXED: P_eps^{-1} evaluated in complex FP32
 *              (vectors, matvec, Arnoldi and residuals stay FP64).
 *   spatial    PCOP_DST (requires a = 1; nx + 1 a power of two, 4..512)
 *              or PCOP_MG (one complex-shifted V-cycle per frequency).
 *   side       PCOP_RIGHT: GMRES on A P^{-1}, stops on the true relative
 *              residual ||b - A x|| / ||b - A x0||;
 *              PCOP_LEFT: GMRES on P^{-1} A, stops on the preconditioned
 *              relative residual (the setting of Section 3);
 *              PCOP_FLEXIBLE: right-preconditioned flexible GMRES that keeps
 *              Z_j = P^{-1} v_j (required with PCOP_MIXED).
 *   restart    Krylov dimension per cycle, 1..40.
 *   maxit      maximum total Arnoldi steps (>= 1).
 *   rtol       relative residual tolerance (> 0).
 *   graph      1: run each group of Arnoldi steps as one captured HIP graph
 *              (needs a non-default stream), 0: plain launches.
 *   graph_chunk Arnoldi steps per graph launch when graph = 1 (>= 1).
 *   reorth_tol a second Gram-Schmidt pass is run for a member when the
 *              coefficients of the new vector against the basis exceed
 *              reorth_tol times its norm (0 = always, < 0 = never).
 *   time_cols  kernels of the two time passes (steps 1 and 3-4 of P_eps^{-1}):
 *              0 automatic; -1 Stockham with two LDS buffers and as many
 *              spatial points per block as fit; -4 / -8 / -16 two buffers
 *              with at most that many points per block; 4 / 8 / 16 in-place
 *              Stockham (one LDS buffer) with at most that many points per
 *              block.  A kind of kernel that does not fit LDS falls back to
 *              the other; +-32 as +-16 with up to 32 points.  When nt - 1
 *              has a prime factor above 17, or no Stockham tile of it fits
 *              LDS (long smooth lengths, e.g. FP64 n = 1152 or 2048), the
 *              chirp-z kernels run instead: 0 / -1 automatic (the
 *              prime-factor kernels below where they exist, else the
 *              three-stage kernels where they exist, convolution lengths up
 *              to 1024, i.e. n <= 512); 32 / -32 the three-stage kernels
 *              with 256 / 512 threads; 4 / 8 / 16 the two-FFT kernels with at
 *              most that many points per block and 256 threads, -4 / -8 /
 *              -16 with 512 threads (a request that fits no kernel falls back
 *              to the automatic choice); 64 / -64 the prime-factor kernels
 *              with 256 / 512 threads (n = 511 = 7 x 73 by the Good-Thomas
 *              split with a Rader transform of 73 points, 8 / 16 points per
 *              block, the automatic choice there; n = 255 = 15 x 17, 15 / 30
 *              points; n = 127 by a Rader transform, 16 / 32 points); for
 *              other n, 64 / -64 are read as 16 / -16 (Stockham) or fall
 *              back to the automatic choice (chirp-z).
 *   dst_kernel sine-transform kernels of step 2 (PCOP_DST): 0 automatic,
 *              1 register-resident lines, 2 lines staged through LDS,
 *              3 register-resident lines with twice as many strided lines
 *              per block (512 threads), 4 strided lines through a
 *              half-length FFT (nx + 1 points; for nx >= 7, else as 1),
 *              5 the half-length FFT for the contiguous lines as well.
 *   tune       1: pcop_setup times the candidates of every kernel choice
 *              left at 0 ("automatic": time_cols, dst_kernel, kkt_jchunk,
 *              krylov_blocks, gs_update) on the context's stream and keeps
 *              the fastest (the Krylov choices per basis size); the choice
 *              is cached per device and shape for the process.  0:
 *              built-in choices.  All choices give
 *              the same iterates up to rounding (the reduction order follows
 *              the block count).
 *   precond    PCOP_PRECOND_EPS: the epsilon-circulant RBD preconditioner
 *              P_eps (Section 2.1; all time levels at once);
 *              PCOP_PRECOND_IDEAL: the ideal RBD preconditioner P of
 *              eq. matrix_P, applied by sequential substitution in time
 *              (n dependent spatial solves with (1 + alpha) I + tau K; the
 *              comparison method of Tables 4 and 8).  time_cols is ignored.
 *   kkt_jchunk KKT matvec kernel: 0 automatic (-8, or the tuner's choice);
 *              1..64 one thread per point marching that many time levels;
 *              -64..-1 LDS-tiled blocks (1024 points and their in-plane
 *              neighbours staged per level) marching -kkt_jchunk levels
 *              (for nx <= 1024, else as 16).
 *   krylov_blocks  blocks per member of the Krylov reductions: 0 automatic
 *              (with tune = 1: chosen per basis size), else 1..4096 for
 *              every size (the reduction order, and so the rounding,
 *              follows it).
 *   gs_update  Gram-Schmidt update kernel: 0 automatic (with tune = 1:
 *              chosen per basis size), 1 one element per thread and step,
 *              2 double2 pairs.
 *   stream     hipStream_t on which all work is enqueued.
 *   mg_smoother  the V-cycle's Gauss-Seidel pre-smoother (PCOP_MG; Section
 *              3, Example 2 names Gauss-Seidel without an ordering): 0
 *              red-black (red = even index sum first; the default), 1 one
 *              sweep in the natural order (x1 fastest), 2 that sweep and
 *              one in the reverse order.  1 and 2 walk the grid's
 *              hyperplanes x1 + x2 (+ x3) = const one after another (one
 *              block per frequency slice), so they are much slower than 0. */
typedef struct {
  int precision;
  int spatial;
  int side;
  int restart;
  int maxit;
  double rtol;
  int graph;
  int graph_chunk;
  double reorth_tol;
  int time_cols;
  int dst_kernel;
  int tune;
  int precond;
  int kkt_jchunk;
  int krylov_blocks;
  int gs_update;
  void* stream;
  int mg_smoother;
} pcop_options;

/* Per-member outcome of pcop_solve. */
typedef struct {
  int iters;            /* Arnoldi steps taken */
  int converged;        /* 1 if the monitored relative residual <= rtol */
  double relres_est;    /* monitored relative residual from the Givens QR */
  double relres_true;   /* ||b - A x|| / ||b|| recomputed at the end */
} pcop_member_info;

/* Validate a problem/options pair without touching the device.
 * Returns PCOP_OK, PCOP_ERR_INVALID_ARG or PCOP_ERR_UNSUPPORTED. */
pcop_status pcop_validate(const pcop_problem* prob, const pcop_options* opts);

/* Fill in the default options (FP64, DST, right, restart 30, maxit 300,
 * rtol 1e-8, no graph, reorth_tol 1e-8, default stream). */
void pcop_default_options(pcop_options* opts);

/* Bytes of device workspace pcop_setup needs for (prob, opts).  Host-only. */
pcop_status pcop_workspace_size(const pcop_problem* prob, const pcop_options* opts,
                                size_t* bytes);

/* Create a context.  workspace: caller-owned device memory of at least
 * pcop_workspace_size bytes, 256-byte aligned, that stays valid and unused
 * by the caller until pcop_destroy.  Host tables are computed in FP64 (long
 * double where the host has it, rounded once) and copied into the workspace
 * on the stream: the factors of eq. decomposition_eps -- D_eps =
 * diag(eps^{(j-1)/n}) and the eigenvalues lambda_k = 1 - eps^{1/n}
 * theta^{-k} of C_{eps,n} -- the sine-mode eigenvalues of K (Section 3,
 * Example 1), the time and sine-transform twiddles, the chirp-z tables,
 * per-member alpha = tau / sqrt(gamma) (eq. matrix_A), and for PCOP_MG the
 * re-discretised tau K_a of every multigrid level.  With tune = 1 the kernel
 * candidates are timed here (see pcop_options). */
pcop_status pcop_setup(pcop_ctx* out, const pcop_problem* prob, const pcop_options* opts,
                       void* workspace, size_t bytes);

/* b = [g-block; -sqrt(gamma) f-block] of eq. main_system from device g, f
 * [batch][n][m] and y0 [batch][m]: b_1^j = tau M g^j, b_2^j = -sqrt(gamma)
 * M (tau f^j + [j = 1] y0) (eq. main_system_before with p^N = 0; M = I for
 * PCOP_MASS_IDENTITY; with PCOP_MASS_Q1 the intermediate without M is
 * staged in the workspace, on the context's stream). */
pcop_status pcop_rhs(pcop_ctx ctx, const double* g, const double* f, const double* y0,
                     double* b);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), eq. matrix_A.
 * x, y: device vectors; they must not overlap. */
pcop_status pcop_kkt_apply(pcop_ctx ctx, const double* x, double* y, int transpose);

/* w = P_eps^{-1} v by the four steps of Section 2.1 (time FFT with the D_eps
 * scaling, shifted spatial solves, inverse FFT, [[I,-I],[I,I]] combination).
 * v, w: device vectors; they may alias. */
pcop_status pcop_precond_apply(pcop_ctx ctx, const double* v, double* w);

/* w = P_eps^{-1} v exactly as pcop_precond_apply (same kernels, same
 * results), for callers that cannot allocate device memory at call time or
 * hand the library scratch per call: code under HIP graph capture, tight
 * serving loops.  The spectrum scratch is not the context's workspace but a
 * file-scope device array of the library, one per device, held until the
 * process ends; the call itself allocates nothing and does no per-kernel
 * timing.
 *   Limit: the spectrum, 2 (n/2 + 1) m complex values per member (16 bytes
 *   each in FP64, 8 with PCOP_MIXED), must fit 64 MiB; larger contexts get
 *   PCOP_ERR_UNSUPPORTED, as do contexts with PCOP_MG or
 *   PCOP_PRECOND_IDEAL.  The current device must be the one current at
 *   pcop_setup (PCOP_ERR_INVALID_ARG otherwise).
 *   Sharing: every call on a device uses that device's one array (the
 *   forward time pass writes all of it before it is read, so nothing needs
 *   clearing); calls that overlap in time on one device -- from different
 *   streams, contexts or threads -- race and must be serialised by the
 *   caller.
 * v, w: device vectors as in pcop_precond_apply; they may alias. */
pcop_status pcop_precond_apply_noalloc(pcop_ctx ctx, const double* v, double* w);

/* Solve A x = b (transpose = 0) or A^T x = b (transpose = 1) with GMRES
 * preconditioned by P_eps (eq. preconditioned_system: the preconditioned
 * system P_eps^{-1} A x = P_eps^{-1} b for PCOP_LEFT, as in Section 3's
 * experiments with zero initial guess and relative tolerance; A P_eps^{-1}
 * for PCOP_RIGHT and PCOP_FLEXIBLE), or by P of eq. matrix_P with
 * PCOP_PRECOND_IDEAL.  A^T = J A J with J = diag(I, -I), so the transposed
 * solve runs the same iteration on J b and returns J times its solution.  x: device vector, initial guess on entry, solution
 * on exit.  b and x must be 16-byte aligned (PCOP_ERR_INVALID_ARG otherwise).  info: host array [batch] (may be NULL).  res_hist: host array
 * [batch][maxit + 1] of monitored relative residuals (may be NULL; entries
 * after a member's last step are left untouched).  Returns
 * PCOP_NOT_CONVERGED (with x and info filled) when a member misses rtol. */
pcop_status pcop_solve(pcop_ctx ctx, const double* b, double* x, int transpose,
                       pcop_member_info* info, double* res_hist);

/* y = x_1 / sqrt(gamma), p = x_2: device [batch][n][m] each. */
pcop_status pcop_unpack(pcop_ctx ctx, const double* x, double* y, double* p);

/* r = [ybar / sqrt(gamma); pbar]: the cotangent of x for a loss of (y, p).
 * ybar, pbar: device [batch][n][m]; r: device vector. */
pcop_status pcop_pack_cotangent(pcop_ctx ctx, const double* ybar, const double* pbar,
                                double* r);

/* Gradients of a loss with respect to the data from lam = A^{-T} dL/dx:
 * dg = tau M lam_1, df = -sqrt(gamma) tau M lam_2, dy0 = -sqrt(gamma) M lam_2^1
 * (the transpose of the map in pcop_rhs; M = I for PCOP_MASS_IDENTITY).
 * Any output may be NULL. */
pcop_status pcop_data_grad(pcop_ctx ctx, const double* lam, double* dg, double* df,
                           double* dy0);

/* End levels of the discrete solution from a solved x (Section 1, the two
 * formulas after eq. Toeplitz_Mat_B, p^N = 0):
 *   (M + tau K) y^N = M (y^{N-1} + tau f^N),   (M + tau K) p^0 = M (p^1 + tau (g^0 - y^0)),
 * M = I for PCOP_MASS_IDENTITY.
 * x: [batch][2][n][m] solution of pcop_solve; fN, g0, y0: [batch][m] data at
 * t = T, t = 0 and the initial state; outputs yN, p0: [batch][m].  All device
 * FP64 pointers.  Solved by iterative refinement with an FP64 residual and
 * the context's spatial solver (sine transforms in FP64, or one V-cycle per
 * step) until the residual stops decreasing or falls below 1e-14 of the
 * initial one.  relres (host [batch], may be NULL) receives the final
 * ||rhs - E z|| / ||rhs||; PCOP_NOT_CONVERGED when any exceeds 1e-10 (outputs
 * still written).  Uses the context's scratch buffers: not concurrent with
 * pcop_solve on the same context.  Synchronises the stream. */
pcop_status pcop_post_solve(pcop_ctx ctx, const double* x, const double* fN, const double* g0,
                            const double* y0, double* yN, double* p0, double* relres);

/* The error e_h of Section 3 per member:
 *   e_h = h^{d/2} max_{1<=j<=N} max(||y^j - y(t_j)||_2, ||p^{j-1} - p(t_{j-1})||_2),
 * with y^j = x_1^j / sqrt(gamma), p^j = x_2^j for 1 <= j <= n and the end
 * levels yN, p0 of pcop_post_solve.  y_exact, p_exact: device
 * [batch][N+1][m] FP64 values of the exact solution at t_j = j tau,
 * j = 0..N (level N of p and level 0 of y are not read).  eh: host [batch].
 * Fixed-order reductions; synchronises the stream. */
pcop_status pcop_error_eh(pcop_ctx ctx, const double* x, const double* yN, const double* p0,
                          const double* y_exact, const double* p_exact, double* eh);

/* Host copy of a few derived scalars: tau, alpha[batch], eps. */
pcop_status pcop_get_params(pcop_ctx ctx, double* tau, double* alpha, double* eps);

/* Kernel choices in effect (after tuning):
 *   time_cols      Stockham: -P (two LDS buffers, P points per block) or
 *                  +P (in place); chirp-z (nt - 1 with a prime factor above
 *                  17, or no Stockham tile fits LDS): +P (P points, 256
 *                  threads) or -P (512 threads), +-64 (prime-factor);
 *                  0 with PCOP_PRECOND_IDEAL (no time transform);
 *   dst_kernel     1 (register-resident), 2 (LDS-staged), 3 (register, wide
 *                  column tiles), 4 (half-length strided transforms), 5
 *                  (half-length transforms on every axis) or 0 (multigrid);
 *   kkt_jchunk     KKT matvec kernel (as in pcop_options);
 *   krylov_blocks  blocks per member of the Krylov multi-dot over the full
 *                  basis (the tuner picks counts per basis size: shorter
 *                  bases may use others);
 *   gs_update      1 (one element per thread) or 2 (double2 pairs), the
 *                  update kernel over the full basis;
 *   tuned_precond_ms  the fastest preconditioner apply measured by the
 *                  tuner, 0 when no tuning ran. */
typedef struct {
  int time_cols;
  int dst_kernel;
  int kkt_jchunk;
  int krylov_blocks;
  int gs_update;
  double tuned_precond_ms;
} pcop_kernel_choice;
pcop_status pcop_get_kernels(pcop_ctx ctx, pcop_kernel_choice* out);

/* Per-kernel timing.  While enabled, every kernel the context launches is
 * bracketed by HIP events on the context's stream; pcop_timing_read
 * synchronises, and returns for each kernel family the number of launches,
 * the summed event time in milliseconds and the summed algorithmic HBM
 * bytes (what the method must read and write: each input and output vector
 * once).  name points to static storage.  Enabling resets the counters.
 * While timing is enabled pcop_solve runs without graphs (graph = 1 is
 * ignored), so that every kernel can be bracketed. */
typedef struct {
  const char* name;
  long long launches;
  double ms;
  double bytes;
} pcop_kernel_stat;

pcop_status pcop_timing_enable(pcop_ctx ctx, int enable);
pcop_status pcop_timing_read(pcop_ctx ctx, pcop_kernel_stat* out, int cap, int* count, int reset);

/* Release the context (does not free the caller's workspace). */
void pcop_destroy(pcop_ctx ctx);

const char* pcop_status_string(pcop_status s);
const char* pcop_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PCOP_H */
