/*
 * gnk.h -- C ABI of the MI355X (gfx950) solver for boundary integral equations
 * with the generalized Neumann kernel (Nasser, "Fast solution of boundary
 * integral equations with the generalized Neumann kernel").
 *
 * Problem statement (paper Sec. 1, eqs. (e:ie), (e:h), (e:ie*)):
 *   (I - N) mu = -M gamma,   h = [M mu - (I - N) gamma] / 2,
 *   (I + N* + J) mu = gamma,
 * discretised by the trapezoidal-rule Nystrom method with singularity
 * subtraction (Sec. 3.1-3.2 and 4.1-4.2):
 *   (2I + diag(B1) - B) mu = -y,  y = (D - diag(D1) + Lhat) gamma    (eqs. (e:sys), (e:y))
 *   h = [(D - diag(D1) + Lhat) mu - (2I + diag(B1) - B) gamma] / 2   (eq. (e:bh))
 *   (diag(e) + B^T + Phat) mu = gamma                                  (eq. (e:sys*))
 * and solved by restarted GMRES (Sec. 3.5, 4.5) whose matrix-vector product is
 * the Cauchy sum (E w)_i = sum_{j != i} w_j / (eta_i - eta_j) (eq. (e:fmm-E)),
 * evaluated directly on the GPU, plus the m+1 circulant blocks L of Sec. 3.3
 * applied by FFT (eq. (e:L-bs)).
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers on the context's device (for example
 *     torch tensor data pointers). Complex arrays are interleaved pairs of
 *     doubles {re, im} (the layout of complex128). Real arrays are double.
 *   - Node ordering is component-major: node i = k*n + p, component
 *     k = 0..m, node p = 0..n-1 at parameter t = 2*pi*p/n (eq. (e:ti-skp)).
 *   - Multi-column arrays (nrhs right-hand sides) are column-major with
 *     leading dimension N = (m+1)*n: column r starts at element r*N.
 *   - The caller owns every input and output buffer. The library owns its
 *     workspace inside the context (grown on demand, released by gnk_destroy)
 *     and keeps no caller pointer after a call returns.
 *   - Work is enqueued on the context stream; every call returns after the
 *     stream has completed that work, so outputs and info are valid on return.
 *   - Errors are reported by status codes; no exception crosses the ABI.
 *     A negative status means no output was written. GNK_NOT_CONVERGED (> 0)
 *     means the best iterate was written (the "flag = 1" of MATLAB's gmres).
 *     gnk_last_error() returns a message for the last failing call.
 *   - One context per host thread; a context is not thread-safe.
 */
#ifndef GNK_H
#define GNK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Exported entry points (the library is built with hidden default visibility). */
#define GNK_API __attribute__((visibility("default")))

typedef struct gnk_ctx gnk_ctx;

typedef enum {
  GNK_OK = 0,
  GNK_NOT_CONVERGED = 1,   /* result written; GMRES stopped at maxit above tol */
  GNK_ERR_ARG = -1,        /* null pointer, bad size, bad option */
  GNK_ERR_ODD_N = -2,      /* n must be even (Sec. 2.4) */
  GNK_ERR_ZERO_A = -3,     /* A(t_i) == 0 at some node */
  GNK_ERR_ZERO_ETAP = -4,  /* eta'(t_i) == 0 where the adjoint equation divides by it */
  GNK_ERR_NONFINITE = -5,  /* NaN or Inf in an input */
  GNK_ERR_HIP = -10,       /* a HIP runtime call failed */
  GNK_ERR_OOM = -11        /* workspace allocation failed or exceeds GNK_WORKSPACE_MB */
} gnk_status;

typedef enum { GNK_FP64 = 0, GNK_MIXED = 1 } gnk_precision;

/* Operators for gnk_apply (x real N x nrhs -> y real N x nrhs). */
typedef enum {
  GNK_OP_FB = 0,    /* (2I + diag(B1) - B) x                    eq. (e:f_B)          */
  GNK_OP_FC = 1,    /* (D - diag(D1) + Lhat) x                  eqs. (e:y), (e:bh)   */
  GNK_OP_GB = 2,    /* (diag(e) + B^T + Phat) x                 eq. (e:g_B)          */
  GNK_OP_FB_T = 3,  /* (2I + diag(B1) - B)^T x                  transpose of FB      */
  GNK_OP_FC_T = 4,  /* (D - diag(D1) + Lhat)^T x = (D^T - diag(D1) - Lhat) x         */
  GNK_OP_GB_T = 5,  /* (diag(e) + B + Phat) x                   transpose of GB      */
  GNK_OP_LHAT = 6,  /* Lhat x, the circulant blocks alone       eq. (e:L-bs)         */
  /* the same equations without singularity subtraction (Example 2's comparison):
   * the kernel N by the trapezoidal rule with its diagonal limit (e:N-tt),
   * Nd_i = (2 pi/n) N(t_i, t_i); need etapp and Ap */
  GNK_OP_FB_U = 7,  /* (I - B - diag(Nd)) x                     (I - N) x, no subtraction   */
  GNK_OP_GB_U = 8   /* (I + B^T + diag(Nd) + Phat) x            (I + N* + J) x, likewise    */
} gnk_op;

/* Boundary data of an (m+1)-connected domain (Sec. 2.1-2.2).
 *   eta, etap : N complex, eta(t_i) and eta'(t_i).
 *   A         : N complex, nonzero; eq. (e:A) gives the admissible choices
 *               e^{i(pi/2-theta)}(eta-alpha) (bounded) and e^{i(pi/2-theta)}
 *               (unbounded); any nonzero values are accepted.
 *   etapp, Ap : N complex, eta'' and A'; used by the adjoint equation and by
 *               the variants without singularity subtraction (may be NULL
 *               for the FBIE entry points otherwise).
 *   c         : +1 bounded, -1 unbounded (eq. (e:c)); adjoint equation only. */
typedef struct {
  int64_t m1;        /* number of boundary components m+1 (>= 1) */
  int64_t n;         /* nodes per component (even, >= 2) */
  const void* eta;
  const void* etap;
  const void* etapp;
  const void* A;
  const void* Ap;
  int c;
} gnk_domain;

/* Solver options (the restart / gmrestol / maxit arguments of Sec. 3.5).
 *   restart    : inner iterations per cycle (1..256); the Krylov basis takes
 *                (restart+1) * N * nrhs doubles of workspace
 *   maxit      : maximum number of restart cycles (>= 1)
 *   tol        : relative residual ||b - A x||_2 / ||b||_2 per right-hand side
 *   prec       : GNK_FP64, or GNK_MIXED: the Arnoldi products switch to FP32
 *                for well-separated 64-node tiles (FP64 for all other pairs,
 *                the epilogues, the orthogonalisation) once every column's
 *                residual estimate is below inner_tol; the residual starting
 *                each restart cycle is recomputed with FP64 products, so
 *                restarts act as FP64 iterative refinement and the same tol
 *                is reached
 *   inner_tol  : GNK_MIXED switch level (0: min(1e-4, 5e6 tol): the mixed
 *                products' relative error, about 1e-8, then adds at most about
 *                tol/2 to the final residual, so no extra restart is needed)
 *   max_refine : GNK_MIXED: at most this many restart cycles take mixed
 *                products (each is followed by the cycle's FP64 residual, one
 *                step of iterative refinement); the cycles after them take
 *                FP64 products. 0: no limit. Ignored for GNK_FP64.
 *   x0         : optional device initial guess (N x nrhs) or NULL for zero
 *   no_subtraction : 0 (the paper's method); 1 solves gnk_fbie / gnk_fbie_ad
 *                without singularity subtraction (GNK_OP_FB_U / GNK_OP_GB_U,
 *                the comparison of Example 2; needs etapp and Ap); the
 *                right-hand side and h use M as in the paper's method
 *   far_tol    : 0 (every pair summed directly); > 0: the Cauchy sums take
 *                their far field from multipole expansions of boxes of
 *                consecutive nodes (a treecode; the paper uses the FMM), each
 *                truncated where (r_box / distance)^p <= far_tol; FP64 only
 *                (prec GNK_FP64), gnk_fbie and gnk_fbie_ad only; 1e-15..0.1
 *   hist, hist_len : optional residual history (the paper reports GMRES's
 *                convergence, Sec. 7): HOST array of hist_len doubles per
 *                right-hand side (column r at hist + r * hist_len, in the order
 *                of the info entries), caller-owned. Per column it receives the
 *                relative true residual (FP64 product) at the start of each
 *                restart cycle, each followed by the relative residual estimate
 *                after each Arnoldi step of that cycle, and finally the true
 *                residual that ended the solve; gnk_info.hist_count entries are
 *                written, the rest are left untouched. hist_len 0 (hist NULL):
 *                no history; hist_len > 0 needs hist. */
typedef struct {
  int restart;
  int maxit;
  double tol;
  int prec;
  double inner_tol;
  int max_refine;
  const double* x0;
  int no_subtraction;
  double far_tol;
  double* hist;
  int hist_len;
} gnk_opts;

/* Per right-hand side outcome (host memory, one entry per column).
 *   flag        : 0 converged, 1 not converged
 *   outer_it    : restart cycles used (0 for a column converged at the start, e.g. b = 0);
 *                 inner_it: total Arnoldi steps
 *   relres      : GMRES residual estimate at exit
 *   true_relres : ||b - A x|| / ||b|| recomputed with an FP64 product
 *   mixed_steps : Arnoldi steps whose product used FP32 far tiles (GNK_MIXED); at most
 *                 inner_it, and in a solve that switches to mixed products part-way it
 *                 may include up to seven speculative steps after the column stopped
 *   refine_steps: GNK_MIXED: restart cycles of this column that took mixed products,
 *                 each followed by an FP64 residual (refinement steps); 0 for GNK_FP64
 *   hist_count  : entries written to this column's residual history (0 without one) */
typedef struct {
  int flag;
  int outer_it;
  int inner_it;
  int mixed_steps;
  double relres;
  double true_relres;
  int refine_steps;
  int hist_count;
} gnk_info;

/* Context lifetime. device: HIP device ordinal. The context owns a blocking
 * stream of default priority, used unless gnk_set_stream installs a caller
 * stream (hipStream_t; NULL selects the context's own stream again). The
 * Arnoldi step of GMRES is captured once per solve into a hipGraph and
 * replayed (GNK_GRAPH=0 disables this; so does profiling with gnk_profile);
 * a caller stream must therefore be capturable (not the legacy null stream). */
/* Environment (all optional):
 *   GNK_WORKSPACE_MB=m   cap the context's workspace at m MiB (GNK_ERR_OOM beyond)
 *   GNK_GRAPH=0          launch every kernel directly instead of replaying graphs
 *   GNK_LOG=1            print each GMRES cycle's true residual to stderr
 *   GNK_TUNE, GNK_TUNE_CACHE   the batched autotuner (see gnk_fbie_batched)
 *   GNK_CAUCHY_TPT=1|2, GNK_CAUCHY_SPLITS=s   override the pair kernels' targets
 *                        per lane and source splits (the planner's choice otherwise)
 *   GNK_MIXED_THETA=t    separation factor of the far-tile test (default 1): a
 *                        source tile is far from a target tile when their
 *                        bounding circles are (1 + t)(r_t + r_s) apart
 *   GNK_TREE_SPLITS=s    override the treecode's splits per target tile
 * The overrides change launch shapes and the near/far split (in mixed precision,
 * which pairs are summed in FP32), never which pairs are summed. */
GNK_API gnk_status gnk_create(gnk_ctx** ctx, int device);
GNK_API gnk_status gnk_destroy(gnk_ctx* ctx);
GNK_API gnk_status gnk_set_stream(gnk_ctx* ctx, void* hip_stream);
GNK_API const char* gnk_last_error(const gnk_ctx* ctx);
/* Library version string (static storage). */
GNK_API const char* gnk_version(void);

/* Timing of the Cauchy-sum launches (the hot kernel), measured with HIP
 * events recorded on the context stream around every launch while enabled.
 *   launches, ms      : all launches and their summed duration
 *   pair_cols         : sum over launches of N(N-1) * columns
 *   flops             : N(N-1) * (16 + 8 (columns - 1)) summed (16 flops per
 *                       pair and column 1, 8 per further column sharing it)
 *   launches1, ms1, pairs1 : the single-column FP64 launches alone
 *   *_mixed           : the mixed-precision launches (also in the totals)
 *   *_tree            : the treecode products (also in the totals; their flops
 *                       field counts the direct sum they replace): launches,
 *                       time, and the work their interaction lists imply,
 *                       8 p_e + 8 flops per target and far box (a p_e-term
 *                       expansion), 16 per near pair, for each column
 *   *_fft             : the circulant products L-hat x (not in the totals):
 *                       launches (one per call, all block lengths), time, and
 *                       algorithmic bytes, 24 per unknown and column (read x,
 *                       read and write y) */
typedef struct {
  int64_t launches;
  double ms;
  double pair_cols;
  double flops;
  int64_t launches1;
  double ms1;
  double pairs1;
  int64_t launches_mixed;   /* mixed-precision launches (any column count) */
  double ms_mixed;
  double pair_cols_mixed;
  int64_t launches_tree;    /* treecode products (any column count) */
  double ms_tree;
  double flops_tree;
  int64_t launches_fft;     /* circulant products */
  double ms_fft;
  double bytes_fft;
} gnk_prof;

/* enable: 1 starts recording, 0 stops (already recorded launches are kept).
 * While enabled, solves launch every kernel directly (no graph replay), and
 * the fully masked speculative Arnoldi steps that GMRES runs after its last
 * column stops (they do no work) are left out of the totals. */
GNK_API gnk_status gnk_profile(gnk_ctx* ctx, int enable);
/* Waits for the stream, folds the recorded launches into the totals, copies
 * them to *out (may be NULL), and clears them when reset != 0. */
GNK_API gnk_status gnk_profile_read(gnk_ctx* ctx, gnk_prof* out, int reset);

/* Cauchy sum S = E w (eq. (e:fmm-E), the product that the paper computes with
 * zfmm2dpart, eq. (e:E-fmm)):  S_i = sum_{j != i} w_j / (eta_i - eta_j).
 *   N     : number of nodes; eta: N complex.
 *   w     : N x nrhs complex; S: N x nrhs complex (output, must not alias w).
 * FP64; every pair is evaluated directly (no far-field approximation).
 * Coincident nodes (eta_i == eta_j, i != j) give non-finite sums. */
GNK_API gnk_status gnk_cauchy_sum(gnk_ctx* ctx, int64_t N, const void* eta, const void* w, int nrhs,
                          void* S);

/* gnk_cauchy_sum for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, layout and results, but the call allocates nothing. Its
 * workspace (node records, split partial sums, tile bounds, work lists) lives
 * in a fixed 64 MiB device array that the library holds on each GPU it runs on
 * until the process ends. That limits the size: the call needs about
 *   N * (40 + 16 (3 + 2 (nrhs + 1)) + 16 s (nrhs + 1)) bytes plus small tables,
 * s being the planner's source splits (1..64, fewer for larger N; the split
 * partial sums dominate): N = 65536 with nrhs = 1 fits, N = 264192 does not.
 * Larger inputs return GNK_ERR_ARG with a message naming the buffer that did
 * not fit, and nothing is written. Every call on one GPU shares that GPU's
 * array and overwrites it: calls that overlap on one GPU (several host threads
 * or contexts) race and must be serialised by the caller. */
GNK_API gnk_status gnk_cauchy_sum_noalloc(gnk_ctx* ctx, int64_t N, const void* eta, const void* w, int nrhs,
                                          void* S);

/* Cauchy integral formula at interior points (Sec. 7, eqs. (e:cauchy5) and
 * (e:cauchy6)): the values f(z_i) at nz points of G of a function analytic in G,
 * from its values at the N = m1 n boundary nodes, by the subtracted form
 *   bounded G:    f(z) = P_f / P_1
 *   unbounded G:  f(z) = (f(inf) - P_f/(n i)) / (1 - P_1/(n i))
 * with P_f = sum_j f_j eta'_j / (z - eta_j) and P_1 = sum_j eta'_j / (z - eta_j)
 * summed directly in FP64 over every node (no far-field approximation).
 *   eta, etap : N complex (device), nodes and derivatives, component-major
 *   f         : N x nrhs complex (device), boundary values, leading dim N
 *   z         : nz complex (device), the points (in G; any layout of them)
 *   finf      : NULL for bounded G; for unbounded G, a HOST array of nrhs
 *               complex values f(infinity)
 *   fz        : nz x nrhs complex (device, output, leading dim nz); must not
 *               alias f, z, eta or etap.
 * n is the number of nodes per boundary component (the weight 2 pi/n); it need
 * not be even here. A point equal to a node gets that node's value (the limit
 * of the ratio); points outside G give the formula's value there (not f).
 * Errors: GNK_ERR_ARG for sizes outside 1..2^30 (N, nz), nrhs outside 1..4096,
 * NULL or aliased pointers; nothing is written then. */
GNK_API gnk_status gnk_fcau(gnk_ctx* ctx, int64_t m1, int64_t n, const void* eta, const void* etap,
                            const void* f, int nrhs, const void* z, int64_t nz, const void* finf, void* fz);

/* Conformal map of a bounded (m+1)-connected domain onto the unit disc with
 * m circular slits (Example 3, theta = pi/2), from one FBIE solve: with
 * A = eta - alpha and gamma = -log|eta - alpha| (alpha in G), the boundary
 * values are f(eta) = exp(-h_0) (eta - alpha) exp(gamma + h + i mu) and the
 * slit radii R_j = exp(h_j - h_0) (h_j the mean of FBIE's h over component j;
 * R_0 = 1), so f(alpha) = 0 and f'(alpha) > 0.
 *   eta, etap : N complex (device), component-major, outer boundary first (ccw),
 *               inner boundaries clockwise
 *   alpha     : host, 2 doubles {Re, Im}, a point of G
 *   opts      : as for gnk_fbie (NULL: defaults); far_tol allowed
 *   f         : N complex (device, output): boundary values of the map
 *   radii     : host array of m1 doubles (output) or NULL
 *   info      : host, one entry (the FBIE solve) or NULL
 * Interior values follow from gnk_fcau with these boundary values.
 * Errors: GNK_ERR_ARG for NULL or aliased pointers, sizes, no_subtraction, and
 * alpha outside G (as for gnk_slit_map, which this is with bounded = 1 and
 * theta = pi/2). */
GNK_API gnk_status gnk_circular_slit_map(gnk_ctx* ctx, int64_t m1, int64_t n, const void* eta, const void* etap,
                                         const double* alpha, const gnk_opts* opts, void* f, double* radii,
                                         gnk_info* info);

/* gnk_fcau with the two Cauchy sums from the treecode (see gnk_opts.far_tol):
 * the nodes' box tree, target tiles of 128 points, far boxes by p_e-term
 * expansions with (r/R)^p_e <= far_tol, near 64-node blocks summed directly.
 * Same arguments, layout and results as gnk_fcau, plus far_tol (1e-15..0.1);
 * GNK_ERR_ARG for far_tol outside that range. For many points around a large
 * boundary (N in the millions), where the direct sums take N nz pairs. */
GNK_API gnk_status gnk_fcau_tree(gnk_ctx* ctx, int64_t m1, int64_t n, const void* eta, const void* etap,
                                 const void* f, int nrhs, const void* z, int64_t nz, const void* finf,
                                 double far_tol, void* fz);

/* Conformal map of an (m+1)-connected domain onto a canonical domain with
 * slits, from one FBIE solve with the piecewise constant theta of eq. (e:A):
 * circular slits for theta_j = pi/2, radial slits for theta_j = 0 (Examples 3
 * and 4), arcs of logarithmic spirals for other values. With
 * rot_j = exp(i (pi/2 - theta_j)), gamma = -Re[rot_j log(eta - alpha)] (the
 * logarithm continued along each component) and h_j the mean of FBIE's h over
 * component j:
 *   bounded G:   A = rot_j (eta - alpha), theta_0 = pi/2,
 *                f(eta) = exp(-h_0) (eta - alpha) exp((gamma + h_j + i mu) / rot_j):
 *                the unit disc with slits, f(alpha) = 0, f'(alpha) > 0,
 *                level_j = h_j - h_0 sin(theta_j) (level_0 = 0);
 *   unbounded G: A = rot_j,
 *                f(eta) = (eta - alpha) exp((gamma + h_j + i mu) / rot_j):
 *                the extended plane with m + 1 slits, f(alpha) = 0,
 *                f(z) = z + O(1) at infinity, level_j = h_j.
 * On Gamma_j, Re[rot_j log f] = level_j: a circle of radius exp(level_j) for
 * theta_j = pi/2, a radial slit at angle -level_j for theta_j = 0.
 *   eta, etap : N complex (device), component-major; bounded: outer boundary
 *               first (ccw), the others clockwise; unbounded: all clockwise
 *   bounded   : 1 for a bounded G, 0 for an unbounded one
 *   alpha     : host, 2 doubles {Re, Im}, a point of G
 *   theta     : host, m1 doubles (theta[0] = pi/2 when bounded); NULL = pi/2 everywhere
 *   opts      : as for gnk_fbie (NULL: defaults); far_tol allowed
 *   f         : N complex (device, output): boundary values of the map
 *   level     : host array of m1 doubles (output) or NULL
 *   info      : host, one entry (the FBIE solve) or NULL
 * Interior values follow from gnk_fcau with these boundary values (for an
 * unbounded G, from those of f(z) - z, whose value at infinity is finite).
 * Errors: GNK_ERR_ARG for NULL or aliased pointers, sizes, bounded not 0 or 1,
 * no_subtraction, theta[0] != pi/2 (bounded) or a non-finite theta, and alpha
 * outside G (found from the winding of each component around alpha: 1 for the
 * outer boundary of a bounded G, 0 for every other component). */
GNK_API gnk_status gnk_slit_map(gnk_ctx* ctx, int64_t m1, int64_t n, const void* eta, const void* etap, int bounded,
                                const double* alpha, const double* theta, const gnk_opts* opts, void* f,
                                double* level, gnk_info* info);

/* gnk_cauchy_sum with the far field from the treecode (see gnk_opts.far_tol):
 * S_i = sum_{j != i} w_j / (eta_i - eta_j), near pairs summed directly, far
 * boxes by p-term expansions with (r/R)^p <= far_tol (1e-15..0.1). Same
 * arguments and layout as gnk_cauchy_sum; GNK_ERR_ARG for far_tol outside
 * that range. */
GNK_API gnk_status gnk_cauchy_sum_tree(gnk_ctx* ctx, int64_t N, const void* eta, const void* w, int nrhs,
                                       double far_tol, void* S);

/* Operator application y = op(x) for one domain (see gnk_op). x and y are
 * real N x nrhs and must not alias. GB and GB_T need etapp, Ap and c.
 * prec: GNK_FP64, or GNK_MIXED (Cauchy sums over well-separated 64-node tiles
 * in FP32 on tile-local coordinates, all other pairs and every epilogue in
 * FP64; the relative error of the product is about 1e-7). */
GNK_API gnk_status gnk_apply(gnk_ctx* ctx, const gnk_domain* dom, int op, int prec, const double* x, int nrhs,
                             double* y);

/* FBIE (Sec. 3): solve (I - N) mu = -M gamma and compute h for nrhs columns.
 *   gam : N x nrhs real (input);  mu, h : N x nrhs real (outputs).
 *   h may be NULL to skip it. info: host array of nrhs entries or NULL. */
GNK_API gnk_status gnk_fbie(gnk_ctx* ctx, const gnk_domain* dom, const double* gam, int nrhs,
                    const gnk_opts* opts, double* mu, double* h, gnk_info* info);

/* FBIEad (Sec. 4): solve (I + N* + J) mu = gamma for nrhs columns.
 * Needs dom->etapp, dom->Ap and dom->c; eta' must be nonzero at every node. */
GNK_API gnk_status gnk_fbie_ad(gnk_ctx* ctx, const gnk_domain* dom, const double* gam, int nrhs,
                       const gnk_opts* opts, double* mu, gnk_info* info);

/* Batched FBIE: ndom independent domains, each with its own nrhs[d] columns,
 * solved together (every Cauchy-sum launch covers all domains and columns;
 * the GMRES steps run for all columns at once, converged columns are masked).
 *   doms  : host array of ndom domains
 *   gam   : host array of ndom device pointers, gam[d] is N_d x nrhs[d]
 *   mu, h : host arrays of ndom device pointers (h may be NULL, or h[d] NULL)
 *   info  : host array of sum(nrhs) entries, domain-major, or NULL
 * The pair-kernel launch shape is chosen by a built-in autotuner (timed once
 * per batch signature; GNK_TUNE=0 disables it, GNK_TUNE_CACHE=path keeps the
 * choices in a text file). opts->x0 must be NULL. */
GNK_API gnk_status gnk_fbie_batched(gnk_ctx* ctx, int ndom, const gnk_domain* doms, const double* const* gam,
                                    const int* nrhs, const gnk_opts* opts, double* const* mu, double* const* h,
                                    gnk_info* info);

/* ------------------------------------------------------------------------
 * Differentiation (reverse mode). L is any real function of the FBIE outputs;
 * g_mu = dL/dmu and g_h = dL/dh are its cotangents. From
 *   Aop mu = -Cop gamma,  h = (Cop mu - Aop gamma)/2,
 *   Aop = 2I + diag(B1) - B (eq. (e:sys)),  Cop = D - diag(D1) + Lhat ((e:y), (e:bh)):
 *   lam       = Aop^{-T} (Cop^T g_h / 2 + g_mu)            (adjoint GMRES)
 *   dL/dgamma = -Aop^T g_h / 2 - Cop^T lam
 *   dL (geometry) = (g_h/2)^T dCop mu - (g_h/2)^T dAop gamma
 *                   - lam^T dAop mu - lam^T dCop gamma
 * The transposes use B^T x = (2/n) Im[(eta'/A) E(A x)] (eq. (e:BTx)) and its
 * real part for D^T, and L^T = -L. Complex gradients follow the convention of
 * torch.autograd: g = dL/dRe z + i dL/dIm z.
 * ------------------------------------------------------------------------ */

/* Adjoint solve of FBIE for nrhs columns.
 *   g_mu, g_h : N x nrhs real cotangents (either may be NULL = zero, not both)
 *   lam       : N x nrhs real output (the adjoint variable above)
 *   g_gam     : N x nrhs real output dL/dgamma (may be NULL)
 *   opts      : GMRES options for the transposed system (opts->x0: initial lam)
 *   info      : host array of nrhs entries or NULL. */
GNK_API gnk_status gnk_fbie_adjoint(gnk_ctx* ctx, const gnk_domain* dom, const double* g_mu, const double* g_h,
                                    int nrhs, const gnk_opts* opts, double* lam, double* g_gam, gnk_info* info);

/* Gradient of s = sum_t coef[t] * u_t^T Op_t v_t with respect to the boundary
 * data eta, eta', A (the operators' dependence through K_ij =
 * (2/n)(A_i/A_j) eta'_j/(eta_j - eta_i), eqs. (e:N), (e:M)).
 *   nterms : 1..64;  ops: host array, each GNK_OP_FB or GNK_OP_FC
 *   coef   : host array of real factors, or NULL (all 1)
 *   u, v   : host arrays of nterms device pointers to real N-vectors (terms
 *            with the same v pointer share work)
 *   g_eta, g_etap, g_A : N complex outputs (overwritten); any may be NULL,
 *            not all. FP64, every pair evaluated directly. */
GNK_API gnk_status gnk_geom_vjp(gnk_ctx* ctx, const gnk_domain* dom, int nterms, const int* ops, const double* coef,
                                const double* const* u, const double* const* v, void* g_eta, void* g_etap,
                                void* g_A);

/* Boundary curves given by Fourier series, m1 components of n nodes:
 *   eta_j(t_p) = sum_{k=kmin}^{kmin+nk-1} c_{j,k} e^{i s k t_p},  t_p = 2 pi p / n,
 * s = +1 (ccw != 0) or -1, with eta' (factor i s k) and eta'' (factor -k^2).
 *   coef : m1 x nk complex (component-major);  eta: m1*n complex output;
 *   etap, etapp: outputs, may be NULL. */
GNK_API gnk_status gnk_fourier_curve(gnk_ctx* ctx, int64_t m1, int64_t n, int kmin, int nk, int ccw,
                                     const void* coef, void* eta, void* etap, void* etapp);

/* Reverse mode of gnk_fourier_curve: g_coef[j,k] = sum_p (g_eta + conj(i s k) g_eta'
 * + conj(-k^2) g_eta'')_p e^{-i s k t_p}; any of g_eta, g_etap, g_etapp may be
 * NULL (zero), not all. g_coef: m1 x nk complex output. */
GNK_API gnk_status gnk_fourier_vjp(gnk_ctx* ctx, int64_t m1, int64_t n, int kmin, int nk, int ccw,
                                   const void* g_eta, const void* g_etap, const void* g_etapp, void* g_coef);

#ifdef __cplusplus
}
#endif

#endif /* GNK_H */
