/*
 * ctmrg.h -- C ABI of the MI355X (gfx950) CTMRG library.
 *
 * The library runs the corner-transfer-matrix renormalization group step of
 * Ueda, Okunishi, Yunoki and Nishino, "Corner transfer matrix renormalization
 * group analysis of the two-dimensional dodecahedron model" (Sec. III,
 * Algorithm 3) for a q-state vector-spin model on the square lattice whose
 * Boltzmann weight sits on every other plaquette (Sec. II, Eqs. 1-2):
 *
 *   W[s,sg,s',sg'] = exp(K (v_s.v_sg + v_sg.v_sg' + v_sg'.v_s' + v_s'.v_s)),  K = 1/T,
 *
 * with the corners of a plaquette in the cyclic order s, sg, sg', s' (s and s'
 * are the two legs that border the same edge of the extended corner).
 *
 * State: the corner matrix is kept diagonal, C = diag(omega) (m values), and the
 * half-row transfer tensor P is stored as q symmetric m x m slices P_s, laid out
 * side by side as the m x (q m) row-major matrix A[gamma][s*m + alpha] = P_s[gamma][alpha]
 * (the paper's P with its (state, spin) column index).  Rows and columns beyond
 * the current kept dimension m_eff are zero.  Every combined index of an
 * (m q) x (m q) matrix is spin-major: row (s, alpha) -> s*m + alpha.
 *
 * One step (ctmrg_step):
 *   1. X_{s sg} = P_s Omega P_sg for all q^2 spin pairs   (Algorithm 3, the product P^t P')
 *   2. C'_{s' sg'} = sum_{s,sg} W[s,sg,s',sg'] X_{s sg}     (the product with w; C' is (mq)x(mq))
 *   3. all eigenvalues of C'; eigenvectors of the m largest |lambda| (the EigenExa call)
 *   4. keep m_eff <= m of them without splitting a multiplet (|l_j|-|l_{j+1}| > gap_tol |l_1|)
 *   5. P~_{sg'} = sum_{s'} U_{s'}^t (sum_{s,sg} W[s,sg,s',sg'] P_s U_sg)  (second Sub-CTMRG and U^t X)
 *   6. P <- P~ / max|P~|;  Omega <- lambda_kept / (sum over all mq eigenvalues of lambda^4)^(1/4)
 *   7. S_E = -sum w^4 ln w^4 over all eigenvalues (Eq. 6), Delta = max_j |w_j^4(k) - w_j^4(k-1)|.
 *
 * Memory and ownership: every call copies its host inputs; outputs go to
 * caller-provided host memory.  The context owns all device memory it uses
 * (allocated by ctmrg_init, freed by ctmrg_destroy).  A context is bound to the
 * device that was current at ctmrg_init and to one HIP stream (its own, or the
 * caller's hip_stream); contexts are not thread-safe, use one per thread.
 *
 * Errors: every call returns a ctmrg_status; no C++ exception crosses the ABI.
 * The message of the last failure is available from ctmrg_last_error.
 */
#ifndef CTMRG_H
#define CTMRG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CTMRG_OK = 0,
    CTMRG_E_INVALID_ARG = 1,   /* bad size, null pointer, non-unit vector, K <= 0, ... */
    CTMRG_E_OUT_OF_MEMORY = 2, /* device or host allocation failed */
    CTMRG_E_HIP = 3,           /* a HIP runtime call failed */
    CTMRG_E_NOT_CONVERGED = 4, /* max_steps reached; the state is kept and can be resumed */
    CTMRG_E_NUMERICAL = 5,     /* NaN/Inf, or a bounded kernel wait hit its limit */
    CTMRG_E_STATE = 6,         /* wrong call order (e.g. observables before two steps) */
    CTMRG_E_UNSUPPORTED = 7    /* option not available in this build */
} ctmrg_status;

/* Precision of the contractions (steps 1, 2 and 5 above).
 *   CTMRG_FP64: FP64 operands on the FP64 matrix cores.
 *   CTMRG_FP32: the mixed path.  P, Omega, U and W are rounded to FP32 operands
 *     (W scaled by e^{-4K} first, so no weight overflows), products run on the
 *     FP32 matrix cores with FP32 accumulation, and C' and P~ are produced in
 *     FP64 with the factor restored.  The state, the eigensolver, the cut, all
 *     normalizations, the log bookkeeping and the observables stay FP64.  The
 *     contraction error is ~1e-7 relative to max|C'|, which also splits
 *     multiplets of C' by that much: use gap_tol >= 1e-6 on this path.
 *   CTMRG_BF16X3: the mixed path with the same FP32 operands, each split into
 *     two bf16 parts (hi = bf16(x), lo = bf16(x - hi), round to nearest even),
 *     and every product taken as hi*hi + hi*lo + lo*hi on the bf16 matrix cores
 *     with FP32 accumulation (the three-term split of Henry, Tang and
 *     Heinecke, ARITH 2019).  The dropped lo*lo term and the rounding of the lo
 *     parts leave a relative error of order 2^-18 per product (2^-16 at
 *     most), so the contraction error is about ten times CTMRG_FP32's (about
 *     5e-6 of max|C'|) and f, E and M reach 1e-5 rather than 1e-6.  Its
 *     rounding splits multiplets of C' by up to about 5e-6 |lambda_1|: a
 *     gap_tol of 1e-5 or more recognizes them where the gaps at the cut are
 *     wider (at q = 20, m = 512, T = 0.4398 they are about 2e-6 |lambda_1|,
 *     below this path's resolution, and a wide gap_tol there merges the whole
 *     tail into one cluster and cuts far below m). */
typedef enum { CTMRG_FP64 = 0, CTMRG_FP32 = 1, CTMRG_BF16X3 = 2 } ctmrg_precision;
typedef enum { CTMRG_BC_FIXED = 0, CTMRG_BC_FREE = 1 } ctmrg_bc;

/* Eigensolver of step 3.
 *   CTMRG_EIG_TWO_STAGE: every step reduces C' to band and tridiagonal form
 *     (all q m eigenvalues exactly; eigenvectors of the m largest |lambda|).
 *   CTMRG_EIG_WARM: from the third step on, the leading k = m + warm_guard
 *     eigenpairs of C' from the previous step's (Chebyshev-filtered subspace
 *     iteration with Rayleigh-Ritz, all FP64; the kept eigenvectors of every
 *     step rotated inside each multiplet to match the step before, so that the
 *     renormalized basis stays in one gauge).  A step whose kept residuals do
 *     not fall below warm_tol |lambda_1| within the pass limit runs the
 *     two-stage solver instead.  The products use the lower triangle of C'
 *     (mirrored into the upper one first), the part the two-stage solver reads.
 *     n_C and S_E (Eq. 6) then come from the k Ritz values plus the part of
 *     sum lambda^4 beyond them (see ctmrg_warm_tail), and the spectrum buffer
 *     holds the k Ritz values ascending followed by NaN. */
typedef enum { CTMRG_EIG_TWO_STAGE = 0, CTMRG_EIG_WARM = 1 } ctmrg_eig_solver;

/* The part of sum lambda^4 beyond the Ritz block of the warm solver.
 *   CTMRG_WARM_TAIL_EXACT: sum lambda^4 = ||C'^2||_F^2, from one product C' C'
 *     (the tiles on and below the diagonal), so n_C is exact to rounding; the
 *     tail's share of S_E lies within a bound (ctmrg_get_eig_stats).
 *   CTMRG_WARM_TAIL_BOUND: no product; sum lambda^2 beyond the block is
 *     ||C'||_F^2 - sum theta^2, each |lambda| is at most |theta_k|, and the
 *     midpoint of the resulting interval for sum lambda^4 is taken.
 *   CTMRG_WARM_TAIL_AUTO (default): the product only in steps where the bound
 *     on the tail's share of sum w^4 exceeds the contractions' own precision
 *     (1e-14 with FP64 contractions, 1e-9 with FP32 or BF16X3), the midpoint otherwise. */
typedef enum { CTMRG_WARM_TAIL_EXACT = 0, CTMRG_WARM_TAIL_BOUND = 1, CTMRG_WARM_TAIL_AUTO = 2 } ctmrg_warm_tail;

typedef struct {
    int precision;        /* ctmrg_precision of the contractions; the eigensolver is always FP64 */
    int bc;               /* ctmrg_bc: fixed (all boundary spins = boundary_spin) or free      */
    int boundary_spin;    /* vertex index of the fixed boundary spin (the paper's s = 1)       */
    int band;             /* eigensolver half-bandwidth: 16 (default) or 32                    */
    double gap_tol;       /* multiplet gap, relative to |lambda_1| (default 1e-10; >= 1e-6 for FP32) */
    double rank_tol;      /* eigenvalues with |l| <= rank_tol |l_1| are never kept (1e-13)     */
    void *hip_stream;     /* hipStream_t to run on; NULL = a stream owned by the context       */
    int eig_solver;       /* ctmrg_eig_solver (default CTMRG_EIG_TWO_STAGE)                    */
    int warm_guard;       /* CTMRG_EIG_WARM: guard vectors below the kept ones (0 = max(8, m/4)) */
    int warm_degree;      /* CTMRG_EIG_WARM: largest Chebyshev degree per pass, 1..8 (0 = 8)   */
    double warm_tol;      /* CTMRG_EIG_WARM: kept residuals below warm_tol |lambda_1|
                             (0 = 1e-12 for FP64 contractions, 1e-8 for FP32 / BF16X3)       */
    int warm_tail;        /* CTMRG_EIG_WARM: ctmrg_warm_tail (default CTMRG_WARM_TAIL_AUTO)    */
    void *workspace;      /* NULL, or device memory of workspace_bytes >= ctmrg_workspace_size()
                             bytes, owned by the caller and kept alive until ctmrg_destroy: every
                             device buffer ctmrg_init would allocate is carved from it instead
                             (256-byte aligned).  Pinned host buffers, and the buffers that
                             ctmrg_observables and the derivative allocate on first use
                             (ctmrg_extra_workspace_size), are still allocated by the library. */
    size_t workspace_bytes;
} ctmrg_options;

typedef struct {
    double f;              /* free energy per site, -(T/2) ln kappa_W                            */
    double E;              /* energy per site from the central plaquette, (1/2) <h_4>           */
    double M;              /* magnetization, Eq. 5 (fixed BC: v_{s0}.v_s; free BC: |<v_s>|)      */
    double S_E;            /* entanglement entropy of the last step, Eq. 6, over all q m eigenvalues
                              of its C' (after a warm-solved step they are computed here)        */
    double ln_kappa_W;     /* ln of the partition function per vertex from the normalizations  */
    double ln_kappa_ratio; /* the same from Z_d Z_b / Z_h^2 on the current state                 */
    double delta;          /* convergence measure of the last step                              */
    double c_paper;        /* |1 - S_E(k)/S_E(k-1)|, the paper's stopping quantity              */
    int m_eff;             /* kept dimension of the last step                                   */
    int steps;             /* steps taken since init / import                                   */
    /* Effective correlation length (Sec. II, last paragraph) from the renormalized
     * row-to-row transfer matrix T = sum_s P_s (x) P_s (m^2 x m^2, the stored P):
     * its two eigenvalues of largest modulus by Lanczos, xi_e = 1 / ln|l1 / l2|
     * in rows of vertices (0 if l2 = 0). */
    double xi_e;
    double tm_lambda1;     /* leading eigenvalue of T                                            */
    double tm_lambda2;     /* second eigenvalue by modulus                                       */
    double tm_residual;    /* max ||T y - l y|| / |l1| of the two Ritz pairs                     */
    int tm_iterations;     /* Lanczos iterations                                                 */
    int tm_converged;      /* 1 if both residual estimates fell below 1e-11 |l1|                 */
} ctmrg_observables_t;

typedef struct ctmrg_ctx ctmrg_ctx;

/* Defaults: FP64, fixed boundary, boundary_spin 0, band 16, gap_tol 1e-10, rank_tol 1e-13,
 * two-stage eigensolver. */
ctmrg_status ctmrg_default_options(ctmrg_options *opt);

/* Create a context for q spins (vertex_vectors: q x dim row-major unit vectors,
 * copied), coupling K = 1/T > 0 and cutoff m >= 1.  opt may be NULL (defaults).
 * The state is initialized as in Algorithm 3: P_s = [delta_{s,s0}] (fixed) or
 * [1] (free), Omega = [1].  Requires a gfx950 device; allocates all memory. */
ctmrg_status ctmrg_init(int q, int dim, const double *vertex_vectors, double K, int m, const ctmrg_options *opt,
                        ctmrg_ctx **out);

/* Change K (rebuilds W) and reset the state to the initial one; buffers are reused. */
ctmrg_status ctmrg_set_K(ctmrg_ctx *ctx, double K);

/* Run nsteps CTMRG steps, each one pass of the loop body of Algorithm 3 (Sec. III): the
 * extension of the corner by the first Sub-CTMRG contraction and the weight, its
 * diagonalization, the cut and normalization (with S_E of Eq. 6), the renormalized half-row
 * by the second Sub-CTMRG contraction and the projection, and its normalization.
 * delta_out (nullable) receives Delta of the last step (the change of the normalized kept
 * spectrum, w_j^4, between consecutive steps, the loop's stopping quantity). */
ctmrg_status ctmrg_step(ctmrg_ctx *ctx, int nsteps, double *delta_out);

/* The loop of Algorithm 3 to its stopping rule: step until Delta < tol (after at least two
 * steps) or max_steps steps were taken.  Returns CTMRG_E_NOT_CONVERGED if max_steps is reached
 * (the state is kept). */
ctmrg_status ctmrg_run_to_fixed_point(ctmrg_ctx *ctx, double tol, int max_steps, int *steps_out, double *delta_out);

/* A sweep over temperatures, the scans of Sec. IV (for one cutoff m: a (T, m) grid is one
 * context per m).  For each T[i] in order: K = 1/T[i]; the state restarts from the boundary
 * (warm_start = 0; as ctmrg_set_K) or is kept from the previous temperature's fixed point
 * (warm_start = 1; W is rebuilt; for T[0], the state the context holds, so that a sweep can be
 * continued by further calls, or the boundary if the context has taken no step since init or
 * ctmrg_set_K); at least two and at most
 * max_steps steps until Delta < tol; then out[i] = ctmrg_observables (M, S_E, xi_e, f, E, ...).
 * steps_out[i] and converged[i] (both nullable) receive the steps taken and whether Delta < tol
 * was reached; a temperature that does not converge is reported and the sweep continues.
 * deriv_out (nullable, n entries; declared below): at every temperature whose run converged
 * (to Delta < min(tol, 1e-6)), deriv_out[i] = ctmrg_fixed_point_derivative with
 * second_order = 1 (dF/dK, d2F/dK2 = dE/dK and dM/dK along the fixed point); zeros elsewhere.
 * A derivative that fails with CTMRG_E_NOT_CONVERGED or CTMRG_E_NUMERICAL leaves zeros with
 * that status in deriv_out[i].status, and the sweep continues.
 * With the environment variable CTMRG_PROGRESS set (to anything but 0), every hundredth step of
 * a temperature is reported on stderr.
 * Errors: CTMRG_E_INVALID_ARG (n < 0, a temperature not positive, max_steps < 2, tol < 0),
 * and those of ctmrg_step, ctmrg_observables and ctmrg_fixed_point_derivative, which stop the
 * sweep. */
struct ctmrg_derivative_s;
ctmrg_status ctmrg_sweep(ctmrg_ctx *ctx, int n, const double *T, double tol, int max_steps, int warm_start,
                         ctmrg_observables_t *out, int *steps_out, int *converged,
                         struct ctmrg_derivative_s *deriv_out);

/* Observables of the current state (Sec. II: Eqs. 3-6 on the fixed-point
 * matrices; the free energy from the normalization history).  Needs >= 1 step
 * since init, set_K, set_state or import_state; f and ln_kappa_W need two and
 * are NaN after one.  kept_spectrum (nullable, m entries) receives omega
 * (normalized kept eigenvalues, zero padded).  After a step solved by the warm
 * eigensolver, whose C' warm mode keeps, S_E is computed here from all
 * eigenvalues of that C' (the two-stage reduction, eigenvalues only), which
 * then also fill the spectrum buffer.
 * Errors: CTMRG_E_STATE before the first step. */
ctmrg_status ctmrg_observables(ctmrg_ctx *ctx, ctmrg_observables_t *out, double *kept_spectrum);

/* Derivatives of the free energy per site F = beta f at the fixed point with
 * respect to K, by implicit differentiation through the fixed-point map
 * (tangent mode).  The state must be converged (Delta < 1e-6; the routine
 * then converges it further in FP64, in the gauge in which the kept
 * eigenvectors of consecutive steps are aligned inside every multiplet, until
 * P repeats element by element).  The tangent t = dx/dK solves (I - J) t = d_K Phi
 * (J: the derivative of one step, with the kept eigenvectors' derivative
 * sum_i u_i (u_i^T dC' u_j) / (lambda_j - lambda_i) over the discarded
 * eigenpairs i of C', and the corner's tangent carried as a full symmetric
 * block, so that rotations inside the kept space -- degenerate or not -- are
 * treated as gauge), and dF/dK follows from F = -1/2 ln ||P~||_F at
 * the fixed point.  The linear system is solved by restarted GMRES (64 Krylov
 * vectors, classical Gram-Schmidt twice) with J t applied matrix-free, to a
 * relative residual of 1e-12 (or, where restarts no longer reduce it, 1e-10),
 * at most 3000 products J t; tangent_change reports max |J t + d_K Phi - t| at
 * the solution.
 * Along the converged tangent the routine also differentiates the impurity
 * energy E of the plaquette (Sec. II; the product rule through the
 * environment sums, with dW/dK = -W h4) and the magnetization M (Eq. 5; the
 * spin weights of U Omega^4 U^T with the tangents of U and of the corner
 * block): dE_dK and dM_dK are always filled.  dF/dK equals E at every fixed
 * point (the CTMRG free energy is stationary in the environment; E and dF_dK
 * agree to the convergence of the fixed point), so d2F/dK2 = dE/dK:
 * second_order == 1 returns it as d2F_dK2 (no further fixed point);
 * second_order == 2 returns instead the central difference of dF/dK at
 * K (1 +- 1e-4), each from its own converged fixed point (a cross-check, three
 * tangent solves).  The context's state, K and weight are left unchanged; work
 * memory (about 16 (q m_eff)^2 doubles, 69 tangent vectors of q m_eff^2 +
 * m_eff^2 doubles for GMRES, and a full eigensolver workspace;
 * ctmrg_extra_workspace_size) is allocated on the first call and kept until
 * ctmrg_destroy.  Runs in FP64 whatever the context's precision.  With the
 * environment variable CTMRG_PROGRESS set (to anything but 0), every tenth
 * aligned step and every twentieth product J t is reported on stderr.
 * Errors: CTMRG_E_STATE if the state is not converged; CTMRG_E_NOT_CONVERGED
 * if the aligned fixed point or the tangent solve does not converge;
 * CTMRG_E_NUMERICAL if the kept dimension changes or a multiplet is larger
 * than 8. */
typedef struct ctmrg_derivative_s {
    double F;              /* beta f = -1/2 ln ||P~||_F at the aligned fixed point           */
    double dF_dK;          /* dF/dK, the energy per site                                      */
    double d2F_dK2;        /* d2F/dK2 (second_order 1: dE/dK; 2: central difference; 0: 0)     */
    double gauge_residual; /* max |P_next - P| of the aligned fixed point                     */
    double tangent_change; /* max |J t + d_K Phi - t| of the tangent solution                 */
    int aligned_steps;     /* FP64 steps taken to the aligned fixed point                     */
    int iterations;        /* products J t of the tangent solve                               */
    int n_eigen;           /* eigenpairs of C' used (those above rank_tol |lambda_1|)          */
    double E;              /* impurity energy of the plaquette at the aligned fixed point      */
    double M;              /* magnetization (Eq. 5) at the aligned fixed point                 */
    double dE_dK;          /* total derivative of E along the fixed point (= d2F/dK2)          */
    double dM_dK;          /* total derivative of M along the fixed point                      */
    int status;            /* CTMRG_OK; in a sweep, the status of a derivative that failed     */
} ctmrg_derivative_t;

ctmrg_status ctmrg_fixed_point_derivative(ctmrg_ctx *ctx, int second_order, ctmrg_derivative_t *out);

/* Backward pass for the observables (f, E, M) of the fixed point as functions
 * of K: *K_bar = obs_bar[0] df/dK + obs_bar[1] dE/dK + obs_bar[2] dM/dK, with
 * f = F/K, dE/dK = d2F/dK2 and dM/dK from one call of
 * ctmrg_fixed_point_derivative (second_order 1); *d2F_dK2 (if non-NULL)
 * receives d2F/dK2.  Same requirements and errors as
 * ctmrg_fixed_point_derivative. */
ctmrg_status ctmrg_backward(ctmrg_ctx *ctx, const double obs_bar[3], double *K_bar, double *d2F_dK2);

/* Checkpoint of the state (P, Omega, the normalization history, step count).
 * Call with host_buf NULL to get the size in *bytes. */
ctmrg_status ctmrg_export_state(ctmrg_ctx *ctx, void *host_buf, size_t *bytes);
ctmrg_status ctmrg_import_state(ctmrg_ctx *ctx, const void *host_buf, size_t bytes);

/* Replace the state by caller data: P as q slices of d x d (P[(s*d + a)*d + b]),
 * omega (d values), d <= m.  The normalization history is reset. */
ctmrg_status ctmrg_set_state(ctmrg_ctx *ctx, int d, const double *P, const double *omega);

/* Device bytes a context with these sizes allocates at init (each buffer rounded up to 256
 * bytes; with dim = 3, an upper bound for smaller dim): the size a caller-owned workspace needs. */
ctmrg_status ctmrg_workspace_size(int q, int m, const ctmrg_options *opt, size_t *bytes);

/* Device bytes a context allocates later, on first use (each once, kept until
 * ctmrg_destroy): *observables_bytes by ctmrg_observables (the Lanczos vectors of
 * xi_e, min(400, m^2) + 1 vectors of m^2 doubles, and the products' buffers), and
 * *derivative_bytes by ctmrg_fixed_point_derivative / ctmrg_backward (the tangent
 * solve's 12 (q m)^2 + 13 q m^2 doubles, its GMRES vectors, 69 of q m^2 + m^2
 * doubles, and an eigensolver workspace for all q m eigenvectors), both at their
 * largest (m_eff = m).  Either pointer may be NULL. */
ctmrg_status ctmrg_extra_workspace_size(int q, int m, const ctmrg_options *opt, size_t *observables_bytes,
                                        size_t *derivative_bytes);

/* Inspection of device buffers (host copies), for tests and checkpoints:
 *  CTMRG_BUF_P        m x (q m)  current P in the A layout above
 *  CTMRG_BUF_OMEGA    m          current omega (zero padded)
 *  CTMRG_BUF_SPECTRUM q m        all eigenvalues of the last C', ascending
 *  CTMRG_BUF_U        (q m) x m  kept eigenvectors of the last step (row-major, zero columns past m_eff)
 *  CTMRG_BUF_CEXT     (q m)^2    C' of the last ctmrg_extend call (row-major)
 *  CTMRG_BUF_W        q^2 x q^2  the weight matrix W[(s,sg),(s',sg')]                  */
typedef enum {
    CTMRG_BUF_P = 0,
    CTMRG_BUF_OMEGA = 1,
    CTMRG_BUF_SPECTRUM = 2,
    CTMRG_BUF_U = 3,
    CTMRG_BUF_CEXT = 4,
    CTMRG_BUF_W = 5
} ctmrg_buffer;
ctmrg_status ctmrg_get_buffer(ctmrg_ctx *ctx, int which, double *host_dst, size_t count);

/* Steps 1-2 only (extension and W-mix) on the current state; C' stays readable
 * through CTMRG_BUF_CEXT until the next step. */
ctmrg_status ctmrg_extend(ctmrg_ctx *ctx);

/* Standalone use of the eigensolver on a host symmetric n x n matrix (row-major,
 * lower triangle read): all eigenvalues ascending (evals, n values) and the k
 * eigenvectors of largest |lambda| (evecs, n x k row-major, sign convention:
 * the first entry of largest magnitude is positive), ordered by descending
 * |lambda|, ties to the larger lambda.  kept_vals receives those k eigenvalues.
 * band as in ctmrg_options (0 = default). */
ctmrg_status ctmrg_eigh_topk(int n, const double *A, int k, int band, double *evals, double *kept_vals,
                             double *evecs);

/* The same computation as ctmrg_eigh_topk, for callers that cannot allocate device
 * memory (code that runs under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): no hipMalloc, hipFree, stream creation or allocating
 * library call.  Every device buffer of the call is carved from one file-scope
 * device array of CTMRG_NOALLOC_BYTES that each GPU the library runs on holds
 * until the process ends.  Sizes: n <= CTMRG_NOALLOC_NMAX, k <= CTMRG_NOALLOC_KMAX
 * (larger sizes return CTMRG_E_INVALID_ARG without touching the device).  Runs
 * on the null stream of the current device and returns when the outputs are in
 * host memory.  All calls on one GPU share that GPU's array: calls that overlap
 * on one GPU (from several host threads) race and must be serialized by the
 * caller.  Arguments, outputs and the other errors as ctmrg_eigh_topk. */
#define CTMRG_NOALLOC_NMAX 1024
#define CTMRG_NOALLOC_KMAX 128
#define CTMRG_NOALLOC_BYTES (96u << 20)
ctmrg_status ctmrg_eigh_topk_noalloc(int n, const double *A, int k, int band, double *evals, double *kept_vals,
                                     double *evecs);

/* Stage timing with HIP events on the context's stream.  While enabled, each
 * step synchronizes once more at its end and accumulates the device time of
 * its stages (milliseconds, summed over the steps since enabling):
 *   0 extension products X        1 W-mix of X (C')          2 dense->band
 *   3 band->tridiagonal           4 bisection (all values)    5 selection/cut/entropy
 *   6 inverse iteration           7 orthonormalization        8 back-transform (band)
 *   9 back-transform (dense)     10 half-row products Y      11 W-mix of Y
 *  12 projection U^T Z           13 normalization            14 whole step
 *  15 warm eigensolver (CTMRG_EIG_WARM; a step that falls back counts its
 *     attempt here and its two-stage solve in stages 2-9)
 * Enabling resets the sums. */
#define CTMRG_NUM_STAGES 16
ctmrg_status ctmrg_set_profiling(ctmrg_ctx *ctx, int enable);
ctmrg_status ctmrg_get_stage_times(ctmrg_ctx *ctx, double *ms, int *nsteps);

/* Counters of the warm eigensolver since ctmrg_init: out[0] steps solved warm, out[1] steps that fell back to the
 * two-stage solver after a warm attempt, out[2] passes, out[3] products C' V of
 * the filter and the Rayleigh-Ritz step, out[4] the largest and out[5] the last
 * share of sum w^4 beyond the Ritz block (exact with CTMRG_WARM_TAIL_EXACT, a
 * bound otherwise; the entropy of that share is known within tail ln(N/tail)), out[6] how the last warm
 * attempt ended (0 converged, 1 no warm start, 2 Gram matrix not positive
 * definite, 3 Rayleigh-Ritz solver error, 4 non-finite residual, 5 pass limit)
 * and out[7] its largest kept residual over |lambda_1|.  While stage timing is
 * enabled (ctmrg_set_profiling, which resets them), out[8] sums the device
 * milliseconds of the solver's products C' V (HIP events around each launch),
 * out[9] their algorithmic flops (2 (q m)^2 columns each) and out[10] counts them.
 * out[11] is S_E as the last warm-solved step gave it (Ritz values plus the
 * bounded tail; ctmrg_observables computes it over all eigenvalues), out[12]
 * the warm steps that took sum lambda^4 from the product C' C'. */
ctmrg_status ctmrg_get_eig_stats(ctmrg_ctx *ctx, double out[13]);

const char *ctmrg_last_error(const ctmrg_ctx *ctx);
void ctmrg_destroy(ctmrg_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* CTMRG_H */
