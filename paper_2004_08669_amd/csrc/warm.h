// Warm-started eigensolver for the extended corner (the diagonalization step of
// Algorithm 3, Sec. III), used from the second step of a run on: the leading
// eigenpairs of C' from the previous step's, without reducing C' to band and
// tridiagonal form.
//
// From one step to the next the extended corner changes little once the
// renormalized basis is kept in one gauge: the kept eigenvectors of every step
// are rotated inside each multiplet (and signed) to best match those of the
// step before (orthogonal Procrustes), so that the basis of the next C' is,
// state by state, the basis of this one.  The previous step's Ritz vectors --
// the kept ones and p guard vectors below them -- are then a close start for
// the top k = m + p eigenvectors of the new C'.  Each pass of the solver
//
//   1. filters the block with a Chebyshev polynomial of degree d in C'/a,
//      a = the smallest |Ritz value| of the block (the damped interval [-a, a]
//      holds the spectrum the block does not track), each column scaled by the
//      polynomial's value at its own Ritz value so that it stays of order one;
//   2. orthonormalizes the block: Cholesky factorization of its Gram matrix
//      (blocked, 64 x 64 diagonal blocks in LDS) and a triangular solve;
//   3. Rayleigh-Ritz: H = Q^T C' Q, all eigenpairs of H (k x k) with the
//      library's two-stage solver, Ritz vectors Q X sorted by descending |theta|;
//   4. measures the residuals ||C' v_j - theta_j v_j|| of the kept Ritz pairs.
//
// It stops when every kept residual is below tol |theta_1|, or after max_passes
// (the caller then runs the two-stage solver on C').  All eigenvalues of C' are
// not computed: n_C and S_E (Eq. 6) take the k Ritz values plus the part of the
// spectrum beyond the block, which the Frobenius norm bounds: with
// t2 = ||C'||_F^2 - sum theta^2 (the sum of the remaining lambda^2), the
// remaining sum of lambda^4 lies in [0, theta_k^2 t2]; its midpoint is used and
// half the interval is reported as the bound.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "eig.h"

namespace ctm {

struct WarmWork {
    int N = 0, m = 0, p = 0, kmax = 0, nb = 0;
    // N x kmax blocks (row-major, ld kmax): the basis / Ritz vectors, a filter buffer,
    // C' Q and C' V
    double *V = nullptr, *Y = nullptr, *CQ = nullptr, *CV = nullptr;
    // kmax x kmax: Gram matrix / Cholesky factor, Rayleigh quotient (and the copy the
    // two-stage solver destroys), Ritz vector coefficients, overlap with the previous U
    double *G = nullptr, *H = nullptr, *Hs = nullptr, *X = nullptr, *Mov = nullptr;
    double *Linv = nullptr;           // inverses of the 64 x 64 diagonal blocks of L
    double *theta = nullptr;          // kmax Ritz values, descending |theta|
    double *zero = nullptr;           // kmax + 8 zeros (the "previous spectrum" of the small solves)
    double *scr = nullptr;            // kmax + 8 scratch (omega of the small solves)
    double *coef = nullptr;           // Chebyshev column coefficients: 2 * dmax * kmax
    double *res = nullptr;            // residual partials (row chunks x kmax), then norms
    double *part = nullptr;           // reduction partials
    double *fro2 = nullptr;           // ||C'||_F^2 (device scalar)
    double *sum4 = nullptr;           // ||C'^2||_F^2 / ||C'||_F^4 = sum lambda^4 / ||C'||_F^4 (device scalar)
    PostOut *rr_post = nullptr;       // post-eigen results of the small solve
    unsigned *err = nullptr;          // flags: 1 = Gram matrix not positive definite
    double *h_theta = nullptr, *h_res = nullptr, *h_coef = nullptr;  // pinned host copies
    PostOut *h_post = nullptr;
    double *h_scal = nullptr;         // pinned host scalars
    double *pbig = nullptr;           // split-K partials of the products with C' (part_elems = 4 N kmax)
    size_t part_elems = 0;
    // live timing of the products with C' (when profiling): event pairs of one pass, the sums
    static constexpr int NEV = 24;
    hipEvent_t ev[2 * NEV] = {};
    int nev = 0;
    double product_ms = 0.0, product_flops = 0.0;
    long product_launches = 0;
    double pending_flops[NEV] = {};
    EigWork rr;                       // two-stage solver for the k x k Rayleigh-Ritz problem
    bool carved = false;              // device buffers carved from a caller's workspace (not freed here)
    // state carried between steps
    int kcur = 0;                     // valid columns of V (0: no warm start)
    double a_prev = 0.0;              // filter bound of the last pass
    // statistics since the last reset
    long steps = 0, fallbacks = 0, passes = 0, products = 0, exact_tails = 0;
    double tail_bound_max = 0.0;
    double last_rmax = 0.0;           // largest kept residual / |theta_1| of the last pass
    // why the last attempt ended: 0 converged, 1 no warm start, 2 Gram matrix not positive
    // definite, 3 Rayleigh-Ritz solver error, 4 non-finite residual, 5 pass limit
    int last_reason = 1;
};

struct WarmParams {
    double gap_tol = 1e-10, rank_tol = 1e-13;
    double tol = 1e-12;               // kept residuals below tol |theta_1|
    int degree = 4;                   // Chebyshev degree per pass
    int max_passes = 8;
    bool profile = false;             // time every product with C' (HIP events)
    // sum lambda^4 from ||C'^2||_F^2 (given the scratch): always, or when the bound on the share
    // of sum w^4 beyond the block exceeds tail_tol
    bool tail_exact = true;
    double tail_tol = 0.0;
};

constexpr int WARM_DMAX = 8;          // largest degree per pass

// k = m + p columns of at most N.  Device buffers through ar (hipMalloc when it does not carve);
// with ar->count_only only ar->used grows.
hipError_t warm_alloc(WarmWork &w, int N, int m, int p, Arena *ar = nullptr, hipStream_t s = nullptr);
void warm_free(WarmWork &w);
size_t warm_bytes(int N, int m, int p);

// One warm solve on C' (N x N row-major, full symmetric, left intact).  On convergence
// (*converged = 1) writes what the two-stage path writes: omega_new (m, zero padded),
// selval (the m_eff kept eigenvalues, descending |lambda|), *post_dev, the kept
// eigenvectors U (N x m, aligned to the previous U, zero padded) and, in spectrum, the k
// Ritz values ascending followed by NaN.  U must hold the previous step's kept vectors
// (m_eff_prev columns) on entry.  V then holds the new Ritz vectors for the next step.  sq
// (N x N scratch, or null): sum lambda^4 is then taken exactly as ||C'^2||_F^2 (one product
// C' C' on the tiles on and below the diagonal; see WarmParams::tail_exact) instead of bounded
// from ||C'||_F.
hipError_t warm_solve(WarmWork &w, const double *C, int N, int m, const WarmParams &prm, const double *omega_prev,
                      double *omega_new, double *selval, PostOut *post_dev, double *U, int m_eff_prev,
                      double *spectrum, double *sq, hipStream_t s, int *converged, std::string *why);

// Upper bound on the share of sum lambda^4 beyond the k values theta (descending |.|), from
// fro2 = ||C'||_F^2.
double tail_share_bound(const double *theta, int k, double fro2);

// Copies the lower triangle of C (N x N, row-major) into the upper one.
hipError_t warm_symmetrize(double *C, int N, hipStream_t s);

// After a two-stage solve whose vectors for the top kk eigenvalues are in w.V (ld kmax,
// sign-fixed) and their values in selk (descending |lambda|): align the first m_eff
// columns to the previous U (m_eff_prev columns; none when 0), copy them into U
// (N x m, zero padded) and keep the block as the next step's warm start.
hipError_t warm_seed(WarmWork &w, int N, int m, int m_eff, int kk, const double *selk, double *U, int m_eff_prev,
                     double gap_tol, hipStream_t s);

// ||C'||_F^2 into w.fro2.
hipError_t warm_frobenius(WarmWork &w, const double *C, long n2, hipStream_t s);

}  // namespace ctm
