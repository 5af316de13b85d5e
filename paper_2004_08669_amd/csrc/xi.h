// Effective correlation length xi_e(T, m) (Sec. II, last paragraph): the leading
// eigenvalues of the renormalized row-to-row transfer matrix built from the
// half-row matrices P_s.
//
// A full row of vertices is two half-rows joined at their common inner end spin s:
// T = sum_s P_s (x) P_s, symmetric of order m^2 (P_s is symmetric).  T is never
// formed; on a vector X (m x m, row-major) it acts as X -> sum_s P_s X P_s, two
// products on the matrix cores: Y = [P_0 X; P_1 X; ...] (N x m, one GEMM with P's
// stored layout read transposed) and T X = sum over (s, b) of Y[s m + i][b] P_s[b][j]
// (one GEMM of inner dimension N = q m, split over K).
//
// The two eigenvalues of largest modulus come from Lanczos with full
// reorthogonalization (classical Gram-Schmidt, twice) from a pseudo-random start
// vector (splitmix64 of the index, so both symmetric and antisymmetric X are
// reached).  Every 8 iterations the tridiagonal matrix is solved on the device
// (Sturm bisection for its two largest and two smallest eigenvalues, inverse
// iteration for the vectors of the two of largest modulus); the iteration stops
// when both residual estimates beta_j |s_j| are below tol |theta_1|.  The Ritz
// vectors are then formed and their residuals ||T y - theta y|| measured with one
// more product each.  xi_e = 1 / ln(|lambda_1| / |lambda_2|), in rows of vertices.
#pragma once

#include <hip/hip_runtime.h>

namespace ctm {

struct XiWork {
    int m = 0, N = 0, jmax = 0;
    long n = 0;                   // m^2
    double *V = nullptr;          // (jmax + 1) x n Lanczos vectors, one per row
    double *Y = nullptr;          // N x m
    double *w = nullptr;          // n: T v, then the next vector before normalization
    double *yv = nullptr;         // 2 x n: Ritz vectors
    double *part = nullptr;       // split-K partials of the second product (part_elems)
    size_t part_elems = 0;
    double *dots = nullptr;       // dot-product partials: chunks x (jmax + 2)
    double *h = nullptr;          // jmax + 2 projections (two passes: 2 x (jmax + 2))
    double *ab = nullptr;         // alpha[0..jmax], beta[0..jmax]
    double *tri = nullptr;        // small solve: theta[2], est[2], then 2 vectors of jmax + 1
    double *tws = nullptr;        // small solve scratch: 2 x 6 x (jmax + 1)
    double *nrm = nullptr;        // device scalars
    double *h_out = nullptr;      // pinned host: theta[2], est[2], res[2], beta
};

struct XiResult {
    double lambda1 = 0.0, lambda2 = 0.0;  // descending modulus, of T built from the stored P
    double xi = 0.0;                      // 1 / ln(|lambda1| / |lambda2|); 0 if lambda2 = 0
    double residual = 0.0;                // max over the two of ||T y - theta y|| / |lambda1|
    int iterations = 0;
    bool converged = false;
};

size_t xi_bytes(int q, int m, int jmax);
hipError_t xi_alloc(XiWork &w, int q, int m, int jmax);
void xi_free(XiWork &w);

// A: P in its stored layout, m x (q m) row-major, A[g][s m + a] = P_s[g][a].
hipError_t xi_solve(XiWork &w, const double *A, int q, int m, double tol, hipStream_t s, XiResult *out);

}  // namespace ctm
