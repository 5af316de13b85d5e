// Derivative of the CTMRG fixed point with respect to the coupling K
// (implicit differentiation through the fixed-point map, tangent mode).
//
// With P normalized by its Frobenius norm (the normalization does not change
// the partition function per vertex, Sec. 3, Algorithm 3), the free energy per
// site at a fixed point x* is F = beta f = -1/2 ln s*, s* = ||P~(x*)||_F.  Its
// total derivative is
//     dF/dK = -1/2 (d s / dK) / s*,   ds/dK = d_K s + d_x s . t,
// where the tangent t = dx*/dK solves (I - J) t = d_K Phi (J = d Phi / dx at x*),
// by restarted GMRES with J t applied matrix-free.  J t is the hand-written directional
// derivative of one step: the product rule through the contractions, and the
// derivative of the kept eigenvectors of C',
//     dU_j = sum_i u_i (u_i^T dC' u_j) / (lambda_j - lambda_i)   (i discarded),
// over all eigenpairs i of C' outside the kept set.  Rotations inside the kept
// space are gauge (only the kept subspace enters the next step), so the tangent
// of the corner is carried as a full symmetric block
//     dOmega = U_k^T dC' U_k / n_C - Lambda dn_C / n_C^2
// instead of the derivative of a diagonal; no (near-)degenerate pair of kept
// states then enters a denominator, and a pair split by the cut cannot occur
// (the cut never splits a multiplet).  The base point is a fixed point in one
// gauge: FP64 steps whose kept eigenvectors are rotated inside each multiplet
// to best match the previous step's (orthogonal Procrustes), until P repeats
// element by element.
//
// Observables along the tangent.  With X = A^T Omega A in the block layout
// (X_{s sg} = P_s Omega P_sg), G = Om~ X Om~ (Om~ = diag(Omega, ..., Omega)),
// C' = W-mix(X) and C'_h = (W h4)-mix(X), the impurity energy of the
// plaquette (Sec. II) is E = 1/2 <G, C'_h> / <G, C'> (Frobenius products).
// Its total derivative along the fixed point, dE/dK = d_K E + d_x E . t,
// follows from the product rule with dW/dK = -W h4 and d(W h4)/dK = -W h4^2:
//   d<G, C'> = 2 <Om~ X dOm~, C'> + <Om~ dX Om~, C'> + <G, dC'>
// (X, C' and dOm~ symmetric), and the same with C'_h.  Since dF/dK equals E
// at every fixed point (the stationarity of the CTMRG free energy; checked by
// the tests to the convergence of the fixed point), d2F/dK2 = dE/dK exactly.
// The magnetization (Eq. 5) weighs the spins by
// prob_s = sum_b (U Omega^4 U^T)[(s,b),(s,b)]; with the corner's tangent a full
// symmetric block dOm, d(Omega^4)[j][k] = dOm[j][k] (w_j^3 + w_j^2 w_k +
// w_j w_k^2 + w_k^3), and
//   d prob_s = sum_b [2 (dU Omega^4 U^T) + U d(Omega^4) U^T][(s,b),(s,b)].
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "eig.h"

namespace ctm {

struct AdjInputs {
    int q = 0, m = 0, d = 0;          // context cutoff m, kept dimension d of the converged state
    const double *W = nullptr;        // q^2 x q^2 weight at K
    const double *WH = nullptr;       // W * h4 (h4 = -sum of the plaquette bonds), so dW/dK = -WH
    const double *A = nullptr;        // m x (q m) state (padded), omega (m), last kept U ((q m) x m)
    const double *omega = nullptr;
    const double *U = nullptr;
    const double *V = nullptr;        // spin vectors (q x dim), for M
    int dim = 0, bc = 0, s0 = 0;      // boundary condition and the boundary spin, for M
    double gap_tol = 1e-10, rank_tol = 1e-13;
    int max_aligned_steps = 500, max_iterations = 3000;  // aligned steps; products J t of the tangent solve
    double gauge_tol = 1e-10;         // element-wise |P_next - P| of the aligned fixed point
    double tangent_tol = 1e-12;       // GMRES: ||d_K Phi - (I - J) t|| / ||d_K Phi||
    int restart = 64;                 // GMRES restart length
};

struct AdjResult {
    double F = 0.0;            // -1/2 ln s*
    double dFdK = 0.0;
    double gauge_residual = 0.0;
    double tangent_change = 0.0;
    int aligned_steps = 0;
    int iterations = 0;
    int n_eigen = 0;           // eigenpairs of C'* used (its rank)
    double E = 0.0, dEdK = 0.0;  // impurity energy at the aligned fixed point and its total derivative
    double M = 0.0, dMdK = 0.0;  // magnetization (Eq. 5) and its total derivative
};

struct AdjWork {
    int q = 0, d = 0, n = 0, band = 32;
    double *A = nullptr, *OA = nullptr, *Pt = nullptr, *om = nullptr, *omn = nullptr, *zero = nullptr;
    double *Ucur = nullptr, *Uprev = nullptr, *Mov = nullptr;
    double *X = nullptr, *C = nullptr, *Y = nullptr, *Z = nullptr, *Cb = nullptr, *Zb = nullptr;
    double *Uall = nullptr, *M3 = nullptr, *lam = nullptr, *sel = nullptr;
    double *dA = nullptr, *dAn = nullptr, *dOA = nullptr, *dom = nullptr, *domn = nullptr;
    double *dX = nullptr, *dC = nullptr, *dY = nullptr, *dZ = nullptr, *dPt = nullptr;
    double *T1 = nullptr, *Bm = nullptr, *R = nullptr, *dU = nullptr;
    double *part = nullptr, *scal = nullptr, *hscal = nullptr;
    double *W2 = nullptr, *obsv = nullptr, *hobsv = nullptr;  // W h4^2 (q^4); prob, d prob (device, host)
    // GMRES of the tangent: Krylov basis (restart + 1 vectors of L = d n + d^2), right-hand side,
    // solution, J times a vector, projections (device, host)
    int restart = 0;
    double *Vk = nullptr, *gb = nullptr, *gx = nullptr, *gy = nullptr, *gh = nullptr, *hgh = nullptr;
    PostOut *post = nullptr, *hpost = nullptr;
    unsigned *err = nullptr;
    EigWork eig;
};

hipError_t adj_alloc(AdjWork &w, int q, int d, int band, int restart = 64);
size_t adj_bytes(int q, int d, int band, int restart = 64);  // what adj_alloc allocates
void adj_free(AdjWork &w);

// Returns 0 on success; otherwise a ctmrg_status value with a message in *msg.
int adjoint_dFdK(AdjWork &w, const AdjInputs &in, AdjResult *res, hipStream_t s, std::string *msg);

}  // namespace ctm
