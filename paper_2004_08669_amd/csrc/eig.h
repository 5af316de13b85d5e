// Symmetric eigensolver for the extended corner matrix (the diagonalization
// step of Algorithm 3, Sec. III): all eigenvalues plus the eigenvectors of
// the m largest in magnitude.
//
//   stage 1  dense -> band (half-bandwidth b): blocked Householder QR of each
//            b-column panel below the band (one kernel per panel whose
//            workgroups, all resident, exchange per-column partial sums through
//            device-coherent slots) and a two-sided compact-WY update of the
//            trailing matrix with GEMMs on the matrix cores; the matrix is held
//            in its lower triangle (the product with it reads the triangle once
//            at b = 16, twice at b = 32; the update writes only tiles on or
//            below the diagonal);
//   stage 2  band -> tridiagonal: bulge chasing, one wave per step, one
//            launch per wavefront of independent steps (a sweep trails its
//            predecessor by three steps);
//   values   all N eigenvalues by Sturm-count bisection;
//   vectors  inverse iteration on the tridiagonal for the kept eigenvalues,
//            re-orthogonalization inside tight clusters, then a Newton-Schulz
//            polar step (GEMMs) for global orthonormality;
//   back     the stage-2 reflectors grouped b sweeps at a time into block
//            reflectors applied in a wavefront order, then the stage-1 panels
//            as GEMMs.
#pragma once

#include <hip/hip_runtime.h>

namespace ctm {

struct EigWork {
    int Nmax = 0, kmax = 0, b = 0, Tmax = 0, nJmax = 0;
    // stage 1
    double *Vx = nullptr;      // explicit V of every panel, concatenated (sum n_p * b)
    double *Tp = nullptr;      // T of every panel (npanel * b * b)
    double *tau1 = nullptr;    // (npanel * b)
    double *VW = nullptr;      // n x 2b  [V | W]
    double *WV = nullptr;      // n x 2b  [W | V]
    double *Y = nullptr;       // n x b
    double *X = nullptr;       // n x b
    double *sm = nullptr;      // 4 * b * b
    double *part = nullptr;    // panel QR: exchange slots (two sets)
    unsigned long pqr_launches = 0;  // panel QR launches so far (the parity picks the slot set)
    int pqr_gprev = 0;         // workgroups of the previous panel QR launch
    int pqr_cap = 0;           // panel QR workgroups the device holds at once
    int ysym_cap = 0;          // single-pass Y workgroups the device holds at once
    size_t lds_bulge_bytes = 0;  // dynamic LDS the in-LDS bulge chasing may use (0: launches only)
    double *splitk = nullptr;  // split-K partials
    size_t splitk_elems = 0;
    // stage 2
    double *band = nullptr;    // N x 2b column-major band
    double *refl = nullptr;    // (N * Tmax * b) reflectors
    double *rtau = nullptr;    // (N * Tmax)
    double *T2 = nullptr;      // nJ * Tmax * b * b
    // back-transform of stage 1: per group of panels, the Gram matrix of its V and its T
    double *bt1_gram = nullptr, *bt1_T = nullptr;
    double *bt1_W = nullptr;   // 2 x (4 b) x kmax: V_G^T Z and T_G V_G^T Z of one group
    // tridiagonal
    double *d = nullptr, *e = nullptr, *e2 = nullptr;  // N
    double *evals = nullptr;   // N, ascending
    double *slices = nullptr;  // spectrum slicing: 2 x 4096 points, then their 2 x 4096 Sturm counts (int)
    double *ZT = nullptr;      // N x kmax (row-major, ld kmax)
    double *Ztmp = nullptr;    // N x kmax
    double *G = nullptr;       // kmax x kmax
    double *lu = nullptr;      // inverse-iteration scratch (5 N kmax, rounded up to 64)
    int *ipiv = nullptr;       // N kmax
    int *clist = nullptr;      // kmax: kept indices in ascending-eigenvalue order
    int *cstart = nullptr;     // kmax + 1 cluster offsets
    unsigned *err = nullptr;   // kernel error flags
    hipEvent_t *marks = nullptr;  // optional stage-boundary events (see MarkId)
    // look-ahead: the update of the rest of the trailing matrix runs on s2 while the next
    // panel's QR runs on the caller's stream
    hipStream_t s2 = nullptr;
    hipEvent_t ev_cols = nullptr, ev_update = nullptr;
    // false when the buffers were carved from caller memory (eig_carve): eig_free then frees nothing
    bool owned = true;
};

// Stage boundaries recorded when EigWork::marks is set (indices into marks).
enum MarkId {
    MK_START = 0, MK_EXT = 1, MK_WMIX1 = 2, MK_STAGE1 = 3, MK_BULGE = 4, MK_BISECT = 5, MK_POST = 6,
    MK_INVIT = 7, MK_NS = 8, MK_BT2 = 9, MK_BT1 = 10, MK_HALF = 11, MK_WMIX2 = 12, MK_PROJ = 13,
    MK_NORM = 14, MK_VEC_START = 15, MK_WARM_END = 16, MK_COUNT = 17
};
inline void mark(const EigWork &w, int id, hipStream_t s)
{
    if (w.marks) (void)hipEventRecord(w.marks[id], s);
}

// Post-eigenvalue results shared with the host (one small struct per step).
struct PostOut {
    int m_eff;
    int rank;
    int nclusters;
    int pad;
    double n_C;
    double S_E;
    double delta;
    double lam1;
    double sum_w4_kept;
    double tail_bound;  // warm solver: bound on the part of sum w^4 beyond its block (0: all eigenvalues known)
};

hipError_t eig_alloc(EigWork &w, int Nmax, int kmax, int b);
// The same buffers laid out in caller memory [base, base + bytes) (at least eig_bytes(Nmax, kmax, b),
// 256-byte aligned); no allocation, no second stream (the look-ahead of stage 1 then runs in order on
// the caller's stream).  The exchange slots and error flags are reset by fill kernels on s.
hipError_t eig_carve(EigWork &w, void *base, size_t bytes, int Nmax, int kmax, int b, hipStream_t s);
// The second stream and its events (the look-ahead of stage 1) for a carved workspace.
hipError_t eig_attach_streams(EigWork &w);
void eig_free(EigWork &w);
size_t eig_bytes(int Nmax, int kmax, int b);

// Stages 1 and 2 plus bisection: A (N x N, row-major, lda) is destroyed.
// On return w.evals holds all eigenvalues in ascending order.
hipError_t eig_values(EigWork &w, double *A, long lda, int N, hipStream_t s);

// Selection of the m largest |lambda| with the multiplet-preserving cut,
// normalization n_C, entropy, convergence measure against the previous kept
// spectrum omega_prev (m entries, zero padded).  Writes omega_new (m entries, zero padded) and out.
hipError_t eig_post(EigWork &w, int N, int m, double gap_tol, double rank_tol, const double *omega4_prev,
                    double *omega_new, double *selval, PostOut *out_dev, hipStream_t s);

// Eigenvectors of the kept eigenvalues selval[0..me) (in kept order), written
// to U (N x ldu row-major; columns me..ldu-1 zeroed), sign-fixed.
// Requires the stage-1/2 data of the last eig_values call on the same matrix.
hipError_t eig_vectors(EigWork &w, const double *A_reflectors, long lda, int N, int me, const double *selval,
                       int nclusters, double *U, int ldu, hipStream_t s);

// Error flags accumulated by the kernels (0 = none); clears them.
unsigned eig_take_errors(EigWork &w);

}  // namespace ctm
