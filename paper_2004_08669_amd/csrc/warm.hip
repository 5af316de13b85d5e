// Warm-started eigensolver for the extended corner; see warm.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "common.h"
#include "gemm.h"
#include "warm.h"

namespace ctm {

namespace {

constexpr int CB = 64;        // diagonal block of the Cholesky factorization
constexpr int RES_CHUNKS = 64;
constexpr int ALIGN_KB = 8;   // largest multiplet the alignment rotates

int grid_for(long n) { return (int)std::max<long>(1, std::min<long>(1024, (n + 255) / 256)); }

// Y_new = alpha[j] acc + beta[j] Y_old, with Y_old read and overwritten in place (per column
// coefficients of the scaled Chebyshev recurrence).
struct EpiCheb {
    double *p; long ld; const double *alpha, *beta;
    __device__ void operator()(int i, int j, double v, int) const
    {
        double *c = p + (long)i * ld + j;
        const double b = beta[j];
        *c = alpha[j] * v + (b != 0.0 ? b * (*c) : 0.0);
    }
};

// C -= alpha[j] acc (the locked part of a deflated product, per column coefficient)
struct EpiSubScaled {
    double *p; long ld; const double *alpha;
    __device__ void operator()(int i, int j, double v, int) const { p[(long)i * ld + j] -= alpha[j] * v; }
};

// T[i][j] *= theta[i]  (rows of Q_L^T Y scaled by the locked Ritz values)
__global__ void scale_rows_by_kernel(double *T, long ld, int rows, int cols, const double *theta)
{
    const long total = (long)rows * cols;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / cols), j = (int)(idx - (long)i * cols);
        T[(long)i * ld + j] *= theta[i];
    }
}

// Cholesky of the CB x CB diagonal block at (p0, p0) of G (lower, row-major ld), in place, and
// the inverse of that factor into Linv (CB x CB, row-major, zero above the diagonal).  A pivot
// that is not positive raises flag 1 and is replaced by a tiny positive number.  The block
// stays in LDS: right-looking by columns, the trailing update on a 16 x 16 thread grid; the
// inverse by forward substitution, one column per thread.
__global__ void __launch_bounds__(256) chol_diag_kernel(double *G, int ld, int p0, int nb, double *Linv, unsigned *err)
{
    __shared__ double A[CB][CB + 1];
    __shared__ double Li[CB][CB + 1];
    __shared__ double dg[CB];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < CB * CB; idx += 256) {
        const int i = idx / CB, j = idx - i * CB;
        A[i][j] = (i < nb && j <= i) ? G[(long)(p0 + i) * ld + p0 + j] : (i == j ? 1.0 : 0.0);
        Li[i][j] = 0.0;
    }
    __syncthreads();
    // Right-looking factorization with one barrier per column: step j reads column j unscaled,
    // updates the trailing lower triangle with A[i][j] A[l][j] / d, and writes the scaled column
    // L[i][j] = A[i][j] / sqrt(d) to the unused upper triangle (A[j][i]) and sqrt(d) to dg[j];
    // nothing a step writes is read in the same step.
    const int tx = tid & 15, ty = tid >> 4;
    for (int j = 0; j < nb; ++j) {
        const double d = A[j][j];
        const bool bad = !(d > 0.0);
        const double dd = bad ? 1e-300 : d;
        const double piv = sqrt(dd), inv = 1.0 / piv, invd = 1.0 / dd;
        if (tid == 0) {
            if (bad) raise_error(err, 1u);
            dg[j] = piv;
        }
        for (int i = j + 1 + ty; i < nb; i += 16) {
            const double aij = A[i][j] * invd;
            for (int l = j + 1 + tx; l <= i; l += 16) A[i][l] -= aij * A[l][j];
        }
        for (int i = j + 1 + tid; i < nb; i += 256) A[j][i] = A[i][j] * inv;
        __syncthreads();
    }
    // L^{-1} by forward substitution, one column per thread (a column depends on itself only)
    if (tid < nb) {
        const int c = tid;
        for (int i = c; i < nb; ++i) {
            double acc = (i == c) ? 1.0 : 0.0;
            for (int t = c; t < i; ++t) acc -= A[t][i] * Li[t][c];
            Li[i][c] = acc / dg[i];
        }
    }
    __syncthreads();
    for (int idx = tid; idx < nb * nb; idx += 256) {
        const int i = idx / nb, j = idx - i * nb;
        G[(long)(p0 + i) * ld + p0 + j] = (j < i) ? A[j][i] : (j == i ? dg[i] : 0.0);
    }
    for (int idx = tid; idx < CB * CB; idx += 256) {
        const int i = idx / CB, j = idx - i * CB;
        Linv[idx] = (i < nb && j < nb) ? Li[i][j] : 0.0;
    }
}

// part[chunk][j] = sum over the chunk's rows of (CV[i][j] - theta_j V[i][j])^2
__global__ void __launch_bounds__(256) resid_partial_kernel(const double *CV, const double *V, const double *theta, int N,
                                                            int k, long ld, double *part)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= k) return;
    const int rows = (N + gridDim.y - 1) / gridDim.y;
    const int r0 = blockIdx.y * rows, r1 = min(N, r0 + rows);
    const double th = theta[j];
    double acc = 0.0;
    for (int i = r0; i < r1; ++i) {
        const double r = CV[(long)i * ld + j] - th * V[(long)i * ld + j];
        acc += r * r;
    }
    part[(long)blockIdx.y * k + j] = acc;
}

__global__ void resid_finalize_kernel(const double *part, int chunks, int k, double *res)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[(long)c * k + j];
    res[j] = sqrt(s);
}

__global__ void __launch_bounds__(256) sumsq_partial_kernel(const double *x, long n, double *part)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) acc += x[i] * x[i];
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void sum_finalize_kernel(const double *part, int np, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += part[i];
    *out = s;
}

// Mirror of the lower triangle of C (N x N, row-major) into the upper one, 64 x 64 tiles
// through LDS: block b takes the tile (I, J), J <= I, of the lower triangle and writes its
// transpose into (J, I) (on the diagonal only the entries above it).  The two-stage solver
// reads the lower triangle only; the mirror makes the products of the warm solver use that
// same symmetric matrix where the contraction leaves C' asymmetric by its rounding.
__global__ void __launch_bounds__(256) mirror_lower_kernel(double *C, int N)
{
    __shared__ double t[64][65];
    const int b = blockIdx.x;
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > b) --I;
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    const int J = b - I * (I + 1) / 2;
    const int r0 = I * 64, c0 = J * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int i = r0 + r, j = c0 + tx;
        t[r][tx] = (i < N && j < N) ? C[(long)i * N + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int i = c0 + r, j = r0 + tx;  // C[i][j] = C[j][i] = t[tx][r]
        if (i < N && j < N && j > i) C[(long)i * N + j] = t[tx][r];
    }
}

// C'^2 on the 128 x 128 tiles on or below the diagonal (row-major, ld N).
struct EpiSquareTiles {
    double *p; long ld;
    static constexpr bool kLowerTiles = true;
    __device__ void operator()(int i, int j, double v, int) const { p[(long)i * ld + j] = v; }
};

// sum_ij (S_ij / f)^2 over the whole symmetric S = C'^2 from its stored tiles: weight 1 on the
// diagonal 128 x 128 tiles, 2 below them; f = ||C'||_F^2 >= lambda_1^2 keeps every term <= 1.
// Partial sums per block (rows strided over the grid).
__global__ void __launch_bounds__(256) sum4_partial_kernel(const double *S, int N, const double *fro2, double *part)
{
    __shared__ double red[4];
    const double inv = 1.0 / *fro2;
    double acc = 0.0;
    for (int i = blockIdx.x; i < N; i += gridDim.x) {
        const int d0 = (i / 128) * 128, end = min(N, d0 + 128);
        const double *row = S + (long)i * N;
        for (int j = threadIdx.x; j < end; j += 256) {
            const double x = row[j] * inv;
            acc += (j < d0 ? 2.0 : 1.0) * (x * x);
        }
    }
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Shift of shifted Cholesky QR: G_ii += 11 (N k + k (k + 1)) u tr(G), u = 2^-53 (tr G bounds
// ||Y||_2^2), which makes the factorization of the Gram matrix of any N x k block succeed.
__global__ void __launch_bounds__(256) gram_shift_kernel(double *G, int k, long ld, int N)
{
    __shared__ double red[4];
    double t = 0.0;
    for (int i = threadIdx.x; i < k; i += 256) t += G[(long)i * ld + i];
    t = block_sum<256>(t, red);
    const double shift = 11.0 * ((double)N * k + (double)k * (k + 1)) * 1.1102230246251565e-16 * t;
    for (int i = threadIdx.x; i < k; i += 256) G[(long)i * ld + i] += shift;
}

// Hs = (H + H^T) / 2  (k x k, ld)
__global__ void symmetrize_kernel(const double *H, double *Hs, int k, long ld)
{
    const long total = (long)k * k;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / k), j = (int)(idx - (long)i * k);
        Hs[(long)i * ld + j] = 0.5 * (H[(long)i * ld + j] + H[(long)j * ld + i]);
    }
}

// U (N x m, row-major) = V[:, :me] (ld kv), zero columns me..m-1
__global__ void copy_kept_kernel(const double *V, long kv, int N, int me, int m, double *U)
{
    const long total = (long)N * m;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / m), j = (int)(idx - (long)i * m);
        U[idx] = (j < me) ? V[(long)i * kv + j] : 0.0;
    }
}

// Symmetric k x k eigendecomposition by cyclic Jacobi (k <= ALIGN_KB, one thread).
__device__ void small_jacobi8(double (&S)[ALIGN_KB][ALIGN_KB], double (&V)[ALIGN_KB][ALIGN_KB], int k)
{
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < k; ++p)
            for (int r = p + 1; r < k; ++r) off += S[p][r] * S[p][r];
        if (off < 1e-60) break;
        for (int p = 0; p < k; ++p)
            for (int r = p + 1; r < k; ++r) {
                if (S[p][r] == 0.0) continue;
                const double th = (S[r][r] - S[p][p]) / (2.0 * S[p][r]);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
                for (int i = 0; i < k; ++i) {
                    const double a = S[i][p], b = S[i][r];
                    S[i][p] = c * a - sn * b;
                    S[i][r] = sn * a + c * b;
                }
                for (int i = 0; i < k; ++i) {
                    const double a = S[p][i], b = S[r][i];
                    S[p][i] = c * a - sn * b;
                    S[r][i] = sn * a + c * b;
                }
                for (int i = 0; i < k; ++i) {
                    const double a = V[i][p], b = V[i][r];
                    V[i][p] = c * a - sn * b;
                    V[i][r] = sn * a + c * b;
                }
            }
    }
}

// Keep one gauge from step to step: the first `me` columns of U (ld ldu) are rotated inside
// each multiplet (|theta_j| - |theta_{j+1}| <= gap_tol |theta_1|) to best match the previous
// vectors, R = M (M^T M)^{-1/2} with M = U_b^T Uprev_b (Mov holds U^T Uprev, me x me).  A
// multiplet larger than ALIGN_KB, or one whose overlap with the previous vectors is
// singular (a state that moved across the cut), is signed instead: its largest entry positive.
// One workgroup per column; only the first column of a multiplet works.
__global__ void __launch_bounds__(64) warm_align_kernel(double *U, int ldu, int N, const double *Mov, int me,
                                                         const double *theta, double gap_tol)
{
    const int j = blockIdx.x;
    const double tol = gap_tol * fabs(theta[0]);
    if (j > 0 && !(fabs(theta[j - 1]) - fabs(theta[j]) > tol)) return;
    int k = 1;
    while (j + k < me && !(fabs(theta[j + k - 1]) - fabs(theta[j + k]) > tol)) ++k;
    __shared__ double R[ALIGN_KB][ALIGN_KB];
    __shared__ int ok;
    if (threadIdx.x == 0) {
        ok = 0;
        if (k <= ALIGN_KB) {
            double M[ALIGN_KB][ALIGN_KB], S[ALIGN_KB][ALIGN_KB], Q[ALIGN_KB][ALIGN_KB];
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) M[a][b] = Mov[(long)(j + a) * me + (j + b)];
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) {
                    double acc = 0.0;
                    for (int c = 0; c < k; ++c) acc += M[c][a] * M[c][b];
                    S[a][b] = acc;
                }
            small_jacobi8(S, Q, k);
            double smax = 0.0, smin = INFINITY;
            for (int a = 0; a < k; ++a) {
                smax = fmax(smax, S[a][a]);
                smin = fmin(smin, S[a][a]);
            }
            if (smin > 1e-6 * smax && smax > 0.0) {
                double T[ALIGN_KB][ALIGN_KB];
                for (int a = 0; a < k; ++a)
                    for (int b = 0; b < k; ++b) {
                        double acc = 0.0;
                        for (int c = 0; c < k; ++c) acc += Q[a][c] * Q[b][c] / sqrt(S[c][c]);
                        T[a][b] = acc;
                    }
                for (int a = 0; a < k; ++a)
                    for (int b = 0; b < k; ++b) {
                        double acc = 0.0;
                        for (int c = 0; c < k; ++c) acc += M[a][c] * T[c][b];
                        R[a][b] = acc;
                    }
                ok = 1;
            }
        }
    }
    __syncthreads();
    if (ok) {
        for (int r = threadIdx.x; r < N; r += 64) {
            double x[ALIGN_KB];
            for (int a = 0; a < k; ++a) x[a] = U[(long)r * ldu + j + a];
            for (int c = 0; c < k; ++c) {
                double acc = 0.0;
                for (int a = 0; a < k; ++a) acc += x[a] * R[a][c];
                U[(long)r * ldu + j + c] = acc;
            }
        }
        return;
    }
    // sign convention per column: the first entry of largest magnitude positive
    __shared__ double sv[64];
    __shared__ int si[64];
    for (int c = 0; c < k; ++c) {
        double best = -1.0;
        int bi = 0;
        for (int r = threadIdx.x; r < N; r += 64) {
            const double a = fabs(U[(long)r * ldu + j + c]);
            if (a > best) { best = a; bi = r; }
        }
        sv[threadIdx.x] = best;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int st = 32; st > 0; st >>= 1) {
            if (threadIdx.x < st) {
                const double a = sv[threadIdx.x + st];
                const int ai = si[threadIdx.x + st];
                if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ai < si[threadIdx.x])) {
                    sv[threadIdx.x] = a;
                    si[threadIdx.x] = ai;
                }
            }
            __syncthreads();
        }
        const bool flip = U[(long)si[0] * ldu + j + c] < 0.0;
        __syncthreads();
        if (flip)
            for (int r = threadIdx.x; r < N; r += 64) U[(long)r * ldu + j + c] = -U[(long)r * ldu + j + c];
        __syncthreads();
    }
}

// The post-eigen pass of a warm solve (one workgroup): cut, n_C, omega, S_E (Eq. 6) with the
// tail's bounded share, Delta, and the spectrum buffer (the k Ritz values ascending, then NaN).
// theta: k values, descending |theta|.  The part of sum lambda^4 beyond the block is exact when
// sum4 (sum lambda^4 / ||C'||_F^4, from ||C'^2||_F^2) is given, else the midpoint of its bounds.
__global__ void __launch_bounds__(256) warm_post_kernel(const double *theta, int k, int N, int m, double gap_tol,
                                                        double rank_tol, const double *fro2, const double *sum4,
                                                        const double *om4_prev, double *omega_new, double *selval,
                                                        PostOut *out, double *spectrum)
{
    __shared__ double red[4];
    __shared__ int s_me;
    const int tid = threadIdx.x;
    const double l1 = fabs(theta[0]);
    if (tid == 0) {
        const int jmax = (k == N) ? min(m, N) : min(m, k - 1);
        int me = -1;
        for (int j = jmax; j >= 1; --j) {
            const double aj = fabs(theta[j - 1]);
            if (aj <= rank_tol * l1) continue;
            if (j == N || aj - fabs(theta[j]) > gap_tol * l1) { me = j; break; }
        }
        if (me < 0) {
            int c = 0;
            for (int j = 0; j < jmax; ++j) c += (fabs(theta[j]) > rank_tol * l1) ? 1 : 0;
            me = max(1, c);
        }
        s_me = me;
    }
    __syncthreads();
    const int me = s_me;
    double s4 = 0.0, s2 = 0.0, rk = 0.0;
    for (int i = tid; i < k; i += 256) {
        const double x = theta[i] / l1;
        s4 += (x * x) * (x * x);
        s2 += theta[i] * theta[i];
        rk += (fabs(theta[i]) > rank_tol * l1) ? 1.0 : 0.0;
    }
    s4 = block_sum<256>(s4, red);
    s2 = block_sum<256>(s2, red);
    rk = block_sum<256>(rk, red);
    // the spectrum beyond the block: sum lambda^2 = ||C'||_F^2 - sum theta^2, each |lambda| <= |theta_k|
    const double thk = fabs(theta[k - 1]) / l1;
    const double t2 = (k < N) ? fmax(0.0, *fro2 / (l1 * l1) - s2 / (l1 * l1)) : 0.0;
    double t4 = 0.5 * thk * thk * t2;  // midpoint of [0, thk^2 t2]
    if (sum4 && k < N) {
        const double F = *fro2 / (l1 * l1);
        t4 = fmax(0.0, (*sum4) * F * F - s4);
    }
    const double nC = l1 * sqrt(sqrt(s4 + t4));
    const double tn = t4 / (s4 + t4);        // tail share of sum w^4 (estimate), bound tn
    double se = 0.0;
    for (int i = tid; i < k; i += 256) {
        const double wv = theta[i] / nC;
        const double w4 = (wv * wv) * (wv * wv);
        if (w4 > 0.0) se -= w4 * log(w4);
    }
    se = block_sum<256>(se, red);
    if (tn > 0.0) {
        // each remaining w^4 is at most u: their entropy lies in [tn ln(1/u), tn ln((N-k)/tn)]
        const double u = (thk * thk) * (thk * thk) * (l1 * l1 * l1 * l1) / ((nC * nC) * (nC * nC));
        const double lo = tn * log(1.0 / u), hi = tn * log((double)(N - k) / tn);
        se += 0.5 * (lo + fmax(lo, hi));
    }
    double dl = 0.0, kept4 = 0.0;
    for (int j = tid; j < m; j += 256) {
        const double om = (j < me) ? theta[j] / nC : 0.0;
        omega_new[j] = om;
        const double o4 = (om * om) * (om * om);
        kept4 += o4;
        const double op = om4_prev[j];
        dl = fmax(dl, fabs(o4 - (op * op) * (op * op)));
    }
    dl = block_max<256>(dl, red);
    kept4 = block_sum<256>(kept4, red);
    for (int j = tid; j < min(k, m + 1); j += 256) selval[j] = theta[j];
    // spectrum: the Ritz values in ascending order (rank by value, ties by index), NaN beyond
    for (int i = tid; i < k; i += 256) {
        const double v = theta[i];
        int r = 0;
        for (int t = 0; t < k; ++t) {
            const double u2 = theta[t];
            r += (u2 < v || (u2 == v && t < i)) ? 1 : 0;
        }
        spectrum[r] = v;
    }
    for (int i = k + tid; i < N; i += 256) spectrum[i] = __longlong_as_double(0x7FF8000000000000LL);
    if (tid == 0) {
        out->m_eff = me;
        out->rank = (int)rk;
        out->nclusters = 0;
        out->n_C = nC;
        out->S_E = se;
        out->delta = dl;
        out->lam1 = l1;
        out->sum_w4_kept = kept4;
        out->tail_bound = tn;
    }
}

// ---------------------------------------------------------------- host helpers

int splits_for_k(long tiles, long K, int kmin)
{
    long s = 1;
    while (tiles * s < 512 && K / (s * 2) >= kmin) s *= 2;
    return (int)s;
}

// C (k x k, ld kmax) = A^T B for two N x k blocks (ld kmax), split over N.
hipError_t gram(WarmWork &w, const double *A, const double *B, double *C, int N, int k, hipStream_t s)
{
    const long tiles = (long)ceil_div(k, 64) * ceil_div(k, 64);
    int sp = splits_for_k(tiles, N, 256);
    while (sp > 1 && (size_t)sp * k * k > w.rr.splitk_elems) sp /= 2;
    return gemm_mfma_splitk(A_T{A, w.kmax}, B_RM{B, w.kmax}, EpiStore{C, w.kmax, 1.0}, k, k, N, sp, w.rr.splitk, s);
}

// Y (N x k, ld kmax) <- Y L^{-T} with L the Cholesky factor of Y^T Y (+ the shift of
// gram_shift_kernel when `shift`): the columns become orthonormal (up to cond(Y)^2 u without the
// shift).
hipError_t chol_qr(WarmWork &w, double *Y, int N, int k, bool shift, hipStream_t s)
{
    const int ld = w.kmax;
    hipError_t e = gram(w, Y, Y, w.G, N, k, s);
    if (e != hipSuccess) return e;
    if (shift) hipLaunchKernelGGL(gram_shift_kernel, dim3(1), dim3(256), 0, s, w.G, k, (long)ld, N);
    const int nblk = ceil_div(k, CB);
    for (int pb = 0; pb < nblk; ++pb) {
        const int p0 = pb * CB, nb = std::min(CB, k - p0), p1 = p0 + nb, nt = k - p1;
        double *Li = w.Linv + (long)pb * CB * CB;
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, w.G, ld, p0, nb, Li, w.err);
        if (nt > 0) {
            // panel below the block: L_ip = G_ip L_pp^{-T}
            e = gemm_mfma(GEMM_SMALL, A_RM{w.G + (long)p1 * ld + p0, ld}, B_T{Li, CB},
                          EpiStore{w.G + (long)p1 * ld + p0, ld, 1.0}, nt, nb, nb, s);
            if (e != hipSuccess) return e;
            // trailing lower triangle: G_22 -= L_21 L_21^T
            e = gemm_mfma_lower(A_RM{w.G + (long)p1 * ld + p0, ld}, B_T{w.G + (long)p1 * ld + p0, ld},
                                EpiAxpbyLower{w.G + (long)p1 * ld + p1, ld, -1.0, 1.0}, nt, nb, s);
            if (e != hipSuccess) return e;
        }
    }
    // Q L^T = Y, column block by column block
    for (int pb = 0; pb < nblk; ++pb) {
        const int p0 = pb * CB, nb = std::min(CB, k - p0);
        const double *Li = w.Linv + (long)pb * CB * CB;
        if (p0 > 0) {
            e = gemm_mfma(GEMM_TALL, A_RM{Y, ld}, B_T{w.G + (long)p0 * ld, ld}, EpiAxpby{Y + p0, ld, -1.0, 1.0}, N, nb,
                          p0, s);
            if (e != hipSuccess) return e;
        }
        e = gemm_mfma(GEMM_SMALL, A_RM{Y + p0, ld}, B_T{Li, CB}, EpiStore{Y + p0, ld, 1.0}, N, nb, nb, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

__global__ void copy_cols_kernel(const double *src, double *dst, long ld, int N, int nc)
{
    const long total = (long)N * nc;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / nc), j = (int)(idx - (long)i * nc);
        dst[(long)i * ld + j] = src[(long)i * ld + j];
    }
}

// dst[:, :nc] = src[:, :nc] (N rows, ld)
hipError_t copy_cols(const double *src, double *dst, long ld, int N, int nc, hipStream_t s)
{
    hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_for((long)N * nc)), dim3(256), 0, s, src, dst, ld, N, nc);
    return hipGetLastError();
}

// A product C' B (N x N times N x ka, ld kmax) with epilogue epi: 128 x 128 tiles, the K range
// split so that at least three rounds of workgroups fill the device (the output alone has
// ceil(N/128) ceil(ka/128) tiles: 400 at N = 10240, ka = 640, for 256 compute units).
template <class EPI>
hipError_t product(WarmWork &w, const double *C, int N, const double *B, int ka, EPI epi, bool timed, hipStream_t s)
{
    const long tiles = (long)ceil_div(N, 128) * ceil_div(ka, 128);
    int sp = 1;
    while (tiles * sp < 1024 && (size_t)(2 * sp) * N * ka <= w.part_elems) sp *= 2;
    const bool rec = timed && w.nev < WarmWork::NEV;
    if (rec) (void)hipEventRecord(w.ev[2 * w.nev], s);
    hipError_t e = (sp == 1) ? gemm_mfma(GEMM_LARGE, A_RM{C, N}, B_RM{B, w.kmax}, epi, N, ka, N, s)
                             : gemm_mfma_splitk(A_RM{C, N}, B_RM{B, w.kmax}, epi, N, ka, N, sp, w.pbig, s, GEMM_LARGE);
    if (rec) {
        (void)hipEventRecord(w.ev[2 * w.nev + 1], s);
        w.pending_flops[w.nev] = 2.0 * N * (double)N * ka;
        w.nev += 1;
    }
    return e;
}

// Adds the timed products of the pass (after the stream has been synchronized).
void collect_product_times(WarmWork &w)
{
    for (int i = 0; i < w.nev; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, w.ev[2 * i], w.ev[2 * i + 1]) == hipSuccess) {
            w.product_ms += ms;
            w.product_flops += w.pending_flops[i];
            w.product_launches += 1;
        }
    }
    w.nev = 0;
}

// The cut of the post kernel, on the host, for the convergence decision.
int host_cut(const double *theta, int k, int N, int m, double gap_tol, double rank_tol)
{
    const double l1 = fabs(theta[0]);
    const int jmax = (k == N) ? std::min(m, N) : std::min(m, k - 1);
    for (int j = jmax; j >= 1; --j) {
        const double aj = fabs(theta[j - 1]);
        if (aj <= rank_tol * l1) continue;
        if (j == N || aj - fabs(theta[j]) > gap_tol * l1) return j;
    }
    int c = 0;
    for (int j = 0; j < jmax; ++j) c += (fabs(theta[j]) > rank_tol * l1) ? 1 : 0;
    return std::max(1, c);
}

// Per-column coefficients of the scaled Chebyshev recurrence of degree d on [-a, a]:
// Yhat_1 = C' V / theta_c, Yhat_j = (2/a) rho_j C' Yhat_{j-1} - rho_{j-1} rho_j Yhat_{j-2},
// rho_1 = 1/x, rho_j = 1/(2x - rho_{j-1}), x = theta_c / a (kept away from [-1, 1]).
void cheb_coefficients(const double *theta, int k, double a, int d, double *coef, int kmax)
{
    for (int c = 0; c < k; ++c) {
        double x = theta[c] / a;
        if (fabs(x) < 1.01) x = (x < 0.0 ? -1.01 : 1.01);
        double rho_prev = 1.0 / x;
        coef[c] = 1.0 / (a * x);       // alpha of degree 1
        coef[kmax + c] = 0.0;          // beta of degree 1
        for (int j = 2; j <= d; ++j) {
            const double rho = 1.0 / (2.0 * x - rho_prev);
            coef[(long)(2 * (j - 1)) * kmax + c] = 2.0 * rho / a;
            coef[(long)(2 * (j - 1) + 1) * kmax + c] = -rho_prev * rho;
            rho_prev = rho;
        }
    }
}

// Rotate/sign the first me columns of U (ld ldu) towards Uprev (N x m, me_prev columns).
hipError_t align_block(WarmWork &w, double *U, int ldu, int N, int me, const double *theta, const double *Uprev,
                       int m, int me_prev, double gap_tol, hipStream_t s)
{
    const int mm = std::min(me, me_prev);
    if (mm < 1) return hipSuccess;
    const long tiles = (long)ceil_div(mm, 64) * ceil_div(mm, 64);
    int sp = splits_for_k(tiles, N, 256);
    while (sp > 1 && (size_t)sp * mm * mm > w.rr.splitk_elems) sp /= 2;
    hipError_t e = gemm_mfma_splitk(A_T{U, ldu}, B_RM{Uprev, m}, EpiStore{w.Mov, mm, 1.0}, mm, mm, N, sp,
                                    w.rr.splitk, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(warm_align_kernel, dim3(mm), dim3(64), 0, s, U, ldu, N, w.Mov, mm, theta, gap_tol);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------- allocation

size_t warm_bytes(int N, int m, int p)
{
    const size_t k = (size_t)std::min(N, m + p);
    const size_t nb = (k + CB - 1) / CB;
    size_t s = sizeof(double) * (8 * (size_t)N * k + 5 * k * k + nb * CB * CB + 3 * (k + 8) + k + 2 * WARM_DMAX * k +
                                 RES_CHUNKS * k + k + 1024 + 24);
    s += sizeof(PostOut) + 64;
    s += eig_bytes((int)k, (int)k, 16);
    return s;
}

hipError_t warm_alloc(WarmWork &w, int N, int m, int p, Arena *ar, hipStream_t s)
{
    Arena own;
    Arena &a = ar ? *ar : own;
    w.N = N;
    w.m = m;
    w.p = p;
    w.kmax = std::min(N, m + p);
    w.nb = ceil_div(w.kmax, CB);
    const size_t k = (size_t)w.kmax;
    struct Req { double **p; size_t n; };
    Req reqs[] = {
        {&w.V, (size_t)N * k}, {&w.Y, (size_t)N * k}, {&w.CQ, (size_t)N * k}, {&w.CV, (size_t)N * k},
        {&w.G, k * k}, {&w.H, k * k}, {&w.Hs, k * k}, {&w.X, k * k}, {&w.Mov, k * k},
        {&w.Linv, (size_t)w.nb * CB * CB}, {&w.theta, k + 8}, {&w.zero, k + 8}, {&w.scr, k + 8},
        {&w.coef, 2 * (size_t)WARM_DMAX * k}, {&w.res, (size_t)RES_CHUNKS * k + k}, {&w.part, 1024}, {&w.fro2, 8}, {&w.sum4, 8},
        {&w.pbig, 4 * (size_t)N * k},
    };
    w.part_elems = 4 * (size_t)N * k;
    w.carved = a.carving();
    for (auto &r : reqs) {
        hipError_t e = a.take((void **)r.p, sizeof(double) * std::max<size_t>(r.n, 1));
        if (e != hipSuccess) return e;
    }
    hipError_t e = a.take((void **)&w.rr_post, sizeof(PostOut));
    if (e == hipSuccess) e = a.take((void **)&w.err, 64);
    // the small solver's workspace
    void *rr_base = nullptr;
    const size_t rr_bytes = eig_bytes(w.kmax, w.kmax, 16);
    if (e == hipSuccess && a.carving()) e = a.take(&rr_base, rr_bytes);
    if (e != hipSuccess || a.count_only) return e;
    e = hipHostMalloc((void **)&w.h_theta, sizeof(double) * (k + 8), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w.h_res, sizeof(double) * (k + 8), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&w.h_coef, sizeof(double) * 2 * WARM_DMAX * k, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w.h_post, sizeof(PostOut), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w.h_scal, sizeof(double) * 8, hipHostMallocDefault);

    if (e == hipSuccess) e = hipMemset(w.zero, 0, sizeof(double) * (k + 8));
    if (e == hipSuccess) e = hipMemset(w.err, 0, 64);
    if (e == hipSuccess) e = rr_base ? eig_carve(w.rr, rr_base, rr_bytes, w.kmax, w.kmax, 16, s)
                                     : eig_alloc(w.rr, w.kmax, w.kmax, 16);
    for (int i = 0; i < 2 * WarmWork::NEV && e == hipSuccess; ++i) e = hipEventCreate(&w.ev[i]);
    return e;
}

void warm_free(WarmWork &w)
{
    double *bufs[] = {w.V, w.Y, w.CQ, w.CV, w.G, w.H, w.Hs, w.X, w.Mov, w.Linv, w.theta, w.zero, w.scr,
                      w.coef, w.res, w.part, w.fro2, w.sum4, w.pbig};
    if (!w.carved) {
        for (double *p : bufs)
            if (p) (void)hipFree(p);
        if (w.rr_post) (void)hipFree(w.rr_post);
        if (w.err) (void)hipFree(w.err);
    }
    if (w.h_theta) (void)hipHostFree(w.h_theta);
    if (w.h_res) (void)hipHostFree(w.h_res);
    if (w.h_coef) (void)hipHostFree(w.h_coef);
    if (w.h_post) (void)hipHostFree(w.h_post);
    if (w.h_scal) (void)hipHostFree(w.h_scal);

    eig_free(w.rr);
    for (int i = 0; i < 2 * WarmWork::NEV; ++i)
        if (w.ev[i]) (void)hipEventDestroy(w.ev[i]);
    w = WarmWork();
}

hipError_t warm_frobenius(WarmWork &w, const double *C, long n2, hipStream_t s)
{
    const int np = grid_for(n2);
    hipLaunchKernelGGL(sumsq_partial_kernel, dim3(np), dim3(256), 0, s, C, n2, w.part);
    hipLaunchKernelGGL(sum_finalize_kernel, dim3(1), dim3(64), 0, s, w.part, np, w.fro2);
    return hipGetLastError();
}

// Upper bound on the share of sum lambda^4 beyond the k Ritz values theta (descending |.|):
// the remaining sum lambda^2 is ||C'||_F^2 - sum theta^2 and each remaining |lambda| <= |theta_k|.
double tail_share_bound(const double *theta, int k, double fro2)
{
    const double l1 = fabs(theta[0]);
    if (!(l1 > 0.0)) return 1.0;
    double s4 = 0.0, s2 = 0.0;
    for (int i = 0; i < k; ++i) {
        const double x = theta[i] / l1;
        s4 += (x * x) * (x * x);
        s2 += x * x;
    }
    const double thk = fabs(theta[k - 1]) / l1;
    const double t4 = thk * thk * std::max(0.0, fro2 / (l1 * l1) - s2);
    return t4 / (s4 + t4);
}

hipError_t warm_symmetrize(double *C, int N, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    const long T = ceil_div(N, 64);
    hipLaunchKernelGGL(mirror_lower_kernel, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, s, C, N);
    return hipGetLastError();
}

hipError_t warm_sum4(WarmWork &w, const double *C, int N, double *sq, hipStream_t s)
{
    hipError_t e = gemm_mfma_lower_large(A_RM{C, N}, B_RM{C, N}, EpiSquareTiles{sq, N}, N, N, s);
    if (e != hipSuccess) return e;
    const int np = std::min(N, 1024);
    hipLaunchKernelGGL(sum4_partial_kernel, dim3(np), dim3(256), 0, s, sq, N, w.fro2, w.part);
    hipLaunchKernelGGL(sum_finalize_kernel, dim3(1), dim3(64), 0, s, w.part, np, w.sum4);
    return hipGetLastError();
}

hipError_t warm_seed(WarmWork &w, int N, int m, int m_eff, int kk, const double *selk, double *U, int m_eff_prev,
                     double gap_tol, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(w.theta, selk, sizeof(double) * kk, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = align_block(w, w.V, w.kmax, N, m_eff, w.theta, U, m, m_eff_prev, gap_tol, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(copy_kept_kernel, dim3(grid_for((long)N * m)), dim3(256), 0, s, w.V, (long)w.kmax, N, m_eff, m, U);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = hipMemcpyAsync(w.h_theta, w.theta, sizeof(double) * kk, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    w.kcur = kk;
    w.a_prev = fabs(w.h_theta[kk - 1]);
    return hipSuccess;
}

// ---------------------------------------------------------------- the solve

hipError_t warm_solve(WarmWork &w, const double *C, int N, int m, const WarmParams &prm, const double *omega_prev,
                      double *omega_new, double *selval, PostOut *post_dev, double *U, int m_eff_prev,
                      double *spectrum, double *sq, hipStream_t s, int *converged, std::string *why)
{
    *converged = 0;
    const int k = w.kcur;
    const int ld = w.kmax;
    const int d = std::max(1, std::min(prm.degree, WARM_DMAX));
    if (k < 2 || N != w.N) {
        *why = "no warm start";
        w.last_reason = 1;
        return hipSuccess;
    }
    hipError_t e = warm_frobenius(w, C, (long)N * N, s);
    if (e != hipSuccess) return e;
    w.steps += 1;
    // Ritz values of the block from the previous step or pass (host copy), descending |theta|
    double a = std::max(w.a_prev, 1e-12 * fabs(w.h_theta[0]));
    // Leading columns whose residual is below the tolerance are locked: later passes filter,
    // orthonormalize (against the locked block) and Rayleigh-Ritz only the columns [nl, k).
    int nl = 0;
    double *resn = w.res + (long)RES_CHUNKS * ld;  // residual norms, one per column
    for (int pass = 0; pass < prm.max_passes; ++pass) {
        w.passes += 1;
        const int ka = k - nl;
        double *QL = w.V;  // the locked columns [0, nl) stay in this buffer
        // 1. Chebyshev filter of the active columns (ping-pong between V and Y; result in `cur`).
        //    The first pass of a step is one plain product: the previous step's vectors carry
        //    components along this step's leading eigenvectors that a higher degree would
        //    amplify by T_d(|lambda_1| / a) past the precision of the block.  Later passes filter
        //    with the operator deflated by the locked pairs, C' - Q_L Theta_L Q_L^T, so that the
        //    leading directions are not amplified again.
        // The degree of a pass: at most d, and low enough that the filter amplifies the largest
        // active Ritz value by no more than 1e8 over the edge of the damped interval (the
        // block's columns keep 8 significant digits of their own direction against
        // rounding-level components along the top of the active range).
        int dp = 1;
        {
            const double xt = std::max(1.0, fabs(w.h_theta[nl]) / a);
            const double ach = acosh(xt);
            while (dp < d && cosh((dp + 1) * ach) <= 1e8) ++dp;
        }
        cheb_coefficients(w.h_theta + nl, ka, a, dp, w.h_coef, ld);
        e = hipMemcpyAsync(w.coef, w.h_coef, sizeof(double) * 2 * dp * ld, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        double *prev = w.V, *cur = w.Y;
        const long ltiles = (long)ceil_div(nl, 64) * ceil_div(ka, 64);
        int lsp = splits_for_k(ltiles, N, 256);
        while (lsp > 1 && (size_t)lsp * nl * ka > w.rr.splitk_elems) lsp /= 2;
        for (int j = 1; j <= dp; ++j) {
            const double *alpha = w.coef + (long)(2 * (j - 1)) * ld, *beta = w.coef + (long)(2 * (j - 1) + 1) * ld;
            // degree 1: Y = alpha C' V;  degree j: (into prev's buffer) alpha C' cur + beta prev
            double *dst = (j == 1) ? cur : prev;
            const double *src = (j == 1) ? prev : cur;
            if (nl > 0) {
                // T = Theta_L Q_L^T src, before dst (which may share src's buffer only for j = 1,
                // where dst is the other buffer) is written
                e = gemm_mfma_splitk(A_T{QL, ld}, B_RM{src + nl, ld}, EpiStore{w.H, ld, 1.0}, nl, ka, N, lsp,
                                     w.rr.splitk, s);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(scale_rows_by_kernel, dim3(grid_for((long)nl * ka)), dim3(256), 0, s, w.H, (long)ld,
                                   nl, ka, w.theta);
            }
            e = product(w, C, N, src + nl, ka, EpiCheb{dst + nl, ld, alpha, beta}, prm.profile, s);
            if (e == hipSuccess && nl > 0)
                e = gemm_mfma(GEMM_LARGE, A_RM{QL, ld}, B_RM{w.H, ld}, EpiSubScaled{dst + nl, ld, alpha}, N, ka, nl, s);
            if (e != hipSuccess) return e;
            w.products += 1;
            if (j > 1) std::swap(prev, cur);
        }
        double *Q = cur, *spare = prev;
        // 2. orthonormal basis of the filtered active columns: twice projected off the locked
        //    block, then shifted Cholesky QR and twice unshifted (the filter leaves the block far
        //    from orthogonal: its columns share the directions of the largest eigenvalues,
        //    amplified by up to T_d(|lambda_1| / a))
        e = hipMemsetAsync(w.err, 0, sizeof(unsigned), s);
        for (int r = 0; r < 2 && nl > 0 && e == hipSuccess; ++r) {
            const long tiles = (long)ceil_div(nl, 64) * ceil_div(ka, 64);
            int sp = splits_for_k(tiles, N, 256);
            while (sp > 1 && (size_t)sp * nl * ka > w.rr.splitk_elems) sp /= 2;
            e = gemm_mfma_splitk(A_T{QL, ld}, B_RM{Q + nl, ld}, EpiStore{w.H, ld, 1.0}, nl, ka, N, sp, w.rr.splitk, s);
            if (e == hipSuccess)
                e = gemm_mfma(GEMM_LARGE, A_RM{QL, ld}, B_RM{w.H, ld}, EpiAxpby{Q + nl, ld, -1.0, 1.0}, N, ka, nl, s);
        }
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = chol_qr(w, Q + nl, N, ka, r == 0, s);
        if (e != hipSuccess) return e;
        // 3. Rayleigh-Ritz on the active columns: H = Q^T C' Q, its eigenpairs, the Ritz vectors
        //    and C' times them
        e = product(w, C, N, Q + nl, ka, EpiStore{w.CQ + nl, ld, 1.0}, prm.profile, s);
        if (e != hipSuccess) return e;
        w.products += 1;
        e = gram(w, Q + nl, w.CQ + nl, w.H, N, ka, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(symmetrize_kernel, dim3(grid_for((long)ka * ka)), dim3(256), 0, s, w.H, w.Hs, ka, (long)ld);
        unsigned flags = 0;
        e = hipMemcpyAsync(w.h_scal + 2, w.err, sizeof(unsigned), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        memcpy(&flags, w.h_scal + 2, sizeof(unsigned));
        if (flags) {
            *why = "the filtered block lost rank (Gram matrix not positive definite)";
            w.last_reason = 2;
            collect_product_times(w);
            return hipSuccess;
        }
        // the small eigenproblem: all eigenpairs of H with the two-stage solver
        e = eig_values(w.rr, w.Hs, ld, ka, s);
        if (e == hipSuccess) e = eig_post(w.rr, ka, ka, -1.0, -1.0, w.zero, w.scr, w.theta + nl, w.rr_post, s);
        if (e == hipSuccess) e = hipMemcpyAsync(w.h_post, w.rr_post, sizeof(PostOut), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (eig_take_errors(w.rr)) {
            *why = "the Rayleigh-Ritz eigensolver raised an error";
            w.last_reason = 3;
            return hipSuccess;
        }
        e = eig_vectors(w.rr, nullptr, 0, ka, ka, w.theta + nl, w.h_post->nclusters, w.X, ld, s);
        if (e != hipSuccess) return e;
        e = gemm_mfma(GEMM_LARGE, A_RM{Q + nl, ld}, B_RM{w.X, ld}, EpiStore{spare + nl, ld, 1.0}, N, ka, ka, s);
        if (e == hipSuccess)
            e = gemm_mfma(GEMM_LARGE, A_RM{w.CQ + nl, ld}, B_RM{w.X, ld}, EpiStore{w.CV + nl, ld, 1.0}, N, ka, ka, s);
        if (e == hipSuccess && nl > 0 && spare != QL) e = copy_cols(QL, spare, ld, N, nl, s);
        if (e != hipSuccess) return e;
        // 4. residuals of the active Ritz pairs
        hipLaunchKernelGGL(resid_partial_kernel, dim3(ceil_div(ka, 256), RES_CHUNKS), dim3(256), 0, s, w.CV + nl,
                           spare + nl, w.theta + nl, N, ka, (long)ld, w.res);
        hipLaunchKernelGGL(resid_finalize_kernel, dim3(ceil_div(ka, 256)), dim3(256), 0, s, w.res, RES_CHUNKS, ka,
                           resn + nl);
        e = hipMemcpyAsync(w.h_theta + nl, w.theta + nl, sizeof(double) * ka, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w.h_res + nl, resn + nl, sizeof(double) * ka, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(w.h_scal + 4, w.fro2, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        collect_product_times(w);
        // the new block becomes the basis
        w.V = spare;
        w.Y = Q;
        a = std::max(fabs(w.h_theta[k - 1]), 1e-12 * fabs(w.h_theta[0]));
        w.a_prev = a;
        if (nl > 0 && fabs(w.h_theta[nl]) > fabs(w.h_theta[nl - 1])) {
            // an active Ritz value above a locked one: the order by |theta| is lost, unlock all
            nl = 0;
            continue;
        }
        const int me = host_cut(w.h_theta, k, N, m, prm.gap_tol, prm.rank_tol);
        double rmax = 0.0;
        for (int j = 0; j < me; ++j) rmax = std::max(rmax, w.h_res[j]);
        w.last_rmax = rmax / fabs(w.h_theta[0]);
        if (!std::isfinite(rmax)) {
            *why = "non-finite residual";
            w.last_reason = 4;
            w.kcur = 0;
            return hipSuccess;
        }
        const double rtol = prm.tol * fabs(w.h_theta[0]);
        if (rmax <= rtol) {
            // sum lambda^4 exactly (||C'^2||_F^2) when asked, or when the bound on the share of
            // sum w^4 beyond the block is above prm.tail_tol
            const double *sum4 = nullptr;
            if (sq && k < N && (prm.tail_exact || tail_share_bound(w.h_theta, k, w.h_scal[4]) > prm.tail_tol)) {
                if ((e = warm_sum4(w, C, N, sq, s)) != hipSuccess) return e;
                sum4 = w.sum4;
                w.exact_tails += 1;
            }
            // 5. outputs: kept vectors in the previous step's gauge, post-eigen quantities
            e = align_block(w, w.V, ld, N, me, w.theta, U, m, m_eff_prev, prm.gap_tol, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(copy_kept_kernel, dim3(grid_for((long)N * m)), dim3(256), 0, s, w.V, (long)ld, N, me,
                               m, U);
            hipLaunchKernelGGL(warm_post_kernel, dim3(1), dim3(256), 0, s, w.theta, k, N, m, prm.gap_tol,
                               prm.rank_tol, w.fro2, sum4, omega_prev, omega_new, selval, post_dev, spectrum);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            *converged = 1;
            w.last_reason = 0;
            return hipSuccess;
        }
        // lock the converged leading columns, never splitting a multiplet
        while (nl < me && w.h_res[nl] <= rtol) ++nl;
        while (nl > 0 && nl < k && !(fabs(w.h_theta[nl - 1]) - fabs(w.h_theta[nl]) > prm.gap_tol * fabs(w.h_theta[0])))
            --nl;
    }
    *why = "not converged in the pass limit";
    w.last_reason = 5;
    return hipSuccess;
}

}  // namespace ctm
