// Derivative of the CTMRG fixed point with respect to K; see adjoint.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "adjoint.h"
#include "blocks.h"
#include "common.h"
#include "contract.h"
#include "ctmrg.h"
#include "gemm.h"

namespace ctm {

namespace {

constexpr int KB = 8;        // largest multiplet the alignment handles
constexpr int NSCAL = 16;    // device scalars: 0 s*, 1 dn_C/n_C^3-scaled, 2 ds, 3 tangent change, 5 gauge residual,
                             // 6 .. 14 the Frobenius products of the energy's tangent

enum { S_NORM = 0, S_DNC = 1, S_DS = 2, S_CHANGE = 3, S_GAUGE = 5, S_OBS = 6 };
enum { OP_SUM = 0, OP_SQRT = 1, OP_MAX = 2, OP_MAX_ACC = 3 };

int grid_for(long n) { return (int)std::max<long>(1, std::min<long>(1024, (n + 255) / 256)); }

// ---------------------------------------------------------------- small kernels

// Ad (d x q d), omd (d), Ud (q d x d) from the padded state A (m x q m), omega (m), U (q m x m).
__global__ void compact_kernel(const double *A, const double *om, const double *U, int q, int m, int d, double *Ad,
                               double *omd, double *Ud)
{
    const long n = (long)q * d;
    const long totA = (long)d * n;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < totA; idx += (long)gridDim.x * blockDim.x) {
        const int g = (int)(idx / n);
        const int c = (int)(idx - (long)g * n);
        const int s = c / d, a = c - s * d;
        Ad[idx] = A[(long)g * q * m + s * m + a];
        const int r = g;  // reuse the index range for U: row c, column r
        Ud[(long)c * d + r] = U[(long)(s * m + a) * m + r];
    }
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < d; i += (long)gridDim.x * blockDim.x) omd[i] = om[i];
}

__global__ void __launch_bounds__(256) dot_partial_kernel(const double *x, const double *y, long n, double *part)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        acc += x[i] * y[i];
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(256) maxdiff_partial_kernel(const double *x, const double *y, long n, double *part)
{
    __shared__ double red[4];
    double mx = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        mx = fmax(mx, fabs(x[i] - y[i]));
    mx = block_max<256>(mx, red);
    if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

__global__ void finalize_kernel(const double *part, int np, double *out, int op, double scale)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    if (op == OP_SUM || op == OP_SQRT) {
        for (int i = 0; i < np; ++i) acc += part[i];
        *out = (op == OP_SQRT) ? sqrt(acc) : scale * acc;
    } else {
        for (int i = 0; i < np; ++i) acc = fmax(acc, part[i]);
        *out = (op == OP_MAX_ACC) ? fmax(*out, acc) : acc;
    }
}

// y = x / *s
__global__ void div_by_kernel(const double *x, double *y, long n, const double *s)
{
    const double inv = 1.0 / *s;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = x[i] * inv;
}

__global__ void axpy_kernel(double *y, const double *x, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] += x[i];
}

// dst (rows x cols, ld_dst) = src (rows x cols, ld_src)
__global__ void copy2d_kernel(const double *src, long ld_src, double *dst, long ld_dst, int rows, int cols)
{
    const long total = (long)rows * cols;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int r = (int)(idx / cols), c = (int)(idx - (long)r * cols);
        dst[r * ld_dst + c] = src[r * ld_src + c];
    }
}

// Symmetric k x k eigendecomposition by cyclic Jacobi (k <= KB, one thread).
__device__ void small_jacobi(double (&S)[KB][KB], double (&V)[KB][KB], int k)
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
                for (int i = 0; i < k; ++i) {  // columns p, r
                    const double a = S[i][p], b = S[i][r];
                    S[i][p] = c * a - sn * b;
                    S[i][r] = sn * a + c * b;
                }
                for (int i = 0; i < k; ++i) {  // rows p, r
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

// Rotate the kept columns of U inside each multiplet to best match the previous
// vectors (orthogonal Procrustes): with M = U_b^T Uprev_b, U_b <- U_b M (M^T M)^{-1/2}.
// lamk: the kept eigenvalues in the order of the columns (descending |lambda|);
// multiplets are separated by gaps |l_j| - |l_{j+1}| > gap_tol |l_1| (the cut rule).
// One workgroup per column; only the first column of a multiplet works.
__global__ void __launch_bounds__(64) align_kernel(double *U, int ldu, int n, const double *Mov, int d,
                                                  const double *lamk, double gap_tol, unsigned *err)
{
    const int j = blockIdx.x;
    const double tol = gap_tol * fabs(lamk[0]);
    if (j > 0 && !(fabs(lamk[j - 1]) - fabs(lamk[j]) > tol)) return;
    int k = 1;
    while (j + k < d && !(fabs(lamk[j + k - 1]) - fabs(lamk[j + k]) > tol)) ++k;
    __shared__ double R[KB][KB];
    __shared__ int ok;
    if (threadIdx.x == 0) {
        ok = 1;
        if (k > KB) {
            ok = 0;
            raise_error(err, KERR_ALIGN);
        } else {
            double M[KB][KB], S[KB][KB], V[KB][KB];
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) M[a][b] = Mov[(long)(j + a) * d + (j + b)];
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) {
                    double acc = 0.0;
                    for (int c = 0; c < k; ++c) acc += M[c][a] * M[c][b];
                    S[a][b] = acc;
                }
            small_jacobi(S, V, k);
            double smax = 0.0, smin = INFINITY;
            for (int a = 0; a < k; ++a) {
                smax = fmax(smax, S[a][a]);
                smin = fmin(smin, S[a][a]);
            }
            if (!(smin > 1e-6 * smax)) {
                ok = 0;
                raise_error(err, KERR_ALIGN);
            } else {
                // R = M V diag(sigma^-1/2) V^T
                double T[KB][KB];
                for (int a = 0; a < k; ++a)
                    for (int b = 0; b < k; ++b) {
                        double acc = 0.0;
                        for (int c = 0; c < k; ++c) acc += V[a][c] * V[b][c] / sqrt(S[c][c]);
                        T[a][b] = acc;
                    }
                for (int a = 0; a < k; ++a)
                    for (int b = 0; b < k; ++b) {
                        double acc = 0.0;
                        for (int c = 0; c < k; ++c) acc += M[a][c] * T[c][b];
                        R[a][b] = acc;
                    }
            }
        }
    }
    __syncthreads();
    if (!ok) return;
    for (int r = threadIdx.x; r < n; r += 64) {
        double x[KB];
        for (int a = 0; a < k; ++a) x[a] = U[(long)r * ldu + j + a];
        for (int c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int a = 0; a < k; ++a) acc += x[a] * R[a][c];
            U[(long)r * ldu + j + c] = acc;
        }
    }
}

// UL[r][c] = U[r][c] lam_c^3 for c < np (row length ld)
__global__ void scale_cols_cube_kernel(const double *U, long ld, int rows, int np, const double *lam, double *UL)
{
    const long total = (long)rows * np;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int r = (int)(idx / np), c = (int)(idx - (long)r * np);
        const double l = lam[c];
        UL[r * ld + c] = U[r * ld + c] * l * l * l;
    }
}

// The eigen part of the tangent, in place on B = U_all^T dC' U_k (np x d):
//   kept rows i < d: the corner block dOm[i][j] = B[i][j] / n_C - delta_ij lam_j dn_C / n_C^2,
//     and G[i][j] = 0 (rotations inside the kept space are gauge: the state carries them in dOm);
//   other rows: G[i][j] = B[i][j] / (lam_j - lam_i) (no kept multiplet reaches past the cut).
// dnc holds dn_C = <C'^3, dC'> / n_C^3.
__global__ void eigen_tangent_kernel(double *B, int np, int d, const double *lam, double nC, const double *dnc,
                                     double *dOm)
{
    const double dn = *dnc;
    const long total = (long)np * d;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / d), j = (int)(idx - (long)i * d);
        const double b = B[idx];
        if (i < d) {
            dOm[(long)i * d + j] = b / nC - (i == j ? lam[j] * dn / (nC * nC) : 0.0);
            B[idx] = 0.0;
        } else {
            B[idx] = b / (lam[j] - lam[i]);
        }
    }
}

// dU[:, j] += R[:, j] / lam_j: the eigenvectors of C' with eigenvalue zero, through
// the complement of the computed ones.
__global__ void nullspace_tangent_kernel(double *dU, const double *R, long n, int d, const double *lam)
{
    const long total = n * d;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int j = (int)(idx % d);
        dU[idx] += R[idx] / lam[j];
    }
}

// dOA = Omega dA (rows scaled; the product dOmega A is added by a GEMM)
__global__ void scale_rows_kernel(const double *om, const double *dA, int d, long n, double *dOA)
{
    const long total = (long)d * n;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x)
        dOA[idx] = om[idx / n] * dA[idx];
}

// P = P~ / s:  dP = dP~ / s - P~ ds / s^2
__global__ void tangent_norm_kernel(const double *dPt, const double *Pt, long total, const double *s, const double *ds,
                                    double *dA)
{
    const double sv = *s, dsv = *ds;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x)
        dA[i] = dPt[i] / sv - Pt[i] * dsv / (sv * sv);
}

// W2 = W h4^2 = (W h4)^2 / W (W > 0)
__global__ void weight_h2_kernel(const double *W, const double *WH, double *W2, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        W2[i] = WH[i] * WH[i] / W[i];
}

// Partial sums of sum_{r,c} w_{r mod d} [w_{c mod d}] M[r][c] C[r][c] over an n x n pair (both = the
// product <Om~ M Om~, C>; else <Om~ M, C>), one per workgroup.
__global__ void __launch_bounds__(256) wdot_partial_kernel(const double *M, const double *C, const double *om, int n,
                                                           int d, int both, double *part)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int r = blockIdx.x; r < n; r += gridDim.x) {
        const double wr = om[r % d];
        const double *mr = M + (long)r * n, *cr = C + (long)r * n;
        double a = 0.0;
        for (int c = threadIdx.x; c < n; c += 256) a += (both ? om[c % d] : 1.0) * mr[c] * cr[c];
        acc += wr * a;
    }
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// D4[j][k] = dOm[j][k] (w_j^3 + w_j^2 w_k + w_j w_k^2 + w_k^3): the derivative of Omega^4 along dOm
__global__ void omega4_tangent_kernel(const double *dOm, const double *om, int d, double *D4)
{
    const long total = (long)d * d;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int j = (int)(idx / d), k = (int)(idx - (long)j * d);
        const double a = om[j], b = om[k];
        D4[idx] = dOm[idx] * (a * a * a + a * a * b + a * b * b + b * b * b);
    }
}

// One workgroup per spin s: out[s] = prob_s = sum_{b,j} U[(s,b),j]^2 w_j^4 and
// out[q + s] = sum_{b,j} U[(s,b),j] (2 dU[(s,b),j] w_j^4 + V1[(s,b),j]), with V1 = U D4.
__global__ void __launch_bounds__(256) spin_tangent_kernel(const double *U, const double *dU, const double *V1,
                                                           const double *om, int q, int d, double *out)
{
    __shared__ double red[4];
    const int s = blockIdx.x;
    double p = 0.0, dp = 0.0;
    const long total = (long)d * d;
    for (long idx = threadIdx.x; idx < total; idx += 256) {
        const int b = (int)(idx / d), j = (int)(idx - (long)b * d);
        const long at = (long)(s * d + b) * d + j;
        const double w = om[j], w4 = (w * w) * (w * w), u = U[at];
        p += u * u * w4;
        dp += u * (2.0 * dU[at] * w4 + V1[at]);
    }
    p = block_sum<256>(p, red);
    dp = block_sum<256>(dp, red);
    if (threadIdx.x == 0) {
        out[s] = p;
        out[q + s] = dp;
    }
}

// part[i][b] = workgroup b's share of <V_i, x> for the nv vectors V_i (stride L) of a Krylov basis
__global__ void __launch_bounds__(256) multi_dot_partial_kernel(const double *V, long L, int nv, const double *x,
                                                                double *part)
{
    __shared__ double red[4];
    for (int i = 0; i < nv; ++i) {
        const double *v = V + (long)i * L;
        double acc = 0.0;
        for (long k = blockIdx.x * 256L + threadIdx.x; k < L; k += (long)gridDim.x * 256) acc += v[k] * x[k];
        acc = block_sum<256>(acc, red);
        if (threadIdx.x == 0) part[(long)i * gridDim.x + blockIdx.x] = acc;
    }
}

// h[i] = sum of the np partials of vector i (fixed order)
__global__ void multi_dot_finalize_kernel(const double *part, int np, int nv, double *h)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double acc = 0.0;
    for (int b = 0; b < np; ++b) acc += part[(long)i * np + b];
    h[i] = acc;
}

// x += sign * sum_i c[i] V_i
__global__ void lincomb_kernel(const double *V, long L, int nv, const double *c, double sign, double *x)
{
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < L; k += (long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < nv; ++i) acc += c[i] * V[(long)i * L + k];
        x[k] += sign * acc;
    }
}

// r = a - b + c
__global__ void amb_kernel(const double *a, const double *b, const double *c, double *r, long n)
{
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        r[k] = a[k] - b[k] + (c ? c[k] : 0.0);
}

// x *= a
__global__ void scal_kernel(double *x, long n, double a)
{
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) x[k] *= a;
}

// ---------------------------------------------------------------- host helpers

hipError_t reduce_dot(const double *x, const double *y, long n, double *part, double *out, int op, double scale,
                      hipStream_t s)
{
    const int np = grid_for(n);
    hipLaunchKernelGGL(dot_partial_kernel, dim3(np), dim3(256), 0, s, x, y, n, part);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, s, part, np, out, op, scale);
    return hipGetLastError();
}

hipError_t reduce_maxdiff(const double *x, const double *y, long n, double *part, double *out, bool acc, hipStream_t s)
{
    const int np = grid_for(n);
    hipLaunchKernelGGL(maxdiff_partial_kernel, dim3(np), dim3(256), 0, s, x, y, n, part);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, s, part, np, out, acc ? OP_MAX_ACC : OP_MAX, 1.0);
    return hipGetLastError();
}

// *out = <Om~ M Om~, C> (both) or <Om~ M, C> over n x n matrices
hipError_t reduce_wdot(const double *M, const double *C, const double *om, int n, int d, bool both, double *part,
                       double *out, hipStream_t s)
{
    const int np = std::min(n, 1024);
    hipLaunchKernelGGL(wdot_partial_kernel, dim3(np), dim3(256), 0, s, M, C, om, n, d, both ? 1 : 0, part);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, s, part, np, out, OP_SUM, 1.0);
    return hipGetLastError();
}

hipError_t copy2d(const double *src, long lds, double *dst, long ldd, int rows, int cols, hipStream_t s)
{
    hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for((long)rows * cols)), dim3(256), 0, s, src, lds, dst, ldd, rows,
                       cols);
    return hipGetLastError();
}

// U (n x d, row stride ldu) rotated inside each kept multiplet towards Uprev (n x d).
hipError_t align_to(AdjWork &w, double *U, int ldu, const double *lamk, double gap_tol, hipStream_t s)
{
    const int n = w.n, d = w.d;
    hipError_t e = gemm_mfma(GEMM_SMALL, A_T{U, ldu}, B_RM{w.Uprev, d}, EpiStore{w.Mov, d, 1.0}, d, d, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(align_kernel, dim3(d), dim3(64), 0, s, U, ldu, n, w.Mov, d, lamk, gap_tol, w.err);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------- allocation

namespace {

struct AdjReq { double **p; size_t n; };

// The device buffers of the derivative (element counts), for n = q d.
std::vector<AdjReq> adj_requests(AdjWork &w, int q, int d, int restart)
{
    const size_t n = (size_t)q * d, dd = (size_t)d;
    const size_t L = dd * n + dd * dd;
    return {
        {&w.A, dd * n}, {&w.OA, dd * n}, {&w.Pt, dd * n}, {&w.om, n + 8}, {&w.omn, n + 8}, {&w.zero, n + 8},
        {&w.Ucur, n * dd}, {&w.Uprev, n * dd}, {&w.Mov, dd * dd},
        {&w.X, n * n}, {&w.C, n * n}, {&w.Y, n * n}, {&w.Z, n * n}, {&w.Cb, n * n}, {&w.Zb, n * n},
        {&w.Uall, n * n}, {&w.M3, n * n}, {&w.lam, n + 8}, {&w.sel, n + 8},
        {&w.dA, dd * n}, {&w.dAn, dd * n}, {&w.dOA, dd * n}, {&w.dom, dd * dd}, {&w.domn, dd * dd},
        {&w.dX, n * n}, {&w.dC, n * n}, {&w.dY, n * n}, {&w.dZ, n * n}, {&w.dPt, dd * n},
        {&w.T1, n * dd}, {&w.Bm, n * dd}, {&w.R, n * dd}, {&w.dU, n * dd},
        {&w.part, std::max<size_t>(1024, 256 * ((size_t)restart + 2))}, {&w.scal, NSCAL + n + 8},
        {&w.W2, (size_t)q * q * q * q}, {&w.obsv, 4 * (size_t)q + 8},
        {&w.Vk, L * ((size_t)restart + 1)}, {&w.gb, L}, {&w.gx, L}, {&w.gy, L}, {&w.gh, 2 * (size_t)restart + 8},
    };
}

}  // namespace

size_t adj_bytes(int q, int d, int band, int restart)
{
    AdjWork w;
    size_t s = 0;
    for (const AdjReq &r : adj_requests(w, q, d, restart)) s += sizeof(double) * std::max<size_t>(r.n, 1);
    s += sizeof(PostOut) + sizeof(unsigned) * 4;
    return s + eig_bytes(q * d, q * d, band);
}

hipError_t adj_alloc(AdjWork &w, int q, int d, int band, int restart)
{
    w.q = q;
    w.d = d;
    w.n = q * d;
    w.band = band;
    w.restart = restart;
    const size_t n = (size_t)w.n;
    for (auto &r : adj_requests(w, q, d, restart)) {
        hipError_t e = hipMalloc((void **)r.p, sizeof(double) * std::max<size_t>(r.n, 1));
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc((void **)&w.post, sizeof(PostOut));
    if (e == hipSuccess) e = hipHostMalloc((void **)&w.hpost, sizeof(PostOut), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w.hscal, sizeof(double) * NSCAL, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w.hobsv, sizeof(double) * (4 * (size_t)q + 8), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w.hgh, sizeof(double) * (2 * (size_t)restart + 8), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void **)&w.err, sizeof(unsigned) * 4);
    if (e == hipSuccess) e = eig_alloc(w.eig, w.n, w.n, band);
    if (e == hipSuccess) e = hipMemset(w.zero, 0, sizeof(double) * (n + 8));
    return e;
}

void adj_free(AdjWork &w)
{
    double *bufs[] = {w.A, w.OA, w.Pt, w.om, w.omn, w.zero, w.Ucur, w.Uprev, w.Mov, w.X, w.C, w.Y, w.Z, w.Cb,
                      w.Zb, w.Uall, w.M3, w.lam, w.sel, w.dA, w.dAn, w.dOA, w.dom, w.domn, w.dX, w.dC, w.dY, w.dZ,
                      w.dPt, w.T1, w.Bm, w.R, w.dU, w.part, w.scal, w.W2, w.obsv, w.Vk, w.gb, w.gx, w.gy, w.gh};
    for (double *p : bufs)
        if (p) (void)hipFree(p);
    if (w.post) (void)hipFree(w.post);
    if (w.hpost) (void)hipHostFree(w.hpost);
    if (w.hscal) (void)hipHostFree(w.hscal);
    if (w.hobsv) (void)hipHostFree(w.hobsv);
    if (w.hgh) (void)hipHostFree(w.hgh);
    if (w.err) (void)hipFree(w.err);
    eig_free(w.eig);
    const int band = w.band;
    w = AdjWork();
    w.band = band;
}

// ---------------------------------------------------------------- the derivative

int adjoint_dFdK(AdjWork &w, const AdjInputs &in, AdjResult *res, hipStream_t s, std::string *msg)
{
    const int q = in.q, d = in.d, n = q * d;
    // with CTMRG_PROGRESS set in the environment, long solves report their progress on stderr
    const char *pe = getenv("CTMRG_PROGRESS");
    const bool progress = pe && *pe && *pe != '0';
    const int q2 = q * q;
    hipError_t e = hipSuccess;
#define ADJ_CK(expr)                                                          \
    do {                                                                      \
        if ((e = (expr)) != hipSuccess) {                                     \
            *msg = std::string(#expr) + ": " + hipGetErrorString(e);          \
            return e == hipErrorOutOfMemory ? CTMRG_E_OUT_OF_MEMORY : CTMRG_E_HIP; \
        }                                                                     \
    } while (0)
    auto fetch_post = [&]() -> hipError_t {
        hipError_t e2 = hipMemcpyAsync(w.hpost, w.post, sizeof(PostOut), hipMemcpyDeviceToHost, s);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        return e2;
    };
    auto fetch_scal = [&]() -> hipError_t {
        hipError_t e2 = hipMemcpyAsync(w.hscal, w.scal, sizeof(double) * NSCAL, hipMemcpyDeviceToHost, s);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        return e2;
    };
    auto take_err = [&]() -> unsigned {
        unsigned h = 0;
        (void)hipMemcpy(&h, w.err, sizeof(unsigned), hipMemcpyDeviceToHost);
        (void)hipMemset(w.err, 0, sizeof(unsigned));
        return h | eig_take_errors(w.eig);
    };
    if (w.q != q || w.d != d || !w.A || w.restart != in.restart) {
        adj_free(w);
        ADJ_CK(adj_alloc(w, q, d, w.band, in.restart));
    }
    ADJ_CK(hipMemsetAsync(w.err, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(compact_kernel, dim3(grid_for((long)d * n)), dim3(256), 0, s, in.A, in.omega, in.U, q, in.m, d,
                       w.A, w.om, w.Uprev);
    ADJ_CK(hipGetLastError());

    // ---- 1. fixed point in the aligned gauge, P normalized by its Frobenius norm
    double resid = INFINITY;
    int k = 0;
    for (k = 0; k < in.max_aligned_steps; ++k) {
        ADJ_CK(extension_products(w.A, w.om, w.OA, w.X, q, d, s));
        ADJ_CK(weight_mix(in.W, w.X, w.C, q, d, s));
        ADJ_CK(eig_values(w.eig, w.C, n, n, s));
        ADJ_CK(eig_post(w.eig, n, d, in.gap_tol, in.rank_tol, w.zero, w.omn, w.sel, w.post, s));
        ADJ_CK(fetch_post());
        const PostOut po = *w.hpost;
        if (po.m_eff != d) {
            *msg = "the kept dimension changed from " + std::to_string(d) + " to " + std::to_string(po.m_eff) +
                   " while converging the aligned fixed point";
            return CTMRG_E_NUMERICAL;
        }
        ADJ_CK(eig_vectors(w.eig, nullptr, 0, n, d, w.sel, po.nclusters, w.Ucur, d, s));
        ADJ_CK(align_to(w, w.Ucur, d, w.sel, in.gap_tol, s));
        ADJ_CK(halfrow_products(w.A, w.Ucur, w.Y, q, d, s));
        ADJ_CK(weight_mix(in.W, w.Y, w.Z, q, d, s));
        ADJ_CK(projection(w.Ucur, w.Z, w.Pt, q, d, nullptr, 0, s));
        ADJ_CK(reduce_dot(w.Pt, w.Pt, (long)d * n, w.part, w.scal + S_NORM, OP_SQRT, 1.0, s));
        hipLaunchKernelGGL(div_by_kernel, dim3(grid_for((long)d * n)), dim3(256), 0, s, w.Pt, w.dAn, (long)d * n,
                           w.scal + S_NORM);
        ADJ_CK(reduce_maxdiff(w.dAn, w.A, (long)d * n, w.part, w.scal + S_GAUGE, false, s));
        ADJ_CK(hipMemcpyAsync(w.A, w.dAn, sizeof(double) * d * n, hipMemcpyDeviceToDevice, s));
        ADJ_CK(hipMemcpyAsync(w.om, w.omn, sizeof(double) * d, hipMemcpyDeviceToDevice, s));
        ADJ_CK(hipMemcpyAsync(w.Uprev, w.Ucur, sizeof(double) * n * d, hipMemcpyDeviceToDevice, s));
        ADJ_CK(fetch_scal());
        if (unsigned ke = take_err()) {
            *msg = "kernel error " + std::to_string(ke) + " in an aligned step (a multiplet larger than 8, or "
                   "subspaces that do not overlap)";
            return CTMRG_E_NUMERICAL;
        }
        resid = w.hscal[S_GAUGE];
        if (!std::isfinite(resid)) {
            *msg = "non-finite state in an aligned step";
            return CTMRG_E_NUMERICAL;
        }
        if (progress && k % 10 == 9)
            fprintf(stderr, "[ctmrg derivative] aligned step %d: |P_next - P| = %.3e\n", k + 1, resid);
        if (k >= 1 && resid < in.gauge_tol) break;
    }
    res->aligned_steps = k + 1;
    res->gauge_residual = resid;
    if (!(resid < in.gauge_tol)) {
        char buf[128];
        snprintf(buf, sizeof(buf), "the aligned fixed point did not converge (|P_next - P| = %.3e after %d steps)", resid,
                 res->aligned_steps);
        *msg = buf;
        return CTMRG_E_NOT_CONVERGED;
    }

    // ---- 2. at x*: all eigenpairs of C'*, the kept block aligned with the last step
    ADJ_CK(extension_products(w.A, w.om, w.OA, w.X, q, d, s));
    ADJ_CK(weight_mix(in.W, w.X, w.C, q, d, s));
    ADJ_CK(eig_values(w.eig, w.C, n, n, s));
    ADJ_CK(eig_post(w.eig, n, n, in.gap_tol, in.rank_tol, w.zero, w.omn, w.sel, w.post, s));
    ADJ_CK(fetch_post());
    const PostOut pa = *w.hpost;
    const int np = pa.m_eff;  // eigenpairs above the rank threshold, all multiplets whole
    if (np < d) {
        *msg = "the spectrum of C' at the fixed point has fewer than d resolvable eigenpairs";
        return CTMRG_E_NUMERICAL;
    }
    const double nC = pa.n_C;
    ADJ_CK(eig_vectors(w.eig, nullptr, 0, n, np, w.sel, pa.nclusters, w.Uall, n, s));
    ADJ_CK(hipMemcpyAsync(w.lam, w.sel, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
    ADJ_CK(copy2d(w.Uall, n, w.Ucur, d, n, d, s));
    ADJ_CK(align_to(w, w.Ucur, d, w.lam, in.gap_tol, s));
    ADJ_CK(copy2d(w.Ucur, d, w.Uall, n, n, d, s));
    // M3 = U diag(lambda^3) U^T = C'^3 (on the resolved spectrum)
    ADJ_CK(hipMemsetAsync(w.dX, 0, sizeof(double) * (size_t)n * n, s));
    hipLaunchKernelGGL(scale_cols_cube_kernel, dim3(grid_for((long)n * np)), dim3(256), 0, s, w.Uall, (long)n, n, np,
                       w.lam, w.dX);
    ADJ_CK(gemm_mfma(GEMM_LARGE, A_RM{w.dX, n}, B_T{w.Uall, n}, EpiStore{w.M3, n, 1.0}, n, n, np, s));
    // P~*, its norm s*, and the K-derivative parts of C' and Z (dW/dK = -WH)
    ADJ_CK(halfrow_products(w.A, w.Ucur, w.Y, q, d, s));
    ADJ_CK(weight_mix(in.W, w.Y, w.Z, q, d, s));
    ADJ_CK(projection(w.Ucur, w.Z, w.Pt, q, d, nullptr, 0, s));
    ADJ_CK(reduce_dot(w.Pt, w.Pt, (long)d * n, w.part, w.scal + S_NORM, OP_SQRT, 1.0, s));
    ADJ_CK(gemm_mfma(GEMM_MIX, A_T{in.WH, q2}, B_Mix{w.X, q, d, n}, EpiMix_<double, true>{w.Cb, q, d, n, -1.0}, q2,
                     d * d, q2, s));
    ADJ_CK(gemm_mfma(GEMM_MIX, A_T{in.WH, q2}, B_Mix{w.Y, q, d, n}, EpiMix_<double, true>{w.Zb, q, d, n, -1.0}, q2,
                     d * d, q2, s));
    ADJ_CK(fetch_scal());
    if (unsigned ke = take_err()) {
        *msg = "kernel error " + std::to_string(ke) + " at the fixed point";
        return CTMRG_E_NUMERICAL;
    }
    const double sstar = w.hscal[S_NORM];
    res->F = -0.5 * log(sstar);
    res->n_eigen = np;

    // ---- 3. the tangent: (I - J) t = d_K Phi (dK = 1), by restarted GMRES
    const long nd = (long)d * n;
    const long L = nd + (long)d * d;  // a tangent vector: dA (d x n), then dOm (d x d)
#define TF_CK(expr)                          \
    do {                                     \
        hipError_t e3 = (expr);              \
        if (e3 != hipSuccess) return e3;     \
    } while (0)
    // The front of one tangent step from (tA, tOm): dX, dC', the eigen part (the next state's
    // corner tangent into oOm, and dU).  with_b adds the K-derivative of the weights (d_K Phi).
    auto tangent_front = [&](const double *tA, const double *tOm, double *oOm, bool with_b) -> hipError_t {
        // dOA = dOmega A + Omega dA (dOmega: the full symmetric corner tangent)
        hipLaunchKernelGGL(scale_rows_kernel, dim3(grid_for(nd)), dim3(256), 0, s, w.om, tA, d, (long)n, w.dOA);
        TF_CK(gemm_mfma(GEMM_SMALL, A_RM{tOm, d}, B_RM{w.A, n}, EpiAxpby{w.dOA, n, 1.0, 1.0}, d, n, d, s));
        // dX = dA^T (Omega A) + A^T (dOmega A + Omega dA)
        TF_CK(gemm_mfma(GEMM_LARGE, A_T{tA, n}, B_RM{w.OA, n}, EpiStore{w.dX, n, 1.0}, n, n, d, s));
        TF_CK(gemm_mfma(GEMM_LARGE, A_T{w.A, n}, B_RM{w.dOA, n}, EpiAxpby{w.dX, n, 1.0, 1.0}, n, n, d, s));
        // dC' = W-mix(dX) (+ W'-mix(X*))
        TF_CK(weight_mix(in.W, w.dX, w.dC, q, d, s));
        if (with_b)
            hipLaunchKernelGGL(axpy_kernel, dim3(grid_for((long)n * n)), dim3(256), 0, s, w.dC, w.Cb, (long)n * n);
        // eigenvector and eigenvalue derivatives
        TF_CK(gemm_mfma(GEMM_TALL, A_RM{w.dC, n}, B_RM{w.Ucur, d}, EpiStore{w.T1, d, 1.0}, n, d, n, s));
        TF_CK(gemm_mfma(GEMM_TALL, A_T{w.Uall, n}, B_RM{w.T1, d}, EpiStore{w.Bm, d, 1.0}, np, d, n, s));
        if (np < n) {
            TF_CK(copy2d(w.T1, d, w.R, d, n, d, s));
            TF_CK(gemm_mfma(GEMM_TALL, A_RM{w.Uall, n}, B_RM{w.Bm, d}, EpiAxpby{w.R, d, -1.0, 1.0}, n, d, np, s));
        }
        TF_CK(reduce_dot(w.M3, w.dC, (long)n * n, w.part, w.scal + S_DNC, OP_SUM, 1.0 / (nC * nC * nC), s));
        hipLaunchKernelGGL(eigen_tangent_kernel, dim3(grid_for((long)np * d)), dim3(256), 0, s, w.Bm, np, d, w.lam,
                           nC, w.scal + S_DNC, oOm);
        TF_CK(gemm_mfma(GEMM_TALL, A_RM{w.Uall, n}, B_RM{w.Bm, d}, EpiStore{w.dU, d, 1.0}, n, d, np, s));
        if (np < n)
            hipLaunchKernelGGL(nullspace_tangent_kernel, dim3(grid_for((long)n * d)), dim3(256), 0, s, w.dU, w.R,
                               (long)n, d, w.lam);
        return hipSuccess;
    };
    // One tangent step y = J x (+ d_K Phi with with_b); x and y are tangent vectors of length L.
    auto step_t = [&](const double *x, double *y, bool with_b) -> hipError_t {
        const double *tA = x, *tOm = x + nd;
        TF_CK(tangent_front(tA, tOm, y + nd, with_b));
        // dY = dA^T U + A^T dU,  dZ = W-mix(dY) (+ W'-mix(Y*)),  dP~ = dU^T Z* + U^T dZ
        TF_CK(gemm_mfma(GEMM_LARGE, A_T{tA, n}, B_Ublk{w.Ucur, d}, EpiStore{w.dY, n, 1.0}, n, n, d, s));
        TF_CK(gemm_mfma(GEMM_LARGE, A_T{w.A, n}, B_Ublk{w.dU, d}, EpiAxpby{w.dY, n, 1.0, 1.0}, n, n, d, s));
        TF_CK(weight_mix(in.W, w.dY, w.dZ, q, d, s));
        if (with_b)
            hipLaunchKernelGGL(axpy_kernel, dim3(grid_for((long)n * n)), dim3(256), 0, s, w.dZ, w.Zb, (long)n * n);
        TF_CK(gemm_mfma(GEMM_LARGE, A_T{w.dU, d}, B_RM{w.Z, n}, EpiStore{w.dPt, n, 1.0}, d, n, n, s));
        TF_CK(gemm_mfma(GEMM_LARGE, A_T{w.Ucur, d}, B_RM{w.dZ, n}, EpiAxpby{w.dPt, n, 1.0, 1.0}, d, n, n, s));
        // normalization by the Frobenius norm (ds into S_DS)
        TF_CK(reduce_dot(w.Pt, w.dPt, nd, w.part, w.scal + S_DS, OP_SUM, 1.0 / sstar, s));
        hipLaunchKernelGGL(tangent_norm_kernel, dim3(grid_for(nd)), dim3(256), 0, s, w.dPt, w.Pt, nd,
                           w.scal + S_NORM, w.scal + S_DS, y);
        return hipGetLastError();
    };
    const int R = std::max(1, in.restart);
    const int ndot = grid_for(L) < 256 ? grid_for(L) : 256;
    // h[0 .. nv) = V[0 .. nv)^T x on the device, and on the host when `fetch`
    auto project = [&](int nv, const double *x, double *h) -> hipError_t {
        hipLaunchKernelGGL(multi_dot_partial_kernel, dim3(ndot), dim3(256), 0, s, w.Vk, L, nv, x, w.part);
        hipLaunchKernelGGL(multi_dot_finalize_kernel, dim3((nv + 63) / 64), dim3(64), 0, s, w.part, ndot, nv, h);
        return hipGetLastError();
    };
    auto norm2 = [&](const double *x) -> double {
        if (reduce_dot(x, x, L, w.part, w.gh + 2 * R + 6, OP_SQRT, 1.0, s) != hipSuccess) return NAN;
        if (hipMemcpyAsync(w.hgh + 2 * R + 6, w.gh + 2 * R + 6, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return NAN;
        return w.hgh[2 * R + 6];
    };
    // b = d_K Phi: the step with the K-derivative applied to t = 0
    ADJ_CK(hipMemsetAsync(w.gx, 0, sizeof(double) * L, s));
    ADJ_CK(step_t(w.gx, w.gb, true));
    const double bnorm = norm2(w.gb);
    if (!std::isfinite(bnorm) || !(bnorm > 0.0)) {
        *msg = "non-finite or zero right-hand side of the tangent";
        return CTMRG_E_NUMERICAL;
    }
    std::vector<double> H((size_t)(R + 1) * R, 0.0), cs(R), sn(R), g(R + 1), yv(R);
    double gres = bnorm, true_prev = INFINITY;
    int it = 0;
    bool converged = false;
    while (!converged && it <= in.max_iterations) {
        // r = b - (x - J x), the first Krylov vector
        if (it == 0) {
            ADJ_CK(hipMemcpyAsync(w.Vk, w.gb, sizeof(double) * L, hipMemcpyDeviceToDevice, s));
        } else {
            ADJ_CK(step_t(w.gx, w.gy, false));
            hipLaunchKernelGGL(amb_kernel, dim3(grid_for(L)), dim3(256), 0, s, w.gb, w.gx, w.gy, w.Vk, L);
        }
        const double beta = norm2(w.Vk);
        if (!std::isfinite(beta)) {
            *msg = "non-finite tangent residual";
            return CTMRG_E_NUMERICAL;
        }
        gres = beta;
        // converged, or a restart that no longer reduces the true residual once it is within 1e-10
        // of the right-hand side (the attainable accuracy of the FP64 products)
        if (beta <= in.tangent_tol * bnorm || (beta <= 1e-10 * bnorm && beta > 0.5 * true_prev)) {
            converged = true;
            break;
        }
        true_prev = beta;
        if (it >= in.max_iterations) break;
        hipLaunchKernelGGL(scal_kernel, dim3(grid_for(L)), dim3(256), 0, s, w.Vk, L, 1.0 / beta);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jn = 0;
        for (int j = 0; j < R && it < in.max_iterations; ++j) {
            double *vj = w.Vk + (long)j * L, *vn = w.Vk + (long)(j + 1) * L;
            // vn = (I - J) vj, orthogonalized twice against v_0 .. v_j (classical Gram-Schmidt)
            ADJ_CK(step_t(vj, w.gy, false));
            hipLaunchKernelGGL(amb_kernel, dim3(grid_for(L)), dim3(256), 0, s, vj, w.gy, (const double *)nullptr, vn, L);
            for (int pass = 0; pass < 2; ++pass) {
                ADJ_CK(project(j + 1, vn, w.gh + pass * (R + 2)));
                hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(L)), dim3(256), 0, s, w.Vk, L, j + 1,
                                   w.gh + pass * (R + 2), -1.0, vn);
            }
            ADJ_CK(hipMemcpyAsync(w.hgh, w.gh, sizeof(double) * 2 * (R + 2), hipMemcpyDeviceToHost, s));
            const double hn = norm2(vn);  // synchronizes the stream
            if (!std::isfinite(hn)) {
                *msg = "non-finite Krylov vector in the tangent solve";
                return CTMRG_E_NUMERICAL;
            }
            ++it;
            double *hc = H.data() + (size_t)j * (R + 1);  // column j of the Hessenberg matrix
            for (int i = 0; i <= j; ++i) hc[i] = w.hgh[i] + w.hgh[R + 2 + i];
            hc[j + 1] = hn;
            // the previous rotations, then a new one that annihilates hc[j + 1]
            for (int i = 0; i < j; ++i) {
                const double a = hc[i], b2 = hc[i + 1];
                hc[i] = cs[i] * a + sn[i] * b2;
                hc[i + 1] = -sn[i] * a + cs[i] * b2;
            }
            const double rr = std::hypot(hc[j], hc[j + 1]);
            cs[j] = rr > 0.0 ? hc[j] / rr : 1.0;
            sn[j] = rr > 0.0 ? hc[j + 1] / rr : 0.0;
            hc[j] = rr;
            hc[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            gres = fabs(g[j + 1]);
            jn = j + 1;
            if (progress && it % 20 == 0)
                fprintf(stderr, "[ctmrg derivative] GMRES product %d: relative residual %.3e\n", it, gres / bnorm);
            if (gres <= in.tangent_tol * bnorm || hn <= 1e-300) break;
            hipLaunchKernelGGL(scal_kernel, dim3(grid_for(L)), dim3(256), 0, s, vn, L, 1.0 / hn);
        }
        // x += V y with H y = g (upper triangular, jn x jn)
        for (int i = jn - 1; i >= 0; --i) {
            double acc = g[i];
            for (int c = i + 1; c < jn; ++c) acc -= H[(size_t)c * (R + 1) + i] * yv[c];
            yv[i] = acc / H[(size_t)i * (R + 1) + i];
        }
        ADJ_CK(hipMemcpyAsync(w.gh, yv.data(), sizeof(double) * jn, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(L)), dim3(256), 0, s, w.Vk, L, jn, w.gh, 1.0, w.gx);
        ADJ_CK(hipStreamSynchronize(s));
        // the next pass through the loop measures the true residual of the updated solution
    }
    // the true residual and dF/dK from one more step t -> J t + d_K Phi of the solution
    ADJ_CK(step_t(w.gx, w.gy, true));
    ADJ_CK(reduce_maxdiff(w.gy, w.gx, L, w.part, w.scal + S_CHANGE, false, s));
    ADJ_CK(fetch_scal());
    const double change = w.hscal[S_CHANGE], ds = w.hscal[S_DS];
    res->iterations = it;
    res->tangent_change = change;
    res->dFdK = -0.5 * ds / sstar;
    if (!std::isfinite(change) || !std::isfinite(ds)) {
        *msg = "non-finite tangent";
        return CTMRG_E_NUMERICAL;
    }
    if (!converged) {
        char buf[160];
        snprintf(buf, sizeof(buf), "the tangent solve did not converge (relative residual %.3e after %d products)",
                 gres / bnorm, it);
        *msg = buf;
        return CTMRG_E_NOT_CONVERGED;
    }
    // the state tangent for the observables below
    ADJ_CK(hipMemcpyAsync(w.dA, w.gx, sizeof(double) * nd, hipMemcpyDeviceToDevice, s));
    ADJ_CK(hipMemcpyAsync(w.dom, w.gx + nd, sizeof(double) * d * d, hipMemcpyDeviceToDevice, s));

    // ---- 4. E and M at x* and their derivatives along the converged tangent (dK = 1)
    ADJ_CK(tangent_front(w.dA, w.dom, w.domn, true));  // dX, dC', domn and dU of the final (dA, dOm)
    // C' (into Z, free now), Om~ X dOm~ (as X reshaped to (q n) x d times dOm, into dY),
    // (W h4^2)-mix(X) (into dZ) and (W h4)-mix(dX) (into Zb)
    ADJ_CK(weight_mix(in.W, w.X, w.Z, q, d, s));
    ADJ_CK(gemm_mfma(GEMM_TALL, A_RM{w.X, d}, B_RM{w.dom, d}, EpiStore{w.dY, d, 1.0}, n * q, d, d, s));
    hipLaunchKernelGGL(weight_h2_kernel, dim3(grid_for((long)q2 * q2)), dim3(256), 0, s, in.W, in.WH, w.W2,
                       (long)q2 * q2);
    ADJ_CK(hipGetLastError());
    ADJ_CK(weight_mix(w.W2, w.X, w.dZ, q, d, s));
    ADJ_CK(weight_mix(in.WH, w.dX, w.Zb, q, d, s));
    // slots: 6 <G,C'>  7 <G,Cb>  8 <Om~X dOm~,C'>  9 <Om~ dX Om~,C'>  10 <G,dC'>
    //        11 <Om~X dOm~,Cb>  12 <Om~ dX Om~,Cb>  13 <G,(W h4)-mix(dX)>  14 <G,(W h4^2)-mix(X)>
    // (Cb = -(W h4)-mix(X))
    double *sc = w.scal + S_OBS;
    ADJ_CK(reduce_wdot(w.X, w.Z, w.om, n, d, true, w.part, sc + 0, s));
    ADJ_CK(reduce_wdot(w.X, w.Cb, w.om, n, d, true, w.part, sc + 1, s));
    ADJ_CK(reduce_wdot(w.dY, w.Z, w.om, n, d, false, w.part, sc + 2, s));
    ADJ_CK(reduce_wdot(w.dX, w.Z, w.om, n, d, true, w.part, sc + 3, s));
    ADJ_CK(reduce_wdot(w.X, w.dC, w.om, n, d, true, w.part, sc + 4, s));
    ADJ_CK(reduce_wdot(w.dY, w.Cb, w.om, n, d, false, w.part, sc + 5, s));
    ADJ_CK(reduce_wdot(w.dX, w.Cb, w.om, n, d, true, w.part, sc + 6, s));
    ADJ_CK(reduce_wdot(w.X, w.Zb, w.om, n, d, true, w.part, sc + 7, s));
    ADJ_CK(reduce_wdot(w.X, w.dZ, w.om, n, d, true, w.part, sc + 8, s));
    // M: prob_s and d prob_s from U*, dU and d(Omega^4) (the next state's corner tangent domn)
    hipLaunchKernelGGL(omega4_tangent_kernel, dim3(grid_for((long)d * d)), dim3(256), 0, s, w.domn, w.om, d, w.Bm);
    ADJ_CK(hipGetLastError());
    ADJ_CK(gemm_mfma(GEMM_TALL, A_RM{w.Ucur, d}, B_RM{w.Bm, d}, EpiStore{w.T1, d, 1.0}, n, d, d, s));
    hipLaunchKernelGGL(spin_tangent_kernel, dim3(q), dim3(256), 0, s, w.Ucur, w.dU, w.T1, w.om, q, d, w.obsv);
    ADJ_CK(hipGetLastError());
    ADJ_CK(hipMemcpyAsync(w.hobsv, w.obsv, sizeof(double) * 2 * q, hipMemcpyDeviceToHost, s));
    ADJ_CK(fetch_scal());
    {
        const double *h = w.hscal + S_OBS;
        const double Zd = h[0], ZH = -h[1];
        const double dZd = 2.0 * h[2] + h[3] + h[4];
        const double dZH = -2.0 * h[5] - h[6] + h[7] - h[8];
        res->E = 0.5 * ZH / Zd;
        res->dEdK = 0.5 * (dZH / Zd - ZH * dZd / (Zd * Zd));
        const double *prob = w.hobsv, *dprob = w.hobsv + q;
        double ps = 0.0, dps = 0.0, mn = 0.0, dmn = 0.0, v[3] = {0, 0, 0}, dv[3] = {0, 0, 0};
        std::vector<double> hv((size_t)q * std::max(in.dim, 1), 0.0);
        if (in.V && in.dim > 0) ADJ_CK(hipMemcpy(hv.data(), in.V, sizeof(double) * q * in.dim, hipMemcpyDeviceToHost));
        for (int sp = 0; sp < q; ++sp) {
            ps += prob[sp];
            dps += dprob[sp];
            double dot = 0.0;
            for (int x = 0; x < in.dim; ++x) dot += hv[(size_t)in.s0 * in.dim + x] * hv[(size_t)sp * in.dim + x];
            mn += prob[sp] * dot;
            dmn += dprob[sp] * dot;
            for (int x = 0; x < std::min(in.dim, 3); ++x) {
                v[x] += prob[sp] * hv[(size_t)sp * in.dim + x];
                dv[x] += dprob[sp] * hv[(size_t)sp * in.dim + x];
            }
        }
        if (in.bc == 0) {
            res->M = mn / ps;
            res->dMdK = (dmn * ps - mn * dps) / (ps * ps);
        } else {
            const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            const double dnv = nv > 0.0 ? (v[0] * dv[0] + v[1] * dv[1] + v[2] * dv[2]) / nv : 0.0;
            res->M = nv / ps;
            res->dMdK = (dnv * ps - nv * dps) / (ps * ps);
        }
        if (!std::isfinite(res->dEdK) || !std::isfinite(res->dMdK)) {
            *msg = "non-finite derivative of E or M";
            return CTMRG_E_NUMERICAL;
        }
    }
    return CTMRG_OK;
#undef TF_CK
#undef ADJ_CK
}

}  // namespace ctm
