// Effective correlation length from the row-to-row transfer matrix; see xi.h.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "gemm.h"
#include "xi.h"

namespace ctm {

namespace {

constexpr int XCH = 1024;  // vector elements per dot-product chunk (4 per thread)
constexpr int XRG = 8;     // Lanczos vectors per dot-product block

int grid_for(long n) { return (int)std::max<long>(1, std::min<long>(1024, (n + 255) / 256)); }

// Y (N x m, rows s m + i) read as the m x N left operand of sum_s Y_s P_s:
// A(i, s m + b) = Y[(s m + i) m + b] = (P_s X)[i][b].
struct A_Yblk {
    using value_type = double;
    const double *p;
    int m;
    static constexpr bool kContigK = true;
    __device__ double operator()(int i, int k) const
    {
        const int s = k / m, b = k - s * m;
        return p[((long)s * m + i) * m + b];
    }
};
// P as the N x m right operand: B(s m + b, j) = P_s[b][j] = A[b][s m + j].
struct B_Pblk {
    using value_type = double;
    const double *p;
    int m;
    long N;
    static constexpr bool kContigK = false;
    __device__ double operator()(int k, int j) const
    {
        const int s = k / m, b = k - s * m;
        return p[(long)b * N + (long)s * m + j];
    }
};

int second_splits(int m, int N)
{
    const long tiles = (long)ceil_div(m, 64) * ceil_div(m, 64);
    int sp = 1;
    while (tiles * sp < 768 && N / (2 * sp) >= 256) sp *= 2;
    return sp;
}

// splitmix64 (Steele, Lea and Flood): a counter-based generator, here of the start vector.
__device__ inline uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void start_vector_kernel(double *v, long n)
{
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        v[t] = 2.0 * ((double)(splitmix64((uint64_t)t) >> 11) * 0x1.0p-53) - 1.0;
}

__global__ void zero_kernel(double *x, long n)
{
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) x[t] = 0.0;
}

__global__ void __launch_bounds__(256) sumsq_kernel(const double *x, long n, double *part)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        acc += x[i] * x[i];
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// *out = sqrt(sum of part[0..np))
__global__ void norm_finalize_kernel(const double *part, int np, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += part[i];
    *out = sqrt(s);
}

// dst = src / *nrm (zero if the norm is zero)
__global__ void scale_by_norm_kernel(double *dst, const double *src, long n, const double *nrm)
{
    const double r = *nrm;
    const double inv = r > 0.0 ? 1.0 / r : 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        dst[t] = src[t] * inv;
}

// part[c * ld + i] = sum over chunk c of V[i][t] w[t], for rows i of the block's group
__global__ void __launch_bounds__(256) dots_kernel(const double *V, long n, int rows, const double *w, double *part,
                                                   int ld)
{
    __shared__ double red[4][XRG];
    const int c = blockIdx.x, r0 = blockIdx.y * XRG;
    const long t0 = (long)c * XCH;
    double wv[XCH / 256];
#pragma unroll
    for (int u = 0; u < XCH / 256; ++u) {
        const long t = t0 + threadIdx.x + u * 256;
        wv[u] = t < n ? w[t] : 0.0;
    }
    double acc[XRG];
#pragma unroll
    for (int r = 0; r < XRG; ++r) {
        acc[r] = 0.0;
        const int i = r0 + r;
        if (i < rows) {
#pragma unroll
            for (int u = 0; u < XCH / 256; ++u) {
                const long t = t0 + threadIdx.x + u * 256;
                if (t < n) acc[r] += V[(long)i * n + t] * wv[u];
            }
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < XRG; ++r) {
        const double v = wave_sum(acc[r]);
        if (lane == 0) red[wave][r] = v;
    }
    __syncthreads();
    if (threadIdx.x < XRG && r0 + (int)threadIdx.x < rows) {
        const int r = threadIdx.x;
        part[(long)c * ld + r0 + r] = red[0][r] + red[1][r] + red[2][r] + red[3][r];
    }
}

// h[i] = sum_c part[c * ld + i], chunks in order
__global__ void dots_reduce_kernel(const double *part, int chunks, int rows, int ld, double *h)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[(long)c * ld + i];
    h[i] = s;
}

// w[t] += sign * sum_i V[i][t] h[i]
__global__ void __launch_bounds__(256) combine_kernel(const double *V, long n, int rows, const double *h, double sign,
                                                      double *w)
{
    __shared__ double hs[512];
    for (int i = threadIdx.x; i < rows; i += 256) hs[i] = h[i];
    __syncthreads();
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < rows; ++i) s += V[(long)i * n + t] * hs[i];
        w[t] += sign * s;
    }
}

// alpha_j = h1[j] + h2[j]
__global__ void set_alpha_kernel(const double *h1, const double *h2, int j, double *alpha)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) alpha[j] = h1[j] + h2[j];
}

// part of ||z - theta y||^2 (theta = tri[idx])
__global__ void __launch_bounds__(256) resid_sumsq_kernel(const double *z, const double *y, const double *tri, int idx,
                                                          long n, double *part)
{
    __shared__ double red[4];
    const double th = tri[idx];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double r = z[i] - th * y[i];
        acc += r * r;
    }
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Sturm count of the tridiagonal (alpha, beta) of order k: eigenvalues below x.
__device__ int sturm_count(const double *alpha, const double *beta, int k, double x, double pivmin)
{
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
        const double b2 = (i > 0) ? beta[i - 1] * beta[i - 1] : 0.0;
        q = alpha[i] - x - ((i > 0) ? b2 / q : 0.0);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0) ? 1 : 0;
    }
    return cnt;
}

// The small Lanczos problem (one workgroup of 64): the tridiagonal T_k (alpha[0..k),
// beta[0..k-1)); its two eigenvalues of largest modulus theta[0..1] (descending |.|),
// their eigenvectors s (inverse iteration) and the residual estimates |beta[k-1] s_{k-1}|.
// out: theta[2], est[2], s_0[ld], s_1[ld].  ws: 2 x 6 x ld scratch.
__global__ void __launch_bounds__(64) small_tridiag_kernel(const double *alpha, const double *beta, int k, int ld,
                                                           double *out, double *ws)
{
    const double beta_k = beta[k - 1];  // the norm of the next Lanczos direction
    __shared__ double vals[4];
    __shared__ int nv;
    __shared__ double sel[2];
    const int t = threadIdx.x;
    double gl = 0.0, gu = 0.0, bmax2 = 0.0;
    for (int i = 0; i < k; ++i) {
        const double bl = (i > 0) ? fabs(beta[i - 1]) : 0.0, br = (i + 1 < k) ? fabs(beta[i]) : 0.0;
        gl = (i == 0) ? alpha[i] - bl - br : fmin(gl, alpha[i] - bl - br);
        gu = (i == 0) ? alpha[i] + bl + br : fmax(gu, alpha[i] + bl + br);
        bmax2 = fmax(bmax2, br * br);
    }
    const double pivmin = 1e-290 * fmax(1.0, bmax2);
    const double span = fmax(fabs(gl), fabs(gu));
    gl -= 2e-15 * span + pivmin;
    gu += 2e-15 * span + pivmin;
    // ascending indices of the two smallest and the two largest (distinct when k >= 4)
    int idx[4], cntv = 0;
    {
        const int cand[4] = {0, 1, k - 2, k - 1};
        for (int c = 0; c < 4; ++c) {
            const int v = cand[c];
            if (v < 0 || v >= k) continue;
            bool dup = false;
            for (int d = 0; d < cntv; ++d) dup = dup || (idx[d] == v);
            if (!dup) idx[cntv++] = v;
        }
    }
    if (t < cntv) {
        double lo = gl, hi = gu;
        for (int it = 0; it < 256; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (hi - lo <= 2.2e-16 * fmax(fabs(lo), fabs(hi)) + pivmin || mid == lo || mid == hi) break;
            if (sturm_count(alpha, beta, k, mid, pivmin) > idx[t]) hi = mid;
            else lo = mid;
        }
        vals[t] = 0.5 * (lo + hi);
    }
    if (t == 0) nv = cntv;
    __syncthreads();
    if (t == 0) {
        // the two of largest modulus, ties by value descending
        int b0 = 0;
        for (int c = 1; c < nv; ++c)
            if (fabs(vals[c]) > fabs(vals[b0]) || (fabs(vals[c]) == fabs(vals[b0]) && vals[c] > vals[b0])) b0 = c;
        int b1 = -1;
        for (int c = 0; c < nv; ++c) {
            if (c == b0) continue;
            if (b1 < 0 || fabs(vals[c]) > fabs(vals[b1]) || (fabs(vals[c]) == fabs(vals[b1]) && vals[c] > vals[b1]))
                b1 = c;
        }
        sel[0] = vals[b0];
        sel[1] = (b1 >= 0) ? vals[b1] : 0.0;
        out[0] = sel[0];
        out[1] = sel[1];
        if (b1 < 0) out[3] = 0.0;
    }
    __syncthreads();
    if (t < 2 && (t == 0 || nv > 1)) {
        // inverse iteration on T_k - theta I: LU with partial pivoting (rows i, i+1), three solves
        const double th = sel[t];
        double *dl = ws + (long)t * 6 * ld, *d = dl + ld, *du = d + ld, *du2 = du + ld, *x = du2 + ld, *pv = x + ld;
        const double tiny = 1e-15 * fmax(span, 1e-300);
        for (int i = 0; i < k; ++i) {
            d[i] = alpha[i] - th;
            if (i + 1 < k) { dl[i] = beta[i]; du[i] = beta[i]; }
            du2[i] = 0.0;
            pv[i] = 0.0;
        }
        for (int i = 0; i + 1 < k; ++i) {
            if (fabs(d[i]) >= fabs(dl[i])) {
                if (d[i] == 0.0) d[i] = tiny;
                const double l = dl[i] / d[i];
                dl[i] = l;
                d[i + 1] -= l * du[i];
            } else {
                const double l = d[i] / dl[i];
                d[i] = dl[i];
                dl[i] = l;
                const double tmp = du[i];
                du[i] = d[i + 1];
                d[i + 1] = tmp - l * d[i + 1];
                if (i + 2 < k) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -l * du[i + 1];
                }
                pv[i] = 1.0;
            }
        }
        if (d[k - 1] == 0.0) d[k - 1] = tiny;
        for (int i = 0; i < k; ++i) x[i] = 1.0 / sqrt((double)k) * ((i & 1) ? -1.0 : 1.0) + 0.5 / k;
        for (int rep = 0; rep < 3; ++rep) {
            for (int i = 0; i + 1 < k; ++i) {
                if (pv[i] == 0.0) {
                    x[i + 1] -= dl[i] * x[i];
                } else {
                    const double tmp = x[i];
                    x[i] = x[i + 1];
                    x[i + 1] = tmp - dl[i] * x[i];
                }
            }
            x[k - 1] /= d[k - 1];
            if (k >= 2) x[k - 2] = (x[k - 2] - du[k - 2] * x[k - 1]) / d[k - 2];
            for (int i = k - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / d[i];
            double nn = 0.0, mx = 0.0;
            for (int i = 0; i < k; ++i) mx = fmax(mx, fabs(x[i]));
            for (int i = 0; i < k; ++i) nn += (x[i] / mx) * (x[i] / mx);
            const double sc = 1.0 / (mx * sqrt(nn));
            for (int i = 0; i < k; ++i) x[i] *= sc;
        }
        double *s = out + 4 + (long)t * ld;
        for (int i = 0; i < k; ++i) s[i] = x[i];
        for (int i = k; i < ld; ++i) s[i] = 0.0;
        out[2 + t] = fabs(beta_k * x[k - 1]);
    }
}

}  // namespace

size_t xi_bytes(int q, int m, int jmax)
{
    const long n = (long)m * m, N = (long)q * m;
    const long chunks = (n + XCH - 1) / XCH;
    const size_t sp = (size_t)second_splits(m, (int)N);
    size_t d = (size_t)(jmax + 1) * n + (size_t)N * m + 3 * (size_t)n + sp * n + (size_t)chunks * (jmax + 2) +
               2 * (size_t)(jmax + 2) + 2 * (size_t)(jmax + 1) + 4 + 2 * (size_t)(jmax + 1) + 12 * (size_t)(jmax + 1) +
               1024 + 8;
    return sizeof(double) * d + 64;
}

hipError_t xi_alloc(XiWork &w, int q, int m, int jmax)
{
    if (jmax < 1 || jmax + 1 > 512) return hipErrorInvalidValue;  // combine_kernel holds <= 512 coefficients
    w.m = m;
    w.N = q * m;
    w.n = (long)m * m;
    w.jmax = jmax;
    const long chunks = (w.n + XCH - 1) / XCH;
    w.part_elems = (size_t)second_splits(m, w.N) * w.n;
    struct Req { double **p; size_t n; };
    Req reqs[] = {
        {&w.V, (size_t)(jmax + 1) * w.n}, {&w.Y, (size_t)w.N * m}, {&w.w, (size_t)w.n}, {&w.yv, 2 * (size_t)w.n},
        {&w.part, w.part_elems}, {&w.dots, (size_t)chunks * (jmax + 2) + 1024}, {&w.h, 2 * (size_t)(jmax + 2)},
        {&w.ab, 2 * (size_t)(jmax + 1)}, {&w.tri, 4 + 2 * (size_t)(jmax + 1)}, {&w.tws, 12 * (size_t)(jmax + 1)},
        {&w.nrm, 8},
    };
    for (auto &r : reqs) {
        hipError_t e = hipMalloc((void **)r.p, sizeof(double) * std::max<size_t>(r.n, 1));
        if (e != hipSuccess) return e;
    }
    return hipHostMalloc((void **)&w.h_out, sizeof(double) * 16, hipHostMallocDefault);
}

void xi_free(XiWork &w)
{
    double *bufs[] = {w.V, w.Y, w.w, w.yv, w.part, w.dots, w.h, w.ab, w.tri, w.tws, w.nrm};
    for (double *p : bufs)
        if (p) (void)hipFree(p);
    if (w.h_out) (void)hipHostFree(w.h_out);
    w = XiWork();
}

namespace {

// dst (m x m) = sum_s P_s X P_s for X = src (m x m)
hipError_t apply_T(XiWork &w, const double *A, int m, const double *src, double *dst, hipStream_t s)
{
    const int N = w.N;
    const long t128 = (long)ceil_div(N, 128) * ceil_div(m, 128);
    hipError_t e = gemm_mfma(t128 >= 512 ? GEMM_LARGE : GEMM_SMALL, A_T{A, N}, B_RM{src, m}, EpiStore{w.Y, m, 1.0}, N, m,
                             m, s);
    if (e != hipSuccess) return e;
    const int sp = second_splits(m, N);
    return gemm_mfma_splitk(A_Yblk{w.Y, m}, B_Pblk{A, m, (long)N}, EpiStore{dst, m, 1.0}, m, m, N, sp, w.part, s,
                            GEMM_SMALL);
}

// w -= V[0..rows) (V[0..rows)^T w), h = the projections
hipError_t project_out(XiWork &w, int rows, double *h, hipStream_t s)
{
    const int chunks = (int)((w.n + XCH - 1) / XCH);
    const int ld = w.jmax + 2;
    hipLaunchKernelGGL(dots_kernel, dim3(chunks, ceil_div(rows, XRG)), dim3(256), 0, s, w.V, w.n, rows, w.w, w.dots,
                       ld);
    hipLaunchKernelGGL(dots_reduce_kernel, dim3(ceil_div(rows, 256)), dim3(256), 0, s, w.dots, chunks, rows, ld, h);
    hipLaunchKernelGGL(combine_kernel, dim3(grid_for(w.n)), dim3(256), 0, s, w.V, w.n, rows, h, -1.0, w.w);
    return hipGetLastError();
}

hipError_t norm_into(XiWork &w, const double *x, long n, double *out, hipStream_t s)
{
    const int np = grid_for(n);
    hipLaunchKernelGGL(sumsq_kernel, dim3(np), dim3(256), 0, s, x, n, w.dots);
    hipLaunchKernelGGL(norm_finalize_kernel, dim3(1), dim3(64), 0, s, w.dots, np, out);
    return hipGetLastError();
}

}  // namespace

hipError_t xi_solve(XiWork &w, const double *A, int q, int m, double tol, hipStream_t s, XiResult *out)
{
    *out = XiResult();
    if (m != w.m || q * m != w.N) return hipErrorInvalidValue;
    const long n = w.n;
    const int jmax = (int)std::min<long>(w.jmax, n);
    const int ld = w.jmax + 1;
    double *alpha = w.ab, *beta = w.ab + ld;
    hipError_t e;
    // v_0: pseudo-random, normalized
    hipLaunchKernelGGL(start_vector_kernel, dim3(grid_for(n)), dim3(256), 0, s, w.w, n);
    if ((e = norm_into(w, w.w, n, w.nrm, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(scale_by_norm_kernel, dim3(grid_for(n)), dim3(256), 0, s, w.V, w.w, n, w.nrm);
    int k = 0;
    bool conv = false;
    for (int j = 0; j < jmax; ++j) {
        const double *vj = w.V + (long)j * n;
        if ((e = apply_T(w, A, m, vj, w.w, s)) != hipSuccess) return e;
        // full reorthogonalization against v_0..v_j (twice); alpha_j from both passes
        if ((e = project_out(w, j + 1, w.h, s)) != hipSuccess) return e;
        if ((e = project_out(w, j + 1, w.h + (jmax + 2), s)) != hipSuccess) return e;
        hipLaunchKernelGGL(set_alpha_kernel, dim3(1), dim3(64), 0, s, w.h, w.h + (jmax + 2), j, alpha);
        if ((e = norm_into(w, w.w, n, beta + j, s)) != hipSuccess) return e;
        if (j + 1 < ld)
            hipLaunchKernelGGL(scale_by_norm_kernel, dim3(grid_for(n)), dim3(256), 0, s, w.V + (long)(j + 1) * n, w.w,
                               n, beta + j);
        k = j + 1;
        const bool check = (k % 8 == 0) || k == jmax;
        if (!check) continue;
        hipLaunchKernelGGL(small_tridiag_kernel, dim3(1), dim3(64), 0, s, alpha, beta, k, ld, w.tri, w.tws);
        if ((e = hipMemcpyAsync(w.h_out, w.tri, sizeof(double) * 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(w.h_out + 6, beta + j, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        const double bk = w.h_out[6];
        const double t1 = fabs(w.h_out[0]);
        if (!(t1 > 0.0) || !std::isfinite(t1)) break;
        if ((w.h_out[2] <= tol * t1 && w.h_out[3] <= tol * t1) || bk <= 1e-15 * t1) {
            conv = true;
            break;
        }
    }
    if (k == 0) return hipErrorInvalidValue;
    // Ritz vectors y_i = sum_t s_i[t] v_t and their residuals ||T y - theta y||
    double res = 0.0;
    const int nsel = (k >= 2) ? 2 : 1;
    for (int i = 0; i < nsel; ++i) {
        double *y = w.yv + (long)i * n;
        hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, n);
        hipLaunchKernelGGL(combine_kernel, dim3(grid_for(n)), dim3(256), 0, s, w.V, n, k, w.tri + 4 + (long)i * ld, 1.0,
                           y);
        if ((e = apply_T(w, A, m, y, w.w, s)) != hipSuccess) return e;
        const int np = grid_for(n);
        hipLaunchKernelGGL(resid_sumsq_kernel, dim3(np), dim3(256), 0, s, w.w, y, w.tri, i, n, w.dots);
        hipLaunchKernelGGL(norm_finalize_kernel, dim3(1), dim3(64), 0, s, w.dots, np, w.nrm + i);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(w.h_out + 4, w.nrm, sizeof(double) * 2, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(w.h_out, w.tri, sizeof(double) * 2, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const double l1 = w.h_out[0], l2 = (nsel > 1) ? w.h_out[1] : 0.0;
    for (int i = 0; i < nsel; ++i) res = std::max(res, w.h_out[4 + i] / fabs(l1));
    out->lambda1 = l1;
    out->lambda2 = l2;
    out->xi = (l2 != 0.0 && fabs(l2) < fabs(l1)) ? 1.0 / log(fabs(l1) / fabs(l2)) : (l2 == 0.0 ? 0.0 : INFINITY);
    out->residual = res;
    out->iterations = k;
    out->converged = conv;
    return hipSuccess;
}

}  // namespace ctm
