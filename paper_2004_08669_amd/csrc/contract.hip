// Contractions and fused elementwise kernels of one CTMRG step; see contract.h.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "contract.h"
#include "gemm.h"
#include "blocks.h"

namespace ctm {

// ---------------------------------------------------------------- accessors (block layout: blocks.h)
// Gram of the extension blocks: A(k1 = (s,sg), n = (i,j)) = w_i w_j X[(s m + i) N + sg m + j]
struct A_MixW {
    using value_type = double;
    const double *X; const double *om; int q, m; long Nc;
    static constexpr bool kContigK = true;
    __device__ double operator()(int k1, int n) const
    {
        const int s = k1 / q, sg = k1 - s * q;
        const int i = n / m, j = n - i * m;
        return om[i] * om[j] * X[(long)(s * m + i) * Nc + sg * m + j];
    }
};
// B(n = (i,j), k2 = (s',sg')) = X[(s' m + i) N + sg' m + j]
struct B_MixT {
    using value_type = double;
    const double *X; int q, m; long Nc;
    static constexpr bool kContigK = true;
    __device__ double operator()(int n, int k2) const
    {
        const int s = k2 / q, sg = k2 - s * q;
        const int i = n / m, j = n - i * m;
        return X[(long)(s * m + i) * Nc + sg * m + j];
    }
};

// ---------------------------------------------------------------- kernels

// W[(s,sg),(s',sg')] = exp(K (g(s,sg) + g(sg,sg') + g(sg',s') + g(s',s))), g = v.v (Eqs. 1-2);
// WH = W * h4 with h4 = -(that sum), the plaquette energy.
__global__ void build_weight_kernel(const double *V, int q, int dim, double K, double *W, double *WH)
{
    const int q2 = q * q;
    const long total = (long)q2 * q2;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int r = (int)(idx / q2), c = (int)(idx - (long)r * q2);
        const int s = r / q, sg = r - s * q, sp = c / q, sgp = c - sp * q;
        auto dot = [&](int a, int b) {
            double acc = 0.0;
            for (int x = 0; x < dim; ++x) acc += V[a * dim + x] * V[b * dim + x];
            return acc;
        };
        const double bonds = dot(s, sg) + dot(sg, sgp) + dot(sgp, sp) + dot(sp, s);
        const double w = exp(K * bonds);
        W[idx] = w;
        WH[idx] = -bonds * w;
    }
}

__global__ void init_state_kernel(double *A, double *omega, int q, int m, int bc, int s0, Book *book)
{
    const long N = (long)q * m;
    const long total = (long)m * N;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int g = (int)(idx / N);
        const long col = idx - (long)g * N;
        const int s = (int)(col / m), a = (int)(col - (long)s * m);
        double v = 0.0;
        if (g == 0 && a == 0) v = (bc == 0) ? (s == s0 ? 1.0 : 0.0) : 1.0;
        A[idx] = v;
    }
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < m; i += (long)gridDim.x * blockDim.x)
        omega[i] = (i == 0) ? 1.0 : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Book b = {};
        b.ln_a = 0.0; b.ln_b = 0.0;
        b.nC_prev = b.nC = b.nP_prev = b.nP = 1.0;
        b.S_prev = b.S = 0.0;
        b.k = 0;
        *book = b;
    }
}

__global__ void scale_rows_kernel(const double *A, const double *omega, double *OA, int m, long N)
{
    const long total = (long)m * N;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int g = (int)(idx / N);
        OA[idx] = omega[g] * A[idx];
    }
}

__global__ void __launch_bounds__(256) absmax_partial_kernel(const double *P, long total, double *partials)
{
    __shared__ double red[4];
    double mx = 0.0;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x)
        mx = fmax(mx, fabs(P[idx]));
    mx = block_max<256>(mx, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = mx;
}

// n_P from the partial maxima; the bookkeeping of the true scale:
//   ln b_k = ln b_{k-1} + 2 ln a_{k-1} + ln n_C(k),  ln a_k = ln a_{k-1} + ln n_P(k).
__global__ void book_kernel(const double *partials, int np, Book *book, const double *nC_dev, const double *S_dev)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double mx = 0.0;
    for (int i = 0; i < np; ++i) mx = fmax(mx, partials[i]);
    Book b = *book;
    const double nC = *nC_dev;
    b.ln_b = b.ln_b + 2.0 * b.ln_a + log(nC);
    b.ln_a = b.ln_a + log(mx);
    b.nC_prev = b.nC; b.nC = nC;
    b.nP_prev = b.nP; b.nP = mx;
    b.S_prev = b.S; b.S = *S_dev;
    b.nP_part_max = mx;
    b.k += 1;
    *book = b;
}

__global__ void scale_by_book_kernel(const double *Pt, double *A, long total, const Book *book)
{
    const double inv = 1.0 / book->nP;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x)
        A[idx] = Pt[idx] * inv;
}

// Magnetization pieces: prob[s] = sum_{b,j} w_j^4 U[(s m + b), j]^2  (one block per spin)
__global__ void __launch_bounds__(256) spin_weight_kernel(const double *U, const double *omega, int m, double *prob)
{
    __shared__ double red[4];
    const int s = blockIdx.x;
    double acc = 0.0;
    const long total = (long)m * m;
    for (long idx = threadIdx.x; idx < total; idx += 256) {
        const int b = (int)(idx / m), j = (int)(idx - (long)b * m);
        const double w = omega[j];
        const double u = U[(long)(s * m + b) * m + j];
        acc += (w * w) * (w * w) * u * u;
    }
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) prob[s] = acc;
}

// Partial sums of the environment scalars, one triple per workgroup:
//   part[3 b + 0] = sum over rows i = b, b + G, ... of sum_{s,j} A[i, (s,j)]^2 w_i^2 w_j^2   (Z_h),
//   part[3 b + 1] = its share of sum W H, part[3 b + 2] of sum W h4 H (the q^4 plaquette sums).
__global__ void __launch_bounds__(256)
env_partials_kernel(const double *A, const double *omega, const double *W, const double *WH, const double *H, int q,
                    int m, double *part)
{
    __shared__ double red[4];
    const long N = (long)q * m;
    const int tid = threadIdx.x;
    double zh = 0.0;
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const double wi = omega[i];
        const double *row = A + (long)i * N;
        double r = 0.0;
        for (int s = 0; s < q; ++s)
            for (int j = tid; j < m; j += 256) {
                const double p = row[(long)s * m + j], wj = omega[j];
                r += p * p * wj * wj;
            }
        zh += r * wi * wi;
    }
    zh = block_sum<256>(zh, red);
    const long q4 = (long)q * q * q * q;
    double zd = 0.0, zdh = 0.0;
    for (long idx = blockIdx.x * 256L + tid; idx < q4; idx += (long)gridDim.x * 256) {
        zd += W[idx] * H[idx];
        zdh += WH[idx] * H[idx];
    }
    zd = block_sum<256>(zd, red);
    zdh = block_sum<256>(zdh, red);
    if (tid == 0) {
        part[3 * blockIdx.x + 0] = zh;
        part[3 * blockIdx.x + 1] = zd;
        part[3 * blockIdx.x + 2] = zdh;
    }
}

// out: [0] Z_b, [1] Z_h, [2] Z_d, [3] Z_d[W h4], [4] sum w^4, [5] M numerator, [6] sum prob
// (the partials of env_partials_kernel summed in workgroup order, so the result does not depend
// on scheduling)
__global__ void __launch_bounds__(256)
env_scalars_kernel(const double *omega, const double *part, int np, const double *prob, const double *V, int q,
                   int dim, int m, int bc, int s0, double *out)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    double zb = 0.0;
    for (int i = tid; i < m; i += 256) {
        const double w = omega[i];
        zb += (w * w) * (w * w);
    }
    zb = block_sum<256>(zb, red);
    if (tid != 0) return;
    double zh = 0.0, zd = 0.0, zdh = 0.0;
    for (int b = 0; b < np; ++b) {
        zh += part[3 * b];
        zd += part[3 * b + 1];
        zdh += part[3 * b + 2];
    }
    double psum = 0.0, mnum = 0.0;
    double vx = 0.0, vy = 0.0, vz = 0.0;
    for (int s = 0; s < q; ++s) {
        psum += prob[s];
        double dp = 0.0;
        for (int x = 0; x < dim; ++x) dp += V[s0 * dim + x] * V[s * dim + x];
        mnum += prob[s] * dp;
        if (dim > 0) vx += prob[s] * V[s * dim + 0];
        if (dim > 1) vy += prob[s] * V[s * dim + 1];
        if (dim > 2) vz += prob[s] * V[s * dim + 2];
    }
    out[0] = zb;
    out[1] = zh;
    out[2] = zd;
    out[3] = zdh;
    out[4] = zb;
    out[5] = (bc == 0) ? mnum : sqrt(vx * vx + vy * vy + vz * vz);
    out[6] = psum;
}

// FP32 operands of the mixed-precision contractions: A32 = A, OA32 = diag(omega) A (rounded once).
__global__ void rows_to_f32_kernel(const double *A, const double *omega, float *A32, float *OA32, int m, long N)
{
    const long total = (long)m * N;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int g = (int)(idx / N);
        const double a = A[idx];
        A32[idx] = (float)a;
        OA32[idx] = (float)(omega[g] * a);
    }
}

// dst = scale * src, rounded to FP32.
__global__ void to_f32_kernel(const double *src, float *dst, long n, double scale)
{
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x)
        dst[idx] = (float)(scale * src[idx]);
}

// ---------------------------------------------------------------- launchers

static int grid_for(long total) { return (int)std::max<long>(1, std::min<long>(4096, (total + 255) / 256)); }

hipError_t build_weight(const double *V, int q, int dim, double K, double *W, double *WH, hipStream_t s)
{
    const long total = (long)q * q * q * q;
    hipLaunchKernelGGL(build_weight_kernel, dim3(grid_for(total)), dim3(256), 0, s, V, q, dim, K, W, WH);
    return hipGetLastError();
}

hipError_t init_state(double *A, double *omega, int q, int m, int bc, int s0, Book *book, hipStream_t s)
{
    hipLaunchKernelGGL(init_state_kernel, dim3(grid_for((long)m * q * m)), dim3(256), 0, s, A, omega, q, m, bc, s0,
                       book);
    return hipGetLastError();
}

hipError_t extension_products(const double *A, const double *omega, double *OA, double *X, int q, int m,
                              hipStream_t s)
{
    const long N = (long)q * m;
    hipLaunchKernelGGL(scale_rows_kernel, dim3(grid_for(m * N)), dim3(256), 0, s, A, omega, OA, m, N);
    return gemm_mfma(GEMM_LARGE, A_T{A, N}, B_RM{OA, N}, EpiStore{X, N, 1.0}, (int)N, (int)N, m, s);
}

hipError_t weight_mix(const double *W, const double *Xin, double *Cout, int q, int m, hipStream_t s)
{
    const long N = (long)q * m;
    const int q2 = q * q;
    // W is symmetric: W^T(i,k) = W[k q2 + i]
    return gemm_mfma(GEMM_MIX, A_T{W, q2}, B_Mix{Xin, q, m, N}, EpiMix_<double, false>{Cout, q, m, N, 1.0}, q2,
                     m * m, q2, s);
}

hipError_t halfrow_products(const double *A, const double *U, double *Y, int q, int m, hipStream_t s)
{
    const long N = (long)q * m;
    return gemm_mfma(GEMM_LARGE, A_T{A, N}, B_Ublk{U, m}, EpiStore{Y, N, 1.0}, (int)N, (int)N, m, s);
}

// Splits of the projection's inner dimension (K = q m, output m x q m): enough workgroups for
// the device, partials within the work buffer (none without one).
static int projection_splits(int m, long N, size_t work_elems)
{
    const long tiles = (long)ceil_div(m, 128) * ceil_div(N, 128);
    int sp = 1;
    while (tiles * sp < 768 && sp < 8 && (size_t)(sp + 1) * m * N <= work_elems && N / (sp + 1) >= 1024) ++sp;
    return sp;
}

hipError_t projection(const double *U, const double *Z, double *Pt, int q, int m, double *work, size_t work_elems,
                      hipStream_t s)
{
    const long N = (long)q * m;
    const int sp = projection_splits(m, N, work ? work_elems : 0);
    return gemm_mfma_splitk(A_T{U, m}, B_RM{Z, N}, EpiStore{Pt, N, 1.0}, m, (int)N, (int)N, sp, work, s, GEMM_LARGE);
}

// ---- mixed precision: FP32 operands on the FP32 matrix cores (or as split-bf16 products on the
// bf16 ones, gemm.h), FP32 accumulation.
// W32 holds W / wscale (wscale = e^{4K} >= max W, so that no weight overflows FP32);
// the factor is restored in FP64 in the epilogues that produce C' and P~.

hipError_t weight_to_f32(const double *W, float *W32, int q, double wscale, hipStream_t s)
{
    const long n = (long)q * q * q * q;
    hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, W, W32, n, 1.0 / wscale);
    return hipGetLastError();
}

hipError_t state_to_f32(const double *A, const double *omega, float *A32, float *OA32, int q, int m, hipStream_t s)
{
    const long N = (long)q * m;
    hipLaunchKernelGGL(rows_to_f32_kernel, dim3(grid_for((long)m * N)), dim3(256), 0, s, A, omega, A32, OA32, m, N);
    return hipGetLastError();
}

hipError_t vectors_to_f32(const double *U, float *U32, int q, int m, hipStream_t s)
{
    const long n = (long)q * m * m;
    hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, U, U32, n, 1.0);
    return hipGetLastError();
}

// The FP32 contractions on the FP32 matrix cores, or as split-bf16 products (x3).
template <GemmShape SH, class LA, class LB, class EPI>
static hipError_t gemm32(bool x3, LA la, LB lb, EPI epi, int M, int N, int K, hipStream_t s)
{
    return x3 ? gemm_bf16x3<SH>(la, lb, epi, M, N, K, s) : gemm_mfma(SH, la, lb, epi, M, N, K, s);
}

hipError_t extension_products_f32(const float *A32, const float *OA32, float *X32, int q, int m, bool x3,
                                  hipStream_t s)
{
    const long N = (long)q * m;
    return gemm32<GEMM_LARGE>(x3, A_Tf{A32, N}, B_RMf{OA32, N}, EpiStoreF{X32, N, 1.0}, (int)N, (int)N, m, s);
}

hipError_t weight_mix_f32_to_f64(const float *W32, const float *X32, double *Cout, int q, int m, double wscale,
                                 bool x3, hipStream_t s)
{
    const long N = (long)q * m;
    const int q2 = q * q;
    return gemm32<GEMM_MIX>(x3, A_Tf{W32, q2}, B_Mixf{X32, q, m, N}, EpiMix_<double, true>{Cout, q, m, N, wscale}, q2,
                            m * m, q2, s);
}

hipError_t halfrow_products_f32(const float *A32, const float *U32, float *Y32, int q, int m, bool x3, hipStream_t s)
{
    const long N = (long)q * m;
    return gemm32<GEMM_LARGE>(x3, A_Tf{A32, N}, B_Ublkf{U32, m}, EpiStoreF{Y32, N, 1.0}, (int)N, (int)N, m, s);
}

hipError_t weight_mix_f32(const float *W32, const float *Y32, float *Z32, int q, int m, bool x3, hipStream_t s)
{
    const long N = (long)q * m;
    const int q2 = q * q;
    return gemm32<GEMM_MIX>(x3, A_Tf{W32, q2}, B_Mixf{Y32, q, m, N}, EpiMix_<float, false>{Z32, q, m, N, 1.0}, q2,
                            m * m, q2, s);
}

hipError_t projection_f32(const float *U32, const float *Z32, double *Pt, int q, int m, double wscale, double *work,
                          size_t work_elems, bool x3, hipStream_t s)
{
    const long N = (long)q * m;
    const int sp = projection_splits(m, N, work ? work_elems : 0);
    if (x3) return gemm_bf16x3<GEMM_LARGE>(A_Tf{U32, m}, B_RMf{Z32, N}, EpiStore{Pt, N, wscale}, m, (int)N, (int)N, s, sp, work);
    return gemm_mfma_splitk(A_Tf{U32, m}, B_RMf{Z32, N}, EpiStore{Pt, N, wscale}, m, (int)N, (int)N, sp, work, s,
                            GEMM_LARGE);
}

hipError_t normalize_and_book(const double *Pt, double *A, int q, int m, double *partials, Book *book,
                              const double *nC_dev, const double *S_dev, hipStream_t s)
{
    const long total = (long)m * q * m;
    const int np = std::min(1024, grid_for(total));
    hipLaunchKernelGGL(absmax_partial_kernel, dim3(np), dim3(256), 0, s, Pt, total, partials);
    hipLaunchKernelGGL(book_kernel, dim3(1), dim3(64), 0, s, partials, np, book, nC_dev, S_dev);
    hipLaunchKernelGGL(scale_by_book_kernel, dim3(grid_for(total)), dim3(256), 0, s, Pt, A, total, book);
    return hipGetLastError();
}

hipError_t observables(const double *A, const double *omega, const double *U, const double *W, const double *WH,
                       const double *V, double *OA, double *X, double *H, double *work, size_t work_elems,
                       int q, int dim, int m, int bc, int s0, double *out, hipStream_t s)
{
    const long N = (long)q * m;
    const int q2 = q * q;
    hipError_t e = extension_products(A, omega, OA, X, q, m, s);
    if (e != hipSuccess) return e;
    // H[(s,sg),(s',sg')] = sum_{i,j} w_i w_j X_{s sg}[i,j] X_{s' sg'}[i,j]
    const long K = (long)m * m;
    const long tiles = (long)ceil_div(q2, 64) * ceil_div(q2, 64);
    int sp = 1;
    while (tiles * sp < 512 && K / (sp * 2) >= 256 && (size_t)(sp * 2) * q2 * q2 <= work_elems) sp *= 2;
    e = gemm_mfma_splitk(A_MixW{X, omega, q, m, N}, B_MixT{X, q, m, N}, EpiStore{H, q2, 1.0}, q2, q2, (int)K, sp, work,
                        s);
    if (e != hipSuccess) return e;
    double *prob = out + 8;
    hipLaunchKernelGGL(spin_weight_kernel, dim3(q), dim3(256), 0, s, U, omega, m, prob);
    // the work buffer is free again once H is formed: it takes the partial sums
    const int np = (int)std::min<size_t>({(size_t)512, (size_t)std::max(m, 1), work_elems / 3});
    if (np < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(env_partials_kernel, dim3(np), dim3(256), 0, s, A, omega, W, WH, H, q, m, work);
    hipLaunchKernelGGL(env_scalars_kernel, dim3(1), dim3(256), 0, s, omega, work, np, prob, V, q, dim, m, bc, s0,
                       out);
    return hipGetLastError();
}

}  // namespace ctm
