// Tiled FP64 / FP32 GEMM on the CDNA matrix cores (gfx950), with operand
// addressing supplied by small accessor structs.  The CTMRG contractions need
// operands whose rows and columns are combined (spin, state) indices; the
// accessors turn the paper's index permutations (its P-Index / P-Index2
// reorderings) into address arithmetic inside the tile loads and the epilogue
// stores, so no permuted copy of any matrix is ever written.
//
// C(i,j) = sum_k A(i,k) B(k,j), then epi(i, j, value, split).
//
// Work decomposition: a workgroup owns a BM x BN output tile and is made of
// WM x WN waves of 64 lanes; each wave owns (BM/WM) x (BN/WN), a grid of 16x16
// MFMA blocks.  K is walked in BK slices staged through LDS.  blockIdx.z splits
// K into chunks (split-K) when the output has too few tiles to fill the chip.
//
// MFMA operand layout of v_mfma_f64_16x16x4_f64 and v_mfma_f32_16x16x4_f32:
//   A fragment: lane l holds A[l%16][l/16]   (row l%16, k l/16)
//   B fragment: lane l holds B[l/16][l%16]   (k l/16, column l%16)
//   D fragment: lane l, register r holds D[row][l%16] with
//               row = l/16 + 4 r    (f64)
//               row = 4 (l/16) + r  (f32)
// The element type of a GEMM is the value type of its accessors: double runs
// on the FP64 matrix cores, float on the FP32 ones with FP32 accumulation.
#pragma once

#include <type_traits>

#include "common.h"

namespace ctm {

static inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------- accessors
// kContigK: consecutive k are adjacent in memory (else consecutive m / n are).

// A row-major M x K: A(i,k) = p[i*ld + k]
template <class T>
struct A_RM_ {
    using value_type = T;
    const T *p; long ld;
    static constexpr bool kContigK = true;
    __device__ T operator()(int i, int k) const { return p[(long)i * ld + k]; }
};
// A stored K x M row-major, used transposed: A(i,k) = p[k*ld + i]
template <class T>
struct A_T_ {
    using value_type = T;
    const T *p; long ld;
    static constexpr bool kContigK = false;
    __device__ T operator()(int i, int k) const { return p[(long)k * ld + i]; }
};
// B row-major K x N: B(k,j) = p[k*ld + j]
template <class T>
struct B_RM_ {
    using value_type = T;
    const T *p; long ld;
    static constexpr bool kContigK = false;
    __device__ T operator()(int k, int j) const { return p[(long)k * ld + j]; }
};
// B stored N x K row-major, used transposed: B(k,j) = p[j*ld + k]
template <class T>
struct B_T_ {
    using value_type = T;
    const T *p; long ld;
    static constexpr bool kContigK = true;
    __device__ T operator()(int k, int j) const { return p[(long)j * ld + k]; }
};
// A symmetric matrix held in its lower triangle (row-major), as two operands:
// the lower triangle with the diagonal, and the strictly lower triangle read
// transposed (its elements above the diagonal).  A . B = A_Lo . B + A_SLoT . B.
// Both restrict the K range of a tile (kRange) to the part that can be nonzero.
struct A_Lo {
    using value_type = double;
    const double *p; long ld;
    static constexpr bool kContigK = true;
    static constexpr bool kRange = true;
    __device__ double operator()(int i, int k) const { return (k <= i) ? p[(long)i * ld + k] : 0.0; }
    __device__ static void range(int m0, int bm, int &klo, int &khi) { khi = min(khi, m0 + bm); }
};
struct A_SLoT {
    using value_type = double;
    const double *p; long ld;
    static constexpr bool kContigK = false;
    static constexpr bool kRange = true;
    __device__ double operator()(int i, int k) const { return (k > i) ? p[(long)k * ld + i] : 0.0; }
    __device__ static void range(int m0, int, int &klo, int &) { klo = max(klo, m0 + 1); }
};

// Work items for a balanced split of the K range of those operands: the K range
// [k_lo, k_hi) of row tile I (rows [bm I, bm I + bm)) is cut into chunks of ch,
// and blockIdx.x enumerates the (tile, chunk) items tile by tile (kItems).
struct A_LoItems : A_Lo {
    static constexpr bool kItems = true;
    __host__ __device__ static int k_lo(int, int) { return 0; }
    __host__ __device__ static int k_hi(int I, int bm, int K) { return K < bm * (I + 1) ? K : bm * (I + 1); }
};
struct A_SLoTItems : A_SLoT {
    static constexpr bool kItems = true;
    __host__ __device__ static int k_lo(int I, int bm) { return bm * I + 1; }
    __host__ __device__ static int k_hi(int, int, int K) { return K; }
};
template <class LA>
__host__ __device__ inline int tile_items(int I, int bm, int K, int ch)
{
    const int lo = LA::k_lo(I, bm), hi = LA::k_hi(I, bm, K);
    return hi > lo ? (hi - lo + ch - 1) / ch : 0;
}

using A_RM = A_RM_<double>;
using A_T = A_T_<double>;
using B_RM = B_RM_<double>;
using B_T = B_T_<double>;
using A_Tf = A_T_<float>;
using B_RMf = B_RM_<float>;

// ---------------------------------------------------------------- epilogues
struct EpiStore {  // C = alpha * acc
    double *p; long ld; double alpha;
    __device__ void operator()(int i, int j, double v, int) const { p[(long)i * ld + j] = alpha * v; }
};
struct EpiAxpby {  // C = alpha * acc + beta * C
    double *p; long ld; double alpha, beta;
    __device__ void operator()(int i, int j, double v, int) const
    {
        double *c = p + (long)i * ld + j;
        *c = alpha * v + beta * (*c);
    }
};
struct EpiStoreF {  // C = alpha * acc, rounded to FP32
    float *p; long ld; double alpha;
    __device__ void operator()(int i, int j, double v, int) const { p[(long)i * ld + j] = (float)(alpha * v); }
};
struct EpiAxpbyLower {  // C = alpha * acc + beta * C on the tiles on or below the diagonal only
    double *p; long ld; double alpha, beta;
    static constexpr bool kLowerTiles = true;
    // C is read before the K loop (the product's inner dimension is short, so a read
    // issued in the epilogue would not overlap any matrix-core work)
    static constexpr bool kPrefetchC = true;
    __device__ double load(int i, int j) const { return p[(long)i * ld + j]; }
    __device__ void store(int i, int j, double v, double c) const { p[(long)i * ld + j] = alpha * v + beta * c; }
    __device__ void operator()(int i, int j, double v, int) const
    {
        double *c = p + (long)i * ld + j;
        *c = alpha * v + beta * (*c);
    }
};
struct EpiItems {  // partial sums of work items (128-row tiles), reduced by reduce_items_kernel
    double *p; long N;
    __device__ void operator()(int i, int j, double v, int item) const { p[((long)item * 128 + (i & 127)) * N + j] = v; }
};
struct EpiPartial {  // split-K partial sums, reduced by reduce_partials
    double *p; long M, N;
    __device__ void operator()(int i, int j, double v, int split) const
    {
        p[((long)split * M + i) * N + j] = v;
    }
};

// ---------------------------------------------------------------- optional traits
template <class T, class = void> struct has_krange : std::false_type {};
template <class T> struct has_krange<T, std::void_t<decltype(T::kRange)>> : std::true_type {};
template <class T, class = void> struct has_items : std::false_type {};
template <class T> struct has_items<T, std::void_t<decltype(T::kItems)>> : std::true_type {};
template <class T, class = void> struct lower_tiles : std::false_type {};
template <class T> struct lower_tiles<T, std::void_t<decltype(T::kLowerTiles)>> : std::true_type {};
template <class T, class = void> struct prefetch_c : std::false_type {};
template <class T> struct prefetch_c<T, std::void_t<decltype(T::kPrefetchC)>> : std::true_type {};

// ---------------------------------------------------------------- MFMA step per element type
template <class T> struct Mfma;
template <> struct Mfma<double> {
    using acc_t = double4_t;
    static __device__ acc_t zero() { return (acc_t){0.0, 0.0, 0.0, 0.0}; }
    static __device__ acc_t mma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
    using acc_t = float4_t;
    static __device__ acc_t zero() { return (acc_t){0.f, 0.f, 0.f, 0.f}; }
    static __device__ acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// ---------------------------------------------------------------- kernel
// PAD: doubles (or floats) of padding per LDS row.  DB: two LDS buffers, so that the next
// K slice is staged while the matrix cores read the current one (one barrier per slice).
// VA, VB: consecutive elements of A and B per thread and load (along k when the operand is
// contiguous in k, else along m / n), so that contiguous operands are read with 16-byte loads.
template <int BM, int BN, int BK, int WM, int WN, class LA, class LB, class EPI, int PAD = 1, bool DB = false,
          int VA = 1, int VB = 1>
__global__ void __launch_bounds__(WM * WN * 64)
gemm_mfma_kernel(LA la, LB lb, EPI epi, int M, int N, int K, int kchunk)
{
    using T = typename LA::value_type;
    static_assert(std::is_same<T, typename LB::value_type>::value, "operand types");
    using MF = Mfma<T>;
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM / 16;
    constexpr int TN = BN / WN / 16;
    static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
    static_assert(BK % 4 == 0 && BK % VA == 0 && BK % VB == 0 && BM % VA == 0 && BN % VB == 0, "BK / VA / VB");
    constexpr int NB = DB ? 2 : 1;
    __shared__ T As[NB][BK][BM + PAD];
    __shared__ T Bs[NB][BK][BN + PAD];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave % WM, wn = wave / WM;
    int tile_m = blockIdx.x, tile_n = blockIdx.y;
    if constexpr (lower_tiles<EPI>::value) {
        // blockIdx.x enumerates the tiles (I, J) with J <= I
        static_assert(BM == BN, "square tiles");
        const int t = blockIdx.x;
        int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while (I * (I + 1) / 2 > t) --I;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        tile_m = I;
        tile_n = t - I * (I + 1) / 2;
    }
    int split = blockIdx.z, kbeg, kend;
    if constexpr (has_items<LA>::value) {
        // blockIdx.x enumerates the work items; kchunk is the chunk length
        int item = blockIdx.x, I = 0;
        const int ntile = (M + BM - 1) / BM;
        for (; I < ntile; ++I) {
            const int cnt = tile_items<LA>(I, BM, K, kchunk);
            if (item < cnt) break;
            item -= cnt;
        }
        tile_m = I;
        split = blockIdx.x;
        kbeg = LA::k_lo(I, BM) + item * kchunk;
        kend = min(LA::k_hi(I, BM, K), kbeg + kchunk);
    } else {
        kbeg = blockIdx.z * kchunk;
        kend = min(K, kbeg + kchunk);
    }
    const int m0 = tile_m * BM, n0 = tile_n * BN;
    if constexpr (has_krange<LA>::value) LA::range(m0, BM, kbeg, kend);

    typename MF::acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::zero();
    // C of this lane's outputs, read ahead of the K loop when the epilogue asks for it
    double cpre[prefetch_c<EPI>::value ? TM : 1][prefetch_c<EPI>::value ? TN : 1][4];
    if constexpr (prefetch_c<EPI>::value) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + (wm * TM + i) * 16 + MF::row(lane, r);
                    const int col = n0 + (wn * TN + j) * 16 + (lane & 15);
                    cpre[i][j][r] = (row < M && col < N) ? epi.load(row, col) : 0.0;
                }
    }

    // Each thread holds its share of the next K slice in registers while the matrix cores
    // work on the current one from LDS.  A thread's share is groups of VA (VB) elements.
    constexpr int GA = BM * BK / VA, GB = BN * BK / VB;
    constexpr int PA = (GA + NT - 1) / NT;
    constexpr int PB = (GB + NT - 1) / NT;
    T ra[PA][VA], rb[PB][VB];
    // group g of A: VA consecutive k of row mm (contiguous in k) or VA consecutive rows at kk
    auto a_pos = [](int g, int &mm, int &kk) {
        if (LA::kContigK) { mm = g / (BK / VA); kk = (g - mm * (BK / VA)) * VA; }
        else { kk = g / (BM / VA); mm = (g - kk * (BM / VA)) * VA; }
    };
    auto b_pos = [](int g, int &nn, int &kk) {
        if (LB::kContigK) { nn = g / (BK / VB); kk = (g - nn * (BK / VB)) * VB; }
        else { kk = g / (BN / VB); nn = (g - kk * (BN / VB)) * VB; }
    };
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int g = tid + u * NT;
            int mm, kk;
            a_pos(g, mm, kk);
            const int gm = m0 + mm, gk = k0 + kk;
            const bool full = g < GA && (LA::kContigK ? (gm < M && gk + VA <= kend) : (gm + VA <= M && gk < kend));
            if (full) {
#pragma unroll
                for (int v = 0; v < VA; ++v) ra[u][v] = LA::kContigK ? la(gm, gk + v) : la(gm + v, gk);
            } else {
#pragma unroll
                for (int v = 0; v < VA; ++v) {
                    const int em = LA::kContigK ? gm : gm + v, ek = LA::kContigK ? gk + v : gk;
                    ra[u][v] = (g < GA && em < M && ek < kend) ? la(em, ek) : T(0);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            const int g = tid + u * NT;
            int nn, kk;
            b_pos(g, nn, kk);
            const int gn = n0 + nn, gk = k0 + kk;
            const bool full = g < GB && (LB::kContigK ? (gn < N && gk + VB <= kend) : (gn + VB <= N && gk < kend));
            if (full) {
#pragma unroll
                for (int v = 0; v < VB; ++v) rb[u][v] = LB::kContigK ? lb(gk + v, gn) : lb(gk, gn + v);
            } else {
#pragma unroll
                for (int v = 0; v < VB; ++v) {
                    const int en = LB::kContigK ? gn : gn + v, ek = LB::kContigK ? gk + v : gk;
                    rb[u][v] = (g < GB && en < N && ek < kend) ? lb(ek, en) : T(0);
                }
            }
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int g = tid + u * NT;
            if (g < GA) {
                int mm, kk;
                a_pos(g, mm, kk);
#pragma unroll
                for (int v = 0; v < VA; ++v) {
                    if (LA::kContigK) As[buf][kk + v][mm] = ra[u][v];
                    else As[buf][kk][mm + v] = ra[u][v];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            const int g = tid + u * NT;
            if (g < GB) {
                int nn, kk;
                b_pos(g, nn, kk);
#pragma unroll
                for (int v = 0; v < VB; ++v) {
                    if (LB::kContigK) Bs[buf][kk + v][nn] = rb[u][v];
                    else Bs[buf][kk][nn + v] = rb[u][v];
                }
            }
        }
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[buf][kk + (lane >> 4)][(wm * TM + i) * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[buf][kk + (lane >> 4)][(wn * TN + j) * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(a[i], b[j], acc[i][j]);
        }
    };
    if constexpr (DB) {
        if (kbeg < kend) {
            fetch(kbeg);
            stage(0);
        }
        __syncthreads();
        int buf = 0;
        for (int k0 = kbeg; k0 < kend; k0 += BK) {
            const bool more = k0 + BK < kend;
            if (more) fetch(k0 + BK);
            compute(buf);
            if (more) stage(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    } else {
        if (kbeg < kend) fetch(kbeg);
        for (int k0 = kbeg; k0 < kend; k0 += BK) {
            stage(0);
            __syncthreads();
            if (k0 + BK < kend) fetch(k0 + BK);
            compute(0);
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + (wm * TM + i) * 16 + MF::row(lane, r);
                const int col = n0 + (wn * TN + j) * 16 + (lane & 15);
                if (row < M && col < N) {
                    if constexpr (prefetch_c<EPI>::value) epi.store(row, col, (double)acc[i][j][r], cpre[i][j][r]);
                    else epi(row, col, (double)acc[i][j][r], split);
                }
            }
}

// Sum split-K partials and apply the final epilogue.
template <class EPI>
__global__ void reduce_partials_kernel(const double *part, int splits, int M, int N, EPI epi)
{
    const long total = (long)M * N;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int z = 0; z < splits; ++z) s += part[(long)z * total + idx];
        const int i = (int)(idx / N), j = (int)(idx - (long)i * N);
        epi(i, j, s, 0);
    }
}

// Y = sum of the work-item partials (EpiItems) of two operands: blockIdx.y is the
// 128-row tile, each thread one output element; the items of the first operand,
// then those of the second, are added in order.
template <class LA1, class LA2>
__global__ void __launch_bounds__(256)
reduce_items_kernel(const double *p1, const double *p2, int M, int N, int K, int ch, double *Y, long ldy)
{
    __shared__ int sred[2][4];
    const int I = blockIdx.y;
    // first item of tile I in each list: sum of the item counts of the tiles before it
    int a1 = 0, a2 = 0;
    for (int t = threadIdx.x; t < I; t += blockDim.x) {
        a1 += tile_items<LA1>(t, 128, K, ch);
        a2 += tile_items<LA2>(t, 128, K, ch);
    }
    for (int off = 32; off > 0; off >>= 1) {
        a1 += __shfl_xor(a1, off, 64);
        a2 += __shfl_xor(a2, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sred[0][threadIdx.x >> 6] = a1;
        sred[1][threadIdx.x >> 6] = a2;
    }
    __syncthreads();
    const int f1 = sred[0][0] + sred[0][1] + sred[0][2] + sred[0][3];
    const int f2 = sred[1][0] + sred[1][1] + sred[1][2] + sred[1][3];
    const int c1 = tile_items<LA1>(I, 128, K, ch), c2 = tile_items<LA2>(I, 128, K, ch);
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = idx / N, j = idx - r * N, i = I * 128 + r;
    if (r >= 128 || i >= M) return;
    const double *q1 = p1 + ((long)f1 * 128 + r) * N + j;
    const double *q2 = p2 + ((long)f2 * 128 + r) * N + j;
    const long step = 128L * N;
    double s = 0.0;
#pragma unroll 8
    for (int u = 0; u < c1; ++u) s += q1[u * step];
#pragma unroll 8
    for (int u = 0; u < c2; ++u) s += q2[u * step];
    Y[(long)i * ldy + j] = s;
}

// ---------------------------------------------------------------- split-bf16 products
// FP32 operands as three bf16 products on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16),
// with FP32 accumulation: each operand value x is split into hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even; x - hi is exact in FP32), and
//   a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi,
// dropping a_lo b_lo and the rounding of the lo parts: at most about 3 * 2^-16 |a b| per
// term (2^-18 for a typical one), on top of the FP32 accumulation; the bf16 products
// themselves are exact in FP32.
//
// Tiles: BK = 32 (one bf16 MFMA per 16 x 16 block and product).  In LDS every row
// (of A: an output row, of B: an output column) holds its 32 k of the slice contiguous,
// hi and lo in separate arrays, padded to 40 entries (80 bytes: eight lanes storing or
// loading 16 bytes in consecutive rows meet disjoint banks).  The fragment of an MFMA is
// then one 16-byte LDS read per lane: lane l takes row l % 16 and the eight k
// 8 (l / 16) .. 8 (l / 16) + 7, for A and B alike (the instruction pairs the same
// lane group and element of both operands, so the products run over the same k).
// D fragment: lane l, register r holds D[4 (l / 16) + r][l % 16].
// A thread stages groups of eight k of one row: along m (n) across the lanes of a wave
// when the operand is contiguous in m (n), along k when it is contiguous in k.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ inline unsigned bf16_rne_bits(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

template <int BM, int BN, int WM, int WN, class LA, class LB, class EPI>
__global__ void __launch_bounds__(WM * WN * 64)
gemm_bf16x3_kernel(LA la, LB lb, EPI epi, int M, int N, int K, int kchunk)
{
    static_assert(std::is_same<typename LA::value_type, float>::value &&
                      std::is_same<typename LB::value_type, float>::value, "FP32 operands");
    static_assert(!has_krange<LA>::value && !has_items<LA>::value && !lower_tiles<EPI>::value &&
                      !prefetch_c<EPI>::value, "plain tiles only");
    constexpr int BK = 32, KP = 40;
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM / 16;
    constexpr int TN = BN / WN / 16;
    static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
    __shared__ __align__(16) unsigned short Ah[BM][KP], Al[BM][KP], Bh[BN][KP], Bl[BN][KP];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave % WM, wn = wave / WM;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int split = blockIdx.z;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);

    float4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = (float4_t){0.f, 0.f, 0.f, 0.f};

    constexpr int GA = BM * (BK / 8), GB = BN * (BK / 8);
    constexpr int PA = (GA + NT - 1) / NT, PB = (GB + NT - 1) / NT;
    float ra[PA][8], rb[PB][8];
    // group g: the eight k kk .. kk + 7 of row r
    auto pos = [](int g, int rows, bool contig_k, int &r, int &kk) {
        if (contig_k) { r = g / (BK / 8); kk = (g - r * (BK / 8)) * 8; }
        else { kk = (g / rows) * 8; r = g - (kk / 8) * rows; }
    };
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int g = tid + u * NT;
            int r, kk;
            pos(g, BM, LA::kContigK, r, kk);
            const int gm = m0 + r, gk = k0 + kk;
            if (g < GA && gm < M && gk + 8 <= kend) {
#pragma unroll
                for (int v = 0; v < 8; ++v) ra[u][v] = la(gm, gk + v);
            } else {
#pragma unroll
                for (int v = 0; v < 8; ++v) ra[u][v] = (g < GA && gm < M && gk + v < kend) ? la(gm, gk + v) : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            const int g = tid + u * NT;
            int r, kk;
            pos(g, BN, LB::kContigK, r, kk);
            const int gn = n0 + r, gk = k0 + kk;
            if (g < GB && gn < N && gk + 8 <= kend) {
#pragma unroll
                for (int v = 0; v < 8; ++v) rb[u][v] = lb(gk + v, gn);
            } else {
#pragma unroll
                for (int v = 0; v < 8; ++v) rb[u][v] = (g < GB && gn < N && gk + v < kend) ? lb(gk + v, gn) : 0.f;
            }
        }
    };
    // split eight values into hi and lo and store each as one 16-byte row segment
    auto put = [](const float (&x)[8], unsigned short *hi, unsigned short *lo) {
        unsigned h[8], l[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            h[v] = bf16_rne_bits(x[v]);
            l[v] = bf16_rne_bits(x[v] - __uint_as_float(h[v] << 16));
        }
        *(uint4 *)hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
        *(uint4 *)lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
    };
    auto stage = [&]() {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int g = tid + u * NT;
            if (g < GA) {
                int r, kk;
                pos(g, BM, LA::kContigK, r, kk);
                put(ra[u], &Ah[r][kk], &Al[r][kk]);
            }
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            const int g = tid + u * NT;
            if (g < GB) {
                int r, kk;
                pos(g, BN, LB::kContigK, r, kk);
                put(rb[u], &Bh[r][kk], &Bl[r][kk]);
            }
        }
    };
    auto compute = [&]() {
        const int kq = (lane >> 4) * 8, rr = lane & 15;
        bf16x8_t ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            ah[i] = __builtin_bit_cast(bf16x8_t, *(const uint4 *)&Ah[(wm * TM + i) * 16 + rr][kq]);
            al[i] = __builtin_bit_cast(bf16x8_t, *(const uint4 *)&Al[(wm * TM + i) * 16 + rr][kq]);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            bh[j] = __builtin_bit_cast(bf16x8_t, *(const uint4 *)&Bh[(wn * TN + j) * 16 + rr][kq]);
            bl[j] = __builtin_bit_cast(bf16x8_t, *(const uint4 *)&Bl[(wn * TN + j) * 16 + rr][kq]);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                // the two small cross terms first
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        stage();
        __syncthreads();
        if (k0 + BK < kend) fetch(k0 + BK);
        compute();
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + (wm * TM + i) * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + (wn * TN + j) * 16 + (lane & 15);
                if (row < M && col < N) epi(row, col, (double)acc[i][j][r], split);
            }
}

// Staging of the tiles per element type (measured on the contraction shapes at q = 20,
// m = 512): FP32 operands are read four at a time (16-byte loads) into LDS rows padded by
// four; FP64 operands one at a time into rows padded by one.  With eight waves per
// 128 x 128 tile, two LDS buffers no longer pay.
template <class T> struct TileCfg {
    static constexpr int PAD = 1, VA = 1, VB = 1;
};
template <> struct TileCfg<float> {
    static constexpr int PAD = 4, VA = 4, VB = 4;
};

// Tile configurations.
enum GemmShape {
    GEMM_LARGE,   // 128 x 128 tile, 4 x 2 waves (each 32 x 64)
    GEMM_TALL,    // 128 x 32 tile, 4 x 1 waves (outputs with few columns)
    GEMM_TALL16,  // 128 x 16 tile, 4 x 1 waves (outputs of 16 columns)
    GEMM_MIX,     // 80 x 128 tile, 1 x 8 waves (the q^2 = 400 rows of the W-mix)
    GEMM_SMALL,   // 64 x 64 tile, 2 x 2 waves
};

template <class LA, class LB, class EPI>
hipError_t gemm_mfma(GemmShape shape, LA la, LB lb, EPI epi, int M, int N, int K, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    using C = TileCfg<typename LA::value_type>;
    switch (shape) {
    case GEMM_LARGE:
        hipLaunchKernelGGL((gemm_mfma_kernel<128, 128, 16, 4, 2, LA, LB, EPI, C::PAD, false, C::VA, C::VB>),
                           dim3(ceil_div(M, 128), ceil_div(N, 128), 1), dim3(512), 0, s, la, lb, epi, M, N, K, K);
        break;
    case GEMM_TALL:
        hipLaunchKernelGGL((gemm_mfma_kernel<128, 32, 16, 4, 1, LA, LB, EPI, C::PAD, false, C::VA, C::VB>),
                           dim3(ceil_div(M, 128), ceil_div(N, 32), 1), dim3(256), 0, s, la, lb, epi, M, N, K, K);
        break;
    case GEMM_TALL16:
        hipLaunchKernelGGL((gemm_mfma_kernel<128, 16, 16, 4, 1, LA, LB, EPI, C::PAD, false, C::VA, C::VB>),
                           dim3(ceil_div(M, 128), ceil_div(N, 16), 1), dim3(256), 0, s, la, lb, epi, M, N, K, K);
        break;
    case GEMM_MIX:
        hipLaunchKernelGGL((gemm_mfma_kernel<80, 128, 16, 1, 8, LA, LB, EPI, C::PAD, false, C::VA, C::VB>),
                           dim3(ceil_div(M, 80), ceil_div(N, 128), 1), dim3(512), 0, s, la, lb, epi, M, N, K, K);
        break;
    case GEMM_SMALL:
        hipLaunchKernelGGL((gemm_mfma_kernel<64, 64, 16, 2, 2, LA, LB, EPI, C::PAD, false, C::VA, C::VB>),
                           dim3(ceil_div(M, 64), ceil_div(N, 64), 1), dim3(256), 0, s, la, lb, epi, M, N, K, K);
        break;
    }
    return hipGetLastError();
}

// C = alpha A B + beta C on the tiles of a square C (M = N) on or below the
// diagonal (64 x 64 tiles); the tiles above it are not touched.
template <class LA, class LB>
hipError_t gemm_mfma_lower(LA la, LB lb, EpiAxpbyLower epi, int N, int K, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    const long T = ceil_div(N, 64);
    hipLaunchKernelGGL((gemm_mfma_kernel<64, 64, 16, 2, 2, LA, LB, EpiAxpbyLower>), dim3((unsigned)(T * (T + 1) / 2), 1, 1),
                       dim3(256), 0, s, la, lb, epi, N, N, K, K);
    return hipGetLastError();
}

// C = A B through EPI (an epilogue with kLowerTiles) on the 128 x 128 tiles of a square C
// (M = N) on or below the diagonal; the tiles above it are not touched.
template <class LA, class LB, class EPI>
hipError_t gemm_mfma_lower_large(LA la, LB lb, EPI epi, int N, int K, hipStream_t s)
{
    static_assert(lower_tiles<EPI>::value, "lower-tile epilogue");
    if (N <= 0) return hipSuccess;
    const long T = ceil_div(N, 128);
    using C = TileCfg<typename LA::value_type>;
    hipLaunchKernelGGL((gemm_mfma_kernel<128, 128, 16, 4, 2, LA, LB, EPI, C::PAD, false, C::VA, C::VB>),
                       dim3((unsigned)(T * (T + 1) / 2), 1, 1), dim3(512), 0, s, la, lb, epi, N, N, K, K);
    return hipGetLastError();
}

// Split-K GEMM: partials go to `work` (splits * M * N doubles), then reduced.
// shape GEMM_SMALL (64 x 64 tiles), GEMM_TALL (128 x 32 tiles, narrow outputs) or GEMM_LARGE.
template <class LA, class LB, class EPI>
hipError_t gemm_mfma_splitk(LA la, LB lb, EPI epi, int M, int N, int K, int splits, double *work, hipStream_t s,
                           GemmShape shape = GEMM_SMALL)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (splits <= 1) return gemm_mfma(shape, la, lb, epi, M, N, K, s);
    int kchunk = ceil_div(ceil_div(K, splits), 16) * 16;
    splits = ceil_div(K, kchunk);
    EpiPartial part{work, M, N};
    using C = TileCfg<typename LA::value_type>;
    if (shape == GEMM_LARGE)
        hipLaunchKernelGGL((gemm_mfma_kernel<128, 128, 16, 4, 2, LA, LB, EpiPartial, C::PAD, false, C::VA, C::VB>),
                           dim3(ceil_div(M, 128), ceil_div(N, 128), splits), dim3(512), 0, s, la, lb, part, M, N, K,
                           kchunk);
    else if (shape == GEMM_TALL)
        hipLaunchKernelGGL((gemm_mfma_kernel<128, 32, 16, 4, 1, LA, LB, EpiPartial, C::PAD, false, C::VA, C::VB>),
                           dim3(ceil_div(M, 128), ceil_div(N, 32), splits), dim3(256), 0, s, la, lb, part, M, N, K,
                           kchunk);
    else
        hipLaunchKernelGGL((gemm_mfma_kernel<64, 64, 16, 2, 2, LA, LB, EpiPartial, C::PAD, false, C::VA, C::VB>),
                           dim3(ceil_div(M, 64), ceil_div(N, 64), splits), dim3(256), 0, s, la, lb, part, M, N, K,
                           kchunk);
    long total = (long)M * N;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(reduce_partials_kernel<EPI>, dim3(blocks), dim3(256), 0, s, work, splits, M, N, epi);
    return hipGetLastError();
}

// The split-bf16 GEMM (FP32 operands, three bf16 products, FP32 accumulation) in the tile
// shape SH (GEMM_LARGE or GEMM_MIX), with an optional split of K (partials in `work`, as in
// gemm_mfma_splitk).
template <GemmShape SH, class LA, class LB, class EPI>
hipError_t gemm_bf16x3(LA la, LB lb, EPI epi, int M, int N, int K, hipStream_t s, int splits = 1,
                       double *work = nullptr)
{
    static_assert(SH == GEMM_LARGE || SH == GEMM_MIX, "tile shape");
    constexpr int BM = SH == GEMM_LARGE ? 128 : 80, WM = SH == GEMM_LARGE ? 4 : 1, WN = SH == GEMM_LARGE ? 2 : 8;
    if (M <= 0 || N <= 0) return hipSuccess;
    if (splits <= 1 || !work) {
        hipLaunchKernelGGL((gemm_bf16x3_kernel<BM, 128, WM, WN, LA, LB, EPI>), dim3(ceil_div(M, BM), ceil_div(N, 128), 1),
                           dim3(512), 0, s, la, lb, epi, M, N, K, K);
        return hipGetLastError();
    }
    const int kchunk = ceil_div(ceil_div(K, splits), 32) * 32;
    splits = ceil_div(K, kchunk);
    EpiPartial part{work, M, N};
    hipLaunchKernelGGL((gemm_bf16x3_kernel<BM, 128, WM, WN, LA, LB, EpiPartial>),
                       dim3(ceil_div(M, BM), ceil_div(N, 128), splits), dim3(512), 0, s, la, lb, part, M, N, K, kchunk);
    const long total = (long)M * N;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(reduce_partials_kernel<EPI>, dim3(blocks), dim3(256), 0, s, work, splits, M, N, epi);
    return hipGetLastError();
}

}  // namespace ctm
