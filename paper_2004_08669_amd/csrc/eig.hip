// Symmetric eigensolver for the extended corner matrix; see eig.h.
#include <float.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "eig.h"
#include "gemm.h"

namespace ctm {

// ============================================================================
// Geometry shared by host and device
// ============================================================================

// Panels of stage 1: panel i covers columns [i*b, i*b + b), its Householder
// vectors act on rows [r0, N) with r0 = i*b + b; panels exist while N - r0 >= 2.
static int num_panels(int N, int b)
{
    int np = 0;
    for (int p = 0; p + b <= N - 2; p += b) ++np;
    return np;
}
__host__ __device__ inline long panel_v_offset(int N, int b, int pi)
{
    long off = 0;
    for (int i = 0; i < pi; ++i) off += (long)(N - (i + 1) * b) * b;
    return off;
}

// Steps of bulge-chasing sweep j (columns j = 0 .. N-3): step t works on rows
// R_t = [r0, r0 + b) with r0 = j + 1 + t b (clipped to N); step 0 always exists and
// step t >= 1 exists while its block has at least two rows: t <= (N - 3 - j) / b.
__host__ __device__ inline int bulge_nsteps(int N, int b, int j) { return 1 + (N - 3 - j) / b; }

static int max_steps(int N, int b) { return N > 2 ? bulge_nsteps(N, b, 0) : 0; }

// ============================================================================
// Stage 1: Householder QR of one panel (all workgroups resident).  Each workgroup holds a
// slice of 128 rows in registers, B / 2 elements per thread.  Per column, every
// workgroup stores its partial products of that column with all columns into
// exchange slots with device-coherent stores, and reads the slots of all the
// others, waiting until none holds the empty marker any more.  There is no
// barrier and no flag: one store and one load separate the columns, and no
// cache is written back or invalidated, so the trailing update running beside
// the panel keeps its caches.  The products with the finished columns give
// V^T v of the compact-WY factor T along the way.
//
// Exchange slots: two sets (launch parity), each [B columns][Gmax workgroups][B]
// partials followed by [B columns][B] copies of panel row i.  A launch fills the
// set of its parity and first returns the other set (filled by the previous
// launch, over its Gprev workgroups) to the marker, so every launch starts on
// an empty set.  Launches on one workspace run one after another.
// ============================================================================

static inline int pqr_rows(int) { return 128; }
static inline int pqr_gmax(int Nmax, int b) { return (Nmax + pqr_rows(b) - 1) / pqr_rows(b); }
__host__ __device__ inline size_t pqr_slot_set(int b, int Gmax) { return (size_t)b * Gmax * b + (size_t)b * b; }

// The empty marker: all bits set (a NaN that arithmetic never produces; computed
// NaNs are stored as the default quiet NaN).
#define PQR_EMPTY (-1LL)

CTMRG_DEVINL bool pqr_empty(double v) { return __double_as_longlong(v) == PQR_EMPTY; }
CTMRG_DEVINL double pqr_publishable(double v) { return v == v ? v : __longlong_as_double(0x7FF8000000000000LL); }

// Value of column i in the caller's row: lanes are grouped B to a row, lane c of a
// group holds column c.
template <int B>
CTMRG_DEVINL double col_bcast(double v, int i, int lane)
{
    if constexpr (B == 32) {
        const int lo = __double2loint(v), hi = __double2hiint(v);
        const int l0 = __builtin_amdgcn_readlane(lo, i), h0 = __builtin_amdgcn_readlane(hi, i);
        const int l1 = __builtin_amdgcn_readlane(lo, i + 32), h1 = __builtin_amdgcn_readlane(hi, i + 32);
        return (lane & 32) ? __hiloint2double(h1, l1) : __hiloint2double(h0, l0);
    } else {
        return __shfl(v, (lane & ~(B - 1)) + i, 64);
    }
}

// Panel columns [p, p + B) of A, rows [r0, r0 + n).  On return the panel holds R on
// and above its diagonal and the Householder vectors below it (unit diagonal
// implied); Vx (n x B, row-major) holds V explicitly, tau_out the B scalars and
// T_out the upper-triangular B x B factor with Q = I - V T V^T.
template <int B>
__global__ void __launch_bounds__(256)
panel_qr_kernel(double *A, long lda, int r0, int p, int n, double *Vx, double *tau_out, double *T_out,
                double *slots, int Gmax, int parity, int Gprev, unsigned *err)
{
    constexpr int RG = 256 / B;    // row groups
    constexpr int KR = B / 2;      // rows per thread: local rows rg + RG k
    constexpr int ROWS = RG * KR;  // 128
    __shared__ double red[4][B];
    __shared__ double rowl[B];
    __shared__ double red2[RG][B];
    __shared__ double gram[B][B + 1];
    __shared__ double tl[B];

    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int c = tid & (B - 1), rg = tid / B;
    const int row0 = g * ROWS;
    const int nloc = min(ROWS, n - row0);
    const long set = (long)pqr_slot_set(B, Gmax);
    double *part = slots + parity * set;       // [B][Gmax][B]
    double *rowv = part + (long)B * Gmax * B;  // [B][B]

    // the previous launch's set back to empty
    {
        double *old = slots + (parity ^ 1) * set;
        const long used = (long)Gprev * B;
        for (long idx = (long)g * 256 + tid; idx < (long)B * used; idx += (long)G * 256) {
            const long ii = idx / used;
            st_coh(&old[ii * Gmax * B + (idx - ii * used)], __longlong_as_double(PQR_EMPTY));
        }
        if (g == 0)
            for (int idx = tid; idx < B * B; idx += 256)
                st_coh(&old[(long)B * Gmax * B + idx], __longlong_as_double(PQR_EMPTY));
    }

    double x[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int r = rg + RG * k;
        x[k] = (r < nloc) ? A[(long)(r0 + row0 + r) * lda + p + c] : 0.0;
    }

    for (int i = 0; i < B; ++i) {
        double *part_i = part + (long)i * Gmax * B;
        double *rowv_i = rowv + i * B;
        // column i in every row, and this thread's share of sum_{rows > i} a_ri a_rc
        double y[KR];
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            y[k] = col_bcast<B>(x[k], i, lane);
            if (row0 + rg + RG * k > i) t += y[k] * x[k];
        }
#pragma unroll
        for (int o = B; o < 64; o <<= 1) t += __shfl_xor(t, o, 64);
        if (lane < B) red[wave][c] = t;
        if (g == 0 && rg == i % RG) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < (B + RG - 1) / RG; ++k)
                if (k == i / RG) v = x[k];
            rowl[c] = v;
        }
        __syncthreads();
        // publish this workgroup's partials (and row i, from workgroup 0)
        if (wave == 0 && lane < B) {
            st_coh(&part_i[(long)g * B + c], pqr_publishable(red[0][c] + red[1][c] + red[2][c] + red[3][c]));
            if (g == 0) st_coh(&rowv_i[c], pqr_publishable(rowl[c]));
        }
        // gather: row group rg adds workgroups rg, rg + RG, ... (the same order everywhere),
        // reading again until no slot it needs is empty
        double ts, arow, alpha;
        {
            unsigned spins = 0;
            for (;;) {
                bool full = true;
                ts = 0.0;
                int gg = rg;
                for (; gg + 3 * RG < G; gg += 4 * RG) {
                    const double v0 = ld_coh(&part_i[(long)gg * B + c]);
                    const double v1 = ld_coh(&part_i[(long)(gg + RG) * B + c]);
                    const double v2 = ld_coh(&part_i[(long)(gg + 2 * RG) * B + c]);
                    const double v3 = ld_coh(&part_i[(long)(gg + 3 * RG) * B + c]);
                    full = full && !pqr_empty(v0) && !pqr_empty(v1) && !pqr_empty(v2) && !pqr_empty(v3);
                    ts += (v0 + v1) + (v2 + v3);
                }
                for (; gg < G; gg += RG) {
                    const double v = ld_coh(&part_i[(long)gg * B + c]);
                    full = full && !pqr_empty(v);
                    ts += v;
                }
                arow = ld_coh(&rowv_i[c]);
                alpha = ld_coh(&rowv_i[i]);
                full = full && !pqr_empty(arow) && !pqr_empty(alpha);
                if (__all(full)) break;
                __builtin_amdgcn_s_sleep(1);
                if (++spins > CTMRG_SPIN_LIMIT) {
                    if (lane == 0) raise_error(err, KERR_WAIT_TIMEOUT);
                    break;
                }
            }
        }
        red2[rg][c] = ts;
        __syncthreads();
        double Sc = 0.0, Si = 0.0;
#pragma unroll
        for (int k = 0; k < RG; ++k) {
            Sc += red2[k][c];
            Si += red2[k][i];
        }
        // reflector of column i (every thread of every workgroup computes the same values)
        double beta, tau, scale;
        if (Si == 0.0) {
            beta = alpha; tau = 0.0; scale = 0.0;
        } else {
            beta = -copysign(sqrt(alpha * alpha + Si), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        const double wc = arow + scale * Sc;  // v_i^T a_c; for c < i this is (V^T V)[c][i]
        if (g == 0) {
            if (rg == 0 && c < i) gram[c][i] = wc;
            if (tid == 0) tl[i] = tau;
        }
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int gr = row0 + rg + RG * k;
            if (c > i) {
                if (gr >= i) x[k] -= tau * ((gr == i) ? 1.0 : y[k] * scale) * wc;
            } else if (c == i) {
                if (gr == i) x[k] = beta;
                else if (gr > i) x[k] = y[k] * scale;
            }
        }
    }

    // R and V back to the panel, and the explicit V
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int r = rg + RG * k, gr = row0 + r;
        if (r < nloc) {
            A[(long)(r0 + gr) * lda + p + c] = x[k];
            Vx[(long)gr * B + c] = (gr == c) ? 1.0 : (gr > c ? x[k] : 0.0);
        }
    }
    if (g != 0) return;
    __syncthreads();
    // T (upper triangular), row j by thread j: T[j][j] = tau_j and, for i > j,
    // T[j][i] = -tau_i sum_{l < i} T[j][l] (V^T V)[l][i]
    if (tid < B) {
        const int j = tid;
        double trow[B];
#pragma unroll
        for (int l = 0; l < B; ++l) trow[l] = (l == j) ? tl[l] : 0.0;
#pragma unroll
        for (int ii = 1; ii < B; ++ii) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < ii; ++l) s += trow[l] * gram[l][ii];
            if (ii > j) trow[ii] = -tl[ii] * s;
        }
#pragma unroll
        for (int l = 0; l < B; ++l) T_out[j * B + l] = trow[l];
        tau_out[j] = tl[j];
    }
}

// The two-sided update of a panel needs W = X - 1/2 V S with X = Y T and
// S = T^T V^T X = T^T (V^T Y) T, i.e. W = [Y | V] [T ; -1/2 S]:
//  * vty_partial_kernel: partial sums of V^T Y (b x b) on the matrix cores, one per
//    workgroup over rows strided by the grid (k-steps of 4 rows);
//  * wy_small_kernel (one workgroup): M0 = sum of the partials, S = T^T M0 T, and
//    the 2b x b right factor [T ; -1/2 S];
//  * one GEMM [Y | V] [T ; -1/2 S] whose epilogue writes [V | W] and [W | V].
constexpr int VTY_WG = 64;

template <int B>
__global__ void __launch_bounds__(256) vty_partial_kernel(const double *V, const double *Y, int n, double *part)
{
    using MF = Mfma<double>;
    constexpr int TB = B / 16;
    // b = 32: wave w forms output block (w / 2, w % 2); b = 16: the one output block, each wave
    // over its own rows (RS row streams per workgroup), the four sums added in LDS in wave order
    constexpr int RS = TB == 1 ? 4 : 1;
    __shared__ double red[RS][16][17];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (TB == 2 && wave >= TB * TB) return;
    const int I = TB == 1 ? 0 : wave / TB, J = TB == 1 ? 0 : wave % TB;
    const int lr = lane >> 4, lc = lane & 15;
    MF::acc_t acc = MF::zero();
    const int stride = gridDim.x * 4 * RS;
    int r0 = (blockIdx.x * RS + (RS == 1 ? 0 : wave)) * 4;
    for (; r0 + 7 * stride + 4 <= n; r0 += 8 * stride) {
        double a[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long r = r0 + u * stride + lr;
            a[u] = V[r * B + 16 * I + lc];
            y[u] = Y[r * B + 16 * J + lc];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = MF::mma(a[u], y[u], acc);
    }
    for (; r0 < n; r0 += stride) {
        const int r = r0 + lr;
        const double a = r < n ? V[(long)r * B + 16 * I + lc] : 0.0;
        const double y = r < n ? Y[(long)r * B + 16 * J + lc] : 0.0;
        acc = MF::mma(a, y, acc);
    }
    double *dst = part + (long)blockIdx.x * B * B;
    if constexpr (RS == 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) dst[(16 * I + lr + 4 * j) * B + 16 * J + lc] = acc[j];
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) red[wave][lr + 4 * j][lc] = acc[j];
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = lr + 4 * j;
                dst[r * B + lc] = ((red[0][r][lc] + red[1][r][lc]) + red[2][r][lc]) + red[3][r][lc];
            }
        }
    }
}

__global__ void __launch_bounds__(1024) wy_small_kernel(const double *part, int nparts, const double *T, int b,
                                                        double *B2)
{
    __shared__ double M0[32][33], Ts[32][33], Mt[32][33];
    const int tid = threadIdx.x;
    const int i = tid / b, j = tid - (tid / b) * b;
    const bool act = tid < b * b;
    if (act) {
        // the partials' loads 32 at a time in flight (nparts <= VTY_WG), summed in a fixed order
        double sum = 0.0;
#pragma unroll 1
        for (int g0 = 0; g0 < VTY_WG; g0 += 32) {
            double v[32];
#pragma unroll
            for (int g = 0; g < 32; ++g) v[g] = g0 + g < nparts ? part[(long)(g0 + g) * b * b + tid] : 0.0;
#pragma unroll
            for (int g = 0; g < 32; ++g) sum += v[g];
        }
        M0[i][j] = sum;
        Ts[i][j] = T[tid];
    }
    __syncthreads();
    if (act) {  // Mt = M0 T
        double t = 0.0;
        for (int k = 0; k < b; ++k) t += M0[i][k] * Ts[k][j];
        Mt[i][j] = t;
    }
    __syncthreads();
    if (act) {  // S = T^T Mt; B2 = [T ; -S/2]
        double t = 0.0;
        for (int k = 0; k < b; ++k) t += Ts[k][i] * Mt[k][j];
        B2[tid] = Ts[i][j];
        B2[b * b + tid] = -0.5 * t;
    }
}

// [Y | V] as one n x 2b operand
struct A_YV {
    using value_type = double;
    const double *Y; const double *V; int b;
    static constexpr bool kContigK = true;
    __device__ double operator()(int i, int k) const { return k < b ? Y[(long)i * b + k] : V[(long)i * b + k - b]; }
};
// Writes [V | W] and [W | V] from W = acc
struct EpiVW {
    const double *V; double *VW; double *WV; int b;
    __device__ void operator()(int i, int j, double w, int) const
    {
        const double v = V[(long)i * b + j];
        VW[(long)i * 2 * b + j] = v;
        VW[(long)i * 2 * b + b + j] = w;
        WV[(long)i * 2 * b + j] = w;
        WV[(long)i * 2 * b + b + j] = v;
    }
};

// b = 16: W = [Y | V] sm (sm = [T ; -1/2 S], 2b x b), the operands [V | W] and [W | V],
// and, when cols is set, the update of the next panel's columns,
// A22[:, 0:b] -= [V | W] [W | V][0:b, :]^T, in one launch.  Every workgroup forms W of
// rows 0..b-1 itself (a b x 2b by 2b x b product), so no workgroup waits for another.
// Workgroup: 32 rows, two elements of each product per thread.
__global__ void __launch_bounds__(256)
vw_cols16_kernel(const double *Y, const double *V, const double *sm, int n, int cols, double *VW, double *WV,
                 double *A22, long lda)
{
    constexpr int B = 16, TR = 32;
    __shared__ double S[2 * B][B];
    __shared__ double W0[B][B + 1];
    __shared__ double V0[B][B + 1];
    __shared__ double Wt[TR][B + 1];
    __shared__ double Vt[TR][B + 1];
    const int tid = threadIdx.x, i0 = blockIdx.x * TR;
    for (int idx = tid; idx < 2 * B * B; idx += 256) S[idx / B][idx % B] = sm[idx];
    {
        const int r = tid / B, c = tid % B;
        V0[r][c] = (r < n) ? V[(long)r * B + c] : 0.0;
    }
    for (int idx = tid; idx < TR * B; idx += 256) {
        const int r = idx / B, c = idx % B;
        Vt[r][c] = (i0 + r < n) ? V[(long)(i0 + r) * B + c] : 0.0;
    }
    __syncthreads();
    {
        const int r = tid / B, c = tid % B;
        double w = 0.0;
        if (r < n) {
#pragma unroll
            for (int k = 0; k < B; ++k) w += Y[(long)r * B + k] * S[k][c];
#pragma unroll
            for (int k = 0; k < B; ++k) w += V0[r][k] * S[B + k][c];
        }
        W0[r][c] = w;
    }
    // W of the tile's rows: thread (r, c) for r = tid / 16 and r + 16
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = tid / B + 16 * h, c = tid % B, i = i0 + r;
        double w = 0.0;
        if (i < n) {
#pragma unroll
            for (int k = 0; k < B; ++k) w += Y[(long)i * B + k] * S[k][c];
#pragma unroll
            for (int k = 0; k < B; ++k) w += Vt[r][k] * S[B + k][c];
            const double v = Vt[r][c];
            VW[(long)i * 2 * B + c] = v;
            VW[(long)i * 2 * B + B + c] = w;
            WV[(long)i * 2 * B + c] = w;
            WV[(long)i * 2 * B + B + c] = v;
        }
        Wt[r][c] = w;
    }
    if (!cols) return;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = tid / B + 16 * h, c = tid % B, i = i0 + r;
        if (i < n) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < B; ++k) a += Vt[r][k] * W0[c][k];
#pragma unroll
            for (int k = 0; k < B; ++k) a += Wt[r][k] * V0[c][k];
            A22[(long)i * lda + c] -= a;
        }
    }
}

// Lower band (r - c in [0, b]) of the stage-1 result into column-major band
// storage with 2b diagonals (the upper b hold the bulges of stage 2).
__global__ void extract_band_kernel(const double *A, long lda, int N, int b, double *band)
{
    const int ld = 2 * b;
    const long total = (long)N * ld;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int c = (int)(idx / ld), k = (int)(idx - (long)c * ld);
        band[idx] = (k <= b && c + k < N) ? A[(long)(c + k) * lda + c] : 0.0;
    }
}

// ============================================================================
// Stage 2: bulge chasing (band to tridiagonal)
// ============================================================================
// Orders this wave's LDS accesses (the LDS unit serves one wave in order).
CTMRG_DEVINL void lane_sync()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// A double moved across lanes by one DPP pattern (both halves with the same control).
template <int CTRL>
CTMRG_DEVINL double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Sum over the 64 lanes of a wave, the same value in every lane: inside each row of
// 16 lanes by DPP (partner lane xor 1, xor 2, then the mirror images within 8 and
// within 16 lanes), then across the rows by two shuffles.  Every lane adds the same
// two operands at every level, so all lanes hold bitwise the same sum.
CTMRG_DEVINL double wave_sum_dpp(double v)
{
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Sum of RPL products x[i] y[i] in four independent chains.
template <int RPL>
CTMRG_DEVINL double dot4(const double *x, const double *y)
{
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < RPL; ++i) a[i & 3] = fma(x[i], y[i], a[i & 3]);
    return (a[0] + a[1]) + (a[2] + a[3]);
}

template <int B>
CTMRG_DEVINL double col_sum(double x)  // over the lanes sharing lane % B
{
    for (int off = B; off < 64; off <<= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// ---------------------------------------------------------------------------
// One bulge-chasing step (sweep j, step t), executed by one wave.  The three
// b x b blocks of the step (the left block whose first column is annihilated,
// the symmetric diagonal block, the block below that receives the new bulge)
// are held in registers and all loaded at the start, so a step costs one
// memory round trip: lane (c, h) = (lane % b, lane / b) owns column c, rows
// h*RPL .. h*RPL + RPL - 1 of the left and diagonal blocks, and row c, columns
// h*RPL .. h*RPL + RPL - 1 of the block below, so that every product with the
// reflector sums within a lane and then over the LPC lanes sharing c.
// vs and ws are two b-element LDS vectors private to the wave.
// ---------------------------------------------------------------------------
template <int B>
CTMRG_DEVINL void bulge_step_pre(double *band, int N, int j, int t, double *refl, double *rtau, int Tmax, double *vs,
                                 double *ws)
{
    constexpr int LPC = 64 / B;
    constexpr int RPL = B / LPC;
    const int lane = threadIdx.x & 63;
    const int c = lane % B, h = lane / B, rb = h * RPL;
    const int ld = 2 * B;
    int r0, c0, ncl;
    if (t == 0) { r0 = j + 1; c0 = j; ncl = 1; }
    else { r0 = j + 1 + t * B; c0 = j + 1 + (t - 1) * B; ncl = B; }
    const int len = min(r0 + B, N) - r0;
    const int n0 = r0 + len, nbl = min(n0 + B, N) - n0;
    const long safe = (long)r0 * ld;  // an in-bounds address for masked-off lanes
    double L[RPL], D[RPL], Bm[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int r = rb + i;
        const bool okl = (c < ncl && r < len);
        const bool okd = (r < len && c < len);
        const bool okb = (c < nbl && r < len);
        const long offd = (r >= c) ? (long)(r0 + c) * ld + (r - c) : (long)(r0 + r) * ld + (c - r);
        const double xl = band[okl ? (long)(c0 + c) * ld + (r0 + r - c0 - c) : safe];
        const double xd = band[okd ? offd : safe];
        const double xb = band[okb ? (long)(r0 + r) * ld + (n0 + c - r0 - r) : safe];
        L[i] = okl ? xl : 0.0;
        D[i] = okd ? xd : 0.0;
        Bm[i] = okb ? xb : 0.0;
    }
    // Householder vector from column 0 of the left block
    const double alpha = __shfl(L[0], 0, 64);
    double part = 0.0;
    if (c == 0) {
        double Lm[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) Lm[i] = (rb + i >= 1) ? L[i] : 0.0;
        part = dot4<RPL>(Lm, Lm);
    }
    const double xs = wave_sum_dpp(part);
    double beta, tau, scale;
    if (xs == 0.0) { beta = alpha; tau = 0.0; scale = 0.0; }
    else {
        beta = -copysign(sqrt(alpha * alpha + xs), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
    // Every band load has arrived before the first store of the step: the vector
    // memory counter covers loads and stores alike, so a late wait for a load would
    // also wait for the reflector stores issued before it.
    __builtin_amdgcn_s_waitcnt(0);
    if (c == 0) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = rb + i;
            const double vr = (r >= len) ? 0.0 : (r == 0 ? 1.0 : L[i] * scale);
            vs[r] = vr;
            refl[((long)j * Tmax + t) * B + r] = vr;
            L[i] = (r == 0) ? beta : 0.0;
        }
    }
    if (lane == 0) rtau[(long)j * Tmax + t] = tau;
    lane_sync();
    const double vc = vs[c];
    // left block, columns >= 1: L[:,c] -= tau v (v^T L[:,c])
    {
        double vl[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) vl[i] = vs[rb + i];
        const double wc = tau * col_sum<B>(dot4<RPL>(vl, L));
        if (c >= 1) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) L[i] -= wc * vs[rb + i];
        }
    }
    // diagonal block: p = tau D v, k = tau v^T p / 2, w = p - k v, D -= v w^T + w v^T
    double vr[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) vr[i] = vs[rb + i];
    const double pc = tau * col_sum<B>(dot4<RPL>(D, vr));
    const double kk = 0.5 * tau * wave_sum_dpp((h == 0 && c < len) ? vc * pc : 0.0);
    const double wc = pc - kk * vc;
    if (h == 0) ws[c] = (c < len) ? wc : 0.0;
    lane_sync();
#pragma unroll
    for (int i = 0; i < RPL; ++i) D[i] -= vs[rb + i] * wc + ws[rb + i] * vc;
    // block below, held transposed (lane (c, h) has row c, columns rb..rb+RPL-1):
    // y = B v, B -= tau y v^T
    {
        const double ty = tau * col_sum<B>(dot4<RPL>(Bm, vr));
#pragma unroll
        for (int i = 0; i < RPL; ++i) Bm[i] -= ty * vs[rb + i];
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int r = rb + i;
        if (c < ncl && r < len) band[(long)(c0 + c) * ld + (r0 + r - c0 - c)] = L[i];
        if (r < len && c < len && r >= c) band[(long)(r0 + c) * ld + (r - c)] = D[i];
        if (c < nbl && r < len) band[(long)(r0 + r) * ld + (n0 + c - r0 - r)] = Bm[i];
    }
}

// Wavefront form: the steps (j, t) with 3 j + t = tau are mutually independent
// (a sweep trails its predecessor by three steps), so one launch per tau runs
// them all, one wave per step; kernel boundaries order the launches.
template <int B>
__global__ void __launch_bounds__(64)
bulge_front_kernel(double *band, int N, int tau, int jlo, double *refl, double *rtau, int Tmax)
{
    __shared__ double vsh[B], wsh[B];
    const int j = jlo + blockIdx.x;
    const int t = tau - 3 * j;
    if (j > N - 3 || t < 0 || t >= bulge_nsteps(N, B, j)) return;
    bulge_step_pre<B>(band, N, j, t, refl, rtau, Tmax, vsh, wsh);
}

// The same wavefront order for a band small enough to live in LDS (one workgroup): the band
// is loaded once, the steps of each tau run on the workgroup's waves, a workgroup barrier
// separates consecutive tau (it orders the LDS accesses as kernel boundaries order the
// launches above), and the band is written back at the end.  Each step is the same
// arithmetic in the same order as in bulge_front_kernel, so the results are identical; what
// goes away is one launch per tau.  Dynamic LDS: (N 2B + 2 * 16 B) doubles.
template <int B>
__global__ void __launch_bounds__(1024)
bulge_lds_kernel(double *band, int N, double *refl, double *rtau, int Tmax)
{
    extern __shared__ double smem[];
    const int ld = 2 * B;
    const long total = (long)N * ld;
    double *sb = smem;
    double *vsh = smem + total, *wsh = vsh + 16 * B;
    for (long i = threadIdx.x; i < total; i += blockDim.x) sb[i] = band[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int taumax = 3 * (N - 3) + bulge_nsteps(N, B, N - 3);
    for (int tau = 0; tau < taumax; ++tau) {
        const int jhi = min(tau / 3, N - 3);
        const int jlo = max(0, (tau - (Tmax - 1)) / 3);
        for (int j = jlo + wave; j <= jhi; j += nw) {
            const int t = tau - 3 * j;
            if (t >= 0 && t < bulge_nsteps(N, B, j))
                bulge_step_pre<B>(sb, N, j, t, refl, rtau, Tmax, vsh + wave * B, wsh + wave * B);
        }
        __syncthreads();
    }
    for (long i = threadIdx.x; i < total; i += blockDim.x) band[i] = sb[i];
}

size_t bulge_lds_bytes(int N, int b) { return sizeof(double) * ((size_t)N * 2 * b + 2 * 16 * (size_t)b); }

__global__ void band_to_tridiag_kernel(const double *band, int N, int b, double *d, double *e, double *e2)
{
    const int ld = 2 * b;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        d[c] = band[(long)c * ld];
        const double ec = (c < N - 1) ? band[(long)c * ld + 1] : 0.0;
        e[c] = ec;
        e2[c] = ec * ec;
    }
}

// ============================================================================
// Eigenvalues: Sturm-count bisection
// ============================================================================

// bounds[0..3] = Gershgorin lower, upper, pivmin, ||T|| (max |row sum|)
__global__ void __launch_bounds__(256) tridiag_bounds_kernel(const double *d, const double *e, int N, double *bounds)
{
    __shared__ double red[4];
    double lo = DBL_MAX, hi = -DBL_MAX, emax2 = 0.0;
    for (int i = threadIdx.x; i < N; i += 256) {
        const double el = (i > 0) ? fabs(e[i - 1]) : 0.0;
        const double er = (i < N - 1) ? fabs(e[i]) : 0.0;
        lo = fmin(lo, d[i] - el - er);
        hi = fmax(hi, d[i] + el + er);
        emax2 = fmax(emax2, er * er);
    }
    lo = -block_max<256>(-lo, red);
    hi = block_max<256>(hi, red);
    emax2 = block_max<256>(emax2, red);
    if (threadIdx.x == 0) {
        const double tn = fmax(fabs(lo), fabs(hi));
        const double slack = 2.0 * DBL_EPSILON * tn + DBL_MIN;
        bounds[0] = lo - slack;
        bounds[1] = hi + slack;
        bounds[2] = DBL_MIN * fmax(1.0, emax2);
        bounds[3] = tn;
    }
}

// Sturm counts of T - x_v I for S shifts at once: the number of negative pivots of
// the LDL^T recurrence q_i = d_i - x - e_{i-1}^2 / q_{i-1} (a tiny pivot is replaced
// by -pivmin).  e2 / q takes the hardware reciprocal and one Newton step: an ulp or
// two, a relative perturbation of e2 of that size, far inside the count's backward
// error.  d and e2 are read in chunks of 16 (the same address in every lane), the
// next chunk's loads issued before the current chunk's recurrence runs.
template <int S>
CTMRG_DEVINL void sturm_counts(const double *d, const double *e2, int N, const double (&x)[S], double pivmin,
                               int (&cnt)[S])
{
    constexpr int C = 16;
    double q[S];
#pragma unroll
    for (int v = 0; v < S; ++v) {
        q[v] = d[0] - x[v];
        cnt[v] = q[v] < 0.0 ? 1 : 0;
    }
    double da[C], ea[C], db[C], eb[C];
    auto load = [&](double (&dd)[C], double (&ee)[C], int i0) {
#pragma unroll
        for (int u = 0; u < C; ++u) {
            const int i = min(i0 + u, N - 1);
            dd[u] = d[i];
            ee[u] = e2[i - 1];
        }
    };
    auto run = [&](const double (&dd)[C], const double (&ee)[C], int i0) {
        const int nI = min(C, N - i0);
#pragma unroll
        for (int u = 0; u < C; ++u) {
            if (u < nI) {
#pragma unroll
                for (int v = 0; v < S; ++v) {
                    double qq = q[v];
                    if (fabs(qq) < pivmin) qq = -pivmin;
                    double r = __builtin_amdgcn_rcp(qq);
                    r = fma(r, fma(-qq, r, 1.0), r);
                    qq = dd[u] - x[v] - ee[u] * r;
                    cnt[v] += qq < 0.0 ? 1 : 0;
                    q[v] = qq;
                }
            }
        }
    };
    int i0 = 1;
    if (i0 < N) load(da, ea, i0);
    while (i0 < N) {
        if (i0 + C < N) load(db, eb, i0 + C);
        run(da, ea, i0);
        i0 += C;
        if (i0 >= N) break;
        if (i0 + C < N) load(da, ea, i0 + C);
        run(db, eb, i0);
        i0 += C;
    }
}

// Spectrum slicing: Sturm counts at two sorted point sets of BIS_SLICE points
// each, one lane per point.  Set 0 is uniform on [lo, hi]; set 1 is geometric
// about zero, +-tn 2^(-s j) down to 2^-46 tn, so that small eigenvalues start
// from a bracket of relative width 1.6%.  bisect_kernel starts eigenvalue k from
// the tighter of the two brackets [x_j, x_j+1) with count(x_j) <= k < count(x_j+1).
constexpr int BIS_SLICE = 4096;

CTMRG_DEVINL double slice_point(int g, const double *bounds)
{
    const double lo = bounds[0], hi = bounds[1], tn = bounds[3];
    const int set = g / BIS_SLICE, j = g - set * BIS_SLICE;
    if (set == 0) return lo + (double)(j + 1) * ((hi - lo) / (double)(BIS_SLICE + 1));
    constexpr int half = BIS_SLICE / 2;
    const double step = 46.0 / (double)(half - 1);
    return j < half ? -tn * exp2(-step * (double)j) : tn * exp2(-step * (double)(half - 1 - (j - half)));
}

__global__ void __launch_bounds__(256) bisect_slice_kernel(const double *d, const double *e2, int N, const double *bounds,
                                                           double *xs, int *cnt)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 2 * BIS_SLICE) return;
    const double pivmin = bounds[2];
    const double x[1] = {slice_point(g, bounds)};
    int c[1];
    sturm_counts<1>(d, e2, N, x, pivmin, c);
    xs[g] = x[0];
    cnt[g] = c[0];
}

// Narrow [lo, hi) for eigenvalue k with one sorted set of slice points (counts
// non-decreasing); a set whose counts disagree around k is ignored.
CTMRG_DEVINL void slice_bracket(const double *xs, const int *cnt, int k, double &lo, double &hi)
{
    int a = -1, b = BIS_SLICE;  // cnt[a] <= k < cnt[b], with a = -1 and b = BIS_SLICE the ends
    while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (cnt[mid] <= k) a = mid;
        else b = mid;
    }
    if (a >= 0 && cnt[a] <= k) lo = fmax(lo, xs[a]);
    if (b < BIS_SLICE && cnt[b] > k) hi = fmin(hi, xs[b]);
}

// Multisection by groups of lanes: LPE lanes work on one eigenvalue index k and
// each evaluates S Sturm counts per pass (their recurrences interleave), so one
// pass over T splits the bracket at LPE*S points and gains log2(LPE*S + 1) bits.
// The group then keeps the sub-interval [largest point with count <= k,
// smallest point with count > k).  All lanes of a wave read the same d[i],
// e2[i] (one broadcast load per wave).
template <int LPE, int S>
__global__ void __launch_bounds__(256) bisect_kernel(const double *d, const double *e2, int N, const double *bounds,
                                                     const double *xs, const int *cnts, double *evals)
{
    constexpr int P = LPE * S;
    const int lane = threadIdx.x & 63;
    const int sub = lane % LPE;
    const int k = (int)((blockIdx.x * (long)blockDim.x + threadIdx.x) / LPE);
    const bool active = k < N;
    double lo = bounds[0], hi = bounds[1];
    if (active) {
        slice_bracket(xs, cnts, k, lo, hi);
        slice_bracket(xs + BIS_SLICE, cnts + BIS_SLICE, k, lo, hi);
        if (!(lo < hi)) { lo = bounds[0]; hi = bounds[1]; }
    }
    const double pivmin = bounds[2], tn = bounds[3];
    const double abstol = DBL_EPSILON * tn;
    bool done = !active;
    for (int it = 0; it < 64; ++it) {
        if (!done && hi - lo <= fmax(abstol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)))) done = true;
        // the whole wave stops when every group has
        if (__all(done)) break;
        const double w = (hi - lo) / (double)(P + 1);
        double x[S];
        int cnt[S];
#pragma unroll
        for (int u = 0; u < S; ++u) x[u] = fmin(hi, lo + (double)(sub * S + u + 1) * w);
        sturm_counts<S>(d, e2, N, x, pivmin, cnt);
        // eigenvalue k lies in [x_a, x_b) with x_a the largest point of count <= k, x_b the smallest of count > k
        double nlo = lo, nhi = hi;
#pragma unroll
        for (int u = 0; u < S; ++u) {
            if (cnt[u] <= k) nlo = fmax(nlo, x[u]);
            else nhi = fmin(nhi, x[u]);
        }
#pragma unroll
        for (int off = 1; off < LPE; off <<= 1) {
            nlo = fmax(nlo, __shfl_xor(nlo, off, 64));
            nhi = fmin(nhi, __shfl_xor(nhi, off, 64));
        }
        if (!done) {
            if (nlo == lo && nhi == hi) done = true;  // no representable point splits the bracket
            lo = nlo;
            hi = nhi;
        }
    }
    if (active && sub == 0) evals[k] = 0.5 * (lo + hi);
}

// ============================================================================
// Selection, cut, normalization, entropy, convergence (one workgroup)
// ============================================================================

__global__ void __launch_bounds__(256)
post_eigen_kernel(const double *ev, int N, int m, double gap_tol, double rank_tol, const double *om4_prev,
                  double *omega_new, double *selval, int *selpos, int *clist, int *cstart, PostOut *out)
{
    __shared__ double red[4];
    __shared__ int s_me, s_nb;
    __shared__ double s_l1;
    const int tid = threadIdx.x;
    const int kk = min(m + 1, N);
    if (tid == 0) {
        // merge from both ends of the ascending list: descending |lambda|, ties to the larger lambda
        int hi = N - 1, lo = 0, nb = 0;
        for (int q = 0; q < kk; ++q) {
            int pick;
            if (lo > hi) break;
            const double a = fabs(ev[hi]), c = fabs(ev[lo]);
            if (a >= c) { pick = hi; --hi; }
            else { pick = lo; ++lo; }
            selval[q] = ev[pick];
            selpos[q] = pick;
        }
        const double l1 = fabs(selval[0]);
        const int jmax = min(m, N);
        int me = -1;
        for (int j = jmax; j >= 1; --j) {
            const double aj = fabs(selval[j - 1]);
            if (aj <= rank_tol * l1) continue;
            if (j == N || aj - fabs(selval[j]) > gap_tol * l1) { me = j; break; }
        }
        if (me < 0) {
            int c = 0;
            for (int j = 0; j < jmax; ++j) c += (fabs(selval[j]) > rank_tol * l1) ? 1 : 0;
            me = max(1, c);
        }
        // the kept set in ascending-eigenvalue order is the bottom run [0, nb) of the
        // ascending list followed by the top run [N - nt, N); bottom picks come in the order 0, 1, 2, ...
        {
            int l = 0, bc = 0;
            for (int q = 0; q < me; ++q) {
                if (selpos[q] == l) { ++l; ++bc; }
            }
            nb = bc;
        }
        const int nt = me - nb;
        for (int q = 0; q < me; ++q) {
            const int pos = selpos[q];
            const int slot = (pos < nb) ? pos : nb + (pos - (N - nt));
            clist[slot] = q;
        }
        int ncl = 0;
        cstart[0] = 0;
        for (int s = 1; s <= me; ++s) {
            bool split = true;
            if (s < me) {
                const int pa = selpos[clist[s - 1]], pb = selpos[clist[s]];
                split = !(pb == pa + 1 && ev[pb] - ev[pa] <= 1e-10 * l1);
            }
            if (split) cstart[++ncl] = s;
        }
        s_me = me;
        s_nb = ncl;
        s_l1 = l1;
        out->m_eff = me;
        out->nclusters = ncl;
        out->lam1 = l1;
    }
    __syncthreads();
    const double l1 = s_l1;
    const int me = s_me;
    double s4 = 0.0, rk = 0.0;
    for (int i = tid; i < N; i += 256) {
        const double x = ev[i] / l1;
        s4 += (x * x) * (x * x);
        rk += (fabs(ev[i]) > rank_tol * l1) ? 1.0 : 0.0;
    }
    s4 = block_sum<256>(s4, red);
    rk = block_sum<256>(rk, red);
    const double nC = l1 * sqrt(sqrt(s4));
    double se = 0.0;
    for (int i = tid; i < N; i += 256) {
        const double wv = ev[i] / nC;
        const double w4 = (wv * wv) * (wv * wv);
        if (w4 > 0.0) se -= w4 * log(w4);
    }
    se = block_sum<256>(se, red);
    double dl = 0.0, kept4 = 0.0;
    for (int j = tid; j < m; j += 256) {
        const double om = (j < me) ? selval[j] / nC : 0.0;
        omega_new[j] = om;
        const double o4 = (om * om) * (om * om);
        kept4 += o4;
        const double op = om4_prev[j];
        dl = fmax(dl, fabs(o4 - (op * op) * (op * op)));
    }
    dl = block_max<256>(dl, red);
    kept4 = block_sum<256>(kept4, red);
    if (tid == 0) {
        out->n_C = nC;
        out->S_E = se;
        out->delta = dl;
        out->rank = (int)rk;
        out->sum_w4_kept = kept4;
        out->tail_bound = 0.0;
    }
}

// ============================================================================
// Eigenvectors of the tridiagonal: inverse iteration
// ============================================================================

// One wave per kept eigenvalue.  The pivoted LU of T - lambda I and the two
// triangular solves of each iteration are recurrences along the rows; the wave
// walks them in chunks of 64 rows.  Lane l loads the operands of row r0 + l
// (one coalesced load per array, the next chunk's loads issued before the
// current chunk runs), every lane evaluates the recurrence with the row's
// operands broadcast from the lane that loaded them (v_readlane), and lane u
// keeps the result of row r0 + u for the chunk's store.  With one wave per
// vector, the m kept vectors occupy m waves across the chip instead of m/64.
// Each vector's scratch is contiguous, with the rows padded to Np = 64
// ceil(N / 64): lu[(5 c + a) Np + i] holds the multipliers (a = 0), the
// reciprocal pivots (1), the first and second superdiagonals of U (2, 3) and
// the iterate (4); ipiv[c Np + i] the row interchanges.  Every row takes the
// same form: the operands past the last row are zero, so the last row keeps
// its pivot and contributes nothing beyond itself, and the padding rows carry
// zero multipliers and superdiagonals, so that the iterate is zero on them
// after each forward pass and stays zero through the backward pass.  All loads
// and stores are unconditional (padded rows, clamped input indices), so the
// memory counters of a chunk are the same on every path and the waits only
// cover the chunk that runs.
// Three iterations from a counter-based random start.  With a shift accurate to
// eps ||T||, only members of an exactly (or nearly exactly) degenerate cluster
// can converge to the same direction; cluster_orth_kernel separates them.
CTMRG_DEVINL double lane_bcast(double v, int u)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), u);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), u);
    return __hiloint2double(hi, lo);
}

__global__ void __launch_bounds__(64)
invit_wave_kernel(const double *d, const double *e, int N, const double *selval, int me, double *ZT, int ldz,
                  double *lu, int *ipiv, const double *bounds, unsigned *err)
{
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= me) return;
    const double lam = selval[c];
    const double tn = bounds[3];
    const double pivmin = fmax(DBL_EPSILON * tn, DBL_MIN);
    const int Np = (N + 63) & ~63;
    const int J = Np / 64;
    double *const DLp = lu + (5L * c + 0) * Np;
    double *const RDp = lu + (5L * c + 1) * Np;
    double *const DUp = lu + (5L * c + 2) * Np;
    double *const DU2p = lu + (5L * c + 3) * Np;
    double *const Xp = lu + (5L * c + 4) * Np;
    int *const IPp = ipiv + (long)c * Np;
    // e has N - 1 entries (none for N = 1); out-of-range operands read a valid entry and are zeroed
    const int elast = max(N - 2, 0);

    // ---- LU with partial pivoting of T - lam I: row i's operands are e_i, d_(i+1) - lam and e_(i+1)
    // (zero past the end); rows i and i+1 are interchanged when |e_i| > |pivot|
    {
        double ddi = d[0] - lam;
        double dui = (N > 1) ? e[0] : 0.0;
        double cl, cd, cu;
        {
            const int i = lane;
            const double a = e[min(i, elast)], b = d[min(i + 1, N - 1)], g = e[min(i + 1, elast)];
            cl = (i < N - 1) ? a : 0.0;
            cd = (i + 1 < N) ? b - lam : 0.0;
            cu = (i + 1 < N - 1) ? g : 0.0;
        }
        for (int j = 0; j < J; ++j) {
            const int r0 = 64 * j;
            double nl, nd, nu;
            {
                const int i = r0 + 64 + lane;  // the next chunk (zero operands past the last chunk)
                const double a = e[min(i, elast)], b = d[min(i + 1, N - 1)], g = e[min(i + 1, elast)];
                nl = (i < N - 1) ? a : 0.0;
                nd = (i + 1 < N) ? b - lam : 0.0;
                nu = (i + 1 < N - 1) ? g : 0.0;
            }
            double oL = 0.0, oR = 0.0, oU = 0.0, oU2 = 0.0;
            int oP = 0;
#pragma unroll 16
            for (int u = 0; u < 64; ++u) {
                const double li = lane_bcast(cl, u), dn = lane_bcast(cd, u), dun = lane_bcast(cu, u);
                const bool keep = fabs(ddi) >= fabs(li);
                const double pv = keep ? ((fabs(ddi) < pivmin) ? (ddi < 0.0 ? -pivmin : pivmin) : ddi) : li;
                const double f = (keep ? li : ddi) / pv;
                const double rd = 1.0 / pv;
                const double du = keep ? dui : dn;
                const double du2 = keep ? 0.0 : dun;
                const double ndd = keep ? dn - f * dui : dui - f * dn;
                const double ndu = keep ? dun : -f * dun;
                const bool mine = lane == u;
                oL = mine ? f : oL;
                oR = mine ? rd : oR;
                oU = mine ? du : oU;
                oU2 = mine ? du2 : oU2;
                oP = mine ? (keep ? 0 : 1) : oP;
                ddi = ndd;
                dui = ndu;
            }
            DLp[r0 + lane] = oL;
            RDp[r0 + lane] = oR;
            DUp[r0 + lane] = oU;
            DU2p[r0 + lane] = oU2;
            IPp[r0 + lane] = oP;
            cl = nl; cd = nd; cu = nu;
        }
    }

    // ---- start vector (counter-based random numbers; zero on the padding rows) and its norm
    const uint64_t key = (uint64_t)(c + 1) << 32;
    double nrm2 = 0.0;
    for (int i = lane; i < Np; i += 64) {
        const double x = (i < N) ? hash_uniform(key ^ (uint64_t)i) : 0.0;
        Xp[i] = x;
        nrm2 += x * x;
    }
    double sc = 1.0 / sqrt(wave_sum(nrm2));  // pending scale of the iterate
    for (int it = 0; it < 3; ++it) {
        // the stores of the previous pass (other lanes' rows included) are visible from here
        __syncthreads();
        // forward: unit lower factor with row interchanges applied to sc x; row i reads x_(i+1)
        {
            double xi = Xp[0] * sc;
            double cdl, cxn;
            int cip;
            {
                const int i = lane;
                const double xr = Xp[min(i + 1, Np - 1)];
                cdl = DLp[i];
                cip = IPp[i];
                cxn = (i + 1 < N) ? xr * sc : 0.0;
            }
            for (int j = 0; j < J; ++j) {
                const int r0 = 64 * j;
                double ndl, nxn;
                int nip;
                {
                    const int i = min(r0 + 64, Np - 64) + lane;  // the next chunk (reloads the last one at the end)
                    const double xr = Xp[min(i + 1, Np - 1)];
                    ndl = DLp[i];
                    nip = IPp[i];
                    nxn = (i + 1 < N) ? xr * sc : 0.0;
                }
                double o = 0.0;
#pragma unroll 16
                for (int u = 0; u < 64; ++u) {
                    const double dl = lane_bcast(cdl, u), xn = lane_bcast(cxn, u);
                    const int ip = __builtin_amdgcn_readlane(cip, u);
                    const double out = ip ? xn : xi;
                    xi = ip ? xi - dl * xn : xn - dl * xi;
                    o = (lane == u) ? out : o;
                }
                Xp[r0 + lane] = o;
                cdl = ndl; cxn = nxn; cip = nip;
            }
        }
        __syncthreads();
        // backward: upper factor with two superdiagonals, rows in reverse order (padding rows are zero)
        {
            double x1 = 0.0, x2 = 0.0, part = 0.0;
            double cxv, cdu, cdu2, crd;
            {
                const int i = Np - 64 + lane;
                cxv = Xp[i];
                cdu = DUp[i];
                cdu2 = DU2p[i];
                crd = RDp[i];
            }
            for (int j = J - 1; j >= 0; --j) {
                const int r0 = 64 * j;
                double nxv, ndu, ndu2, nrd;
                {
                    const int i = max(r0 - 64, 0) + lane;  // the next chunk down (reloads the first at the end)
                    nxv = Xp[i];
                    ndu = DUp[i];
                    ndu2 = DU2p[i];
                    nrd = RDp[i];
                }
                double o = 0.0;
#pragma unroll 16
                for (int u = 63; u >= 0; --u) {
                    const double xv = lane_bcast(cxv, u), du = lane_bcast(cdu, u);
                    const double du2 = lane_bcast(cdu2, u), rd = lane_bcast(crd, u);
                    const double xn = (xv - du2 * x2 - du * x1) * rd;
                    x2 = x1;
                    x1 = xn;
                    o = (lane == u) ? xn : o;
                }
                Xp[r0 + lane] = o;
                part += o * o;
                cxv = nxv; cdu = ndu; cdu2 = ndu2; crd = nrd;
            }
            nrm2 = wave_sum(part);
        }
        if (!(nrm2 > 0.0) || !isfinite(nrm2)) {
            if (lane == 0) raise_error(err, KERR_NONFINITE);
            nrm2 = 1.0;
        }
        sc = 1.0 / sqrt(nrm2);
    }
    __syncthreads();
    // the normalized vector, column c of ZT (eight rows per lane in flight)
    for (int i0 = 0; i0 < Np; i0 += 512) {
        double v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = Xp[min(i0 + 64 * t, Np - 64) + lane];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int i = i0 + 64 * t + lane;
            if (i < N) ZT[(long)i * ldz + c] = v[t] * sc;
        }
    }
}

// Modified Gram-Schmidt inside each tight cluster (members in ascending
// eigenvalue order, as listed by clist), one workgroup per cluster.
__global__ void __launch_bounds__(256)
cluster_orth_kernel(double *Z, int ldz, int N, const int *clist, const int *cstart)
{
    __shared__ double red[4];
    const int b0 = cstart[blockIdx.x], b1 = cstart[blockIdx.x + 1];
    if (b1 - b0 < 2) return;
    for (int k = b0; k < b1; ++k) {
        const int qk = clist[k];
        for (int p = b0; p < k; ++p) {
            const int qp = clist[p];
            double sdot = 0.0;
            for (int i = threadIdx.x; i < N; i += 256) sdot += Z[(long)i * ldz + qp] * Z[(long)i * ldz + qk];
            sdot = block_sum<256>(sdot, red);
            for (int i = threadIdx.x; i < N; i += 256) Z[(long)i * ldz + qk] -= sdot * Z[(long)i * ldz + qp];
        }
        double n2 = 0.0;
        for (int i = threadIdx.x; i < N; i += 256) {
            const double z = Z[(long)i * ldz + qk];
            n2 += z * z;
        }
        n2 = block_sum<256>(n2, red);
        const double scale = (n2 > 0.0) ? 1.0 / sqrt(n2) : 0.0;
        for (int i = threadIdx.x; i < N; i += 256) Z[(long)i * ldz + qk] *= scale;
    }
}

// H = 1.5 I - 0.5 G (Newton-Schulz step for the polar factor)
__global__ void ns_matrix_kernel(double *G, int k)
{
    const long total = (long)k * k;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / k), j = (int)(idx - (long)i * k);
        G[idx] = (i == j ? 1.5 : 0.0) - 0.5 * G[idx];
    }
}

// ============================================================================
// Back-transform of stage 2: grouped block reflectors in wavefront order
// ============================================================================
//
// Group (J, t) = reflectors of sweeps J b .. J b + b - 1 at step t; they act on
// rows [J b + 1 + t b, J b + 1 + t b + 2b - 1).  The stage-2 transform applied to
// Z is, group J from last to first, G(J,0) then G(J,1) ... , where
// G(J,t) = H(Jb,t) H(Jb+1,t) ... = I - V T V^T (forward compact WY).
// G(J,t) only has to follow G(J,t-1) and G(J+1,t), so all groups with the same
// t + (nJ - 1 - J) are applied by one launch.

__global__ void __launch_bounds__(256)
bt2_tfactor_kernel(const double *refl, const double *rtau, int N, int b, int Tmax, int nJ, double *T2)
{
    extern __shared__ double sh[];
    double *V = sh;              // [2b][b]
    double *gram = V + 2 * b * b; // [b][b]
    double *Tm = gram + b * b;   // [b][b]
    double *tl = Tm + b * b;     // [b]
    const int J = blockIdx.x / Tmax, t = blockIdx.x - (blockIdx.x / Tmax) * Tmax;
    if (J >= nJ) return;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 2 * b * b; idx += 256) {
        const int i = idx / (2 * b), r = idx - (idx / (2 * b)) * (2 * b);
        const int j = J * b + i;
        double val = 0.0;
        if (j < N - 2 && t < bulge_nsteps(N, b, j) && r - i >= 0 && r - i < b)
            val = refl[((long)j * Tmax + t) * b + (r - i)];
        V[r * b + i] = val;
    }
    for (int i = tid; i < b; i += 256) {
        const int j = J * b + i;
        tl[i] = (j < N - 2 && t < bulge_nsteps(N, b, j)) ? rtau[(long)j * Tmax + t] : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < b * b; idx += 256) {
        const int i = idx / b, k = idx - (idx / b) * b;
        double s = 0.0;
        for (int r = 0; r < 2 * b; ++r) s += V[r * b + i] * V[r * b + k];
        gram[idx] = s;
        Tm[idx] = 0.0;
    }
    __syncthreads();
    for (int i = 0; i < b; ++i) {
        if (tid < i) {
            double s = 0.0;
            for (int l = tid; l < i; ++l) s += Tm[tid * b + l] * gram[l * b + i];
            Tm[tid * b + i] = -tl[i] * s;
        } else if (tid == i) {
            Tm[i * b + i] = tl[i];
        }
        __syncthreads();
    }
    double *dst = T2 + ((long)J * Tmax + t) * b * b;
    for (int idx = tid; idx < b * b; idx += 256) dst[idx] = Tm[idx];
}

// Application of one group G(J,t) = I - V T V^T to 64 columns of Z on the
// matrix cores.  V is 2b x b (banded: V[r][i] is nonzero for 0 <= r - i < b) and T
// is b x b upper triangular; both sit in LDS.  Each wave owns 16 columns and keeps
// them in registers through the three products W = V^T Z, W2 = T W, Z -= V W2:
// the accumulator layout of v_mfma_f64_16x16x4_f64 (lane l, register j: row
// l/16 + 4 j, column l%16) is the B-operand layout of k-step j, so W and W2 feed
// the next product without leaving the registers, and Z, loaded as row
// 4 s + l/16 in register s, takes the update of output tile R in registers 4 R + j.
constexpr int BT2_NC = 64;

template <int B>
__global__ void __launch_bounds__(256)
bt2_apply_kernel(double *Z, int ldz, int N, int ncols, int Tmax, int nJ, int wave, const double *refl,
                 const double *T2)
{
    constexpr int KS = B / 2;   // k-steps over the 2B rows of a group; Z values per lane
    constexpr int BT = B / 16;  // 16-row tiles of W
    using MF = Mfma<double>;
    __shared__ double V[2 * B][B + 1];
    __shared__ double Tm[B][B + 1];
    const int J = blockIdx.x;
    const int t = wave - (nJ - 1 - J);
    if (t < 0 || t >= Tmax) return;
    if (J * B >= N - 2 || t >= bulge_nsteps(N, B, J * B)) return;
    const int base = J * B + 1 + t * B;
    const int nrow = min(2 * B - 1, N - base);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int idx = tid; idx < 2 * B * B; idx += 256) {
        const int i = idx / (2 * B), r = idx - i * (2 * B);
        const int j = J * B + i;
        double val = 0.0;
        if (r < nrow && j < N - 2 && t < bulge_nsteps(N, B, j) && r - i >= 0 && r - i < B)
            val = refl[((long)j * Tmax + t) * B + (r - i)];
        V[r][i] = val;
    }
    const double *Ts = T2 + ((long)J * Tmax + t) * B * B;
    for (int idx = tid; idx < B * B; idx += 256) Tm[idx / B][idx % B] = Ts[idx];
    const int col = blockIdx.y * BT2_NC + wv * 16 + (lane & 15);
    const bool okc = col < ncols;
    const int lr = lane >> 4, lc = lane & 15;
    double z[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int r = 4 * s + lr;
        z[s] = (okc && r < nrow) ? Z[(long)(base + r) * ldz + col] : 0.0;
    }
    __syncthreads();
    // W = V^T Z
    MF::acc_t w[BT];
#pragma unroll
    for (int I = 0; I < BT; ++I) {
        w[I] = MF::zero();
#pragma unroll
        for (int s = 0; s < KS; ++s) w[I] = MF::mma(V[4 * s + lr][16 * I + lc], z[s], w[I]);
    }
    // W2 = T W (T upper triangular: blocks below the diagonal are zero)
    MF::acc_t w2[BT];
#pragma unroll
    for (int I2 = 0; I2 < BT; ++I2) {
        w2[I2] = MF::zero();
#pragma unroll
        for (int I = I2; I < BT; ++I)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) w2[I2] = MF::mma(Tm[16 * I2 + lc][16 * I + 4 * s4 + lr], w[I][s4], w2[I2]);
    }
    // Z -= V W2
#pragma unroll
    for (int R = 0; R < 2 * BT; ++R) {
        MF::acc_t d = MF::zero();
#pragma unroll
        for (int I = 0; I < BT; ++I)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) d = MF::mma(V[16 * R + lc][16 * I + 4 * s4 + lr], w2[I][s4], d);
#pragma unroll
        for (int j = 0; j < 4; ++j) z[4 * R + j] -= d[j];
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int r = 4 * s + lr;
        if (okc && r < nrow) Z[(long)(base + r) * ldz + col] = z[s];
    }
}

// ============================================================================
// Back-transform of stage 1: panels grouped 128 columns (128 / b panels) at a time
// ============================================================================
//
// Group k holds panels p = k G .. k G + G - 1 (fewer, or none, at the end); their
// product Q_p Q_p+1 ... = I - V_G T_G V_G^T with V_G = [V_p | V_p+1 | ...] (panel
// p + j starts j b rows below panel p) and T_G the compact-WY factor of the G b
// reflectors in order: T[0:i, i] = -tau_i T[0:i, 0:i] (V_G^T V_G)[0:i, i].  One
// group then costs one pass of three GEMMs over Z instead of G passes.
__host__ __device__ constexpr int bt1_g(int b) { return 128 / b; }

// V_G as a function of (row r from the first panel's first row, column c).
template <int B>
struct VGroup {
    const double *V[bt1_g(B)];  // explicit V of each panel (n_j x B, row-major), or null
    int n0;                  // rows of the first panel
    __device__ double at(int r, int c) const
    {
        const int j = c / B, lc = c % B, lr = r - j * B;
        const double *v = V[0];
#pragma unroll
        for (int u = 1; u < bt1_g(B); ++u)
            if (j == u) v = V[u];
        return (v != nullptr && lr >= 0 && lr < n0 - j * B) ? v[(long)lr * B + lc] : 0.0;
    }
};
template <int B>
struct A_VG {  // V_G, n x G B
    using value_type = double;
    VGroup<B> g;
    static constexpr bool kContigK = true;
    __device__ double operator()(int i, int k) const { return g.at(i, k); }
};
template <int B>
struct A_VGT {  // V_G^T, G B x n
    using value_type = double;
    VGroup<B> g;
    static constexpr bool kContigK = false;
    __device__ double operator()(int i, int k) const { return g.at(k, i); }
};

// Gram matrix V_G^T V_G (upper 16 x 16 tiles) of every group on the matrix cores,
// as BT1_RS partial sums over row chunks: workgroup (group, chunk), wave w owning
// the tile rows TR w .. TR w + TR - 1; four k-steps of loads are issued at once.
constexpr int BT1_RS = 16;

template <int B>
__global__ void __launch_bounds__(256) bt1_gram_kernel(const double *Vx, int N, int np, double *gram)
{
    using MF = Mfma<double>;
    constexpr int GB = bt1_g(B) * B, GT = GB / 16, TR = GT / 4, U = 4;
    static_assert(TR * 4 == GT, "four waves");
    const int grp = blockIdx.x, chunk = blockIdx.y, p0 = grp * bt1_g(B);
    VGroup<B> vg;
    long off = panel_v_offset(N, B, p0);
    for (int j = 0; j < bt1_g(B); ++j) {
        vg.V[j] = (p0 + j < np) ? Vx + off : nullptr;
        off += (long)(N - (p0 + j + 1) * B) * B;
    }
    vg.n0 = N - (p0 + 1) * B;
    const int steps = (vg.n0 + 3) / 4, per = (steps + BT1_RS - 1) / BT1_RS;
    const int s_lo = chunk * per, s_hi = min(steps, s_lo + per);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane >> 4, lc = lane & 15;
    const int I0 = TR * wave;
    MF::acc_t acc[TR][GT];
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int J = 0; J < GT; ++J) acc[a][J] = MF::zero();
    for (int s0 = s_lo; s0 < s_hi; s0 += U) {
        double av[U][TR], bv[U][GT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = 4 * (s0 + u) + lr;
            const bool ok = s0 + u < s_hi;
#pragma unroll
            for (int a = 0; a < TR; ++a) av[u][a] = ok ? vg.at(r, 16 * (I0 + a) + lc) : 0.0;
#pragma unroll
            for (int J = 0; J < GT; ++J) bv[u][J] = (ok && J >= I0) ? vg.at(r, 16 * J + lc) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int J = 0; J < GT; ++J)
                if (J >= I0)
#pragma unroll
                    for (int a = 0; a < TR; ++a)
                        if (J >= I0 + a) acc[a][J] = MF::mma(av[u][a], bv[u][J], acc[a][J]);
    }
    double *G = gram + ((long)grp * BT1_RS + chunk) * GB * GB;
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int J = 0; J < GT; ++J)
            if (J >= I0 + a)
#pragma unroll
                for (int q = 0; q < 4; ++q) G[(16 * (I0 + a) + lr + 4 * q) * GB + 16 * J + lc] = acc[a][J][q];
}

// T_G of every group from its Gram matrix and the taus (zero for missing panels);
// column i of T in LDS, one column per step.
template <int B>
__global__ void __launch_bounds__(256) bt1_tg_kernel(const double *gram, const double *tau1, int np, double *TG)
{
    constexpr int GB = bt1_g(B) * B;
    extern __shared__ double sh[];
    double *T = sh;              // [GB][GB + 1]
    double *gc = T + GB * (GB + 1);  // [GB]
    const int grp = blockIdx.x, p0 = grp * bt1_g(B);
    const double *G = gram + (long)grp * BT1_RS * GB * GB;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < GB * (GB + 1); idx += 256) T[idx] = 0.0;
    __syncthreads();
    for (int i = 0; i < GB; ++i) {
        const int pj = p0 + i / B;
        const double tau = (pj < np) ? tau1[(long)p0 * B + i] : 0.0;
        for (int l = tid; l < i; l += 256) {
            double g = 0.0;
            for (int ch = 0; ch < BT1_RS; ++ch) g += G[(long)ch * GB * GB + l * GB + i];
            gc[l] = g;
        }
        __syncthreads();
        if (tid < i) {
            double s = 0.0;
            for (int l = tid; l < i; ++l) s += T[tid * (GB + 1) + l] * gc[l];
            T[tid * (GB + 1) + i] = -tau * s;
        } else if (tid == i) {
            T[i * (GB + 1) + i] = tau;
        }
        __syncthreads();
    }
    double *dst = TG + (long)grp * GB * GB;
    for (int idx = tid; idx < GB * GB; idx += 256) dst[idx] = T[(idx / GB) * (GB + 1) + idx % GB];
}

// ============================================================================
// Final copy with sign convention: each eigenvector is negated if its first
// entry of largest magnitude is negative.
// ============================================================================
__global__ void __launch_bounds__(256)
sign_fix_copy_kernel(const double *Z, int ldz, int N, int me, double *U, int ldu)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    if (j >= me) {
        for (int i = tid; i < N; i += 256) U[(long)i * ldu + j] = 0.0;
        return;
    }
    double best = -1.0;
    int bi = 0;
    for (int i = tid; i < N; i += 256) {
        const double a = fabs(Z[(long)i * ldz + j]);
        if (a > best) { best = a; bi = i; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            const double a = sv[tid + s];
            const int ai = si[tid + s];
            if (a > sv[tid] || (a == sv[tid] && ai < si[tid])) { sv[tid] = a; si[tid] = ai; }
        }
        __syncthreads();
    }
    const double sg = (Z[(long)si[0] * ldz + j] < 0.0) ? -1.0 : 1.0;
    for (int i = tid; i < N; i += 256) U[(long)i * ldu + j] = sg * Z[(long)i * ldz + j];
}

// ============================================================================
// Host drivers
// ============================================================================

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Split-K and work-item partials.  The stage-1 products take at most 64 Nmax max(b, 64)
// doubles; a split-K product whose splits come from splits_for() has tiles * splits < 1024
// and at most 64 x 64 outputs per tile, so it never needs more than 1024 * 64 * 64.
static size_t splitk_elems_for(int Nmax, int b)
{
    return std::max<size_t>((size_t)64 * Nmax * std::max(b, 64), (size_t)1024 * 64 * 64);
}

__global__ void __launch_bounds__(256)
ysym_items_kernel(const double *A, long lda, const double *V, int n, int ch, double *P1, double *P2);

namespace {
struct EigReq {
    void **p;
    size_t bytes;
};
}  // namespace

// Sizes, in the order the buffers are laid out; every entry is rounded to 256 bytes when carved.
static std::vector<EigReq> eig_requests(EigWork &w, int Nmax, int kmax, int b)
{
    const int np = num_panels(Nmax, b);
    const size_t npad = ((size_t)Nmax + 63) / 64 * 64;  // rows of invit_wave_kernel's scratch
    w.Nmax = Nmax;
    w.kmax = kmax;
    w.b = b;
    w.Tmax = max_steps(Nmax, b) + 1;
    w.nJmax = (Nmax + b - 1) / b;
    w.splitk_elems = splitk_elems_for(Nmax, b);
    return {
        {(void **)&w.part, sizeof(double) * 2 * pqr_slot_set(b, pqr_gmax(Nmax, b))},
        {(void **)&w.err, 64},
        {(void **)&w.Vx, sizeof(double) * (size_t)panel_v_offset(Nmax, b, np) + 8},
        {(void **)&w.Tp, sizeof(double) * (size_t)np * b * b + 8},
        {(void **)&w.tau1, sizeof(double) * (size_t)np * b + 8},
        {(void **)&w.VW, sizeof(double) * (size_t)Nmax * 2 * b},
        {(void **)&w.WV, sizeof(double) * (size_t)Nmax * 2 * b},
        {(void **)&w.Y, sizeof(double) * (size_t)Nmax * b},
        {(void **)&w.X, sizeof(double) * (size_t)Nmax * b},
        {(void **)&w.sm, sizeof(double) * 4 * b * b},
        {(void **)&w.splitk, sizeof(double) * w.splitk_elems},
        {(void **)&w.band, sizeof(double) * (size_t)Nmax * 2 * b},
        {(void **)&w.refl, sizeof(double) * (size_t)Nmax * w.Tmax * b},
        {(void **)&w.rtau, sizeof(double) * (size_t)Nmax * w.Tmax},
        {(void **)&w.T2, sizeof(double) * (size_t)w.nJmax * w.Tmax * b * b},
        {(void **)&w.bt1_gram, sizeof(double) * (size_t)ceil_div(np, bt1_g(b)) * BT1_RS * bt1_g(b) * b * bt1_g(b) * b + 8},
        {(void **)&w.bt1_T, sizeof(double) * (size_t)ceil_div(np, bt1_g(b)) * bt1_g(b) * b * bt1_g(b) * b + 8},
        {(void **)&w.bt1_W, sizeof(double) * 2 * (size_t)bt1_g(b) * b * kmax},
        {(void **)&w.d, sizeof(double) * (size_t)Nmax},
        {(void **)&w.e, sizeof(double) * (size_t)Nmax},
        {(void **)&w.e2, sizeof(double) * (size_t)Nmax},
        {(void **)&w.evals, sizeof(double) * (size_t)Nmax},
        {(void **)&w.slices, sizeof(double) * 4 * BIS_SLICE},
        {(void **)&w.ZT, sizeof(double) * (size_t)Nmax * kmax},
        {(void **)&w.Ztmp, sizeof(double) * (size_t)Nmax * kmax},
        {(void **)&w.G, sizeof(double) * (size_t)kmax * kmax},
        {(void **)&w.lu, sizeof(double) * 5 * npad * (size_t)kmax},
        {(void **)&w.ipiv, sizeof(int) * npad * (size_t)kmax},
        {(void **)&w.clist, sizeof(int) * (size_t)(kmax + 2) * 2},
        {(void **)&w.cstart, sizeof(int) * (size_t)(kmax + 2)},
    };
}

size_t eig_bytes(int Nmax, int kmax, int b)
{
    EigWork w;
    size_t s = 0;
    for (const EigReq &r : eig_requests(w, Nmax, kmax, b)) s += align_up(r.bytes);
    return s;
}

// Occupancy-derived limits and the kernel attributes the solver needs (no allocation).
static hipError_t eig_setup_limits(EigWork &w, int b)
{
    const size_t tg_smem = sizeof(double) * ((size_t)bt1_g(b) * b * (bt1_g(b) * b + 1) + bt1_g(b) * b);
    hipError_t e = hipFuncSetAttribute(b == 32 ? (const void *)bt1_tg_kernel<32> : (const void *)bt1_tg_kernel<16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)tg_smem);
    // panel QR workgroups that the device holds at once
    int per_cu = 0, dev = 0, cus = 0;
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, b == 32 ? (const void *)panel_qr_kernel<32> : (const void *)panel_qr_kernel<16>, 256, 0);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    w.pqr_cap = per_cu * cus;
    int ys_cu = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ys_cu, (const void *)ysym_items_kernel, 256, 0);
    w.ysym_cap = std::max(1, ys_cu * cus);
    // the largest dynamic LDS a workgroup may opt into: the bulge chasing of small bands in LDS
    int lds_max = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeSharedMemPerBlockOptin, dev);
    w.lds_bulge_bytes = 0;
    if (e == hipSuccess && lds_max > 0) {
        const size_t want = std::min<size_t>((size_t)lds_max, bulge_lds_bytes(w.Nmax, b));
        e = hipFuncSetAttribute(b == 32 ? (const void *)bulge_lds_kernel<32> : (const void *)bulge_lds_kernel<16>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)want);
        if (e == hipSuccess) w.lds_bulge_bytes = want;
    }
    return e;
}

__global__ void fill_u64_kernel(unsigned long long *p, size_t n, unsigned long long v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// The panel-QR exchange slots to the empty marker, the error flags to zero (fill kernels on s).
static hipError_t eig_reset_flags(EigWork &w, hipStream_t s)
{
    const size_t nslot = 2 * pqr_slot_set(w.b, pqr_gmax(w.Nmax, w.b));
    hipLaunchKernelGGL(fill_u64_kernel, dim3(std::min<size_t>(1024, (nslot + 255) / 256)), dim3(256), 0, s,
                       (unsigned long long *)w.part, nslot, ~0ull);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, s, (unsigned long long *)w.err, (size_t)8, 0ull);
    w.pqr_launches = 0;
    w.pqr_gprev = 0;
    return hipGetLastError();
}

hipError_t eig_alloc(EigWork &w, int Nmax, int kmax, int b)
{
    w.owned = true;
    for (const EigReq &r : eig_requests(w, Nmax, kmax, b)) {
        hipError_t e = hipMalloc(r.p, r.bytes);
        if (e != hipSuccess) {
            eig_free(w);
            return e;
        }
    }
    (void)hipMemset(w.part, 0xFF, sizeof(double) * 2 * pqr_slot_set(b, pqr_gmax(Nmax, b)));  // all slots empty
    (void)hipMemset(w.err, 0, 64);
    hipError_t e = eig_setup_limits(w, b);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&w.s2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w.ev_cols, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w.ev_update, hipEventDisableTiming);
    if (e != hipSuccess) {
        eig_free(w);
        return e;
    }
    return hipSuccess;
}

hipError_t eig_carve(EigWork &w, void *base, size_t bytes, int Nmax, int kmax, int b, hipStream_t s)
{
    w = EigWork();
    w.owned = false;
    char *p = static_cast<char *>(base);
    size_t used = 0;
    for (const EigReq &r : eig_requests(w, Nmax, kmax, b)) {
        const size_t sz = align_up(r.bytes);
        if (used + sz > bytes) return hipErrorInvalidValue;
        *r.p = p + used;
        used += sz;
    }
    hipError_t e = eig_setup_limits(w, b);
    if (e == hipSuccess) e = eig_reset_flags(w, s);
    return e;
}

hipError_t eig_attach_streams(EigWork &w)
{
    hipError_t e = hipStreamCreateWithFlags(&w.s2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w.ev_cols, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w.ev_update, hipEventDisableTiming);
    return e;
}

void eig_free(EigWork &w)
{
    void *ptrs[] = {w.Vx, w.Tp, w.tau1, w.VW, w.WV, w.Y, w.X, w.sm, w.part, w.splitk, w.band, w.refl, w.rtau,
                    w.T2, w.bt1_gram, w.bt1_T, w.bt1_W, w.d, w.e, w.e2, w.evals, w.slices, w.ZT, w.Ztmp, w.G, w.lu, w.ipiv, w.clist,
                    w.cstart, w.err};
    if (w.owned)
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
    if (w.ev_cols) (void)hipEventDestroy(w.ev_cols);
    if (w.ev_update) (void)hipEventDestroy(w.ev_update);
    if (w.s2) (void)hipStreamDestroy(w.s2);
    w = EigWork();
}

unsigned eig_take_errors(EigWork &w)
{
    unsigned e = 0;
    (void)hipMemcpy(&e, w.err, sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e) (void)hipMemset(w.err, 0, sizeof(unsigned));
    return e;
}

static int splits_for(long tiles, long K, int kmin)
{
    long s = 1;
    while (tiles * s < 512 && K / (s * 2) >= kmin) s *= 2;
    return (int)s;
}


static hipError_t panel_qr(EigWork &w, double *A, long lda, int N, int pi, hipStream_t s)
{
    const int b = w.b;
    const int p = pi * b, r0 = p + b, n = N - r0;
    const int rows = pqr_rows(b);
    double *Vp = w.Vx + panel_v_offset(N, b, pi);
    double *Tp = w.Tp + (long)pi * b * b;
    double *taup = w.tau1 + (long)pi * b;
    int G = (n + rows - 1) / rows;
    int Gmax = pqr_gmax(w.Nmax, b), parity = (int)(w.pqr_launches & 1), Gprev = w.pqr_gprev;
    if (G > Gmax) return hipErrorInvalidValue;
    // The workgroups wait for each other's partial sums, so all of them must be able to be
    // resident at once: the grid fits the device (checked against the occupancy at set-up),
    // and the only kernels beside it (the trailing update on the second stream) wait on
    // nothing, so they retire and leave room for any workgroup not yet started.  A plain
    // launch is used: a cooperative launch costs about 13 us more per panel here.
    if (G > w.pqr_cap) return hipErrorCooperativeLaunchTooLarge;
    void *args[] = {&A, &lda, (void *)&r0, (void *)&p, (void *)&n, &Vp, &taup, &Tp, &w.part, &Gmax, &parity, &Gprev, &w.err};
    const void *fn = b == 32 ? (const void *)panel_qr_kernel<32> : (const void *)panel_qr_kernel<16>;
    hipError_t e = hipLaunchKernel(fn, dim3(G), dim3(256), args, 0, s);
    if (e == hipSuccess) {
        ++w.pqr_launches;
        w.pqr_gprev = G;
    }
    return e;
}

// Y = A22 V in one pass over the lower triangle of A22 (b = 16).  The work items are
// those of A_LoItems: row tile I (rows R = [128 I, 128 I + 128)) and a chunk
// [k0, k0 + ch) of its K range [0, min(n, 128 I + 128)).  From each 128 x 16 slice of
// A in LDS an item forms both its rows' part L[R, slice] V[slice] (accumulated over the
// chunk into P1, 128 x 16 per item) and the mirrored part (A[R, slice] with i > k)^T V[R]
// of the slice's rows (written to P2, ch x 16 per item).  Row r of Y is then the sum of
// the P1 rows of its tile's items plus, for every tile I' >= tile(r), the P2 row of the
// item (I', chunk of r) (ysym_reduce_kernel).  Wave w forms P1 for tile rows
// 32 w .. 32 w + 31 and the mirrored product over those same rows, whose V it keeps in
// registers as matrix-core B fragments for the whole item.
__global__ void __launch_bounds__(256)
ysym_items_kernel(const double *A, long lda, const double *V, int n, int ch, double *P1, double *P2)
{
    using MF = Mfma<double>;
    constexpr int B = 16, BM = 128, BK = 16;
    constexpr int PA = BM * BK / 256;  // 8
    __shared__ double As[BK][BM + 1];  // As[kk][mm] = A[m0 + mm][k0 + kk] where k <= i, else 0
    __shared__ double Bs[BK][B];       // V of the slice's rows
    __shared__ double red[3][16][B];   // mirrored partials of waves 1..3

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int item = blockIdx.x, I = 0;
    const int ntile = (n + BM - 1) / BM;
    for (; I < ntile; ++I) {
        const int cnt = tile_items<A_LoItems>(I, BM, n, ch);
        if (item < cnt) break;
        item -= cnt;
    }
    const int m0 = I * BM;
    const int kbeg = item * ch, kend = min(A_LoItems::k_hi(I, BM, n), kbeg + ch);

    // k-step s of the mirrored product covers tile rows 32 w + 4 s .. + 3 (row 32 w + 4 s + lane / 16 in this lane)
    double vf[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) {
        const int row = m0 + 32 * wave + 4 * st + (lane >> 4);
        vf[st] = (row < n) ? V[(long)row * B + (lane & 15)] : 0.0;
    }
    double ra[PA], rb;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int idx = tid + u * 256, mm = idx / BK, kk = idx - mm * BK;
            const int gm = m0 + mm, gk = k0 + kk;
            ra[u] = (gm < n && gk < kend && gk <= gm) ? A[(long)gm * lda + gk] : 0.0;
        }
        const int kk = tid / B, j = tid - kk * B, gk = k0 + kk;
        rb = (gk < kend) ? V[(long)gk * B + j] : 0.0;
    };
    MF::acc_t acc1[2];
    acc1[0] = MF::zero();
    acc1[1] = MF::zero();
    fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int idx = tid + u * 256, mm = idx / BK, kk = idx - mm * BK;
            As[kk][mm] = ra[u];
        }
        Bs[tid / B][tid % B] = rb;
        __syncthreads();
        if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const double bv = Bs[kk + (lane >> 4)][lane & 15];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                acc1[i] = MF::mma(As[kk + (lane >> 4)][(wave * 2 + i) * 16 + (lane & 15)], bv, acc1[i]);
        }
        MF::acc_t acc2 = MF::zero();
#pragma unroll
        for (int st = 0; st < 8; ++st)
            acc2 = MF::mma(As[lane & 15][32 * wave + 4 * st + (lane >> 4)], vf[st], acc2);
        if (wave > 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave - 1][(lane >> 4) + 4 * r][lane & 15] = acc2[r];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int kk = (lane >> 4) + 4 * r, col = lane & 15, k = k0 + kk;
                double v = acc2[r] + red[0][kk][col] + red[1][kk][col] + red[2][kk][col];
                // the slice held the diagonal element A[k][k]; the mirrored part excludes it
                if (k >= m0 && k < m0 + BM && k < kend) v -= As[kk][k - m0] * V[(long)k * B + col];
                if (k < kend) P2[((long)blockIdx.x * ch + (k - kbeg)) * B + col] = v;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = (wave * 2 + i) * 16 + (lane >> 4) + 4 * r, col = lane & 15;
            P1[((long)blockIdx.x * BM + row) * B + col] = acc1[i][r];
        }
}

// Y (n x 16) from the partials of ysym_items_kernel: blockIdx.y is the row tile K,
// each thread one element; the tile's P1 rows, then the P2 rows of tiles K, K + 1, ...
// are added in that order (loads issued sixteen at a time).  At most 1024 row tiles.
__global__ void __launch_bounds__(256)
ysym_reduce_kernel(const double *P1, const double *P2, int n, int ch, double *Y)
{
    constexpr int B = 16, U = 16;
    __shared__ int first[1025];  // first item of each row tile
    const int K = blockIdx.y, ntile = (n + 127) / 128;
    if (threadIdx.x == 0) {
        int f = 0;
        for (int I = 0; I < ntile; ++I) {
            first[I] = f;
            f += tile_items<A_LoItems>(I, 128, n, ch);
        }
        first[ntile] = f;
    }
    __syncthreads();
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = idx / B, j = idx - r * B, row = K * 128 + r;
    if (r >= 128 || row >= n) return;
    double s = 0.0;
    const double *q1 = P1 + ((long)first[K] * 128 + r) * B + j;
    const int c1 = first[K + 1] - first[K];
    for (int u0 = 0; u0 < c1; u0 += U) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = (u0 + u < c1) ? q1[(long)(u0 + u) * 128 * B] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) s += t[u];
    }
    const int c = row / ch, off = row - c * ch;
    for (int I0 = K; I0 < ntile; I0 += U) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            t[u] = (I0 + u < ntile) ? P2[((long)(first[I0 + u] + c) * ch + off) * B + j] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) s += t[u];
    }
    Y[(long)row * B + j] = s;
}

// Dense -> band.  Look-ahead: once the next panel's b columns have their
// update, its QR (on s) overlaps the update of the rest of the trailing matrix
// (on w.s2); s waits for that update before the next product with the trailing
// matrix.
static hipError_t stage1(EigWork &w, double *A, long lda, int N, hipStream_t s)
{
    const int b = w.b;
    const int np = num_panels(N, b);
    const GemmShape tall = b == 16 ? GEMM_TALL16 : GEMM_TALL;  // products with b output columns
    hipError_t e;
    if (np == 0) return hipSuccess;
    e = panel_qr(w, A, lda, N, 0, s);
    if (e != hipSuccess) return e;
    for (int pi = 0; pi < np; ++pi) {
        const int p = pi * b, r0 = p + b, n = N - r0;
        double *Vp = w.Vx + panel_v_offset(N, b, pi);
        double *Tp = w.Tp + (long)pi * b * b;
        double *A22 = A + (long)r0 * lda + r0;
        // Y = A22 V, with A22 held in its lower triangle: Y = L V + (strictly lower)^T V.
        // The K range of each 128-row tile (a triangle's worth) is cut into equal
        // chunks, so every workgroup streams the same number of slices.
        {
            const int ch = n >= 4096 ? 512 : 256;
            const int nt = ceil_div(n, 128);
            int n1 = 0, n2 = 0;
            for (int I = 0; I < nt; ++I) {
                n1 += tile_items<A_LoItems>(I, 128, n, ch);
                n2 += tile_items<A_SLoTItems>(I, 128, n, ch);
            }
            // single pass: the chunk length that puts the items through the device in the fewest
            // rounds of equal work (rounds x chunk length; ties to the longer chunk)
            int ych = ch, yn1 = n1;
            if (b == 16) {
                long best = -1;
                for (int c = 128; c <= 2048; c += 128) {
                    long it = 0;
                    for (int I = 0; I < nt; ++I) it += tile_items<A_LoItems>(I, 128, n, c);
                    const long cost = (it + w.ysym_cap - 1) / w.ysym_cap * c;
                    if (best < 0 || cost <= best) {
                        best = cost;
                        ych = c;
                        yn1 = (int)it;
                    }
                }
            }
            if (b == 16 && nt <= 1024 && (size_t)yn1 * (128 + ych) * b <= w.splitk_elems) {
                // one pass over the triangle (the form that pays at b = 16, where the two-pass
                // products are bound by memory rather than by the matrix cores)
                double *p1 = w.splitk, *p2 = w.splitk + (long)yn1 * 128 * b;
                hipLaunchKernelGGL(ysym_items_kernel, dim3(yn1), dim3(256), 0, s, A22, lda, Vp, n, ych, p1, p2);
                hipLaunchKernelGGL(ysym_reduce_kernel, dim3(ceil_div(128 * b, 256), nt), dim3(256), 0, s, p1, p2,
                                   n, ych, w.Y);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            } else {
                if ((size_t)(n1 + n2) * 128 * b > w.splitk_elems) return hipErrorInvalidValue;
                double *p1 = w.splitk, *p2 = w.splitk + (long)n1 * 128 * b;
                // (the output tile is b columns wide: a wider one would only add matrix-core work)
                if (b == 16) {
                    if (n1 > 0)
                        hipLaunchKernelGGL((gemm_mfma_kernel<128, 16, 32, 4, 1, A_LoItems, B_RM, EpiItems>), dim3(n1),
                                           dim3(256), 0, s, A_LoItems{{A22, lda}}, B_RM{Vp, b}, EpiItems{p1, b}, n, b, n, ch);
                    if (n2 > 0)
                        hipLaunchKernelGGL((gemm_mfma_kernel<128, 16, 32, 4, 1, A_SLoTItems, B_RM, EpiItems>), dim3(n2),
                                           dim3(256), 0, s, A_SLoTItems{{A22, lda}}, B_RM{Vp, b}, EpiItems{p2, b}, n, b, n,
                                           ch);
                } else {
                    if (n1 > 0)
                        hipLaunchKernelGGL((gemm_mfma_kernel<128, 32, 32, 4, 1, A_LoItems, B_RM, EpiItems>), dim3(n1),
                                           dim3(256), 0, s, A_LoItems{{A22, lda}}, B_RM{Vp, b}, EpiItems{p1, b}, n, b, n, ch);
                    if (n2 > 0)
                        hipLaunchKernelGGL((gemm_mfma_kernel<128, 32, 32, 4, 1, A_SLoTItems, B_RM, EpiItems>), dim3(n2),
                                           dim3(256), 0, s, A_SLoTItems{{A22, lda}}, B_RM{Vp, b}, EpiItems{p2, b}, n, b, n,
                                           ch);
                }
                hipLaunchKernelGGL((reduce_items_kernel<A_LoItems, A_SLoTItems>), dim3(ceil_div(128 * b, 256), nt),
                                   dim3(256), 0, s, p1, p2, n, b, n, ch, w.Y, (long)b);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
        }
        // W = [Y | V] [T ; -1/2 S] with S = T^T (V^T Y) T, and the operands [V|W], [W|V]
        {
            const int gv = std::min(VTY_WG, std::max(1, ceil_div(n, 4)));
            if (b == 32)
                hipLaunchKernelGGL(vty_partial_kernel<32>, dim3(gv), dim3(256), 0, s, Vp, w.Y, n, w.splitk);
            else
                hipLaunchKernelGGL(vty_partial_kernel<16>, dim3(gv), dim3(256), 0, s, Vp, w.Y, n, w.splitk);
            hipLaunchKernelGGL(wy_small_kernel, dim3(1), dim3(1024), 0, s, w.splitk, gv, Tp, b, w.sm);
            if (b == 16) {
                // with the next panel's columns (rows 0..n-1, columns 0..b-1 of A22) updated in the same launch
                hipLaunchKernelGGL(vw_cols16_kernel, dim3(ceil_div(n, 32)), dim3(256), 0, s, w.Y, Vp, w.sm, n,
                                   pi + 1 < np ? 1 : 0, w.VW, w.WV, A22, lda);
                e = hipGetLastError();
            } else {
                e = gemm_mfma(tall, A_YV{w.Y, Vp, b}, B_RM{w.sm, b}, EpiVW{Vp, w.VW, w.WV, b}, n, b, 2 * b, s);
            }
            if (e != hipSuccess) return e;
        }
        // A22 -= [V|W] [W|V]^T on the lower triangle (the only part later read)
        if (pi + 1 < np) {
            // the next panel's columns first (rows 0..n-1, columns 0..b-1 of A22) ...
            if (b != 16) {
                e = gemm_mfma(tall, A_RM{w.VW, 2 * b}, B_T{w.WV, 2 * b}, EpiAxpby{A22, lda, -1.0, 1.0}, n, b, 2 * b,
                              s);
                if (e != hipSuccess) return e;
            }
            // ... then the rest of the update on s2, beside the next panel's QR on s (the QR is on
            // the critical path; the update ends first, so the wait for it costs nothing).  Without a
            // second stream (carved workspace) the two run in order on s.
            if (!w.s2) {
                e = gemm_mfma_lower(A_RM{w.VW + (long)b * 2 * b, 2 * b}, B_T{w.WV + (long)b * 2 * b, 2 * b},
                                    EpiAxpbyLower{A22 + (long)b * lda + b, lda, -1.0, 1.0}, n - b, 2 * b, s);
                if (e == hipSuccess) e = panel_qr(w, A, lda, N, pi + 1, s);
                if (e != hipSuccess) return e;
                continue;
            }
            if ((e = hipEventRecord(w.ev_cols, s)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(w.s2, w.ev_cols, 0)) != hipSuccess) return e;
            e = gemm_mfma_lower(A_RM{w.VW + (long)b * 2 * b, 2 * b}, B_T{w.WV + (long)b * 2 * b, 2 * b},
                                EpiAxpbyLower{A22 + (long)b * lda + b, lda, -1.0, 1.0}, n - b, 2 * b, w.s2);
            if (e != hipSuccess) return e;
            if ((e = hipEventRecord(w.ev_update, w.s2)) != hipSuccess) return e;
            e = panel_qr(w, A, lda, N, pi + 1, s);
            if (e != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s, w.ev_update, 0)) != hipSuccess) return e;
        } else {
            e = gemm_mfma_lower(A_RM{w.VW, 2 * b}, B_T{w.WV, 2 * b}, EpiAxpbyLower{A22, lda, -1.0, 1.0}, n, 2 * b, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t eig_values(EigWork &w, double *A, long lda, int N, hipStream_t s)
{
    if (N > w.Nmax) return hipErrorInvalidValue;
    const int b = w.b;
    hipError_t e = stage1(w, A, lda, N, s);
    if (e != hipSuccess) return e;
    mark(w, MK_STAGE1, s);
    hipLaunchKernelGGL(extract_band_kernel, dim3(std::min(4096, ceil_div((long)N * 2 * b, 256))), dim3(256), 0, s, A,
                       lda, N, b, w.band);
    if (N > 2) {
        const int Tmax = w.Tmax;
        // one launch per wavefront tau = 3 j + t of independent steps, or one workgroup over
        // them all when the band fits in its LDS
        const int taumax = 3 * (N - 3) + bulge_nsteps(N, b, N - 3);
        const size_t lb = bulge_lds_bytes(N, b);
        if (lb <= w.lds_bulge_bytes) {
            if (b == 32)
                hipLaunchKernelGGL(bulge_lds_kernel<32>, dim3(1), dim3(1024), lb, s, w.band, N, w.refl, w.rtau, Tmax);
            else
                hipLaunchKernelGGL(bulge_lds_kernel<16>, dim3(1), dim3(1024), lb, s, w.band, N, w.refl, w.rtau, Tmax);
        }
        for (int tau = 0; tau < taumax && lb > w.lds_bulge_bytes; ++tau) {
            const int jhi = std::min(tau / 3, N - 3);
            const int jlo = std::max(0, (tau - (Tmax - 1)) / 3);
            if (jhi < jlo) continue;
            if (b == 32)
                hipLaunchKernelGGL(bulge_front_kernel<32>, dim3(jhi - jlo + 1), dim3(64), 0, s, w.band, N, tau, jlo,
                                   w.refl, w.rtau, Tmax);
            else
                hipLaunchKernelGGL(bulge_front_kernel<16>, dim3(jhi - jlo + 1), dim3(64), 0, s, w.band, N, tau, jlo,
                                   w.refl, w.rtau, Tmax);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    mark(w, MK_BULGE, s);
    hipLaunchKernelGGL(band_to_tridiag_kernel, dim3(ceil_div(N, 256)), dim3(256), 0, s, w.band, N, b, w.d, w.e, w.e2);
    double *bounds = w.sm + 3 * b * b;
    hipLaunchKernelGGL(tridiag_bounds_kernel, dim3(1), dim3(256), 0, s, w.d, w.e, N, bounds);
    double *xs = w.slices;
    int *cnts = (int *)(w.slices + 2 * BIS_SLICE);
    hipLaunchKernelGGL(bisect_slice_kernel, dim3(2 * BIS_SLICE / 256), dim3(256), 0, s, w.d, w.e2, N, bounds, xs, cnts);
    constexpr int LPE = 16, SH = 1;  // 16 lanes per eigenvalue, 1 shift each: 16 points per pass (fastest measured)
    hipLaunchKernelGGL((bisect_kernel<LPE, SH>), dim3(ceil_div((long)N * LPE, 256)), dim3(256), 0, s, w.d, w.e2, N,
                       bounds, xs, cnts, w.evals);
    mark(w, MK_BISECT, s);
    return hipGetLastError();
}

hipError_t eig_post(EigWork &w, int N, int m, double gap_tol, double rank_tol, const double *omega4_prev,
                    double *omega_new, double *selval, PostOut *out_dev, hipStream_t s)
{
    if (m > w.kmax) return hipErrorInvalidValue;
    int *selpos = w.clist + (w.kmax + 2);
    hipLaunchKernelGGL(post_eigen_kernel, dim3(1), dim3(256), 0, s, w.evals, N, m, gap_tol, rank_tol, omega4_prev,
                       omega_new, selval, selpos, w.clist, w.cstart, out_dev);
    return hipGetLastError();
}

// Z[r0:, :] -= V_G T_G V_G^T Z[r0:, :] for panel group k.
template <int B>
static hipError_t bt1_apply_group(EigWork &w, double *Z, int ldz, int N, int me, int np, int k, hipStream_t s)
{
    constexpr int GB = bt1_g(B) * B;
    const int p0 = k * bt1_g(B), r0 = p0 * B + B, n = N - r0;
    VGroup<B> vg;
    long off = panel_v_offset(N, B, p0);
    for (int j = 0; j < bt1_g(B); ++j) {
        vg.V[j] = (p0 + j < np) ? w.Vx + off : nullptr;
        off += (long)(N - (p0 + j + 1) * B) * B;
    }
    vg.n0 = n;
    const double *TG = w.bt1_T + (long)k * GB * GB;
    double *Zs = Z + (long)r0 * ldz;
    double *W1 = w.bt1_W, *W2 = w.bt1_W + (long)GB * me;
    const long tiles = (long)ceil_div(GB, 64) * ceil_div(me, 64);
    int sp = splits_for(tiles, n, 128);
    while (sp > 1 && (size_t)sp * GB * me > w.splitk_elems) sp /= 2;
    hipError_t e = gemm_mfma_splitk(A_VGT<B>{vg}, B_RM{Zs, ldz}, EpiStore{W1, me, 1.0}, GB, me, n, sp, w.splitk, s);
    if (e != hipSuccess) return e;
    e = gemm_mfma(GEMM_SMALL, A_RM{TG, GB}, B_RM{W1, me}, EpiStore{W2, me, 1.0}, GB, me, GB, s);
    if (e != hipSuccess) return e;
    return gemm_mfma(GEMM_LARGE, A_VG<B>{vg}, B_RM{W2, me}, EpiAxpby{Zs, ldz, -1.0, 1.0}, n, me, GB, s);
}

hipError_t eig_vectors(EigWork &w, const double *, long, int N, int me, const double *selval, int nclusters,
                       double *U, int ldu, hipStream_t s)
{
    const int b = w.b;
    const int ldz = w.kmax;
    const double *bounds = w.sm + 3 * b * b;
    hipError_t e;
    mark(w, MK_VEC_START, s);
    if (me > 0)
        hipLaunchKernelGGL(invit_wave_kernel, dim3(me), dim3(64), 0, s, w.d, w.e, N, selval, me, w.ZT, ldz, w.lu,
                           w.ipiv, bounds, w.err);
    if (nclusters < me)
        hipLaunchKernelGGL(cluster_orth_kernel, dim3(nclusters), dim3(256), 0, s, w.ZT, ldz, N, w.clist, w.cstart);
    mark(w, MK_INVIT, s);
    // Newton-Schulz polar orthonormalization: Z <- Z (3/2 I - 1/2 Z^T Z)
    double *Z = w.ZT, *Zo = w.Ztmp;
    for (int it = 0; it < 3; ++it) {
        const long tiles = (long)ceil_div(me, 64) * ceil_div(me, 64);
        int sp = splits_for(tiles, N, 256);
        while (sp > 1 && (size_t)sp * me * me > w.splitk_elems) sp /= 2;
        e = gemm_mfma_splitk(A_T{Z, ldz}, B_RM{Z, ldz}, EpiStore{w.G, me, 1.0}, me, me, N, sp, w.splitk, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(ns_matrix_kernel, dim3(std::max(1, std::min(1024, ceil_div((long)me * me, 256)))), dim3(256), 0,
                           s, w.G, me);
        e = gemm_mfma(GEMM_LARGE, A_RM{Z, ldz}, B_RM{w.G, me}, EpiStore{Zo, ldz, 1.0}, N, me, me, s);
        if (e != hipSuccess) return e;
        std::swap(Z, Zo);
    }
    mark(w, MK_NS, s);
    // stage-2 back-transform
    if (N > 2) {
        const int nJ = ceil_div(N - 2, b);
        const int Tmax = w.Tmax;
        hipLaunchKernelGGL(bt2_tfactor_kernel, dim3(nJ * Tmax), dim3(256), sizeof(double) * (4 * b * b + b), s, w.refl,
                           w.rtau, N, b, Tmax, nJ, w.T2);
        const int nwave = nJ + Tmax - 1;
        for (int wv = 0; wv < nwave; ++wv) {
            if (b == 32)
                hipLaunchKernelGGL(bt2_apply_kernel<32>, dim3(nJ, ceil_div(me, BT2_NC)), dim3(256), 0, s, Z, ldz, N, me,
                                   Tmax, nJ, wv, w.refl, w.T2);
            else
                hipLaunchKernelGGL(bt2_apply_kernel<16>, dim3(nJ, ceil_div(me, BT2_NC)), dim3(256), 0, s, Z, ldz, N, me,
                                   Tmax, nJ, wv, w.refl, w.T2);
        }
    }
    mark(w, MK_BT2, s);
    // stage-1 back-transform, groups of bt1_g(b) panels, last group first
    const int np = num_panels(N, b);
    if (np > 0) {
        const int ngr = ceil_div(np, bt1_g(b)), GB = bt1_g(b) * b;
        if (b == 32) {
            hipLaunchKernelGGL(bt1_gram_kernel<32>, dim3(ngr, BT1_RS), dim3(256), 0, s, w.Vx, N, np, w.bt1_gram);
            hipLaunchKernelGGL(bt1_tg_kernel<32>, dim3(ngr), dim3(256), sizeof(double) * (GB * (GB + 1) + GB), s,
                               w.bt1_gram, w.tau1, np, w.bt1_T);
        } else {
            hipLaunchKernelGGL(bt1_gram_kernel<16>, dim3(ngr, BT1_RS), dim3(256), 0, s, w.Vx, N, np, w.bt1_gram);
            hipLaunchKernelGGL(bt1_tg_kernel<16>, dim3(ngr), dim3(256), sizeof(double) * (GB * (GB + 1) + GB), s,
                               w.bt1_gram, w.tau1, np, w.bt1_T);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int k = ngr - 1; k >= 0; --k) {
            e = b == 32 ? bt1_apply_group<32>(w, Z, ldz, N, me, np, k, s) : bt1_apply_group<16>(w, Z, ldz, N, me, np, k, s);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(sign_fix_copy_kernel, dim3(ldu), dim3(256), 0, s, Z, ldz, N, me, U, ldu);
    mark(w, MK_BT1, s);
    return hipGetLastError();
}

}  // namespace ctm
