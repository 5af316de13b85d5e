// Context, step orchestration and the C ABI declared in include/ctmrg.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "adjoint.h"
#include "common.h"
#include "contract.h"
#include "ctmrg.h"
#include "eig.h"
#include "warm.h"
#include "xi.h"

using namespace ctm;

struct ctmrg_ctx {
    int q = 0, dim = 0, m = 0, N = 0;
    double K = 0.0;
    ctmrg_options opt{};
    std::vector<double> V;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // device state and work buffers
    double *dV = nullptr, *dW = nullptr, *dWH = nullptr;
    double *dA = nullptr, *dOA = nullptr, *dPt = nullptr;
    double *dOmega = nullptr, *dOmNew = nullptr, *dSel = nullptr;
    double *dX = nullptr, *dC = nullptr, *dU = nullptr;
    double *dPart = nullptr, *dObs = nullptr, *dH = nullptr, *dWork = nullptr;
    size_t work_elems = 0;
    // mixed precision (FP32 contractions): W / wscale, A, diag(omega) A and U in FP32
    float *dW32 = nullptr, *dA32 = nullptr, *dOA32 = nullptr, *dU32 = nullptr;
    double wscale = 1.0;
    Book *dBook = nullptr;
    PostOut *dPost = nullptr;
    PostOut *hPost = nullptr;
    EigWork eig;
    // warm-started eigensolver: its workspace, the top-k selection of a fallback step
    WarmWork warm;
    int warm_p = 0, warm_k = 0;
    double *dSelK = nullptr, *dOmK = nullptr;
    PostOut *dPostK = nullptr, *hPostK = nullptr;
    int m_eff_prev2 = 0;  // kept dimension of the step before the last
    // N x N: the half-row Z of a warm-mode step, which leaves that step's C' in dC
    double *dZ = nullptr;
    bool last_warm = false;  // the last step was solved warm (its C' is intact in dC)
    bool carved = false;     // the device buffers of init are carved from the caller's workspace
    // effective correlation length (Lanczos on the row-to-row transfer matrix), allocated on first use
    XiWork xi;
    // fixed-point derivative: its workspace and the weight at K +- dK
    AdjWork adj;
    double *dWd = nullptr, *dWHd = nullptr;
    // host-side status
    int m_eff = 1;
    int steps = 0;
    double delta = INFINITY;
    double c_paper = INFINITY;
    double S_last = 0.0;
    bool have_U = false;
    bool cext_valid = false;
    // stage timing (HIP events on the context's stream)
    bool profile = false;
    hipEvent_t ev[MK_COUNT] = {};
    double stage_ms[MK_COUNT] = {};
    int timed_steps = 0;
    double warm_last_tail = 0.0;
    double warm_last_SE = 0.0;        // S_E as the last warm step gave it (bounded tail)
    std::string err;
};

namespace {

const uint32_t kStateMagic = 0x534d5443u;  // "CTMS"

struct StateHeader {
    uint32_t magic, version;
    int32_t q, m, m_eff, steps, bc, s0;
    double K, delta, c_paper;
    Book book;
};

ctmrg_status fail(ctmrg_ctx *c, ctmrg_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

ctmrg_status hip_fail(ctmrg_ctx *c, hipError_t e, const char *where)
{
    return fail(c, e == hipErrorOutOfMemory ? CTMRG_E_OUT_OF_MEMORY : CTMRG_E_HIP,
                std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                   \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

bool valid_band(int b) { return b == 16 || b == 32; }

bool valid_eig_options(const ctmrg_options &o)
{
    if (o.eig_solver != CTMRG_EIG_TWO_STAGE && o.eig_solver != CTMRG_EIG_WARM) return false;
    if (o.warm_guard < 0 || o.warm_degree < 0 || o.warm_degree > WARM_DMAX || !(o.warm_tol >= 0.0)) return false;
    if (o.warm_tail != CTMRG_WARM_TAIL_EXACT && o.warm_tail != CTMRG_WARM_TAIL_BOUND &&
        o.warm_tail != CTMRG_WARM_TAIL_AUTO)
        return false;
    return true;
}

ctmrg_status check_device(ctmrg_ctx *c)
{
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(c, hipGetDeviceProperties(&prop, dev));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(c, CTMRG_E_UNSUPPORTED, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
    c->device = dev;
    return CTMRG_OK;
}

void free_all(ctmrg_ctx *c)
{
    xi_free(c->xi);
    double *bufs[] = {c->dV, c->dW, c->dWH, c->dA, c->dOA, c->dPt, c->dOmega, c->dOmNew, c->dSel,
                      c->dX, c->dC, c->dU, c->dPart, c->dObs, c->dH, c->dWork, c->dZ, c->dSelK, c->dOmK};
    float *fbufs[] = {c->dW32, c->dA32, c->dOA32, c->dU32};
    if (!c->carved) {
        for (double *p : bufs)
            if (p) (void)hipFree(p);
        for (float *p : fbufs)
            if (p) (void)hipFree(p);
        if (c->dBook) (void)hipFree(c->dBook);
        if (c->dPost) (void)hipFree(c->dPost);
        if (c->dPostK) (void)hipFree(c->dPostK);
    }
    if (c->hPost) (void)hipHostFree(c->hPost);
    if (c->hPostK) (void)hipHostFree(c->hPostK);
    warm_free(c->warm);
    eig_free(c->eig);
    adj_free(c->adj);
    if (c->dWd) (void)hipFree(c->dWd);
    if (c->dWHd) (void)hipFree(c->dWHd);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    for (int i = 0; i < MK_COUNT; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
}

int warm_guard(const ctmrg_options &o, int m) { return o.warm_guard > 0 ? o.warm_guard : std::max(8, m / 4); }

// Every device buffer a context allocates at init, through the arena, in one fixed order (a
// count-only pass gives the bytes of the carving).
hipError_t alloc_device(ctmrg_ctx *c, Arena &a)
{
    const int q = c->q, m = c->m, dim = c->dim;
    const long N = c->N;
    const ctmrg_options &o = c->opt;
    const size_t q4 = (size_t)q * q * q * q;
    c->work_elems = 64 * q4;
    struct Req { double **p; size_t n; };
    Req reqs[] = {
        {&c->dV, (size_t)q * dim}, {&c->dW, q4}, {&c->dWH, q4},
        {&c->dA, (size_t)m * N}, {&c->dOA, (size_t)m * N}, {&c->dPt, (size_t)m * N},
        {&c->dOmega, (size_t)m}, {&c->dOmNew, (size_t)m}, {&c->dSel, (size_t)m + 8},
        {&c->dX, (size_t)N * N}, {&c->dC, (size_t)N * N}, {&c->dU, (size_t)N * m},
        {&c->dPart, 4096}, {&c->dObs, (size_t)64 + q}, {&c->dH, q4}, {&c->dWork, c->work_elems},
    };
    hipError_t e = hipSuccess;
    for (auto &r : reqs)
        if (e == hipSuccess) e = a.take((void **)r.p, sizeof(double) * std::max<size_t>(r.n, 1));
    if (o.precision != CTMRG_FP64) {
        struct ReqF { float **p; size_t n; };
        ReqF fr[] = {{&c->dW32, q4}, {&c->dA32, (size_t)m * N}, {&c->dOA32, (size_t)m * N}, {&c->dU32, (size_t)N * m}};
        for (auto &r : fr)
            if (e == hipSuccess) e = a.take((void **)r.p, sizeof(float) * std::max<size_t>(r.n, 1));
    }
    if (e == hipSuccess) e = a.take((void **)&c->dBook, sizeof(Book));
    if (e == hipSuccess) e = a.take((void **)&c->dPost, sizeof(PostOut));
    const bool warm = o.eig_solver == CTMRG_EIG_WARM;
    if (warm) {
        c->warm_p = warm_guard(o, m);
        c->warm_k = (int)std::min<long>(N, (long)m + c->warm_p);
    }
    // the eigensolver's workspace: one block when carving
    const int kk = warm ? c->warm_k : m;
    if (e == hipSuccess) {
        if (a.carving()) {
            void *base = nullptr;
            const size_t eb = eig_bytes((int)N, kk, o.band);
            e = a.take(&base, eb);
            if (e == hipSuccess && !a.count_only) e = eig_carve(c->eig, base, eb, (int)N, kk, o.band, c->stream);
            if (e == hipSuccess && !a.count_only) e = eig_attach_streams(c->eig);
        } else {
            e = eig_alloc(c->eig, (int)N, kk, o.band);
        }
    }
    if (warm) {
        if (e == hipSuccess) e = warm_alloc(c->warm, (int)N, m, c->warm_p, &a, c->stream);
        if (e == hipSuccess) e = a.take((void **)&c->dSelK, sizeof(double) * ((size_t)c->warm_k + 8));
        if (e == hipSuccess) e = a.take((void **)&c->dOmK, sizeof(double) * ((size_t)c->warm_k + 8));
        if (e == hipSuccess) e = a.take((void **)&c->dPostK, sizeof(PostOut));
        if (e == hipSuccess) e = a.take((void **)&c->dZ, sizeof(double) * (size_t)N * N);
    }
    return e;
}

// The bytes alloc_device carves (each buffer rounded up to 256 bytes).
size_t context_bytes(int q, int m, int dim, const ctmrg_options &o)
{
    ctmrg_ctx t;
    t.q = q;
    t.m = m;
    t.dim = dim;
    t.N = q * m;
    t.opt = o;
    Arena a;
    a.count_only = true;
    (void)alloc_device(&t, a);
    return a.used;
}

ctmrg_status reset_state(ctmrg_ctx *c)
{
    HIPCHK(c, init_state(c->dA, c->dOmega, c->q, c->m, c->opt.bc, c->opt.boundary_spin, c->dBook, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->m_eff = 1;
    c->steps = 0;
    c->delta = INFINITY;
    c->c_paper = INFINITY;
    c->S_last = 0.0;
    c->have_U = false;
    c->cext_valid = false;
    c->warm.kcur = 0;
    c->m_eff_prev2 = 0;
    c->last_warm = false;
    return CTMRG_OK;
}

ctmrg_status check_kernel_errors(ctmrg_ctx *c)
{
    unsigned e = eig_take_errors(c->eig);
    if (e & KERR_WAIT_TIMEOUT)
        return fail(c, CTMRG_E_NUMERICAL, "a bounded kernel wait hit its spin limit (code " + std::to_string(e) + ")");
    if (e & KERR_NONFINITE) return fail(c, CTMRG_E_NUMERICAL, "inverse iteration produced a non-finite vector");
    return CTMRG_OK;
}

// C' = W-mix(A^T Omega A) into dC, in the context's precision (marks MK_EXT between the two products).
hipError_t extend_corner(ctmrg_ctx *c)
{
    const int q = c->q, m = c->m;
    hipStream_t s = c->stream;
    hipError_t e;
    if (c->opt.precision != CTMRG_FP64) {
        const bool x3 = c->opt.precision == CTMRG_BF16X3;
        float *X32 = reinterpret_cast<float *>(c->dX);
        e = state_to_f32(c->dA, c->dOmega, c->dA32, c->dOA32, q, m, s);
        if (e == hipSuccess) e = extension_products_f32(c->dA32, c->dOA32, X32, q, m, x3, s);
        mark(c->eig, MK_EXT, s);
        if (e == hipSuccess) e = weight_mix_f32_to_f64(c->dW32, X32, c->dC, q, m, c->wscale, x3, s);
    } else {
        e = extension_products(c->dA, c->dOmega, c->dOA, c->dX, q, m, s);
        mark(c->eig, MK_EXT, s);
        if (e == hipSuccess) e = weight_mix(c->dW, c->dX, c->dC, q, m, s);
    }
    return e;
}

// W (FP64, and its scaled FP32 copy on the mixed path) for the context's K.
hipError_t make_weight(ctmrg_ctx *c)
{
    hipError_t e = build_weight(c->dV, c->q, c->dim, c->K, c->dW, c->dWH, c->stream);
    if (e != hipSuccess || c->opt.precision == CTMRG_FP64) return e;
    // every plaquette sum of four dot products of unit vectors is at most 4
    c->wscale = exp(4.0 * c->K);
    return weight_to_f32(c->dW, c->dW32, c->q, c->wscale, c->stream);
}

ctmrg_status one_step(ctmrg_ctx *c)
{
    const int q = c->q, m = c->m, N = c->N;
    hipStream_t s = c->stream;
    c->eig.marks = c->profile ? c->ev : nullptr;
    mark(c->eig, MK_START, s);
    // extension: X = A^T Omega A, C' = W-mix(X)
    HIPCHK(c, extend_corner(c));
    mark(c->eig, MK_WMIX1, s);
    c->cext_valid = false;
    const bool warm_mode = c->opt.eig_solver == CTMRG_EIG_WARM;
    const int m_eff_prev = c->have_U ? c->m_eff : 0;
    // warm-started solve from the previous step's block when the last two steps kept the same
    // dimension, or (m >= 64) both kept all but at most one multiplet (<= 8 states) of m: a flip
    // of the cut by a multiplet near m is handled inside (the block holds m + p vectors, and the
    // gauge is aligned over the states both steps kept), while the early steps, whose kept
    // dimension still grows and whose C' has few nonzero eigenvalues, reseed from the two-stage
    // solver
    int warm_done = 0;
    const bool same_dim = c->m_eff == c->m_eff_prev2 ||
                          (c->m >= 64 && c->m_eff_prev2 > 0 && std::min(c->m_eff, c->m_eff_prev2) >= c->m - 8);
    if (warm_mode && c->warm.kcur > 0 && c->have_U && same_dim) {
        WarmParams prm;
        prm.gap_tol = c->opt.gap_tol;
        prm.rank_tol = c->opt.rank_tol;
        prm.degree = c->opt.warm_degree > 0 ? c->opt.warm_degree : 8;
        // residual tolerance: on the mixed paths C' itself carries a rounding error of about 1e-6 of
        // |lambda_1| (Frobenius), so residuals below 1e-8 |lambda_1| leave the kept pairs as accurate as
        // C' allows
        prm.tol = c->opt.warm_tol > 0.0 ? c->opt.warm_tol : (c->opt.precision != CTMRG_FP64 ? 1e-8 : 1e-12);
        prm.profile = c->profile;
        // the exact tail only where the bound could matter at the contractions' own precision
        prm.tail_exact = c->opt.warm_tail == CTMRG_WARM_TAIL_EXACT;
        prm.tail_tol = c->opt.precision != CTMRG_FP64 ? 1e-9 : 1e-14;
        std::string why;
        const long attempts = c->warm.steps;
        // dX (N x N) is free between the extension and the half-row products
        HIPCHK(c, warm_symmetrize(c->dC, N, s));
        double *sq = (c->opt.warm_tail != CTMRG_WARM_TAIL_BOUND) ? c->dX : nullptr;
        HIPCHK(c, warm_solve(c->warm, c->dC, N, m, prm, c->dOmega, c->dOmNew, c->dSel, c->dPost, c->dU, m_eff_prev,
                             c->eig.evals, sq, s, &warm_done, &why));
        if (!warm_done && c->warm.steps > attempts) c->warm.fallbacks += 1;
    }
    mark(c->eig, MK_WARM_END, s);
    if (warm_done) {
        // the two-stage stages take no time in this step
        static const int skipped[] = {MK_STAGE1, MK_BULGE, MK_BISECT, MK_POST, MK_VEC_START, MK_INVIT, MK_NS,
                                      MK_BT2, MK_BT1};
        for (int id : skipped) mark(c->eig, id, s);
        HIPCHK(c, hipMemcpyAsync(c->hPost, c->dPost, sizeof(PostOut), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    } else {
        // eigenvalues, selection, normalization, entropy, convergence
        HIPCHK(c, eig_values(c->eig, c->dC, N, N, s));
        HIPCHK(c, eig_post(c->eig, N, m, c->opt.gap_tol, c->opt.rank_tol, c->dOmega, c->dOmNew, c->dSel, c->dPost, s));
        // warm mode: the top k = m + p as well (the next step's start), into separate outputs
        if (warm_mode)
            HIPCHK(c, eig_post(c->eig, N, c->warm_k, c->opt.gap_tol, c->opt.rank_tol, c->warm.zero, c->dOmK, c->dSelK,
                               c->dPostK, s));
        mark(c->eig, MK_POST, s);
        HIPCHK(c, hipMemcpyAsync(c->hPost, c->dPost, sizeof(PostOut), hipMemcpyDeviceToHost, s));
        if (warm_mode) HIPCHK(c, hipMemcpyAsync(c->hPostK, c->dPostK, sizeof(PostOut), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    ctmrg_status st = check_kernel_errors(c);
    if (st != CTMRG_OK) return st;
    const PostOut po = *c->hPost;
    if (!std::isfinite(po.n_C) || !(po.n_C > 0.0) || !std::isfinite(po.S_E))
        return fail(c, CTMRG_E_NUMERICAL, "non-finite spectrum of the extended corner");
    if (warm_done) {
        c->warm.tail_bound_max = std::max(c->warm.tail_bound_max, po.tail_bound);
        c->warm_last_tail = po.tail_bound;
        c->warm_last_SE = po.S_E;
    } else if (warm_mode) {
        // eigenvectors of the top k (kept first), kept ones aligned with the previous step's
        const PostOut pk = *c->hPostK;
        HIPCHK(c, eig_vectors(c->eig, nullptr, 0, N, pk.m_eff, c->dSelK, pk.nclusters, c->warm.V, c->warm.kmax, s));
        HIPCHK(c, warm_seed(c->warm, N, m, po.m_eff, pk.m_eff, c->dSelK, c->dU, m_eff_prev, c->opt.gap_tol, s));
        c->warm_last_tail = 0.0;
    } else {
        // eigenvectors of the kept states
        HIPCHK(c, eig_vectors(c->eig, nullptr, 0, N, po.m_eff, c->dSel, po.nclusters, c->dU, m, s));
    }
    // half-row: Y = A^T U~, Z = W-mix(Y), P~ = U^T Z
    // warm mode keeps this step's C' (for the exact S_E of ctmrg_observables): Z goes to dZ
    double *Zb = warm_mode ? c->dZ : c->dC;
    c->last_warm = warm_done != 0;
    if (c->opt.precision != CTMRG_FP64) {
        const bool x3 = c->opt.precision == CTMRG_BF16X3;
        float *Y32 = reinterpret_cast<float *>(c->dX), *Z32 = reinterpret_cast<float *>(Zb);
        HIPCHK(c, vectors_to_f32(c->dU, c->dU32, q, m, s));
        HIPCHK(c, halfrow_products_f32(c->dA32, c->dU32, Y32, q, m, x3, s));
        mark(c->eig, MK_HALF, s);
        HIPCHK(c, weight_mix_f32(c->dW32, Y32, Z32, q, m, x3, s));
        mark(c->eig, MK_WMIX2, s);
        // dX (Y32) is free once Z is formed: it takes the projection's split-K partials
        HIPCHK(c, projection_f32(c->dU32, Z32, c->dPt, q, m, c->wscale, c->dX, (size_t)N * N, x3, s));
    } else {
        HIPCHK(c, halfrow_products(c->dA, c->dU, c->dX, q, m, s));
        mark(c->eig, MK_HALF, s);
        HIPCHK(c, weight_mix(c->dW, c->dX, Zb, q, m, s));
        mark(c->eig, MK_WMIX2, s);
        HIPCHK(c, projection(c->dU, Zb, c->dPt, q, m, c->dX, (size_t)N * N, s));
    }
    mark(c->eig, MK_PROJ, s);
    HIPCHK(c, normalize_and_book(c->dPt, c->dA, q, m, c->dPart, c->dBook, &c->dPost->n_C, &c->dPost->S_E, s));
    HIPCHK(c, hipMemcpyAsync(c->dOmega, c->dOmNew, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    mark(c->eig, MK_NORM, s);
    // the eigenvector kernels raise their error flags after the mid-step check above:
    // drain them before the step is reported as done
    HIPCHK(c, hipStreamSynchronize(s));
    st = check_kernel_errors(c);
    if (st != CTMRG_OK) return st;
    if (c->profile) {
        // stage i spans marks (from[i], to[i])
        static const int from[] = {MK_START, MK_EXT, MK_WARM_END, MK_STAGE1, MK_BULGE, MK_BISECT, MK_VEC_START,
                                   MK_INVIT, MK_NS, MK_BT2, MK_BT1, MK_HALF, MK_WMIX2, MK_PROJ};
        static const int to[] = {MK_EXT, MK_WMIX1, MK_STAGE1, MK_BULGE, MK_BISECT, MK_POST, MK_INVIT, MK_NS,
                                 MK_BT2, MK_BT1, MK_HALF, MK_WMIX2, MK_PROJ, MK_NORM};
        for (int i = 0; i < 14; ++i) {
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev[from[i]], c->ev[to[i]]));
            c->stage_ms[i] += ms;
        }
        float tot = 0.f, wm = 0.f;
        HIPCHK(c, hipEventElapsedTime(&tot, c->ev[MK_START], c->ev[MK_NORM]));
        HIPCHK(c, hipEventElapsedTime(&wm, c->ev[MK_WMIX1], c->ev[MK_WARM_END]));
        c->stage_ms[14] += tot;
        c->stage_ms[15] += wm;
        c->timed_steps += 1;
    }
    c->eig.marks = nullptr;
    c->c_paper = (c->steps > 0 && c->S_last != 0.0) ? fabs(1.0 - po.S_E / c->S_last) : INFINITY;
    c->S_last = po.S_E;
    c->m_eff_prev2 = c->m_eff;
    c->m_eff = po.m_eff;
    c->delta = po.delta;
    c->have_U = true;
    c->steps += 1;
    return CTMRG_OK;
}

}  // namespace

extern "C" {

ctmrg_status ctmrg_default_options(ctmrg_options *opt)
{
    if (!opt) return CTMRG_E_INVALID_ARG;
    opt->precision = CTMRG_FP64;
    opt->bc = CTMRG_BC_FIXED;
    opt->boundary_spin = 0;
    opt->band = 16;
    opt->gap_tol = 1e-10;
    opt->rank_tol = 1e-13;
    opt->hip_stream = nullptr;
    opt->eig_solver = CTMRG_EIG_TWO_STAGE;
    opt->warm_guard = 0;
    opt->warm_degree = 0;
    opt->warm_tol = 0.0;
    opt->warm_tail = CTMRG_WARM_TAIL_AUTO;
    return CTMRG_OK;
}

ctmrg_status ctmrg_extra_workspace_size(int q, int m, const ctmrg_options *opt, size_t *observables_bytes,
                                        size_t *derivative_bytes)
{
    if (q < 2 || m < 1) return CTMRG_E_INVALID_ARG;
    ctmrg_options o;
    ctmrg_default_options(&o);
    if (opt) o = *opt;
    if (!valid_band(o.band)) return CTMRG_E_INVALID_ARG;
    if (observables_bytes) *observables_bytes = xi_bytes(q, m, (int)std::min<long>(400, (long)m * m));
    if (derivative_bytes) *derivative_bytes = adj_bytes(q, m, o.band);
    return CTMRG_OK;
}

ctmrg_status ctmrg_workspace_size(int q, int m, const ctmrg_options *opt, size_t *bytes)
{
    if (q < 2 || m < 1 || !bytes) return CTMRG_E_INVALID_ARG;
    ctmrg_options o;
    ctmrg_default_options(&o);
    if (opt) o = *opt;
    if (!valid_band(o.band)) return CTMRG_E_INVALID_ARG;
    if (o.precision != CTMRG_FP64 && o.precision != CTMRG_FP32 && o.precision != CTMRG_BF16X3)
        return CTMRG_E_INVALID_ARG;
    if (!valid_eig_options(o)) return CTMRG_E_INVALID_ARG;
    *bytes = context_bytes(q, m, 3, o);
    return CTMRG_OK;
}

ctmrg_status ctmrg_init(int q, int dim, const double *vertex_vectors, double K, int m, const ctmrg_options *opt,
                        ctmrg_ctx **out)
{
    if (!out) return CTMRG_E_INVALID_ARG;
    *out = nullptr;
    if (q < 2 || dim < 1 || dim > 3 || m < 1 || !vertex_vectors || !(K > 0.0) || !std::isfinite(K))
        return CTMRG_E_INVALID_ARG;
    for (int s = 0; s < q; ++s) {
        double n2 = 0.0;
        for (int x = 0; x < dim; ++x) n2 += vertex_vectors[s * dim + x] * vertex_vectors[s * dim + x];
        if (fabs(sqrt(n2) - 1.0) > 1e-10) return CTMRG_E_INVALID_ARG;
    }
    ctmrg_options o;
    ctmrg_default_options(&o);
    if (opt) o = *opt;
    if (!valid_band(o.band) || o.boundary_spin < 0 || o.boundary_spin >= q || (o.bc != 0 && o.bc != 1))
        return CTMRG_E_INVALID_ARG;
    if (o.precision != CTMRG_FP64 && o.precision != CTMRG_FP32 && o.precision != CTMRG_BF16X3)
        return CTMRG_E_INVALID_ARG;
    if (!valid_eig_options(o)) return CTMRG_E_INVALID_ARG;
    const long N = (long)q * m;
    if (N > 65536) return CTMRG_E_INVALID_ARG;

    ctmrg_ctx *c = new (std::nothrow) ctmrg_ctx();
    if (!c) return CTMRG_E_OUT_OF_MEMORY;
    c->q = q; c->dim = dim; c->m = m; c->N = (int)N; c->K = K; c->opt = o;
    c->V.assign(vertex_vectors, vertex_vectors + (size_t)q * dim);
    ctmrg_status st = check_device(c);
    if (st != CTMRG_OK) { *out = c; return st; }
    if (o.hip_stream) {
        c->stream = (hipStream_t)o.hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            *out = c;
            return fail(c, CTMRG_E_HIP, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    Arena arena;
    if (o.workspace) {
        const size_t need = context_bytes(q, m, dim, o);
        if (o.workspace_bytes < need) {
            *out = c;
            return fail(c, CTMRG_E_INVALID_ARG, "workspace smaller than ctmrg_workspace_size");
        }
        arena.base = static_cast<char *>(o.workspace);
        arena.cap = o.workspace_bytes;
        c->carved = true;
    }
    hipError_t e = alloc_device(c, arena);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->hPost, sizeof(PostOut), hipHostMallocDefault);
    if (e == hipSuccess && o.eig_solver == CTMRG_EIG_WARM)
        e = hipHostMalloc((void **)&c->hPostK, sizeof(PostOut), hipHostMallocDefault);
    if (e != hipSuccess) { *out = c; return hip_fail(c, e, "allocation"); }
    e = hipMemcpy(c->dV, c->V.data(), sizeof(double) * q * dim, hipMemcpyHostToDevice);
    if (e != hipSuccess) { *out = c; return hip_fail(c, e, "hipMemcpy"); }
    e = make_weight(c);
    if (e != hipSuccess) { *out = c; return hip_fail(c, e, "build_weight"); }
    st = reset_state(c);
    *out = c;
    return st;
}

ctmrg_status ctmrg_set_K(ctmrg_ctx *c, double K)
{
    if (!c) return CTMRG_E_INVALID_ARG;
    if (!(K > 0.0) || !std::isfinite(K)) return fail(c, CTMRG_E_INVALID_ARG, "K must be positive");
    c->K = K;
    HIPCHK(c, make_weight(c));
    return reset_state(c);
}

// The flags that the last step's eigenvector kernels may have raised (each step checks those of
// the step before): drained once the stream is idle, before a stepping call returns.
static ctmrg_status finish_steps(ctmrg_ctx *c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_kernel_errors(c);
}

ctmrg_status ctmrg_step(ctmrg_ctx *c, int nsteps, double *delta_out)
{
    if (!c || nsteps < 0) return CTMRG_E_INVALID_ARG;
    for (int i = 0; i < nsteps; ++i) {
        ctmrg_status st = one_step(c);
        if (st != CTMRG_OK) return st;
    }
    if (nsteps > 0) {
        const ctmrg_status st = finish_steps(c);
        if (st != CTMRG_OK) return st;
    }
    if (delta_out) *delta_out = c->delta;
    return CTMRG_OK;
}

ctmrg_status ctmrg_run_to_fixed_point(ctmrg_ctx *c, double tol, int max_steps, int *steps_out, double *delta_out)
{
    if (!c || max_steps < 0 || !(tol >= 0.0)) return CTMRG_E_INVALID_ARG;
    int taken = 0;
    ctmrg_status st = CTMRG_E_NOT_CONVERGED;
    while (taken < max_steps) {
        ctmrg_status s1 = one_step(c);
        if (s1 != CTMRG_OK) { st = s1; break; }
        ++taken;
        if (c->steps >= 2 && c->delta < tol) { st = CTMRG_OK; break; }
    }
    if (taken > 0 && (st == CTMRG_OK || st == CTMRG_E_NOT_CONVERGED)) {
        const ctmrg_status sf = finish_steps(c);
        if (sf != CTMRG_OK) st = sf;
    }
    if (steps_out) *steps_out = taken;
    if (delta_out) *delta_out = c->delta;
    if (st == CTMRG_E_NOT_CONVERGED) c->err = "max_steps reached before Delta < tol";
    return st;
}

ctmrg_status ctmrg_sweep(ctmrg_ctx *c, int n, const double *T, double tol, int max_steps, int warm_start,
                         ctmrg_observables_t *out, int *steps_out, int *converged, ctmrg_derivative_t *deriv_out)
{
    if (!c || n < 0 || (n > 0 && (!T || !out)) || max_steps < 2 || !(tol >= 0.0)) return CTMRG_E_INVALID_ARG;
    for (int i = 0; i < n; ++i)
        if (!(T[i] > 0.0) || !std::isfinite(T[i])) return fail(c, CTMRG_E_INVALID_ARG, "temperatures must be positive");
    // with CTMRG_PROGRESS set in the environment, every hundredth step is reported on stderr
    const char *pe = getenv("CTMRG_PROGRESS");
    const bool progress = pe && *pe && *pe != '0';
    for (int i = 0; i < n; ++i) {
        const double K = 1.0 / T[i];
        if (warm_start && (i > 0 || c->steps > 0)) {
            // the previous temperature's fixed point (or the state the context holds) is the
            // start: new weights, same state
            c->K = K;
            HIPCHK(c, make_weight(c));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        } else {
            const ctmrg_status st = ctmrg_set_K(c, K);
            if (st != CTMRG_OK) return st;
        }
        // at least two steps at each temperature: Delta then compares two steps at the same K
        int taken = 0;
        bool conv = false;
        while (taken < max_steps) {
            const ctmrg_status st = one_step(c);
            if (st != CTMRG_OK) return st;
            ++taken;
            if (progress && taken % 100 == 0)
                fprintf(stderr, "[ctmrg sweep] T = %.6f: step %d, Delta %.3e\n", T[i], taken, c->delta);
            if (taken >= 2 && c->delta < tol) {
                conv = true;
                break;
            }
        }
        if (steps_out) steps_out[i] = taken;
        if (converged) converged[i] = conv ? 1 : 0;
        const ctmrg_status st = ctmrg_observables(c, out + i, nullptr);
        if (st != CTMRG_OK) return st;
        if (deriv_out) {
            deriv_out[i] = ctmrg_derivative_t{};
            if (conv && c->delta < 1e-6) {
                const ctmrg_status sd = ctmrg_fixed_point_derivative(c, 1, deriv_out + i);
                if (sd == CTMRG_E_NOT_CONVERGED || sd == CTMRG_E_NUMERICAL) {
                    deriv_out[i] = ctmrg_derivative_t{};
                    deriv_out[i].status = sd;
                    if (progress) fprintf(stderr, "[ctmrg sweep] T = %.6f: derivative: %s\n", T[i], c->err.c_str());
                } else if (sd != CTMRG_OK) {
                    return sd;
                }
            }
        }
    }
    return CTMRG_OK;
}

ctmrg_status ctmrg_observables(ctmrg_ctx *c, ctmrg_observables_t *out, double *kept_spectrum)
{
    if (!c || !out) return CTMRG_E_INVALID_ARG;
    if (c->steps < 1 || !c->have_U) return fail(c, CTMRG_E_STATE, "observables need at least one step");
    if (c->last_warm) {
        // S_E (Eq. 6) over all eigenvalues of the last step's C' (left in dC by a warm step)
        const size_t n2 = (size_t)c->N * c->N;
        HIPCHK(c, hipMemcpyAsync(c->dX, c->dC, sizeof(double) * n2, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, eig_values(c->eig, c->dX, c->N, c->N, c->stream));
        HIPCHK(c, eig_post(c->eig, c->N, c->warm_k, c->opt.gap_tol, c->opt.rank_tol, c->warm.zero, c->dOmK, c->dSelK,
                           c->dPostK, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->hPostK, c->dPostK, sizeof(PostOut), hipMemcpyDeviceToHost, c->stream));
    }
    if (!c->xi.V) HIPCHK(c, xi_alloc(c->xi, c->q, c->m, (int)std::min<long>(400, (long)c->m * c->m)));
    XiResult xr;
    HIPCHK(c, xi_solve(c->xi, c->dA, c->q, c->m, 1e-11, c->stream, &xr));
    HIPCHK(c, observables(c->dA, c->dOmega, c->dU, c->dW, c->dWH, c->dV, c->dOA, c->dX, c->dH, c->dWork,
                          c->work_elems, c->q, c->dim, c->m, c->opt.bc, c->opt.boundary_spin, c->dObs, c->stream));
    double obs[8];
    Book bk;
    HIPCHK(c, hipMemcpyAsync(obs, c->dObs, sizeof(obs), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&bk, c->dBook, sizeof(Book), hipMemcpyDeviceToHost, c->stream));
    if (kept_spectrum)
        HIPCHK(c, hipMemcpyAsync(kept_spectrum, c->dOmega, sizeof(double) * c->m, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    {
        // flags of the last step's eigenvector kernels and of this call's eigenvalue solve
        const ctmrg_status st = check_kernel_errors(c);
        if (st != CTMRG_OK) return st;
    }
    const double T = 1.0 / c->K;
    // the free energy is a ratio of the normalizations of two consecutive steps
    out->ln_kappa_W = c->steps >= 2 ? log(bk.nP_prev) + 0.5 * log(bk.nC / bk.nC_prev) : NAN;
    out->f = -0.5 * T * out->ln_kappa_W;
    out->ln_kappa_ratio = log(obs[2]) + log(obs[0]) - 2.0 * log(obs[1]);
    out->E = 0.5 * obs[3] / obs[2];
    out->M = obs[5] / obs[6];
    out->S_E = c->last_warm ? c->hPostK->S_E : bk.S;
    out->delta = c->delta;
    out->c_paper = (bk.S_prev != 0.0) ? fabs(1.0 - bk.S / bk.S_prev) : INFINITY;
    out->m_eff = c->m_eff;
    out->steps = c->steps;
    out->xi_e = xr.xi;
    out->tm_lambda1 = xr.lambda1;
    out->tm_lambda2 = xr.lambda2;
    out->tm_residual = xr.residual;
    out->tm_iterations = xr.iterations;
    out->tm_converged = xr.converged ? 1 : 0;
    return CTMRG_OK;
}

namespace {

ctmrg_status derivative_at(ctmrg_ctx *c, const double *W, const double *WH, AdjResult *r)
{
    AdjInputs in;
    in.q = c->q;
    in.m = c->m;
    in.d = c->m_eff;
    in.W = W;
    in.WH = WH;
    in.A = c->dA;
    in.omega = c->dOmega;
    in.U = c->dU;
    in.V = c->dV;
    in.dim = c->dim;
    in.bc = c->opt.bc;
    in.s0 = c->opt.boundary_spin;
    in.gap_tol = c->opt.gap_tol;
    in.rank_tol = c->opt.rank_tol;
    c->adj.band = c->opt.band;
    std::string msg;
    const int st = adjoint_dFdK(c->adj, in, r, c->stream, &msg);
    if (st != CTMRG_OK) return fail(c, (ctmrg_status)st, "fixed-point derivative: " + msg);
    return CTMRG_OK;
}

}  // namespace

ctmrg_status ctmrg_fixed_point_derivative(ctmrg_ctx *c, int second_order, ctmrg_derivative_t *out)
{
    if (!c || !out) return CTMRG_E_INVALID_ARG;
    if (c->steps < 2 || !c->have_U || !(c->delta < 1e-6))
        return fail(c, CTMRG_E_STATE, "the state is not converged (Delta >= 1e-6 or fewer than two steps)");
    AdjResult r;
    ctmrg_status st = derivative_at(c, c->dW, c->dWH, &r);
    if (st != CTMRG_OK) return st;
    *out = ctmrg_derivative_t{};
    out->F = r.F;
    out->dF_dK = r.dFdK;
    out->gauge_residual = r.gauge_residual;
    out->tangent_change = r.tangent_change;
    out->aligned_steps = r.aligned_steps;
    out->iterations = r.iterations;
    out->n_eigen = r.n_eigen;
    out->E = r.E;
    out->M = r.M;
    out->dM_dK = r.dMdK;
    out->dE_dK = r.dEdK;
    out->status = CTMRG_OK;
    if (second_order == 1) out->d2F_dK2 = r.dEdK;
    if (second_order == 2) {
        const size_t q4 = (size_t)c->q * c->q * c->q * c->q;
        if (!c->dWd) HIPCHK(c, hipMalloc((void **)&c->dWd, sizeof(double) * q4));
        if (!c->dWHd) HIPCHK(c, hipMalloc((void **)&c->dWHd, sizeof(double) * q4));
        const double h = 1e-4 * c->K;
        double dF[2];
        for (int side = 0; side < 2; ++side) {
            const double Ks = c->K + (side == 0 ? h : -h);
            HIPCHK(c, build_weight(c->dV, c->q, c->dim, Ks, c->dWd, c->dWHd, c->stream));
            AdjResult rs;
            st = derivative_at(c, c->dWd, c->dWHd, &rs);
            if (st != CTMRG_OK) return st;
            dF[side] = rs.dFdK;
        }
        out->d2F_dK2 = (dF[0] - dF[1]) / (2.0 * h);
    }
    return CTMRG_OK;
}

ctmrg_status ctmrg_backward(ctmrg_ctx *c, const double *obs_bar, double *K_bar, double *d2F_dK2)
{
    if (!c || !obs_bar || !K_bar) return CTMRG_E_INVALID_ARG;
    ctmrg_derivative_t d;
    ctmrg_status st = ctmrg_fixed_point_derivative(c, 1, &d);
    if (st != CTMRG_OK) return st;
    const double K = c->K;
    const double dfdK = d.dF_dK / K - d.F / (K * K);  // f = F / K
    *K_bar = obs_bar[0] * dfdK + obs_bar[1] * d.d2F_dK2 + obs_bar[2] * d.dM_dK;
    if (d2F_dK2) *d2F_dK2 = d.d2F_dK2;
    return CTMRG_OK;
}

ctmrg_status ctmrg_export_state(ctmrg_ctx *c, void *host_buf, size_t *bytes)
{
    if (!c || !bytes) return CTMRG_E_INVALID_ARG;
    const size_t need = sizeof(StateHeader) + sizeof(double) * ((size_t)c->m * c->N + c->m);
    if (!host_buf) { *bytes = need; return CTMRG_OK; }
    if (*bytes < need) return fail(c, CTMRG_E_INVALID_ARG, "buffer too small");
    StateHeader h{};
    h.magic = kStateMagic; h.version = 1; h.q = c->q; h.m = c->m; h.m_eff = c->m_eff; h.steps = c->steps;
    h.bc = c->opt.bc; h.s0 = c->opt.boundary_spin; h.K = c->K; h.delta = c->delta; h.c_paper = c->c_paper;
    HIPCHK(c, hipMemcpyAsync(&h.book, c->dBook, sizeof(Book), hipMemcpyDeviceToHost, c->stream));
    char *p = (char *)host_buf;
    double *pa = (double *)(p + sizeof(StateHeader));
    HIPCHK(c, hipMemcpyAsync(pa, c->dA, sizeof(double) * (size_t)c->m * c->N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(pa + (size_t)c->m * c->N, c->dOmega, sizeof(double) * c->m, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    memcpy(p, &h, sizeof(h));
    *bytes = need;
    return CTMRG_OK;
}

ctmrg_status ctmrg_import_state(ctmrg_ctx *c, const void *host_buf, size_t bytes)
{
    if (!c || !host_buf) return CTMRG_E_INVALID_ARG;
    const size_t need = sizeof(StateHeader) + sizeof(double) * ((size_t)c->m * c->N + c->m);
    if (bytes < need) return fail(c, CTMRG_E_INVALID_ARG, "state buffer too small");
    StateHeader h;
    memcpy(&h, host_buf, sizeof(h));
    if (h.magic != kStateMagic || h.version != 1 || h.q != c->q || h.m != c->m)
        return fail(c, CTMRG_E_INVALID_ARG, "state does not match this context");
    const double *pa = (const double *)((const char *)host_buf + sizeof(StateHeader));
    HIPCHK(c, hipMemcpyAsync(c->dA, pa, sizeof(double) * (size_t)c->m * c->N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dOmega, pa + (size_t)c->m * c->N, sizeof(double) * c->m, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dBook, &h.book, sizeof(Book), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->m_eff = h.m_eff; c->steps = h.steps; c->delta = h.delta; c->c_paper = h.c_paper;
    c->have_U = false;
    c->cext_valid = false;
    c->warm.kcur = 0;
    c->m_eff_prev2 = 0;
    c->last_warm = false;
    return CTMRG_OK;
}

ctmrg_status ctmrg_set_state(ctmrg_ctx *c, int d, const double *P, const double *omega)
{
    if (!c || !P || !omega || d < 1 || d > c->m) return CTMRG_E_INVALID_ARG;
    const int q = c->q, m = c->m;
    const long N = c->N;
    std::vector<double> A((size_t)m * N, 0.0), om(m, 0.0);
    for (int s = 0; s < q; ++s)
        for (int g = 0; g < d; ++g)
            for (int a = 0; a < d; ++a) A[(size_t)g * N + (size_t)s * m + a] = P[((size_t)s * d + g) * d + a];
    for (int i = 0; i < d; ++i) om[i] = omega[i];
    HIPCHK(c, hipMemcpyAsync(c->dA, A.data(), sizeof(double) * A.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dOmega, om.data(), sizeof(double) * m, hipMemcpyHostToDevice, c->stream));
    Book b{};
    b.nC_prev = b.nC = b.nP_prev = b.nP = 1.0;
    HIPCHK(c, hipMemcpyAsync(c->dBook, &b, sizeof(Book), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->m_eff = d; c->steps = 0; c->delta = INFINITY; c->c_paper = INFINITY;
    c->have_U = false; c->cext_valid = false;
    c->warm.kcur = 0; c->m_eff_prev2 = 0; c->last_warm = false;
    return CTMRG_OK;
}

ctmrg_status ctmrg_extend(ctmrg_ctx *c)
{
    if (!c) return CTMRG_E_INVALID_ARG;
    HIPCHK(c, extend_corner(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cext_valid = true;
    c->last_warm = false;
    return CTMRG_OK;
}

ctmrg_status ctmrg_get_buffer(ctmrg_ctx *c, int which, double *dst, size_t count)
{
    if (!c || !dst) return CTMRG_E_INVALID_ARG;
    const size_t N = c->N, m = c->m;
    const double *src = nullptr;
    size_t n = 0;
    switch (which) {
    case CTMRG_BUF_P: src = c->dA; n = m * N; break;
    case CTMRG_BUF_OMEGA: src = c->dOmega; n = m; break;
    case CTMRG_BUF_SPECTRUM: src = c->eig.evals; n = N; break;
    case CTMRG_BUF_U:
        if (!c->have_U) return fail(c, CTMRG_E_STATE, "no eigenvectors yet");
        src = c->dU; n = N * m; break;
    case CTMRG_BUF_CEXT:
        if (!c->cext_valid) return fail(c, CTMRG_E_STATE, "call ctmrg_extend first");
        src = c->dC; n = N * N; break;
    case CTMRG_BUF_W: src = c->dW; n = (size_t)c->q * c->q * c->q * c->q; break;
    default: return fail(c, CTMRG_E_INVALID_ARG, "unknown buffer");
    }
    if (count < n) return fail(c, CTMRG_E_INVALID_ARG, "destination too small");
    HIPCHK(c, hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CTMRG_OK;
}

ctmrg_status ctmrg_eigh_topk(int n, const double *A, int k, int band, double *evals, double *kept_vals,
                             double *evecs)
{
    if (n < 1 || k < 1 || k > n || !A || !evals || !kept_vals || !evecs) return CTMRG_E_INVALID_ARG;
    if (band == 0) band = 16;
    if (!valid_band(band)) return CTMRG_E_INVALID_ARG;
    ctmrg_ctx tmp;
    ctmrg_status st = check_device(&tmp);
    if (st != CTMRG_OK) return st;
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return CTMRG_E_HIP;
    EigWork w;
    double *dA = nullptr, *dU = nullptr, *dom = nullptr, *domn = nullptr, *dsel = nullptr;
    PostOut *dpo = nullptr;
    PostOut po{};
    hipError_t e = eig_alloc(w, n, k, band);
    if (e == hipSuccess) e = hipMalloc((void **)&dA, sizeof(double) * (size_t)n * n);
    if (e == hipSuccess) e = hipMalloc((void **)&dU, sizeof(double) * (size_t)n * k);
    if (e == hipSuccess) e = hipMalloc((void **)&dom, sizeof(double) * (size_t)k);
    if (e == hipSuccess) e = hipMalloc((void **)&domn, sizeof(double) * (size_t)k);
    if (e == hipSuccess) e = hipMalloc((void **)&dsel, sizeof(double) * (size_t)k + 8 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&dpo, sizeof(PostOut));
    if (e == hipSuccess) e = hipMemsetAsync(dom, 0, sizeof(double) * k, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dA, A, sizeof(double) * (size_t)n * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = eig_values(w, dA, n, n, s);
    if (e == hipSuccess) e = eig_post(w, n, k, -1.0, -1.0, dom, domn, dsel, dpo, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&po, dpo, sizeof(PostOut), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    unsigned kerr = 0;
    if (e == hipSuccess) kerr = eig_take_errors(w);
    if (e == hipSuccess && kerr == 0) e = eig_vectors(w, nullptr, 0, n, po.m_eff, dsel, po.nclusters, dU, k, s);
    if (e == hipSuccess) e = hipMemcpyAsync(evals, w.evals, sizeof(double) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(kept_vals, dsel, sizeof(double) * k, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(evecs, dU, sizeof(double) * (size_t)n * k, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && kerr == 0) kerr = eig_take_errors(w);
    (void)hipFree(dA); (void)hipFree(dU); (void)hipFree(dom); (void)hipFree(domn); (void)hipFree(dsel); (void)hipFree(dpo);
    eig_free(w);
    (void)hipStreamDestroy(s);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? CTMRG_E_OUT_OF_MEMORY : CTMRG_E_HIP;
    if (kerr) return CTMRG_E_NUMERICAL;
    return CTMRG_OK;
}

ctmrg_status ctmrg_set_profiling(ctmrg_ctx *c, int enable)
{
    if (!c) return CTMRG_E_INVALID_ARG;
    if (enable && !c->ev[0]) {
        for (int i = 0; i < MK_COUNT; ++i) HIPCHK(c, hipEventCreate(&c->ev[i]));
    }
    c->profile = enable != 0;
    c->warm.product_ms = c->warm.product_flops = 0.0;
    c->warm.product_launches = 0;
    for (int i = 0; i < MK_COUNT; ++i) c->stage_ms[i] = 0.0;
    c->timed_steps = 0;
    return CTMRG_OK;
}

ctmrg_status ctmrg_get_stage_times(ctmrg_ctx *c, double *ms, int *nsteps)
{
    if (!c || !ms || !nsteps) return CTMRG_E_INVALID_ARG;
    for (int i = 0; i < CTMRG_NUM_STAGES; ++i) ms[i] = c->stage_ms[i];
    *nsteps = c->timed_steps;
    return CTMRG_OK;
}

ctmrg_status ctmrg_get_eig_stats(ctmrg_ctx *c, double *out)
{
    if (!c || !out) return CTMRG_E_INVALID_ARG;
    out[0] = (double)(c->warm.steps - c->warm.fallbacks);
    out[1] = (double)c->warm.fallbacks;
    out[2] = (double)c->warm.passes;
    out[3] = (double)c->warm.products;
    out[4] = c->warm.tail_bound_max;
    out[5] = c->warm_last_tail;
    out[6] = (double)c->warm.last_reason;
    out[7] = c->warm.last_rmax;
    out[11] = c->warm_last_SE;
    out[12] = (double)c->warm.exact_tails;
    out[8] = c->warm.product_ms;
    out[9] = c->warm.product_flops;
    out[10] = (double)c->warm.product_launches;
    return CTMRG_OK;
}

const char *ctmrg_last_error(const ctmrg_ctx *c) { return c ? c->err.c_str() : "null context"; }

void ctmrg_destroy(ctmrg_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

}  // extern "C"
