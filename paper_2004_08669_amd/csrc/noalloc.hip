// The standalone eigensolver without allocation: ctmrg_eigh_topk_noalloc (include/ctmrg.h).
//
// Every device buffer of the call -- the working copy of the matrix, the eigenvectors, the
// selection and the whole eigensolver workspace -- is laid out in one file-scope device array,
// `scratch`, of CTMRG_NOALLOC_BYTES.  Each GPU the library runs on holds its own copy until the
// process ends.  Host code never passes the array's name to a kernel or a copy: at the first
// call on a device, with that device current, its address on that device is taken once with
// hipGetSymbolAddress and kept per device; every later use goes through that address.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "ctmrg.h"
#include "eig.h"

namespace {

constexpr size_t kScratchBytes = (size_t)CTMRG_NOALLOC_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The device address of this device's copy of the scratch array (taken once per device).
hipError_t scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

__global__ void zero_kernel(double *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

}  // namespace

extern "C" ctmrg_status ctmrg_eigh_topk_noalloc(int n, const double *A, int k, int band, double *evals,
                                                 double *kept_vals, double *evecs)
{
    using namespace ctm;
    if (n < 1 || k < 1 || k > n || !A || !evals || !kept_vals || !evecs) return CTMRG_E_INVALID_ARG;
    if (n > CTMRG_NOALLOC_NMAX || k > CTMRG_NOALLOC_KMAX) return CTMRG_E_INVALID_ARG;
    if (band == 0) band = 16;
    if (band != 16 && band != 32) return CTMRG_E_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CTMRG_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return CTMRG_E_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return CTMRG_E_UNSUPPORTED;
    void *base = nullptr;
    if (scratch_address(dev, &base) != hipSuccess) return CTMRG_E_HIP;

    // layout of this call: A (n x n), U (n x k), omega_prev, omega_new, selection, PostOut, solver workspace
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = p + off;
        off += align256(bytes);
        return q;
    };
    double *dA = (double *)take(sizeof(double) * (size_t)n * n);
    double *dU = (double *)take(sizeof(double) * (size_t)n * k);
    double *dom = (double *)take(sizeof(double) * (size_t)k);
    double *domn = (double *)take(sizeof(double) * (size_t)k);
    double *dsel = (double *)take(sizeof(double) * ((size_t)k + 8));
    PostOut *dpo = (PostOut *)take(sizeof(PostOut));
    if (off + eig_bytes(n, k, band) > kScratchBytes) return CTMRG_E_INVALID_ARG;

    hipStream_t s = nullptr;  // the null stream: no stream is created
    EigWork w;
    hipError_t e = eig_carve(w, p + off, kScratchBytes - off, n, k, band, s);
    PostOut po{};
    if (e == hipSuccess) e = hipMemcpy(dA, A, sizeof(double) * (size_t)n * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, s, dom, k);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = eig_values(w, dA, n, n, s);
    if (e == hipSuccess) e = eig_post(w, n, k, -1.0, -1.0, dom, domn, dsel, dpo, s);
    if (e == hipSuccess) e = hipMemcpy(&po, dpo, sizeof(PostOut), hipMemcpyDeviceToHost);
    unsigned kerr = 0;
    if (e == hipSuccess) kerr = eig_take_errors(w);
    if (e == hipSuccess && kerr == 0) e = eig_vectors(w, nullptr, 0, n, po.m_eff, dsel, po.nclusters, dU, k, s);
    if (e == hipSuccess) e = hipMemcpy(evals, w.evals, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(kept_vals, dsel, sizeof(double) * k, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(evecs, dU, sizeof(double) * (size_t)n * k, hipMemcpyDeviceToHost);
    if (e == hipSuccess && kerr == 0) kerr = eig_take_errors(w);
    if (e != hipSuccess) return CTMRG_E_HIP;
    if (kerr) return CTMRG_E_NUMERICAL;
    return CTMRG_OK;
}
