// Shared device helpers for the CTMRG library (gfx950, HIP).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

#define CTMRG_DEVINL __device__ __forceinline__

// Device-coherent accesses (relaxed, agent scope): the load or store is coherent
// across the L2s of all XCDs, and no cache is written back or invalidated.  Data
// that the workgroups of one launch exchange goes through these.
CTMRG_DEVINL double ld_coh(const double *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
CTMRG_DEVINL void st_coh(double *p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Error flags raised by kernels (bitwise OR into a device word).
enum {
    KERR_WAIT_TIMEOUT = 1,
    KERR_NONFINITE = 4,
    KERR_NO_CONVERGENCE = 8,
    KERR_ALIGN = 16,
};
CTMRG_DEVINL void raise_error(unsigned *err, unsigned code)
{
    __hip_atomic_fetch_or(err, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin limit of every bounded wait (each iteration sleeps ~64 clocks).
#define CTMRG_SPIN_LIMIT (1u << 26)

// Block-wide sum of one double per thread (blockDim.x a multiple of 64, <= 1024).
CTMRG_DEVINL double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
CTMRG_DEVINL double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <int NT>
CTMRG_DEVINL double block_sum(double v, double *red /* >= NT/64 doubles */)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

template <int NT>
CTMRG_DEVINL double block_max(double v, double *red)
{
    v = wave_max(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < NT / 64; ++i) s = fmax(s, red[i]);
    return s;
}

// Counter-based uniform random number in [-1, 1) (SplitMix64 finalizer of a 64-bit key).
CTMRG_DEVINL double hash_uniform(uint64_t key)
{
    uint64_t z = key + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Device buffers of a context either from hipMalloc (no base) or carved, 256-byte aligned, from
// one block of device memory the caller owns (base, cap).  count_only: only add up the bytes the
// carving would use (no HIP call).
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    bool count_only = false;
    static size_t round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
    bool carving() const { return base != nullptr || count_only; }
    hipError_t take(void **p, size_t bytes)
    {
        const size_t sz = round(bytes > 0 ? bytes : 1);
        if (count_only) {
            *p = nullptr;
            used += sz;
            return hipSuccess;
        }
        if (!base) return hipMalloc(p, sz);
        if (used + sz > cap) return hipErrorOutOfMemory;
        *p = base + used;
        used += sz;
        return hipSuccess;
    }
};
