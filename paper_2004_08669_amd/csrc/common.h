// Shared device helpers for the CTMRG library (gfx950, HIP).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

#define CTMRG_DEVINL __device__ __forceinline__

// Agent-scope fences: make this thread's global stores visible to every
// workgroup of the device, and make other workgroups' stores visible to it.
CTMRG_DEVINL void fence_release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
CTMRG_DEVINL void fence_acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

CTMRG_DEVINL unsigned atomic_load_acquire(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
CTMRG_DEVINL void atomic_store_release(unsigned *p, unsigned v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
CTMRG_DEVINL unsigned atomic_add_acqrel(unsigned *p, unsigned v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-coherent accesses (relaxed, agent scope: the load or store is coherent
// across the L2s of all XCDs, with no cache writeback or invalidate).  Data that
// workgroups exchange inside one launch goes through these; a writer makes its
// coherent stores complete (wait_mem) before it stores the flag that publishes
// them, and a reader issues its coherent loads after it has seen the flag.
CTMRG_DEVINL double ld_coh(const double *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
CTMRG_DEVINL void st_coh(double *p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
CTMRG_DEVINL unsigned ldu_coh(const unsigned *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
CTMRG_DEVINL void stu_coh(unsigned *p, unsigned v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
// Wait until this thread's outstanding memory operations have completed.
CTMRG_DEVINL void wait_mem()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Error flags raised by kernels (bitwise OR into a device word).
enum {
    KERR_BARRIER_TIMEOUT = 1,
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

// Grid-wide barrier for a launch whose workgroups are all resident (cooperative
// launch).  bar[0] counts arrivals, bar[1] is the generation.  `gen` is the
// generation this workgroup read at kernel start; it is advanced on each call.
// Every thread's memory operations complete before the workgroup arrives.
// With FENCED, one thread per workgroup performs the agent-scope release before
// arriving and the acquire after the wait, so plain loads after the barrier see
// every workgroup's plain stores made before it.  Without it no cache is written
// back or invalidated: only data exchanged through the device-coherent accesses
// above (st_coh / ld_coh) is ordered by the barrier, which leaves the caches of
// concurrently running kernels alone.  Polling uses relaxed loads (an acquire
// load in the loop would invalidate the cache on every iteration).  Returns
// false (and raises KERR_BARRIER_TIMEOUT) if the wait hit the spin limit.
template <bool FENCED = true>
CTMRG_DEVINL bool grid_barrier(unsigned *bar, unsigned nblocks, unsigned &gen, unsigned *err)
{
    __shared__ int ok_shared;
    wait_mem();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        if (FENCED) fence_release_agent();
        unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            stu_coh(&bar[0], 0u);
            wait_mem();
            stu_coh(&bar[1], gen + 1u);
        } else {
            unsigned spins = 0;
            while (ldu_coh(&bar[1]) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > CTMRG_SPIN_LIMIT) {
                    raise_error(err, KERR_BARRIER_TIMEOUT);
                    ok = 0;
                    break;
                }
            }
        }
        if (FENCED) fence_acquire_agent();
        ok_shared = ok;
    }
    gen += 1u;
    __syncthreads();
    return ok_shared != 0;
}

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
