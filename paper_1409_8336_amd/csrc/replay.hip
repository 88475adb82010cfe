// Roofline measurement of the transport: replay kernels that re-issue the
// transport's own memory operations -- one voxel-record gather and one FP64
// tally add per condensed-history step (Sec. II.B.3: the dose is accumulated
// per step) -- in the order a traced transport run issued them, with the same
// grid, workgroups, lanes and epochs, but none of the physics; plus a plain
// stream read (achievable HBM bandwidth) and a plain copy (the reference that
// scales the HBM byte counters).
//
// The trace holds, per loop iteration and lane, the tally element the step
// deposited into (voxel * K + group; 0xFFFFFFFF: no step), see kTrace.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cache.hpp"
#include "device.hpp"

namespace pmc {

namespace {

constexpr int kReplayGather = 1, kReplayAtomic = 2, kReplayCache = 4;

// kMode: kReplayGather re-issues the voxel-record gathers; kReplayAtomic the
// deposits as FP64 atomics straight to the tally; kReplayAtomic|kReplayCache
// the deposits through the workgroup's LDS cache with its epoch flushes, as
// the transport does them.  Mode 0 only streams the trace.  The tally gets
// +0.0 per deposit (unchanged).
template <int kMode>
__global__ void __launch_bounds__(1024) replay_kernel(const uint32_t* __restrict__ trace,
                                                      unsigned long long trace_iters,
                                                      unsigned long long lanes,
                                                      const uint32_t* __restrict__ epochs, int epoch_iters,
                                                      uint32_t k_magic, uint32_t K,
                                                      const uint2* __restrict__ vox, double* tally,
                                                      int n_slots, int probes, unsigned long long* sink)
{
    extern __shared__ double cval[];   // n_slots sums, then n_slots u32 keys
    constexpr bool kCache = (kMode & kReplayCache) != 0;
    uint32_t* ckey = reinterpret_cast<uint32_t*>(cval + n_slots);
    if constexpr (kCache) {
        for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
            cval[i] = 0.0;
            ckey[i] = kTraceNone;
        }
        __syncthreads();
    }
    const unsigned long long g = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
    const uint32_t ne = epochs[blockIdx.x];
    uint32_t acc = 0;
    unsigned long long n = 0;
    for (uint32_t e = 0; e < ne; ++e) {
        for (int it = 0; it < epoch_iters && n < trace_iters; ++it, ++n) {
            const uint32_t key = trace[n * lanes + g];
            acc += key;
            if (key == kTraceNone) continue;
            if constexpr ((kMode & kReplayGather) != 0) {
                // voxel = key / K: a high-product estimate within one of the
                // quotient, corrected (an estimate one too high could index
                // past the grid)
                uint32_t v = __umulhi(key, k_magic);
                v -= (uint32_t)((unsigned long long)v * K > key);
                v += (uint32_t)((unsigned long long)(v + 1u) * K <= key);
                const uint2 r = vox[v];
                acc += r.x ^ r.y;
            }
            if constexpr ((kMode & kReplayAtomic) != 0) {
                if constexpr (kCache) {
                    const int slot = cache_slot(ckey, key, key * 0x9E3779B1u, (uint32_t)n_slots, probes);
                    if (slot >= 0) {
                        unsafeAtomicAdd(&cval[slot], 0.0);
                        continue;
                    }
                }
                __hip_atomic_fetch_add(tally + key, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if constexpr (kCache) {
            __syncthreads();
            for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
                const uint32_t key = ckey[i];
                if (key != kTraceNone) {
                    unsafeAtomicAdd(&tally[key], cval[i]);
                    ckey[i] = kTraceNone;
                    cval[i] = 0.0;
                }
            }
            __syncthreads();
        }
    }
    if (acc == 0x9E3779B1u) sink[0] = acc;   // keeps the loads live
}

__global__ void stream_read_kernel(const uint4* __restrict__ p, unsigned long long n, unsigned long long* sink)
{
    uint32_t acc = 0;
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        const uint4 v = p[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9E3779B1u) sink[0] = acc;
}

__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, unsigned long long n)
{
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, unsigned long long n, uint32_t v)
{
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// trace entries that hold a step
__global__ void count_steps_kernel(const uint32_t* __restrict__ trace, unsigned long long n, unsigned long long* out)
{
    unsigned long long c = 0;
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        c += trace[i] != kTraceNone;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

template <int kMode>
hipError_t launch_mode(const uint32_t* trace, unsigned long long trace_iters, unsigned long long lanes,
                       const uint32_t* epochs, int epoch_iters, int K, const uint2* vox, double* tally,
                       int n_slots, int probes, int grid, int block, unsigned long long* sink, hipStream_t st)
{
    const size_t lds = (kMode & kReplayCache) ? (size_t)n_slots * 12 : 0;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)replay_kernel<kMode>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const uint32_t k_magic = (uint32_t)((0x100000000ull + (unsigned)K - 1) / (unsigned)K);
    hipLaunchKernelGGL(replay_kernel<kMode>, dim3(grid), dim3(block), lds, st, trace, trace_iters, lanes, epochs,
                       epoch_iters, k_magic, (uint32_t)K, vox, tally, n_slots, probes, sink);
    return hipGetLastError();
}

}  // namespace

// mode: 0 trace only, 1 gathers, 2 direct atomics, 3 gathers + direct atomics, 6 cached atomics,
// 7 gathers + cached atomics
hipError_t launch_replay(int mode, const uint32_t* trace, unsigned long long trace_iters, unsigned long long lanes,
                         const uint32_t* epochs, int epoch_iters, int K, const uint2* vox, double* tally,
                         int n_slots, int probes, int grid, int block, unsigned long long* sink, hipStream_t st)
{
    switch (mode) {
    case 0: return launch_mode<0>(trace, trace_iters, lanes, epochs, epoch_iters, K, vox, tally, n_slots, probes,
                                  grid, block, sink, st);
    case 1: return launch_mode<1>(trace, trace_iters, lanes, epochs, epoch_iters, K, vox, tally, n_slots, probes,
                                  grid, block, sink, st);
    case 2: return launch_mode<2>(trace, trace_iters, lanes, epochs, epoch_iters, K, vox, tally, n_slots, probes,
                                  grid, block, sink, st);
    case 3: return launch_mode<3>(trace, trace_iters, lanes, epochs, epoch_iters, K, vox, tally, n_slots, probes,
                                  grid, block, sink, st);
    case 6: return launch_mode<6>(trace, trace_iters, lanes, epochs, epoch_iters, K, vox, tally, n_slots, probes,
                                  grid, block, sink, st);
    case 7: return launch_mode<7>(trace, trace_iters, lanes, epochs, epoch_iters, K, vox, tally, n_slots, probes,
                                  grid, block, sink, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stream_read(const void* p, size_t bytes, unsigned long long* sink, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(256), 0, st, (const uint4*)p,
                       (unsigned long long)(bytes / 16), sink);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, st, (const uint4*)src, (uint4*)dst,
                       (unsigned long long)(bytes / 16));
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, unsigned long long n, uint32_t v, hipStream_t st)
{
    unsigned long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_count_steps(const uint32_t* trace, unsigned long long n, unsigned long long* out, hipStream_t st)
{
    hipLaunchKernelGGL(count_steps_kernel, dim3(8192), dim3(256), 0, st, trace, n, out);
    return hipGetLastError();
}

}  // namespace pmc
