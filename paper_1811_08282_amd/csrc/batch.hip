// batch.hip -- persistent kernel of the batched swept launch (table and
// ordering described in batch.h).  One workgroup (256 or 512 threads) runs
// one work item at a time with the same tile-phase bodies as the per-phase
// kernels, so a problem solved in a batch is bit-identical to the same
// problem solved alone with the same width.
//
// Every dependency wait is bounded in wall-clock time (s_memrealtime ticks):
// a wait that exceeds the bound records status 1 and makes every workgroup
// leave, so the launch always terminates.
#include "batch.h"
#include "kernels.h"
#include "tile_euler.h"
#include "tile_flat.h"
#include "tile_heat.h"

namespace sw {
namespace {

__device__ __forceinline__ int load_acquire(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_release(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// copy-out of a single-phase problem: level 1 sits in slot 1 of ws0
template <int NT>
__device__ void copy_out(const BatchProblem &P, int tile)
{
    const int64_t c0 = (int64_t)tile * P.w;
    if (P.eq == 0) {  // heat binary64: slot1 = ws0 + n doubles
        const double *src = (const double *)P.ws0 + P.n;
        double *dst = (double *)P.state;
        for (int i = threadIdx.x; i < P.w; i += NT)
            dst[c0 + i] = src[c0 + i];
    } else {          // heat binary32: u1 = ws0 + n floats, c = ws0 + 2n floats
        const float *src = (const float *)P.ws0;
        float *dst = (float *)P.state;
        for (int i = threadIdx.x; i < P.w; i += NT) {
            dst[c0 + i] = src[P.n + c0 + i];
            dst[P.n + c0 + i] = src[2 * P.n + c0 + i];
        }
    }
}

// Tile bodies compiled into a persistent kernel: all of them, or only one
// heat body.  A kernel holds the registers of its largest body, so a batch
// of heat problems alone runs a kernel without the Euler bodies and fits
// twice the workgroups per CU.
enum Bodies { kAllBodies = 0, kHeatF64Only = 1, kHeatF32Only = 2 };

template <int NT, int BODIES>
__global__ void __launch_bounds__(NT) k_batch_persistent(BatchTables b)
{
    extern __shared__ double lds[];
    __shared__ long long s_item;
    __shared__ int s_abort;
    const int tid = threadIdx.x;

    for (;;) {
        if (tid == 0)
            s_item = (long long)atomicAdd(b.ticket, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= b.n_items)
            return;  // uniform: every thread read the same s_item
        const BatchItem it = batch_item(b.problems, b.n_problems, item);
        const BatchProblem &P = b.problems[it.problem];
        const int k = it.phase;
        const int t = it.tile;

        if (tid == 0) {
            int abort = 0;
            int deps[3];
            const int nd = batch_deps(k, t, P.tiles, P.single_phase, deps);
            for (int d = 0; d < nd && !abort; ++d) {
                const int *f = b.flags + P.flag_off + deps[d];
                const long long t0 = __builtin_amdgcn_s_memrealtime();
                while (load_acquire(f) < k - 1) {
                    if (load_acquire(b.status) != 0 ||
                        (long long)__builtin_amdgcn_s_memrealtime() - t0 > b.wait_limit) {
                        store_release(b.status, 1);
                        abort = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            s_abort = abort;
        }
        __syncthreads();
        if (s_abort)
            return;  // uniform
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

        if (P.single_phase && k == 2) {
            copy_out<NT>(P, t);
        } else {
            const int64_t half = P.w / (2 * P.radius);
            const PhaseRange pr = phase_range(k, P.final_level, half, P.radius);
            TileJob jb;
            jb.state = P.state;
            jb.ws_in = (k % 2 == 0) ? P.ws0 : P.ws1;
            jb.ws_out = (k % 2 == 1) ? P.ws0 : P.ws1;
            jb.n = P.n;
            jb.g0 = pr.offset + (int64_t)t * P.w - P.radius;
            jb.base = pr.base;
            jb.coef = P.coef;
            jb.w = P.w;
            jb.j_first = pr.j_first;
            jb.j_last = pr.j_last;
            jb.first = (k == 1);
            jb.last = (k == P.phases) && !P.single_phase;
            jb.final_level = P.final_level;
            if constexpr (BODIES == kHeatF64Only) {
                heat_f64_tile<NT>(jb, lds);
            } else if constexpr (BODIES == kHeatF32Only) {
                heat_f32_tile<NT>(jb, (float *)lds);
            } else {
                // compile-time LDS offsets for the common Euler widths: 256
                // and 512 in four-wave workgroups, 512 and 1024 in eight-wave
                constexpr int kWideA = NT >= 512 ? 1024 : 512;
                constexpr int kWideB = NT >= 512 ? 512 : 256;
                switch (P.eq) {
                case 0: heat_f64_tile<NT>(jb, lds); break;
                case 1: heat_f32_tile<NT>(jb, (float *)lds); break;
                case 2:
                    if (P.w == kWideA)
                        euler_f64_tile<NT, kWideA>(jb, lds);
                    else if (P.w == kWideB)
                        euler_f64_tile<NT, kWideB>(jb, lds);
                    else
                        euler_f64_tile<NT>(jb, lds);
                    break;
                case 3:
                    if (P.w == kWideA)
                        euler_f32_tile<NT, kWideA>(jb, lds);
                    else if (P.w == kWideB)
                        euler_f32_tile<NT, kWideB>(jb, lds);
                    else
                        euler_f32_tile<NT>(jb, lds);
                    break;
                case 4: flat_f64_tile<NT>(jb, lds); break;
                default: flat_f32_tile<NT>(jb, lds); break;
                }
            }
        }
        // publish: every thread's stores reach device scope before the flag
        __threadfence();
        __syncthreads();
        if (tid == 0)
            store_release(b.flags + P.flag_off + t, k);
    }
}

// zero the ticket, the status word and every tile flag (a plain kernel, so
// the sequence can be captured into a graph and replayed)
__global__ void k_batch_reset(unsigned long long *ticket, int *status, int *flags, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *ticket = 0ull;
        *status = 0;
    }
    for (int64_t j = i; j < count; j += (int64_t)gridDim.x * blockDim.x)
        flags[j] = 0;
}

// Table upload carried in the launch arguments: no host buffer has to outlive
// the call, so the upload can be captured into a graph and replayed.
constexpr int kPutWords = 256;  // 2 KiB of payload per launch

struct PutChunk {
    int64_t offset;  // destination byte offset, a multiple of 8
    int64_t words;   // 8-byte words in this chunk, <= kPutWords
    uint64_t data[kPutWords];
};

__global__ void k_batch_put(char *dst, PutChunk c)
{
    uint64_t *d = (uint64_t *)(dst + c.offset);
    for (int64_t i = threadIdx.x; i < c.words; i += blockDim.x)
        d[i] = c.data[i];
}

// After a persistent launch that holds the caller's own state (swept_solve
// routes large heat grids through one): if the launch aborted a dependency
// wait, fill the state with all-ones words (a NaN in binary64 and binary32),
// so that the failure of an asynchronous call shows in its result.
__global__ void k_poison_on_abort(const int *status, uint32_t *state, int64_t words)
{
    if (*status == 0)
        return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        state[i] = 0xffffffffu;
}

template <typename T>
__global__ void k_fill(T *p, int64_t count, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
hipError_t fill(T *p, int64_t count, T v, hipStream_t s)
{
    const int64_t b = (count + 255) / 256;
    const unsigned blocks = (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

template <int NT>
hipError_t occupancy_of(int bodies, size_t lds_bytes, int *blocks_per_cu)
{
    if (bodies == kHeatF64Only)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            blocks_per_cu, k_batch_persistent<NT, kHeatF64Only>, NT, lds_bytes);
    if (bodies == kHeatF32Only)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            blocks_per_cu, k_batch_persistent<NT, kHeatF32Only>, NT, lds_bytes);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks_per_cu, k_batch_persistent<NT, kAllBodies>, NT, lds_bytes);
}

template <int NT>
void launch_persistent(int bodies, int blocks, size_t lds_bytes, hipStream_t s,
                       const BatchTables &t)
{
    if (bodies == kHeatF64Only)
        hipLaunchKernelGGL((k_batch_persistent<NT, kHeatF64Only>), dim3((unsigned)blocks), dim3(NT),
                           lds_bytes, s, t);
    else if (bodies == kHeatF32Only)
        hipLaunchKernelGGL((k_batch_persistent<NT, kHeatF32Only>), dim3((unsigned)blocks), dim3(NT),
                           lds_bytes, s, t);
    else
        hipLaunchKernelGGL((k_batch_persistent<NT, kAllBodies>), dim3((unsigned)blocks), dim3(NT),
                           lds_bytes, s, t);
}

} // namespace

hipError_t poison_on_abort(const void *ws, void *state, size_t bytes, hipStream_t s)
{
    hipLaunchKernelGGL(k_poison_on_abort, dim3(256), dim3(256), 0, s,
                       (const int *)((const char *)ws + 8), (uint32_t *)state,
                       (int64_t)(bytes / 4));
    return hipGetLastError();
}

hipError_t fill_f64(double *p, int64_t count, double v, hipStream_t s) { return fill(p, count, v, s); }
hipError_t fill_f32(float *p, int64_t count, float v, hipStream_t s) { return fill(p, count, v, s); }

hipError_t batch_put(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes % 8 != 0)
        return hipErrorInvalidValue;
    const uint64_t *w = (const uint64_t *)src;
    const int64_t total = (int64_t)(bytes / 8);
    for (int64_t at = 0; at < total; at += kPutWords) {
        PutChunk c;
        c.offset = at * 8;
        c.words = total - at < kPutWords ? total - at : kPutWords;
        for (int64_t i = 0; i < c.words; ++i)
            c.data[i] = w[at + i];
        hipLaunchKernelGGL(k_batch_put, dim3(1), dim3(256), 0, s, (char *)dst, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t batch_occupancy(size_t lds_bytes, int threads, int bodies, int *blocks_per_cu)
{
    return threads == 512 ? occupancy_of<512>(bodies, lds_bytes, blocks_per_cu)
                          : occupancy_of<256>(bodies, lds_bytes, blocks_per_cu);
}

hipError_t batch_launch(const BatchTables &t, int64_t n_flags, int blocks, int threads,
                        int bodies, size_t lds_bytes, hipStream_t s)
{
    const int64_t rb = (n_flags + 255) / 256;
    const unsigned reset_blocks = (unsigned)(rb < 1 ? 1 : (rb > 4096 ? 4096 : rb));
    hipLaunchKernelGGL(k_batch_reset, dim3(reset_blocks), dim3(256), 0, s, t.ticket, t.status,
                       t.flags, n_flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (threads == 512)
        launch_persistent<512>(bodies, blocks, lds_bytes, s, t);
    else
        launch_persistent<256>(bodies, blocks, lds_bytes, s, t);
    return hipGetLastError();
}

} // namespace sw
