// tile_job.h -- description of one tile of one swept phase, shared by the
// per-phase kernels and the persistent batch kernel.
//
// The tile bodies take the workgroup size NT and, optionally, the tile width
// WT as template parameters: with WT > 0 every LDS offset and loop bound is a
// compile-time constant (the common widths are instantiated; others use the
// run-time width of the job).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

struct TileJob {
    void *state;         // caller state (read when first, written when last)
    const void *ws_in;   // working arrays written by the previous phase
    void *ws_out;        // working arrays of this phase
    int64_t n;           // cells of the problem
    int64_t g0;          // global cell of LDS index 0 (tile start - 1, unwrapped)
    int64_t base;        // (k - 1) * w/2
    double coef;         // r (heat) or lambda (Euler)
    int w;               // tile width
    int j_first, j_last; // relative levels swept by this phase
    int first, last;     // phase 1 / final phase
    int64_t final_level; // F when this phase is cut flat at F, else its top level
};

__host__ __device__ __forceinline__ int64_t wrap_cell(int64_t g, int64_t n)
{
    if (g < 0)
        return g + n;
    if (g >= n)
        return g - n;
    return g;
}

} // namespace sw

namespace sw {

template <typename K, typename... Args>
inline hipError_t launch_kernel(K k, dim3 grid, int threads, size_t lds, hipStream_t s,
                                Args... args)
{
    hipLaunchKernelGGL(k, grid, dim3(threads), lds, s, args...);
    return hipGetLastError();
}

} // namespace sw
