// lds_probe.hip -- LDS throughput of the access patterns the heat tile could
// use, measured on the device it runs on (the CDNA4 LDS bandwidth is not a
// published figure).  A standalone program, not part of the library: the
// build step compiles it into tests/lds_probe, tests/test_gpu_lds_probe.py
// runs it, and bench.py's LDS roofline takes its 16-byte read and write
// rates as the peak.
//
// Each workgroup (256 threads) fills a 64 KiB LDS array and then streams
// through it with one access pattern; every index is masked into the array,
// so every access stays in bounds.  Reported per pattern: bytes per clock per
// CU at the nominal 2.4 GHz clock, or cell-updates per clock per CU for the
// two update patterns:
//   level   three neighbour reads (i-1, i, i+1) and one write per update, the
//           pattern of one heat level in LDS
//   pair    each thread updates two adjacent cells: a 16-byte read of the
//           pair, two 8-byte neighbour reads, one 16-byte write
// and, for the neighbour exchange across lanes instead of through LDS, the
// rate of 32-bit lane moves each followed by a dependent add: DPP row shift
// (row_shr:1), DPP whole-wave shift (wave_shr:1) and ds_bpermute.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kThreads = 256;
constexpr int kDoubles = 8192;  // 64 KiB of LDS per workgroup
constexpr int kIter = 4096;

#define CHECK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

enum Pattern { kReadB64, kReadB128, kWriteB64, kWriteB128, kLevel, kPair, kPatterns };

template <int P>
__global__ void __launch_bounds__(kThreads) k_probe(double *out, double seed)
{
    __shared__ double s[kDoubles];
    const int tid = threadIdx.x;
    for (int i = tid; i < kDoubles; i += kThreads)
        s[i] = seed + i;
    __syncthreads();
    double acc0 = 0.0, acc1 = 0.0;
    if (P == kReadB64) {
#pragma unroll 8
        for (int k = 0; k < kIter; ++k)
            acc0 += s[(tid + k * kThreads) & (kDoubles - 1)];
    } else if (P == kReadB128) {
#pragma unroll 8
        for (int k = 0; k < kIter / 2; ++k) {
            const double2 v = *(const double2 *)&s[(2 * tid + 2 * k * kThreads) & (kDoubles - 1)];
            acc0 += v.x;
            acc1 += v.y;
        }
    } else if (P == kWriteB64) {
#pragma unroll 8
        for (int k = 0; k < kIter; ++k)
            s[(tid + k * kThreads) & (kDoubles - 1)] = seed + k;
        __syncthreads();
        acc0 = s[tid];
    } else if (P == kWriteB128) {
#pragma unroll 8
        for (int k = 0; k < kIter / 2; ++k)
            *(double2 *)&s[(2 * tid + 2 * k * kThreads) & (kDoubles - 1)] =
                make_double2(seed + k, seed - k);
        __syncthreads();
        acc0 = s[tid];
    } else if (P == kLevel) {
        // reads from [0, kDoubles/2], writes to [kDoubles/2, kDoubles)
#pragma unroll 4
        for (int k = 0; k < kIter / 4; ++k) {
            const int i = 1 + ((tid + k * kThreads) & (kDoubles / 2 - 1));
            const double v = s[i] + 0.25 * ((s[i + 1] - s[i]) + (s[i - 1] - s[i]));
            s[kDoubles / 2 + i - 1] = v;
        }
        __syncthreads();
        acc0 = s[kDoubles / 2 + tid];
    } else {
        // pair at even index c in [2, kDoubles/2]: reads [c-1, c+2], writes
        // [kDoubles/2 + c - 2, kDoubles/2 + c - 1]
#pragma unroll 4
        for (int k = 0; k < kIter / 8; ++k) {
            const int c = 2 + 2 * ((tid + k * kThreads) & (kDoubles / 4 - 1));
            const double2 x = *(const double2 *)&s[c];
            const double l = s[c - 1], r = s[c + 2];
            const double v1 = x.x + 0.25 * ((x.y - x.x) + (l - x.x));
            const double v2 = x.y + 0.25 * ((r - x.y) + (x.x - x.y));
            *(double2 *)&s[kDoubles / 2 + c - 2] = make_double2(v1, v2);
        }
        __syncthreads();
        acc0 = s[kDoubles / 2 + tid];
    }
    out[(size_t)blockIdx.x * kThreads + tid] = acc0 + acc1;
}

enum Move { kRowShr, kWaveShr, kPermute, kMoves };

template <int M>
__global__ void __launch_bounds__(kThreads) k_moves(int *out, int seed)
{
    int a = (int)threadIdx.x + seed, b = a * 3 + 1, c = a ^ 0x55, d = a + 7;
    const int lane = threadIdx.x & 63;
    const int from = (lane == 0 ? 63 : lane - 1) * 4;  // byte address of lane - 1
#pragma unroll 8
    for (int k = 0; k < kIter; ++k) {
        if (M == kRowShr) {
            a = __builtin_amdgcn_mov_dpp(a, 0x111, 0xf, 0xf, true) + 1;
            b = __builtin_amdgcn_mov_dpp(b, 0x111, 0xf, 0xf, true) + 1;
            c = __builtin_amdgcn_mov_dpp(c, 0x111, 0xf, 0xf, true) + 1;
            d = __builtin_amdgcn_mov_dpp(d, 0x111, 0xf, 0xf, true) + 1;
        } else if (M == kWaveShr) {
            a = __builtin_amdgcn_mov_dpp(a, 0x138, 0xf, 0xf, true) + 1;
            b = __builtin_amdgcn_mov_dpp(b, 0x138, 0xf, 0xf, true) + 1;
            c = __builtin_amdgcn_mov_dpp(c, 0x138, 0xf, 0xf, true) + 1;
            d = __builtin_amdgcn_mov_dpp(d, 0x138, 0xf, 0xf, true) + 1;
        } else {
            a = __builtin_amdgcn_ds_bpermute(from, a) + 1;
            b = __builtin_amdgcn_ds_bpermute(from, b) + 1;
            c = __builtin_amdgcn_ds_bpermute(from, c) + 1;
            d = __builtin_amdgcn_ds_bpermute(from, d) + 1;
        }
    }
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = a + b + c + d;
}

template <int M>
float time_moves(int blocks, int *d)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    hipLaunchKernelGGL(k_moves<M>, dim3(blocks), dim3(kThreads), 0, 0, d, 1);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(a, 0));
    for (int r = 0; r < 5; ++r)
        hipLaunchKernelGGL(k_moves<M>, dim3(blocks), dim3(kThreads), 0, 0, d, 1);
    CHECK(hipEventRecord(b, 0));
    CHECK(hipEventSynchronize(b));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return ms / 5.0f;
}

template <int P>
float time_pattern(int blocks, double *d)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    hipLaunchKernelGGL(k_probe<P>, dim3(blocks), dim3(kThreads), 0, 0, d, 1.0);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(a, 0));
    for (int r = 0; r < 5; ++r)
        hipLaunchKernelGGL(k_probe<P>, dim3(blocks), dim3(kThreads), 0, 0, d, 1.0);
    CHECK(hipEventRecord(b, 0));
    CHECK(hipEventSynchronize(b));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return ms / 5.0f;
}

} // namespace

int main()
{
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const int blocks = cus * 16;
    double *d = nullptr;
    CHECK(hipMalloc(&d, sizeof(double) * (size_t)blocks * kThreads));
    const double lanes = (double)blocks * kThreads;
    const double clk = (double)cus * 2.4e9;  // CU-clocks per second at 2.4 GHz
    std::printf("device %s, %d CUs\n", prop.gcnArchName, cus);
    const char *names[] = {"read_b64", "read_b128", "write_b64", "write_b128"};
    float ms[kPatterns];
    ms[kReadB64] = time_pattern<kReadB64>(blocks, d);
    ms[kReadB128] = time_pattern<kReadB128>(blocks, d);
    ms[kWriteB64] = time_pattern<kWriteB64>(blocks, d);
    ms[kWriteB128] = time_pattern<kWriteB128>(blocks, d);
    ms[kLevel] = time_pattern<kLevel>(blocks, d);
    ms[kPair] = time_pattern<kPair>(blocks, d);
    for (int p = 0; p < 4; ++p) {
        const double bytes = lanes * kIter * 8.0;
        std::printf("%-10s %8.3f ms  %7.1f TB/s  %6.1f B/clk/CU\n", names[p], ms[p],
                    bytes / (ms[p] * 1e-3) / 1e12, bytes / (ms[p] * 1e-3) / clk);
    }
    const double lv = lanes * (kIter / 4), pr = lanes * (kIter / 8) * 2;
    std::printf("%-10s %8.3f ms  %.3e cell-updates/s  %5.2f per clk per CU\n", "level", ms[kLevel],
                lv / (ms[kLevel] * 1e-3), lv / (ms[kLevel] * 1e-3) / clk);
    std::printf("%-10s %8.3f ms  %.3e cell-updates/s  %5.2f per clk per CU\n", "pair", ms[kPair],
                pr / (ms[kPair] * 1e-3), pr / (ms[kPair] * 1e-3) / clk);
    int *di = nullptr;
    CHECK(hipMalloc(&di, sizeof(int) * (size_t)blocks * kThreads));
    const char *mnames[] = {"row_shr", "wave_shr", "bpermute"};
    float mms[kMoves];
    mms[kRowShr] = time_moves<kRowShr>(blocks, di);
    mms[kWaveShr] = time_moves<kWaveShr>(blocks, di);
    mms[kPermute] = time_moves<kPermute>(blocks, di);
    const double moves = (double)blocks * (kThreads / 64) * kIter * 4;  // wave-level moves
    for (int m = 0; m < kMoves; ++m)
        std::printf("%-10s %8.3f ms  %5.3f wave moves (+ add) per clk per CU\n", mnames[m], mms[m],
                    moves / (mms[m] * 1e-3) / clk);
    CHECK(hipFree(di));
    CHECK(hipFree(d));
    return 0;
}
