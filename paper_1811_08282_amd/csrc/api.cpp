// api.cpp -- host side of the C ABI: argument checks, the swept planner,
// working-array management and the launch sequences of both methods.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "../../include/swept.h"
#include "geom.h"
#include "host.h"
#include "kernels.h"

namespace sw {
namespace host {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return SW_OK;
}

const char *last_error() { return g_err.c_str(); }

bool valid_eq(int eq) { return eq >= SW_HEAT_F64 && eq <= SW_KS_F64; }
bool is_euler(int eq) { return eq >= SW_EULER_F64 && eq <= SW_EULER_F32_FLAT; }
bool is_heat(int eq) { return eq == SW_HEAT_F64 || eq == SW_HEAT_F32; }

bool persistent_route(int eq, int64_t n, int w)
{
    return is_heat(eq) && w >= kPersistentMinWidth && n / w > kPersistentMinTiles;
}
bool is_flat(int eq) { return eq == SW_EULER_F64_FLAT || eq == SW_EULER_F32_FLAT; }
bool is_f32(int eq) { return eq == SW_HEAT_F32 || eq == SW_EULER_F32 || eq == SW_EULER_F32_FLAT; }
int substeps(int eq) { return is_flat(eq) ? 2 : (is_euler(eq) ? 4 : 1); }
int radius(int eq) { return (is_flat(eq) || eq == SW_KS_F64) ? 2 : 1; }

constexpr int64_t kMaxCells = (int64_t)1 << 40;
constexpr int64_t kMaxWidth = 8192;
constexpr uint64_t kMaxLaunchItems = 0xFFFFFFFFull;  // work-items of one HIP launch
constexpr size_t kNaiveGroup = 256;                  // workgroup size of the classic kernels

int lds_per_cell(int eq)
{
    switch (eq) {
    case SW_HEAT_F64: return sw::kLdsPerCellHeatF64;
    case SW_HEAT_F32: return sw::kLdsPerCellHeatF32;
    case SW_EULER_F64: return sw::kLdsPerCellEulerF64;
    case SW_EULER_F32: return sw::kLdsPerCellEulerF32;
    case SW_EULER_F64_FLAT: return sw::kLdsPerCellFlatF64;
    case SW_KS_F64: return sw::kLdsPerCellKsF64;
    default: return sw::kLdsPerCellFlatF32;
    }
}

int struct_bytes(int eq)
{
    switch (eq) {
    case SW_HEAT_F64: return sw::kStructBytesHeatF64;
    case SW_HEAT_F32: return sw::kStructBytesHeatF32;
    case SW_EULER_F64: return sw::kStructBytesEulerF64;
    case SW_EULER_F32: return sw::kStructBytesEulerF32;
    case SW_EULER_F64_FLAT: return sw::kStructBytesFlatF64;
    case SW_KS_F64: return sw::kStructBytesKsF64;
    default: return sw::kStructBytesFlatF32;
    }
}

// measured on MI355X (2^24 cells): heat best at 2048 in both precisions
// (the register-blocked level sweep), Euler at 1024 with 512-thread
// workgroups (flattened binary32 equally fast at 2048); sw_autotune refines
// per grid size
int preferred_width(int eq)
{
    if (!is_euler(eq) || eq == SW_EULER_F32_FLAT)
        return 2048;
    return 1024;
}

// the same for the batch kernel, whose workgroups have 256 threads:
// lengthened Euler is best at 512 there, heat at 2048 (a phase of a lone
// 2^22-cell heat problem is then 2048 items, which the persistent launch
// overlaps with the next phase's)
int preferred_batch_width(int eq)
{
    if (!is_euler(eq))
        return 2048;
    return is_flat(eq) ? 1024 : 512;
}

// workgroup size of a swept phase when the caller gives none: Euler tiles of
// 1000 cells or more and Kuramoto-Sivashinsky tiles of 2048 or more run 512
// threads (twice the resident waves per compute unit at the same LDS;
// measured faster), everything else W rounded up to whole waves, at most 256
int default_threads(int eq, int w)
{
    if ((is_euler(eq) && w >= 1000) || (eq == SW_KS_F64 && w >= 2048))
        return 512;
    return sw::default_phase_threads(w);
}


size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int max_width(int eq)
{
    const int step = 2 * radius(eq);
    int64_t w = sw::kLdsBytes / lds_per_cell(eq) - sw::lds_tile_cells(is_heat(eq), 0, radius(eq));
    if (w > kMaxWidth)
        w = kMaxWidth;
    return (int)(w - w % step);
}

bool width_ok(int eq, int64_t n, int64_t w)
{
    const int step = 2 * radius(eq);
    return w >= step && (w % step) == 0 && w <= max_width(eq) && (n % w) == 0 && n / w >= 2;
}

int default_width(int eq, int64_t n, bool batch)
{
    for (int64_t w = batch ? preferred_batch_width(eq) : preferred_width(eq); w >= 2; w -= 2)
        if (width_ok(eq, n, w))
            return (int)w;
    return 0;
}

size_t state_bytes(int eq, int64_t n)
{
    switch (eq) {
    case SW_HEAT_F64: return (size_t)n * 8;
    case SW_HEAT_F32: return (size_t)n * 8;
    case SW_KS_F64: return (size_t)n * 8;
    default: return (size_t)n * 24;  // Euler, every precision and layout
    }
}

// one copy of the swept working arrays, 256-byte rounded
size_t swept_copy_bytes(int eq, int64_t n) { return round_up((size_t)n * struct_bytes(eq), 256); }

size_t naive_ws_bytes(int eq, int64_t n)
{
    switch (eq) {
    case SW_HEAT_F64: return round_up((size_t)n * 8, 256);
    case SW_HEAT_F32: return round_up((size_t)n * 4, 256);
    case SW_EULER_F64: return round_up((size_t)n * 24, 256) + round_up((size_t)n * 8, 256);
    case SW_EULER_F32: return round_up((size_t)n * 12, 256) + round_up((size_t)n * 8, 256);
    case SW_EULER_F64_FLAT: return round_up((size_t)n * 24, 256);
    case SW_KS_F64: return round_up((size_t)n * 8, 256);
    default: return round_up((size_t)n * 12, 256);
    }
}

// ---- argument checks (no HIP call) -----------------------------------------

int check_common(int eq, int64_t n, int64_t steps, double dt, double dx, const void *state,
                 int64_t min_cells)
{
    if (!valid_eq(eq))
        return fail(SW_ERR_ARG, "invalid equation id %d", eq);
    if (n < min_cells || n > kMaxCells)
        return fail(SW_ERR_ARG, "n_cells %lld out of range [%lld, 2^40]", (long long)n,
                    (long long)min_cells);
    if (steps < 0 || steps > INT64_MAX / 8)
        return fail(SW_ERR_ARG, "n_steps %lld out of range", (long long)steps);
    if (!(dt > 0.0) || !isfinite(dt))
        return fail(SW_ERR_ARG, "dt must be finite and > 0");
    if (!(dx > 0.0) || !isfinite(dx))
        return fail(SW_ERR_ARG, "dx must be finite and > 0");
    if (!state)
        return fail(SW_ERR_ARG, "d_state is NULL");
    if (((uintptr_t)state & 15) != 0)
        return fail(SW_ERR_ARG, "d_state must be 16-byte aligned");
    return SW_OK;
}

// ---- device-side checks and working arrays ------------------------------------

int check_device_pointer(const void *p, int *dev_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "hipGetDevice failed");
    }
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_ARG, "d_state is not a HIP device pointer");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(SW_ERR_ARG, "d_state is not device memory");
    if (attr.device != dev)
        return fail(SW_ERR_ARG, "d_state lives on device %d, current device is %d", attr.device,
                    dev);
    *dev_out = dev;
    return SW_OK;
}

struct CachedWs {
    void *ptr = nullptr;
    size_t bytes = 0;
};

std::mutex g_ws_mutex;
std::map<std::pair<int, void *>, CachedWs> g_ws;  // (device, stream) -> arrays

// Working arrays for a call: the caller's (opts) or the cache of this
// (device, stream).  Growing the cache synchronises the device first, so no
// earlier launch still uses the old arrays when they are freed.
int get_workspace(int dev, hipStream_t stream, size_t need, const sw_opts *o, void **out)
{
    if (o && o->d_workspace) {
        if (o->workspace_bytes < need)
            return fail(SW_ERR_ARG, "workspace of %zu bytes is smaller than the %zu needed",
                        o->workspace_bytes, need);
        if (((uintptr_t)o->d_workspace & 255) != 0)
            return fail(SW_ERR_ARG, "workspace must be 256-byte aligned");
        *out = o->d_workspace;
        return SW_OK;
    }
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    CachedWs &c = g_ws[std::make_pair(dev, (void *)stream)];
    if (c.bytes >= need) {
        *out = c.ptr;
        return SW_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "hipStreamIsCapturing failed");
    }
    if (cs != hipStreamCaptureStatusNone)
        return fail(SW_ERR_CAPTURE,
                    "stream is capturing and the cached working arrays are too small; pass a "
                    "workspace in sw_opts");
    if (c.ptr) {
        if (hipDeviceSynchronize() != hipSuccess || hipFree(c.ptr) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SW_ERR_HIP, "releasing old working arrays failed");
        }
        c.ptr = nullptr;
        c.bytes = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_NOMEM, "hipMalloc of %zu bytes for working arrays failed", need);
    }
    c.ptr = p;
    c.bytes = need;
    *out = p;
    return SW_OK;
}

int launched(hipError_t e, const char *what)
{
    if (e != hipSuccess)
        return fail(SW_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return SW_OK;
}

void ks_coefficients(double dt, double dx, double *a, double *b, double *c)
{
    *a = dt / (2.0 * dx);
    *b = dt / (dx * dx);
    *c = dt / ((dx * dx) * (dx * dx));
}

hipError_t swept_phase_launch(int eq, const sw::PhaseLaunch &p, void *state, const void *in,
                              void *out, double dt, double dx, hipStream_t s)
{
    const double r64 = dt / (dx * dx);
    const double lam64 = dt / dx;
    hipError_t e = hipSuccess;
    switch (eq) {
    case SW_HEAT_F64:
        e = sw::heat_f64_swept_phase(p, (double *)state, (const double *)in, (double *)out, r64, s);
        break;
    case SW_HEAT_F32:
        e = sw::heat_f32_swept_phase(p, (float *)state, (const float *)in, (float *)out,
                                     (float)r64, s);
        break;
    case SW_EULER_F64:
        e = sw::euler_f64_swept_phase(p, (double *)state, (const double *)in, (double *)out,
                                      lam64, s);
        break;
    case SW_EULER_F32:
        e = sw::euler_f32_swept_phase(p, (float *)state, in, out, (float)lam64, s);
        break;
    case SW_EULER_F64_FLAT:
        e = sw::flat_f64_swept_phase(p, (double *)state, (const double *)in, (double *)out, lam64,
                                     s);
        break;
    case SW_KS_F64: {
        double a, b, c;
        ks_coefficients(dt, dx, &a, &b, &c);
        e = sw::ks_f64_swept_phase(p, (double *)state, (const double *)in, (double *)out, a, b, c,
                                   s);
        break;
    }
    default:
        e = sw::flat_f32_swept_phase(p, (float *)state, (const float *)in, (float *)out,
                                     (float)lam64, s);
        break;
    }
    return e;
}

} // namespace host
} // namespace sw

namespace {

using namespace sw::host;

// ---- the two methods ---------------------------------------------------------

int run_swept(int eq, int64_t n, int64_t steps, double dt, double dx, void *state,
              hipStream_t s, int w, int threads, void *ws)
{
    const int64_t final_level = steps * substeps(eq);
    const int rad = radius(eq);
    const int64_t half = w / (2 * rad);
    const int64_t phases = sw::phase_count(final_level, half);
    const size_t copy = swept_copy_bytes(eq, n);
    char *ws_a = (char *)ws;
    char *ws_b = ws_a + copy;
    for (int64_t k = 1; k <= phases; ++k) {
        const sw::PhaseRange pr = sw::phase_range(k, final_level, half, rad);
        sw::PhaseLaunch p;
        p.n = n;
        p.w = w;
        p.offset = pr.offset;
        p.tiles = n / w;
        p.base = pr.base;
        p.j_first = pr.j_first;
        p.j_last = pr.j_last;
        p.threads = threads;
        p.first = (k == 1);
        // A single phase (heat, one step) may not write the caller's state:
        // its tiles read their halos from that same state.  It writes the
        // working array, and level 1 (slot 1) is copied back below.
        p.last = (k == phases) && phases > 1;
        char *in = (k % 2 == 0) ? ws_a : ws_b;
        char *out = (k % 2 == 1) ? ws_a : ws_b;
        const hipError_t e = swept_phase_launch(eq, p, state, in, out, dt, dx, s);
        if (e != hipSuccess)
            return launched(e, "swept phase launch");
    }
    if (phases == 1) {
        // only heat and Kuramoto-Sivashinsky reach here (one step: final
        // level 1); copy slot 1 (and the binary32 compensation) from working
        // array A to the state
        hipError_t e = hipSuccess;
        if (eq == SW_HEAT_F64 || eq == SW_KS_F64) {
            e = hipMemcpyAsync(state, ws_a + (size_t)n * 8, (size_t)n * 8, hipMemcpyDeviceToDevice,
                               s);
        } else if (eq == SW_HEAT_F32) {
            e = hipMemcpyAsync(state, ws_a + (size_t)n * 4, (size_t)n * 8, hipMemcpyDeviceToDevice,
                               s);
        } else {
            return fail(SW_ERR_HIP, "internal: single-phase schedule for a four-sub-step scheme");
        }
        if (e != hipSuccess)
            return launched(e, "swept single-phase copy");
    }
    return SW_OK;
}

int run_naive(int eq, int64_t n, int64_t steps, double dt, double dx, void *state,
              hipStream_t s, void *ws)
{
    const double r64 = dt / (dx * dx);
    const double lam64 = dt / dx;
    hipError_t e = hipSuccess;
    if (eq == SW_HEAT_F64 || eq == SW_HEAT_F32) {
        const size_t elem = (eq == SW_HEAT_F64) ? 8 : 4;
        char *cur = (char *)state, *nxt = (char *)ws;
        for (int64_t t = 0; t < steps && e == hipSuccess; ++t) {
            if (eq == SW_HEAT_F64)
                e = sw::heat_f64_naive_step((const double *)cur, (double *)nxt, n, r64, s);
            else
                e = sw::heat_f32_naive_step((const float *)cur, (float *)nxt,
                                            (float *)state + n, n, (float)r64, s);
            std::swap(cur, nxt);
        }
        if (e == hipSuccess && cur != (char *)state)
            e = hipMemcpyAsync(state, cur, (size_t)n * elem, hipMemcpyDeviceToDevice, s);
        return launched(e, "naive heat launch");
    }
    if (eq == SW_KS_F64) {
        double a, b, c;
        ks_coefficients(dt, dx, &a, &b, &c);
        double *cur = (double *)state, *nxt = (double *)ws;
        for (int64_t t = 0; t < steps && e == hipSuccess; ++t) {
            e = sw::ks_f64_naive_step(cur, nxt, n, a, b, c, s);
            std::swap(cur, nxt);
        }
        if (e == hipSuccess && cur != (double *)state)
            e = hipMemcpyAsync(state, cur, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
        return launched(e, "naive Kuramoto-Sivashinsky launch");
    }
    if (eq == SW_EULER_F64) {
        double *q0 = (double *)state;
        double *q1 = (double *)ws;
        double *pr = (double *)((char *)ws + round_up((size_t)n * 24, 256));
        for (int64_t t = 0; t < steps && e == hipSuccess; ++t)
            for (int sub = 0; sub < 4 && e == hipSuccess; ++sub)
                e = sw::euler_f64_naive_substep(sub, q0, q1, pr, n, lam64, s);
        return launched(e, "naive euler launch");
    }
    if (eq == SW_EULER_F64_FLAT) {
        double *q0 = (double *)state;
        double *q1 = (double *)ws;
        for (int64_t t = 0; t < steps && e == hipSuccess; ++t)
            for (int sub = 0; sub < 2 && e == hipSuccess; ++sub)
                e = sw::flat_f64_naive_substep(sub, q0, q1, n, lam64, s);
        return launched(e, "naive flattened euler launch");
    }
    if (eq == SW_EULER_F32_FLAT) {
        float *q0c = (float *)state;
        float *q1 = (float *)ws;
        for (int64_t t = 0; t < steps && e == hipSuccess; ++t)
            for (int sub = 0; sub < 2 && e == hipSuccess; ++sub)
                e = sw::flat_f32_naive_substep(sub, q0c, q1, n, (float)lam64, s);
        return launched(e, "naive flattened euler launch");
    }
    float *q0c = (float *)state;
    float *q1 = (float *)ws;
    double *pr = (double *)((char *)ws + round_up((size_t)n * 12, 256));
    for (int64_t t = 0; t < steps && e == hipSuccess; ++t)
        for (int sub = 0; sub < 4 && e == hipSuccess; ++sub)
            e = sw::euler_f32_naive_substep(sub, q0c, q1, pr, n, (float)lam64, s);
    return launched(e, "naive euler launch");
}

int solve(int method, int eq, int64_t n, int64_t steps, double dt, double dx, void *state,
          sw_stream stream, const sw_opts *o)
{
    int rc = check_common(eq, n, steps, dt, dx, state, method == SW_METHOD_SWEPT ? 4 : 3);
    if (rc)
        return rc;
    int w = 0;
    int tuned_threads = 0;
    bool tuned = false;  // the autotuner recorded this launch (workgroup size 0: persistent)
    if (method == SW_METHOD_SWEPT) {
        if (o && o->width) {
            if (!width_ok(eq, n, o->width))
                return fail(SW_ERR_ARG,
                            "width %d invalid for n_cells %lld (even, >= 2, divides n_cells, "
                            "n_cells/width >= 2, <= %d)",
                            o->width, (long long)n, max_width(eq));
            w = o->width;
        } else {
            w = chosen_width(-1, eq, n, &tuned_threads, false, &tuned);
            if (!w)
                return fail(SW_ERR_UNSUPPORTED, "no valid triangle width for n_cells %lld",
                            (long long)n);
        }
    }
    if (o && o->threads && o->threads != 64 && o->threads != 128 && o->threads != 256 &&
        o->threads != 512)
        return fail(SW_ERR_ARG, "threads must be 0, 64, 128, 256 or 512");
    if (o && o->d_workspace && ((uintptr_t)o->d_workspace & 255) != 0)
        return fail(SW_ERR_ARG, "workspace must be 256-byte aligned");
    if (o && (o->work_factor < 0 || o->host_threads < 0 || o->host_threads > kMaxHostThreads))
        return fail(SW_ERR_ARG, "work_factor must be >= 0 and host_threads in [0, %d]",
                    kMaxHostThreads);
    if (o && o->work_factor > 0) {
        if (method != SW_METHOD_SWEPT)
            return fail(SW_ERR_ARG, "work_factor applies to the swept method only");
        const int64_t tiles = n / w;
        const int p = o->host_threads ? o->host_threads : kDefaultHostThreads;
        if (tiles / ((int64_t)o->work_factor + p) < 1)
            return fail(SW_ERR_ARG,
                        "work_factor %d with %d host threads leaves no tile for the host (%lld "
                        "tiles of %d cells)",
                        o->work_factor, p, (long long)tiles, w);
    }
    const int threads = (o && o->threads) ? o->threads
                        : (tuned_threads ? tuned_threads : default_threads(eq, w));
    // a launch holds at most 2^32 - 1 work-items: one workgroup per tile in
    // a swept phase, at most one work-item per cell in a classic sub-step
    if (method == SW_METHOD_SWEPT
            ? (uint64_t)(n / w) * (uint64_t)threads > kMaxLaunchItems
            : (uint64_t)round_up((size_t)n, kNaiveGroup) > kMaxLaunchItems)
        return fail(SW_ERR_ARG,
                    method == SW_METHOD_SWEPT
                        ? "n_cells %lld in tiles of %d cells needs more than 2^32 work-items in "
                          "one launch; use a wider tile"
                        : "n_cells %lld exceeds the classic kernels' limit of 2^32 - 256 cells",
                    (long long)n, w);
    if (steps == 0)
        return ok();
    int dev = 0;
    rc = check_device_pointer(state, &dev);
    if (rc)
        return rc;
    hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    if (method == SW_METHOD_SWEPT && persistent_route(eq, n, w) &&
        !(o && (o->d_workspace || o->threads || o->work_factor)) &&
        (!tuned || tuned_threads == 0) &&
        sw::phase_count(steps, w / 2) >= 2) {
        sw_problem p{};
        p.eq = eq;
        p.width = w;
        p.n_cells = n;
        p.n_steps = steps;
        p.dt = dt;
        p.dx = dx;
        p.d_state = state;
        // 0 when the batch's limits refuse the problem (2^31 - 2 phases):
        // the phase launches below take it
        const size_t pneed = persistent_workspace_bytes(p);
        if (pneed) {
            rc = get_workspace(dev, s, pneed, nullptr, &ws);
            if (rc)
                return rc;
            rc = run_swept_persistent(p, ws, pneed, s);
            return rc ? rc : ok();
        }
    }
    const size_t need = (method == SW_METHOD_SWEPT) ? 2 * swept_copy_bytes(eq, n)
                                                    : naive_ws_bytes(eq, n);
    rc = get_workspace(dev, s, need, o, &ws);
    if (rc)
        return rc;
    if (method == SW_METHOD_SWEPT && o && o->work_factor > 0 &&
        sw::phase_count(steps * substeps(eq), w / (2 * radius(eq))) >= 2)
        rc = run_swept_shared(eq, n, steps, dt, dx, state, s, w, threads, ws, o->work_factor,
                              o->host_threads);
    else
        rc = (method == SW_METHOD_SWEPT) ? run_swept(eq, n, steps, dt, dx, state, s, w, threads, ws)
                                         : run_naive(eq, n, steps, dt, dx, state, s, ws);
    return rc ? rc : ok();
}

} // namespace

// ---- static working arrays of the allocation-free entry point ----------------
//
// One file-scope device array per GPU the library runs on (the code object
// holds it from its load until the process ends).  In host code `scratch`
// names a host-side stand-in, not the device address: the address is taken
// once per device with hipGetSymbolAddress, with that device current, and
// only that address is ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[SW_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (dev is the current device).
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SW_ERR_UNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(SW_ERR_HIP, "hipGetSymbolAddress of the static working arrays failed: %s",
                        hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SW_OK;
}

} // namespace

extern "C" {

size_t sw_state_bytes(int eq, int64_t n_cells)
{
    if (!valid_eq(eq) || n_cells <= 0 || n_cells > kMaxCells)
        return 0;
    return state_bytes(eq, n_cells);
}

size_t sw_workspace_bytes(int eq, int64_t n_cells, int width, int method)
{
    (void)width;
    if (!valid_eq(eq) || n_cells <= 0 || n_cells > kMaxCells)
        return 0;
    if (method == SW_METHOD_SWEPT)
        return 2 * swept_copy_bytes(eq, n_cells);
    if (method == SW_METHOD_NAIVE)
        return naive_ws_bytes(eq, n_cells);
    return 0;
}

int sw_max_width(int eq) { return valid_eq(eq) ? max_width(eq) : 0; }

int sw_default_width(int eq, int64_t n_cells)
{
    if (!valid_eq(eq) || n_cells < 4 || n_cells > kMaxCells)
        return 0;
    return default_width(eq, n_cells, false);
}

int sw_default_threads(int eq, int width)
{
    if (!valid_eq(eq) || width < 2 * radius(eq) || width > max_width(eq) ||
        width % (2 * radius(eq)) != 0)
        return 0;
    return default_threads(eq, width);
}

int swept_solve(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx, void *d_state,
                sw_stream stream)
{
    return guarded([&] {
        return solve(SW_METHOD_SWEPT, eq, n_cells, n_steps, dt, dx, d_state, stream, nullptr);
    });
}

int naive_solve(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx, void *d_state,
                sw_stream stream)
{
    return guarded([&] {
        return solve(SW_METHOD_NAIVE, eq, n_cells, n_steps, dt, dx, d_state, stream, nullptr);
    });
}

int swept_solve_ex(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx,
                   void *d_state, sw_stream stream, const sw_opts *opts)
{
    return guarded([&] {
        return solve(SW_METHOD_SWEPT, eq, n_cells, n_steps, dt, dx, d_state, stream, opts);
    });
}

int naive_solve_ex(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx,
                   void *d_state, sw_stream stream, const sw_opts *opts)
{
    return guarded([&] {
        return solve(SW_METHOD_NAIVE, eq, n_cells, n_steps, dt, dx, d_state, stream, opts);
    });
}

int64_t sw_phase_count(int64_t final_level, int width, int radius)
{
    if (final_level < 0 || radius < 1 || radius > 2 || width < 2 * radius ||
        width % (2 * radius) != 0)
        return -1;
    return sw::phase_count(final_level, width / (2 * radius));
}

int sw_phase_info(int64_t k, int64_t final_level, int width, int radius, int64_t *offset,
                  int64_t *first_level, int64_t *last_level)
{
    const int64_t phases = sw_phase_count(final_level, width, radius);
    if (phases < 0 || k < 1 || k > phases || !offset || !first_level || !last_level)
        return fail(SW_ERR_ARG, "invalid phase query");
    const sw::PhaseRange p = sw::phase_range(k, final_level, width / (2 * radius), radius);
    *offset = p.offset;
    *first_level = p.base + p.j_first;
    *last_level = p.base + p.j_last;
    return ok();
}

int sw_phase_interval(int64_t k, int64_t final_level, int width, int radius, int64_t level,
                      int *lo, int *hi)
{
    const int64_t phases = sw_phase_count(final_level, width, radius);
    if (phases < 0 || k < 1 || k > phases || !lo || !hi)
        return fail(SW_ERR_ARG, "invalid phase query");
    const sw::PhaseRange p = sw::phase_range(k, final_level, width / (2 * radius), radius);
    const int64_t j = level - p.base;
    if (j < p.j_first || j > p.j_last) {
        *lo = 0;
        *hi = 0;
        return ok();
    }
    const int a = sw::window_margin((int)j, radius);
    *lo = a;
    *hi = width - a;
    return ok();
}

const char *sw_last_error(void) { return sw::host::last_error(); }

void sw_release(void)
{
    release_host_arrays();
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_ws) {
        if (!kv.second.ptr)
            continue;
        (void)hipSetDevice(kv.first.first);
        (void)hipDeviceSynchronize();
        (void)hipFree(kv.second.ptr);
    }
    g_ws.clear();
    (void)hipSetDevice(cur);
    (void)hipGetLastError();
}

int swept_solve_noalloc(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx,
                        void *d_state, sw_stream stream)
{
    int rc = check_common(eq, n_cells, n_steps, dt, dx, d_state, 4);
    if (rc)
        return rc;
    // every cell's working struct is written by the phase that reads it next,
    // so the arrays need no clearing between calls
    const size_t need = 2 * swept_copy_bytes(eq, n_cells);
    if (need > (size_t)SW_NOALLOC_SCRATCH_BYTES)
        return fail(SW_ERR_ARG,
                    "swept_solve_noalloc: %lld cells need %zu bytes of working arrays, more than "
                    "the %zu of its static arrays (use swept_solve_ex with a workspace)",
                    (long long)n_cells, need, (size_t)SW_NOALLOC_SCRATCH_BYTES);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "hipGetDevice failed");
    }
    void *ws = nullptr;
    rc = scratch_address(dev, &ws);
    if (rc)
        return rc;
    sw_opts o{};
    o.d_workspace = ws;
    o.workspace_bytes = SW_NOALLOC_SCRATCH_BYTES;
    return guarded(
        [&] { return solve(SW_METHOD_SWEPT, eq, n_cells, n_steps, dt, dx, d_state, stream, &o); });
}

} // extern "C"
