// tune_batch.cpp -- host side of the autotuner and of the batched persistent
// launch.
//
// Autotuner: the paper recommends tuning the block width on a limited number
// of time steps before a long run, starting from wide blocks (Sec. 6).
// sw_autotune times short probe solves over the valid widths (multiples of 64
// up to the LDS limit) and workgroup sizes, keeps the fastest per
// (device architecture, equation, cell count) in a process-wide table, and,
// when SWEPT_TUNE_CACHE names a file, persists the table there as text lines
// "<arch> <eq> <n_cells> <width> <threads> <ms_per_cell_update>".
//
// Batch: sw_batch_create builds the work-item tables (batch.h), allocates the
// working arrays of every problem and captures the reset kernel and the
// persistent kernel into a hipGraph; sw_batch_run launches that graph.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/swept.h"
#include "batch.h"
#include "geom.h"
#include "host.h"
#include "kernels.h"

namespace sw {

// bodies: 0 every tile body, 1 heat binary64 only, 2 heat binary32 only
hipError_t batch_occupancy(size_t lds_bytes, int threads, int bodies, int *blocks_per_cu);
hipError_t batch_launch(const BatchTables &t, int64_t n_flags, int blocks, int threads,
                        int bodies, size_t lds_bytes, hipStream_t s);
hipError_t fill_f64(double *p, int64_t count, double v, hipStream_t s);
hipError_t fill_f32(float *p, int64_t count, float v, hipStream_t s);

namespace host {

struct TuneEntry {
    int width;
    int threads;
    double ms_per_update;
};

std::mutex g_tune_mutex;
std::map<std::tuple<std::string, int, int64_t>, TuneEntry> g_tune;
// the latest entry recorded per (arch, eq, size class floor(log2 n)): used for
// cell counts of that class that have no entry of their own
std::map<std::tuple<std::string, int, int>, TuneEntry> g_tune_class;
bool g_tune_loaded = false;

int size_class(int64_t n)
{
    int c = 0;
    while (n > 1) {
        n >>= 1;
        ++c;
    }
    return c;
}

void record_tune_locked(const std::string &arch, int eq, int64_t n, const TuneEntry &e)
{
    g_tune[std::make_tuple(arch, eq, n)] = e;
    g_tune_class[std::make_tuple(arch, eq, size_class(n))] = e;
}

std::string arch_name(int dev)
{
    static std::map<int, std::string> cache;  // guarded by g_tune_mutex
    auto it = cache.find(dev);
    if (it != cache.end())
        return it->second;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    a = colon == std::string::npos ? a : a.substr(0, colon);
    cache[dev] = a;
    return a;
}

void load_tune_file_locked()
{
    if (g_tune_loaded)
        return;
    g_tune_loaded = true;
    const char *path = getenv("SWEPT_TUNE_CACHE");
    if (!path || !*path)
        return;
    FILE *f = fopen(path, "r");
    if (!f)
        return;
    char arch[64];
    int eq, w, t;
    long long n;
    double ms;
    while (fscanf(f, "%63s %d %lld %d %d %lf", arch, &eq, &n, &w, &t, &ms) == 6) {
        if (valid_eq(eq) && width_ok(eq, n, w) && (t == 64 || t == 128 || t == 256 || t == 512))
            record_tune_locked(std::string(arch), eq, (int64_t)n, TuneEntry{w, t, ms});
    }
    fclose(f);
}

void store_tune_file_locked(const std::string &arch, int eq, int64_t n, const TuneEntry &e)
{
    const char *path = getenv("SWEPT_TUNE_CACHE");
    if (!path || !*path)
        return;
    FILE *f = fopen(path, "a");
    if (!f)
        return;
    fprintf(f, "%s %d %lld %d %d %.9e\n", arch.c_str(), eq, (long long)n, e.width, e.threads,
            e.ms_per_update);
    fclose(f);
}

int chosen_width(int dev, int eq, int64_t n, int *threads, bool batch)
{
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        load_tune_file_locked();
        if (!g_tune.empty()) {
            if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
                (void)hipGetLastError();
                dev = 0;
            }
            const std::string arch = arch_name(dev);
            auto it = g_tune.find(std::make_tuple(arch, eq, n));
            if (it != g_tune.end()) {
                if (threads)
                    *threads = it->second.threads;
                return it->second.width;
            }
            auto ic = g_tune_class.find(std::make_tuple(arch, eq, size_class(n)));
            if (ic != g_tune_class.end() && width_ok(eq, n, ic->second.width)) {
                if (threads)
                    *threads = ic->second.threads;
                return ic->second.width;
            }
        }
    }
    const int w = default_width(eq, n, batch);
    if (threads)
        *threads = default_threads(eq, w);
    return w;
}

// width candidates: multiples of 64 dividing n (largest first), else every
// valid even width (at most 24 of them, largest first)
std::vector<int> width_candidates(int eq, int64_t n)
{
    std::vector<int> out;
    for (int w = max_width(eq); w >= 64; --w)
        if (w % 64 == 0 && width_ok(eq, n, w))
            out.push_back(w);
    if (out.empty())
        for (int w = max_width(eq); w >= 2 && out.size() < 24; --w)
            if (width_ok(eq, n, w))
                out.push_back(w);
    return out;
}

hipError_t fill_state(int eq, void *state, int64_t n, hipStream_t s)
{
    hipError_t e = hipSuccess;
    switch (eq) {
    case SW_HEAT_F64: e = fill_f64((double *)state, n, 1.0, s); break;
    case SW_HEAT_F32:
        e = fill_f32((float *)state, n, 1.0f, s);
        if (e == hipSuccess)
            e = fill_f32((float *)state + n, n, 0.0f, s);
        break;
    case SW_EULER_F64:
    case SW_EULER_F64_FLAT:
        e = fill_f64((double *)state, n, 1.0, s);
        if (e == hipSuccess)
            e = fill_f64((double *)state + n, n, 0.0, s);
        if (e == hipSuccess)
            e = fill_f64((double *)state + 2 * n, n, 2.5, s);
        break;
    default:
        e = fill_f32((float *)state, n, 1.0f, s);
        if (e == hipSuccess)
            e = fill_f32((float *)state + n, 2 * n, 0.0f, s);
        if (e == hipSuccess)
            e = fill_f32((float *)state + 2 * n, n, 2.5f, s);
        if (e == hipSuccess)
            e = fill_f32((float *)state + 3 * n, 3 * n, 0.0f, s);
        break;
    }
    return e;
}

} // namespace host
} // namespace sw

using namespace sw::host;

// ---- batch handle -------------------------------------------------------------

struct sw_batch_impl {
    int device = 0;
    void *tables = nullptr;      // problems, segments, ticket, status, flags
    void *arrays = nullptr;      // every problem's working arrays
    size_t array_bytes = 0;
    size_t table_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int *d_status = nullptr;
    int64_t items = 0;
    int64_t flags = 0;
    int blocks = 0;
    int threads = 256;
    int bodies = 0;
    std::vector<int> widths;
};

namespace {

void free_batch(sw_batch_impl *b)
{
    if (!b)
        return;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->tables)
        (void)hipFree(b->tables);
    if (b->arrays)
        (void)hipFree(b->arrays);
    (void)hipGetLastError();
    delete b;
}

} // namespace

extern "C" {

int sw_autotune(int eq, int64_t n_cells, int64_t probe_steps, sw_stream stream, sw_opts *best,
                double *best_ms_per_update)
{
    if (!valid_eq(eq))
        return fail(SW_ERR_ARG, "invalid equation id %d", eq);
    if (n_cells < 4 || n_cells > ((int64_t)1 << 40))
        return fail(SW_ERR_ARG, "n_cells out of range");
    if (probe_steps < 0 || probe_steps > 1000000)
        return fail(SW_ERR_ARG, "probe_steps out of range");
    if (!best)
        return fail(SW_ERR_ARG, "best is NULL");
    const std::vector<int> cands = width_candidates(eq, n_cells);
    if (cands.empty())
        return fail(SW_ERR_UNSUPPORTED, "no valid triangle width for n_cells %lld",
                    (long long)n_cells);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "hipGetDevice failed");
    }
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return fail(SW_ERR_CAPTURE, "sw_autotune cannot run during stream capture");
    }
    // enough sub-steps for four phases at the widest candidate
    const int64_t sub = substeps(eq);
    int64_t steps = probe_steps;
    if (steps == 0)
        steps = std::max<int64_t>(8, (2 * (int64_t)cands.front() + sub - 1) / sub);
    void *state = nullptr, *ws = nullptr;
    const size_t sbytes = sw_state_bytes(eq, n_cells);
    const size_t wbytes = sw_workspace_bytes(eq, n_cells, 0, SW_METHOD_SWEPT);
    if (hipMalloc(&state, sbytes) != hipSuccess || hipMalloc(&ws, wbytes) != hipSuccess) {
        (void)hipGetLastError();
        if (state)
            (void)hipFree(state);
        return fail(SW_ERR_NOMEM, "autotune scratch allocation failed");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SW_OK;
    TuneEntry top{0, 0, INFINITY};
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        fill_state(eq, state, n_cells, s) != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(SW_ERR_HIP, "autotune setup failed");
    }
    const double dt = 0.1, dx = 1.0;
    for (size_t ci = 0; ci < cands.size() && rc == SW_OK; ++ci) {
        const int w = cands[ci];
        for (int threads = 512; threads >= 64 && rc == SW_OK; threads /= 2) {
            if (threads > 64 && threads / 2 >= w)
                continue;  // wider workgroups than the tile only idle
            sw_opts o{w, threads, ws, wbytes};
            rc = swept_solve_ex(eq, n_cells, steps, dt, dx, state, stream, &o);  // warm-up
            if (rc)
                break;
            float ms = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess) {
                rc = fail(SW_ERR_HIP, "hipEventRecord failed");
                break;
            }
            rc = swept_solve_ex(eq, n_cells, steps, dt, dx, state, stream, &o);
            if (rc)
                break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                (void)hipGetLastError();
                rc = fail(SW_ERR_HIP, "autotune timing failed");
                break;
            }
            const double per = (double)ms / ((double)n_cells * (double)steps);
            if (per < top.ms_per_update)
                top = TuneEntry{w, threads, per};
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(state);
    (void)hipFree(ws);
    (void)hipGetLastError();
    if (rc)
        return rc;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        load_tune_file_locked();
        const std::string arch = arch_name(dev);
        record_tune_locked(arch, eq, n_cells, top);
        store_tune_file_locked(arch, eq, n_cells, top);
    }
    best->width = top.width;
    best->threads = top.threads;
    best->d_workspace = nullptr;
    best->workspace_bytes = 0;
    if (best_ms_per_update)
        *best_ms_per_update = top.ms_per_update;
    return ok();
}

int sw_tuned_width(int eq, int64_t n_cells, int *width, int *threads)
{
    if (!valid_eq(eq) || !width)
        return fail(SW_ERR_ARG, "invalid tuned-width query");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "hipGetDevice failed");
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    load_tune_file_locked();
    auto it = g_tune.find(std::make_tuple(arch_name(dev), eq, n_cells));
    if (it == g_tune.end())
        return fail(SW_ERR_UNSUPPORTED, "no tuned width recorded");
    *width = it->second.width;
    if (threads)
        *threads = it->second.threads;
    return ok();
}

void sw_tune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune.clear();
    g_tune_class.clear();
    g_tune_loaded = true;  // do not reload the file after an explicit clear
}

int sw_batch_create(int n_problems, const sw_problem *problems, const sw_batch_opts *opts,
                    sw_batch *out)
{
    if (!out)
        return fail(SW_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_problems < 1 || !problems)
        return fail(SW_ERR_ARG, "empty problem list");
    if (opts && (opts->blocks_per_cu < 0 || opts->wait_limit_us < 0))
        return fail(SW_ERR_ARG, "invalid batch options");
    if (opts && opts->threads != 0 && opts->threads != 256 && opts->threads != 512)
        return fail(SW_ERR_ARG, "batch threads must be 0, 256 or 512");
    const int threads = (opts && opts->threads) ? opts->threads : 256;
    for (int i = 0; i < n_problems; ++i) {
        const sw_problem &p = problems[i];
        int rc = check_common(p.eq, p.n_cells, p.n_steps, p.dt, p.dx, p.d_state, 4);
        if (rc)
            return fail(rc, "problem %d: %s", i, last_error());
        if (p.width && !width_ok(p.eq, p.n_cells, p.width))
            return fail(SW_ERR_ARG, "problem %d: width %d invalid for n_cells %lld", i, p.width,
                        (long long)p.n_cells);
    }
    int dev = 0;
    int rc = check_device_pointer(problems[0].d_state, &dev);
    if (rc)
        return rc;
    for (int i = 1; i < n_problems; ++i) {
        int d = 0;
        rc = check_device_pointer(problems[i].d_state, &d);
        if (rc)
            return fail(rc, "problem %d: %s", i, last_error());
    }

    std::vector<sw::BatchProblem> hp(n_problems);
    std::vector<int> widths(n_problems);
    size_t array_bytes = 0, max_lds = 0;
    int64_t flags = 0;
    int64_t max_phase = 0;
    for (int i = 0; i < n_problems; ++i) {
        const sw_problem &p = problems[i];
        int w = p.width;
        if (!w) {
            w = chosen_width(dev, p.eq, p.n_cells, nullptr, true);
            if (!w)
                return fail(SW_ERR_UNSUPPORTED, "problem %d: no valid width for n_cells %lld", i,
                            (long long)p.n_cells);
        }
        if (p.n_cells / w > (int64_t)INT32_MAX)
            return fail(SW_ERR_ARG, "problem %d: %lld tiles of %d cells exceed 2^31 - 1", i,
                        (long long)(p.n_cells / w), w);
        widths[i] = w;
        sw::BatchProblem &b = hp[i];
        b.state = p.d_state;
        b.n = p.n_cells;
        b.w = w;
        b.eq = p.eq;
        b.tiles = (int)(p.n_cells / w);
        b.final_level = p.n_steps * substeps(p.eq);
        b.radius = radius(p.eq);
        b.phases = sw::phase_count(b.final_level, w / (2 * b.radius));
        b.single_phase = (b.phases == 1);
        b.coef = is_euler(p.eq) ? p.dt / p.dx : p.dt / (p.dx * p.dx);
        if (is_f32(p.eq))
            b.coef = (double)(float)b.coef;
        b.flag_off = flags;
        flags += b.tiles;
        array_bytes += 2 * swept_copy_bytes(p.eq, p.n_cells);
        max_lds = std::max(max_lds, (size_t)(w + 2 * b.radius) * (size_t)lds_per_cell(p.eq));
        max_phase = std::max<int64_t>(max_phase, b.phases + (b.single_phase ? 1 : 0));
    }
    // segments, phase-major
    std::vector<sw::BatchSegment> segs;
    int64_t items = 0;
    for (int64_t k = 1; k <= max_phase; ++k)
        for (int i = 0; i < n_problems; ++i) {
            const int64_t pk = hp[i].phases + (hp[i].single_phase ? 1 : 0);
            if (k > pk)
                continue;
            segs.push_back(sw::BatchSegment{items, i, (int)k});
            items += hp[i].tiles;
        }

    sw_batch_impl *b = new sw_batch_impl();
    // a batch of heat problems of one precision runs the kernel compiled with
    // that body alone (fewer registers, more resident workgroups)
    int bodies = 0;
    {
        bool all64 = true, all32 = true;
        for (int i = 0; i < n_problems; ++i) {
            all64 = all64 && problems[i].eq == SW_HEAT_F64;
            all32 = all32 && problems[i].eq == SW_HEAT_F32;
        }
        bodies = all64 ? 1 : (all32 ? 2 : 0);
    }
    b->device = dev;
    b->threads = threads;
    b->bodies = bodies;
    b->widths = widths;
    b->items = items;
    b->flags = flags;
    const size_t off_seg = round_up(sizeof(sw::BatchProblem) * n_problems, 256);
    const size_t off_ticket = off_seg + round_up(sizeof(sw::BatchSegment) * std::max<size_t>(segs.size(), 1), 256);
    const size_t off_status = off_ticket + 256;
    const size_t off_flags = off_status + 256;
    b->table_bytes = off_flags + round_up(sizeof(int) * std::max<int64_t>(flags, 1), 256);
    b->array_bytes = array_bytes;
    if (hipMalloc(&b->tables, b->table_bytes) != hipSuccess ||
        (array_bytes && hipMalloc(&b->arrays, array_bytes) != hipSuccess)) {
        const size_t table_bytes = b->table_bytes;
        free_batch(b);
        return fail(SW_ERR_NOMEM, "batch allocation of %zu + %zu bytes failed", table_bytes,
                    array_bytes);
    }
    char *arr = (char *)b->arrays;
    for (int i = 0; i < n_problems; ++i) {
        const size_t copy = swept_copy_bytes(hp[i].eq, hp[i].n);
        hp[i].ws0 = arr;
        hp[i].ws1 = arr + copy;
        arr += 2 * copy;
    }
    char *tb = (char *)b->tables;
    // the ticket and the status word start at zero, so that sw_batch_wait
    // before any run reports success (each run resets them on the device)
    if (hipMemcpy(tb, hp.data(), sizeof(sw::BatchProblem) * n_problems, hipMemcpyHostToDevice) !=
            hipSuccess ||
        (!segs.empty() && hipMemcpy(tb + off_seg, segs.data(), sizeof(sw::BatchSegment) * segs.size(),
                                    hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemset(tb + off_ticket, 0, off_flags - off_ticket) != hipSuccess) {
        free_batch(b);
        return fail(SW_ERR_HIP, "uploading batch tables failed");
    }
    sw::BatchTables t;
    t.problems = (const sw::BatchProblem *)tb;
    t.segments = (const sw::BatchSegment *)(tb + off_seg);
    t.n_segments = (int64_t)segs.size();
    t.n_items = items;
    t.ticket = (unsigned long long *)(tb + off_ticket);
    t.status = (int *)(tb + off_status);
    t.flags = (int *)(tb + off_flags);
    const long long limit_us = (opts && opts->wait_limit_us) ? opts->wait_limit_us : 10000000LL;
    t.wait_limit = limit_us * 100;  // s_memrealtime runs at 100 MHz
    b->d_status = t.status;

    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        sw::batch_occupancy(max_lds, threads, bodies, &per_cu) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        free_batch(b);
        return fail(SW_ERR_HIP, "batch occupancy query failed (LDS %zu bytes)", max_lds);
    }
    if (opts && opts->blocks_per_cu)
        per_cu = std::min(per_cu, opts->blocks_per_cu);
    int64_t blocks = (int64_t)cus * per_cu;
    if (blocks > items)
        blocks = std::max<int64_t>(items, 1);
    b->blocks = (int)blocks;

    // capture reset + persistent kernel into a graph on a private stream
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = sw::batch_launch(t, flags, b->blocks, threads, bodies, max_lds, cap);
        e = hipStreamEndCapture(cap, &b->graph);
        if (le != hipSuccess)
            e = le;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiateWithFlags(&b->exec, b->graph, 0);
    if (cap)
        (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_batch(b);
        return fail(SW_ERR_HIP, "building the batch graph failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return ok();
}

int sw_batch_run(sw_batch b, sw_stream stream)
{
    if (!b)
        return fail(SW_ERR_ARG, "batch is NULL");
    if (b->items == 0)
        return ok();
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? ok() : launched(e, "hipGraphLaunch of the batch");
}

int sw_batch_wait(sw_batch b, sw_stream stream)
{
    if (!b)
        return fail(SW_ERR_ARG, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    int status = 0;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipMemcpy(&status, b->d_status, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return launched(e, "waiting for the batch");
    if (status)
        return fail(SW_ERR_HIP, "batch aborted: a dependency wait exceeded its time bound");
    return ok();
}

int sw_batch_info(sw_batch b, int64_t *items, int *blocks, size_t *array_bytes)
{
    if (!b)
        return fail(SW_ERR_ARG, "batch is NULL");
    if (items)
        *items = b->items;
    if (blocks)
        *blocks = b->blocks;
    if (array_bytes)
        *array_bytes = b->array_bytes;
    return ok();
}

int sw_batch_width(sw_batch b, int problem)
{
    if (!b || problem < 0 || problem >= (int)b->widths.size())
        return 0;
    return b->widths[problem];
}

void sw_batch_destroy(sw_batch b)
{
    if (!b)
        return;
    (void)hipDeviceSynchronize();
    free_batch(b);
}

int sw_batch_item_deps(int phase, int tile, int tiles, int single_phase, int *deps)
{
    if (!deps || tiles < 2 || tile < 0 || tile >= tiles || phase < 1)
        return -1;
    return sw::batch_deps(phase, tile, tiles, single_phase, deps);
}

int swept_solve_batch(int n_problems, const sw_problem *problems, sw_stream stream)
{
    sw_batch b = nullptr;
    int rc = sw_batch_create(n_problems, problems, nullptr, &b);
    if (rc)
        return rc;
    rc = sw_batch_run(b, stream);
    if (rc == SW_OK)
        rc = sw_batch_wait(b, stream);
    const std::string msg = last_error();
    sw_batch_destroy(b);
    return rc ? fail(rc, "%s", msg.c_str()) : ok();
}

int sw_batch_autotune(int n_problems, sw_problem *problems, int64_t probe_steps,
                      sw_stream stream, sw_batch_opts *best, double *best_ms_per_update)
{
    if (!best)
        return fail(SW_ERR_ARG, "best is NULL");
    if (n_problems < 1 || !problems)
        return fail(SW_ERR_ARG, "empty problem list");
    if (probe_steps < 0 || probe_steps > 1000000)
        return fail(SW_ERR_ARG, "probe_steps out of range");
    const int only_threads = best->threads;  // 0: try both workgroup sizes
    if (only_threads != 0 && only_threads != 256 && only_threads != 512)
        return fail(SW_ERR_ARG, "best->threads must be 0, 256 or 512");
    for (int i = 0; i < n_problems; ++i) {
        const sw_problem &p = problems[i];
        int rc = check_common(p.eq, p.n_cells, p.n_steps, p.dt, p.dx, p.d_state, 4);
        if (rc)
            return fail(rc, "problem %d: %s", i, last_error());
        if (p.width && !width_ok(p.eq, p.n_cells, p.width))
            return fail(SW_ERR_ARG, "problem %d: width %d invalid for n_cells %lld", i, p.width,
                        (long long)p.n_cells);
    }
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return fail(SW_ERR_CAPTURE, "sw_batch_autotune cannot run during stream capture");
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "device query failed");
    }
    std::vector<int> widths(n_problems);
    for (int i = 0; i < n_problems; ++i) {
        widths[i] = problems[i].width ? problems[i].width
                                      : chosen_width(dev, problems[i].eq, problems[i].n_cells, nullptr, true);
        if (!widths[i])
            return fail(SW_ERR_UNSUPPORTED, "problem %d: no valid width for n_cells %lld", i,
                        (long long)problems[i].n_cells);
    }

    // scratch copies of the states: every probe runs on these
    std::vector<size_t> offs(n_problems);
    size_t total = 0;
    for (int i = 0; i < n_problems; ++i) {
        offs[i] = total;
        total += round_up(sw_state_bytes(problems[i].eq, problems[i].n_cells), 256);
    }
    char *buf = nullptr;
    if (hipMalloc(&buf, total) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_NOMEM, "batch autotune scratch states (%zu bytes) failed", total);
    }
    int rc = SW_OK;
    for (int i = 0; i < n_problems && rc == SW_OK; ++i) {
        if (hipMemcpyAsync(buf + offs[i], problems[i].d_state,
                           sw_state_bytes(problems[i].eq, problems[i].n_cells),
                           hipMemcpyDeviceToDevice, s) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(SW_ERR_HIP, "copying problem %d to the scratch state failed", i);
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == SW_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        (void)hipGetLastError();
        rc = fail(SW_ERR_HIP, "hipEventCreate failed");
    }

    // the same steps per problem in every probe, so that the probes do the
    // same work: probe_steps, or (0) four phases at the widest power-of-two
    // cap of the problem's equation
    std::vector<int64_t> steps(n_problems);
    double work = 0.0;
    for (int i = 0; i < n_problems; ++i) {
        const int e = problems[i].eq;
        int cap = 64;
        while (cap * 2 <= max_width(e))
            cap *= 2;
        const int64_t sub = substeps(e);
        const int64_t four = (4 * (cap / (2 * radius(e))) + sub - 1) / sub;
        steps[i] = std::min(problems[i].n_steps, probe_steps ? probe_steps : four);
        work += (double)problems[i].n_cells * (double)steps[i];
    }

    // one probe: the batch with widths `ws`, `bpc` workgroups per CU of
    // `threads` threads; the result is the ms of the timed run (after one
    // warm-up run)
    int max_bpc = 0;
    auto probe = [&](const std::vector<int> &ws, int bpc, int threads, double *ms_out) -> int {
        std::vector<sw_problem> sp(problems, problems + n_problems);
        for (int i = 0; i < n_problems; ++i) {
            sp[i].d_state = buf + offs[i];
            sp[i].width = ws[i];
            sp[i].n_steps = steps[i];
        }
        sw_batch_opts o{bpc, threads, 0};
        sw_batch b = nullptr;
        int r = sw_batch_create(n_problems, sp.data(), &o, &b);
        if (r)
            return r;
        int64_t items = 0;
        int blocks = 0;
        size_t bytes = 0;
        sw_batch_info(b, &items, &blocks, &bytes);
        if (bpc == 0)
            max_bpc = std::max(1, (blocks + cus - 1) / std::max(cus, 1));
        float ms = 0.f;
        r = sw_batch_run(b, stream);  // warm-up
        if (r == SW_OK)
            r = sw_batch_wait(b, stream);
        if (r == SW_OK && hipEventRecord(e0, s) != hipSuccess)
            r = fail(SW_ERR_HIP, "hipEventRecord failed");
        if (r == SW_OK)
            r = sw_batch_run(b, stream);
        if (r == SW_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            r = fail(SW_ERR_HIP, "batch autotune timing failed");
        if (r == SW_OK)
            r = sw_batch_wait(b, stream);
        const std::string msg = last_error();
        sw_batch_destroy(b);
        (void)hipGetLastError();
        if (r)
            return fail(r, "%s", msg.c_str());
        *ms_out = ms;
        return SW_OK;
    };

    // For each workgroup size (four and eight waves):
    // 1. widths, one equation at a time: every problem of that equation that
    //    leaves its width to the library takes the largest valid width up to
    //    a cap; caps 64, 128, ... up to the equation's widest tile (eight-wave
    //    workgroups start from the four-wave choice and try caps from 512 up:
    //    narrower tiles leave most of their waves idle);
    // 2. resident workgroups per CU for those widths (0 = occupancy limit).
    // The fastest (widths, workgroup size, workgroups per CU) wins.
    std::vector<int> eqs;
    for (int i = 0; i < n_problems; ++i)
        if (!problems[i].width && std::find(eqs.begin(), eqs.end(), problems[i].eq) == eqs.end())
            eqs.push_back(problems[i].eq);
    const std::vector<int> start = widths;
    double best_ms = INFINITY;
    int best_bpc = 0, best_threads = 256;
    for (int threads = 256; threads <= 512 && rc == SW_OK; threads *= 2) {
        if (only_threads && threads != only_threads)
            continue;
        std::vector<int> ws = best_ms < INFINITY ? widths : start;
        double top = INFINITY;
        rc = probe(ws, 0, threads, &top);
        for (size_t k = 0; k < eqs.size() && rc == SW_OK; ++k) {
            const int e = eqs[k];
            const int step = 2 * radius(e);
            for (int cap = threads >= 512 ? 512 : 64; cap <= max_width(e) && rc == SW_OK;
                 cap *= 2) {
                std::vector<int> cand = ws;
                for (int i = 0; i < n_problems; ++i) {
                    if (problems[i].width || problems[i].eq != e)
                        continue;
                    for (int w = cap - cap % step; w >= step; w -= step)
                        if (width_ok(e, problems[i].n_cells, w)) {
                            cand[i] = w;
                            break;
                        }
                }
                if (cand == ws)
                    continue;
                double t = 0.0;
                rc = probe(cand, 0, threads, &t);
                if (rc == SW_OK && t < top) {
                    top = t;
                    ws = cand;
                }
            }
        }
        int top_bpc = 0;
        if (rc == SW_OK)
            rc = probe(ws, 0, threads, &top);  // also sets max_bpc for these widths
        for (int bpc = 1; bpc < max_bpc && rc == SW_OK; ++bpc) {
            double t = 0.0;
            rc = probe(ws, bpc, threads, &t);
            if (rc == SW_OK && t < top) {
                top = t;
                top_bpc = bpc;
            }
        }
        if (rc == SW_OK && top < best_ms) {
            best_ms = top;
            best_bpc = top_bpc;
            best_threads = threads;
            widths = ws;
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    (void)hipGetLastError();
    if (rc)
        return rc;
    for (int i = 0; i < n_problems; ++i)
        if (!problems[i].width)
            problems[i].width = widths[i];
    best->blocks_per_cu = best_bpc;
    best->threads = best_threads;
    best->wait_limit_us = 0;
    if (best_ms_per_update)
        *best_ms_per_update = work > 0.0 ? best_ms / work : 0.0;
    return ok();
}

} // extern "C"
