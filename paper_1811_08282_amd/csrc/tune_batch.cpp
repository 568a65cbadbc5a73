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
// Batch: a problem list is planned on the host into one table (batch.h,
// batch_plan.h) and a workspace layout (header, table, tile flags, working
// arrays).  swept_solve_batch enqueues the table upload, the reset kernel and
// the persistent kernel into a caller-owned workspace; sw_batch_create
// allocates the workspace itself, uploads the table once and captures the
// reset and persistent kernels into a hipGraph that sw_batch_run launches.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/swept.h"
#include "batch.h"
#include "batch_plan.h"
#include "geom.h"
#include "host.h"
#include "kernels.h"

namespace sw {

// bodies: 0 every tile body, 1 heat binary64 only, 2 heat binary32 only
hipError_t batch_occupancy(size_t lds_bytes, int threads, int bodies, int *blocks_per_cu);
hipError_t batch_launch(const BatchTables &t, int64_t n_flags, int blocks, int threads,
                        int bodies, size_t lds_bytes, hipStream_t s);
// copy `bytes` (a multiple of 8) from host memory to device memory `dst` by
// kernels that carry the data in their arguments (capturable, no host buffer
// has to outlive the call)
hipError_t batch_put(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t poison_on_abort(const void *ws, void *state, size_t bytes, hipStream_t s);
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
        const bool sized = t == 64 || t == 128 || t == 256 || t == 512;
        if (valid_eq(eq) && width_ok(eq, n, w) && (sized || (t == 0 && persistent_route(eq, n, w))))
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

int chosen_width(int dev, int eq, int64_t n, int *threads, bool batch, bool *tuned)
{
    if (tuned)
        *tuned = false;
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
                if (tuned)
                    *tuned = true;
                return it->second.width;
            }
            auto ic = g_tune_class.find(std::make_tuple(arch, eq, size_class(n)));
            if (ic != g_tune_class.end() && width_ok(eq, n, ic->second.width)) {
                if (threads)
                    *threads = ic->second.threads;
                if (tuned)
                    *tuned = true;
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

// ---- batch planning and launch ---------------------------------------------

namespace {

constexpr size_t kHeaderBytes = 256;  // ticket (8 B at 0) and status word (4 B at 8)
constexpr int64_t kMaxBatchPhase = (int64_t)INT32_MAX - 1;

// Byte layout of a batch workspace: header, sorted problem table, tile
// flags, every problem's two working arrays.  All parts are 256-byte aligned.
struct PreparedBatch {
    sw::BatchPlan plan;
    std::vector<int> widths;        // caller order
    std::vector<size_t> array_off;  // caller order, within the array part
    size_t array_bytes = 0;
    size_t max_lds = 0;
    int bodies = 0;                 // 0 every tile body, 1 heat binary64 only, 2 heat binary32 only
    size_t off_table = 0, off_flags = 0, off_arrays = 0, total = 0;
};

int check_batch_opts(const sw_batch_opts *opts)
{
    if (opts && (opts->blocks_per_cu < 0 || opts->wait_limit_us < 0))
        return fail(SW_ERR_ARG, "invalid batch options");
    if (opts && opts->threads != 0 && opts->threads != 256 && opts->threads != 512)
        return fail(SW_ERR_ARG, "batch threads must be 0, 256 or 512");
    return SW_OK;
}

// Validate the problems and plan the batch (host only; no HIP call unless a
// tuned width has been recorded, whose lookup asks for the current device).
int prepare_batch(int n_problems, const sw_problem *problems, PreparedBatch *pb)
{
    if (n_problems < 1 || !problems)
        return fail(SW_ERR_ARG, "empty problem list");
    std::vector<sw::BatchProblem> in(n_problems);
    pb->widths.assign(n_problems, 0);
    pb->array_off.assign(n_problems, 0);
    size_t arrays = 0;
    bool all64 = true, all32 = true;
    for (int i = 0; i < n_problems; ++i) {
        const sw_problem &p = problems[i];
        int rc = check_common(p.eq, p.n_cells, p.n_steps, p.dt, p.dx, p.d_state, 4);
        if (rc)
            return fail(rc, "problem %d: %s", i, last_error());
        if (p.eq == SW_KS_F64)
            return fail(SW_ERR_UNSUPPORTED,
                        "problem %d: the batched launch has no Kuramoto-Sivashinsky tile body", i);
        if (p.width && !width_ok(p.eq, p.n_cells, p.width))
            return fail(SW_ERR_ARG, "problem %d: width %d invalid for n_cells %lld", i, p.width,
                        (long long)p.n_cells);
        const int w = p.width ? p.width : chosen_width(-1, p.eq, p.n_cells, nullptr, true);
        if (!w)
            return fail(SW_ERR_UNSUPPORTED, "problem %d: no valid width for n_cells %lld", i,
                        (long long)p.n_cells);
        if (p.n_cells / w > (int64_t)INT32_MAX)
            return fail(SW_ERR_ARG, "problem %d: %lld tiles of %d cells exceed 2^31 - 1", i,
                        (long long)(p.n_cells / w), w);
        sw::BatchProblem &b = in[i];
        b = sw::BatchProblem{};
        b.state = p.d_state;
        b.n = p.n_cells;
        b.w = w;
        b.eq = p.eq;
        b.tiles = (int)(p.n_cells / w);
        b.final_level = p.n_steps * substeps(p.eq);
        b.radius = radius(p.eq);
        b.phases = sw::phase_count(b.final_level, w / (2 * b.radius));
        b.single_phase = (b.phases == 1);
        if (b.phases + b.single_phase > kMaxBatchPhase)
            return fail(SW_ERR_ARG, "problem %d: %lld phases exceed 2^31 - 2 (use a wider tile)",
                        i, (long long)b.phases);
        b.item_phases = (int)(b.phases + b.single_phase);
        b.coef = is_euler(p.eq) ? p.dt / p.dx : p.dt / (p.dx * p.dx);
        if (is_f32(p.eq))
            b.coef = (double)(float)b.coef;
        pb->widths[i] = w;
        pb->array_off[i] = arrays;
        arrays += 2 * swept_copy_bytes(p.eq, p.n_cells);
        pb->max_lds = std::max(pb->max_lds, (size_t)sw::lds_tile_cells(is_heat(p.eq), w, b.radius) *
                                                (size_t)lds_per_cell(p.eq));
        all64 = all64 && p.eq == SW_HEAT_F64;
        all32 = all32 && p.eq == SW_HEAT_F32;
    }
    if (!sw::plan_batch(in, &pb->plan))
        return fail(SW_ERR_ARG, "the batch has more than 2^63 work items");
    // a batch of heat problems of one precision runs the kernel compiled with
    // that body alone (fewer registers, more resident workgroups)
    pb->bodies = all64 ? 1 : (all32 ? 2 : 0);
    pb->array_bytes = arrays;
    pb->off_table = kHeaderBytes;
    pb->off_flags = pb->off_table + round_up(sizeof(sw::BatchProblem) * (size_t)n_problems, 256);
    pb->off_arrays = pb->off_flags + round_up(sizeof(int) * (size_t)pb->plan.n_flags, 256);
    pb->total = pb->off_arrays + arrays;
    return SW_OK;
}

// Every problem's state on the current device (HIP queries, no allocation).
int check_batch_pointers(int n_problems, const sw_problem *problems, int *dev)
{
    for (int i = 0; i < n_problems; ++i) {
        int d = 0;
        int rc = check_device_pointer(problems[i].d_state, &d);
        if (rc)
            return fail(rc, "problem %d: %s", i, last_error());
        *dev = d;
    }
    return SW_OK;
}

// Working-array pointers of the table entries inside workspace `ws`.
void place_arrays(PreparedBatch *pb, char *ws)
{
    for (size_t s = 0; s < pb->plan.table.size(); ++s) {
        sw::BatchProblem &b = pb->plan.table[s];
        const int i = pb->plan.order[s];
        const size_t copy = swept_copy_bytes(b.eq, b.n);
        b.ws0 = ws + pb->off_arrays + pb->array_off[i];
        b.ws1 = (char *)b.ws0 + copy;
    }
}

sw::BatchTables device_tables(const PreparedBatch &pb, char *ws, const sw_batch_opts *opts)
{
    sw::BatchTables t;
    t.problems = (const sw::BatchProblem *)(ws + pb.off_table);
    t.n_problems = (int)pb.plan.table.size();
    t.n_items = pb.plan.n_items;
    t.ticket = (unsigned long long *)ws;
    t.status = (int *)(ws + 8);
    t.flags = (int *)(ws + pb.off_flags);
    const long long limit_us = (opts && opts->wait_limit_us) ? opts->wait_limit_us : 10000000LL;
    t.wait_limit = limit_us * 100;  // s_memrealtime runs at 100 MHz
    return t;
}

// Resident workgroups of the persistent launch: CUs x occupancy (capped by
// opts->blocks_per_cu), at most one per item.
int batch_blocks(const PreparedBatch &pb, int dev, int threads, const sw_batch_opts *opts,
                 int *blocks)
{
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        sw::batch_occupancy(pb.max_lds, threads, pb.bodies, &per_cu) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "batch occupancy query failed (LDS %zu bytes)", pb.max_lds);
    }
    if (opts && opts->blocks_per_cu)
        per_cu = std::min(per_cu, opts->blocks_per_cu);
    int64_t b = (int64_t)cus * per_cu;
    if (b > pb.plan.n_items)
        b = std::max<int64_t>(pb.plan.n_items, 1);
    *blocks = (int)b;
    return SW_OK;
}

// Table upload: kernels that carry the table in their launch arguments, so
// no host buffer outlives the call and the upload can be captured.
int upload_table(const PreparedBatch &pb, char *ws, hipStream_t s)
{
    return launched(sw::batch_put(ws + pb.off_table, pb.plan.table.data(),
                                  sizeof(sw::BatchProblem) * pb.plan.table.size(), s),
                    "batch table upload");
}

// The reset kernel and the persistent kernel on `s`: nothing is allocated,
// nothing waits, and the pair can be captured into a graph.
int launch_run(const PreparedBatch &pb, char *ws, const sw_batch_opts *opts, int blocks,
               int threads, hipStream_t s)
{
    const sw::BatchTables t = device_tables(pb, ws, opts);
    return launched(sw::batch_launch(t, pb.plan.n_flags, blocks, threads, pb.bodies, pb.max_lds, s),
                    "batch launch");
}

} // namespace

// ---- batch handle -------------------------------------------------------------

struct sw_batch_impl {
    int device = 0;
    char *ws = nullptr;          // header, table, flags, working arrays
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t items = 0;
    int blocks = 0;
    size_t array_bytes = 0;
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
    if (b->ws)
        (void)hipFree(b->ws);
    (void)hipGetLastError();
    delete b;
}

int batch_create(int n_problems, const sw_problem *problems, const sw_batch_opts *opts,
                 sw_batch *out)
{
    if (!out)
        return fail(SW_ERR_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_batch_opts(opts);
    if (rc)
        return rc;
    const int threads = (opts && opts->threads) ? opts->threads : 256;
    PreparedBatch pb;
    rc = prepare_batch(n_problems, problems, &pb);
    if (rc)
        return rc;
    int dev = 0;
    rc = check_batch_pointers(n_problems, problems, &dev);
    if (rc)
        return rc;
    int blocks = 0;
    rc = batch_blocks(pb, dev, threads, opts, &blocks);
    if (rc)
        return rc;

    sw_batch_impl *b = new sw_batch_impl();
    b->device = dev;
    b->widths = pb.widths;
    b->items = pb.plan.n_items;
    b->blocks = blocks;
    b->array_bytes = pb.array_bytes;
    if (hipMalloc(&b->ws, pb.total) != hipSuccess) {
        (void)hipGetLastError();
        b->ws = nullptr;
        free_batch(b);
        return fail(SW_ERR_NOMEM, "batch allocation of %zu bytes failed", pb.total);
    }
    place_arrays(&pb, b->ws);
    // the table is uploaded once; the ticket and the status word start at
    // zero so that sw_batch_wait before any run reports success (each run
    // resets them on the device).  Then the reset and persistent kernels are
    // captured into a graph on the same private stream.
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipMemsetAsync(b->ws, 0, kHeaderBytes, cap);
    if (e == hipSuccess && upload_table(pb, b->ws, cap) != SW_OK)
        e = hipErrorLaunchFailure;
    if (e == hipSuccess)
        e = hipStreamSynchronize(cap);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = launch_run(pb, b->ws, opts, blocks, threads, cap);
        e = hipStreamEndCapture(cap, &b->graph);
        if (rc != SW_OK && e == hipSuccess)
            e = hipErrorLaunchFailure;
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

int batch_solve(int n_problems, const sw_problem *problems, const sw_batch_opts *opts,
                void *d_ws, size_t ws_bytes, hipStream_t s)
{
    int rc = check_batch_opts(opts);
    if (rc)
        return rc;
    const int threads = (opts && opts->threads) ? opts->threads : 256;
    PreparedBatch pb;
    rc = prepare_batch(n_problems, problems, &pb);
    if (rc)
        return rc;
    if (!d_ws)
        return fail(SW_ERR_ARG, "d_ws is NULL (size it with sw_batch_workspace_bytes)");
    if (((uintptr_t)d_ws & 255) != 0)
        return fail(SW_ERR_ARG, "d_ws must be 256-byte aligned");
    if (ws_bytes < pb.total)
        return fail(SW_ERR_ARG, "workspace of %zu bytes is smaller than the %zu the batch needs",
                    ws_bytes, pb.total);
    if (pb.plan.n_items == 0)
        return ok();
    int dev = 0;
    rc = check_batch_pointers(n_problems, problems, &dev);
    if (rc)
        return rc;
    int wdev = 0;
    rc = check_device_pointer(d_ws, &wdev);
    if (rc)
        return fail(rc, "d_ws: %s", last_error());
    int blocks = 0;
    rc = batch_blocks(pb, dev, threads, opts, &blocks);
    if (rc)
        return rc;
    place_arrays(&pb, (char *)d_ws);
    rc = upload_table(pb, (char *)d_ws, s);
    if (rc == SW_OK)
        rc = launch_run(pb, (char *)d_ws, opts, blocks, threads, s);
    return rc ? rc : ok();
}

} // namespace

namespace sw {
namespace host {

size_t persistent_workspace_bytes(const sw_problem &p)
{
    PreparedBatch pb;
    return prepare_batch(1, &p, &pb) == SW_OK ? pb.total : 0;
}

int run_swept_persistent(const sw_problem &p, void *ws, size_t ws_bytes, hipStream_t s)
{
    sw_batch_opts bo{};
    bo.threads = 256;
    // the bound of one dependency wait (microseconds); a test forces the
    // abort path with a tiny one
    if (const char *v = getenv("SW_WAIT_LIMIT_US")) {
        const long long us = strtoll(v, nullptr, 10);
        if (us > 0)
            bo.wait_limit_us = us;
    }
    const int rc = batch_solve(1, &p, &bo, ws, ws_bytes, s);
    if (rc)
        return rc;
    return launched(sw::poison_on_abort(ws, p.d_state, state_bytes(p.eq, p.n_cells), s),
                    "the abort check of the persistent launch");
}

} // namespace host
} // namespace sw

extern "C" {

static int autotune_impl(int eq, int64_t n_cells, int64_t probe_steps, sw_stream stream,
                         sw_opts *best, double *best_ms_per_update)
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
    // one warm-up solve, then one timed solve: ms per cell-update
    // one warm-up solve, then one timed solve: ms per cell-update
    auto probe = [&](auto &&solve_once, double *per) -> int {
        int r = solve_once();
        if (r)
            return r;
        if (hipEventRecord(e0, s) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SW_ERR_HIP, "hipEventRecord failed");
        }
        r = solve_once();
        if (r)
            return r;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SW_ERR_HIP, "autotune timing failed");
        }
        *per = (double)ms / ((double)n_cells * (double)steps);
        return SW_OK;
    };
    for (size_t ci = 0; ci < cands.size() && rc == SW_OK; ++ci) {
        const int w = cands[ci];
        double per = 0.0;
        for (int threads = 512; threads >= 64 && rc == SW_OK; threads /= 2) {
            if (threads > 64 && threads / 2 >= w)
                continue;  // wider workgroups than the tile only idle
            const sw_opts o{w, threads, ws, wbytes};
            rc = probe([&] { return swept_solve_ex(eq, n_cells, steps, dt, dx, state, stream, &o); },
                       &per);
            if (rc == SW_OK && per < top.ms_per_update)
                top = TuneEntry{w, threads, per};
        }
        // the one persistent launch swept_solve takes at this width (recorded
        // as workgroup size 0), on working arrays of its own allocated here
        if (rc == SW_OK && persistent_route(eq, n_cells, w) &&
            sw::phase_count(steps * substeps(eq), w / 2) >= 2) {
            sw_problem p{};
            p.eq = eq;
            p.width = w;
            p.n_cells = n_cells;
            p.n_steps = steps;
            p.dt = dt;
            p.dx = dx;
            p.d_state = state;
            const size_t pneed = persistent_workspace_bytes(p);
            void *pws = nullptr;
            if (pneed && hipMalloc(&pws, pneed) == hipSuccess) {
                rc = probe([&] { return run_swept_persistent(p, pws, pneed, s); }, &per);
                (void)hipStreamSynchronize(s);
                (void)hipFree(pws);
                if (rc == SW_OK && per < top.ms_per_update)
                    top = TuneEntry{w, 0, per};
            } else {
                (void)hipGetLastError();  // no room: the phase launches stand
            }
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

int sw_autotune(int eq, int64_t n_cells, int64_t probe_steps, sw_stream stream, sw_opts *best,
                double *best_ms_per_update)
{
    return guarded(
        [&] { return autotune_impl(eq, n_cells, probe_steps, stream, best, best_ms_per_update); });
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
    return guarded([&] { return batch_create(n_problems, problems, opts, out); });
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
    return sw_batch_check(b->ws, stream);
}

int sw_batch_check(const void *d_ws, sw_stream stream)
{
    if (!d_ws)
        return fail(SW_ERR_ARG, "d_ws is NULL");
    int status = 0;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess)
        e = hipMemcpy(&status, (const char *)d_ws + 8, sizeof(int), hipMemcpyDeviceToHost);
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

size_t sw_batch_workspace_bytes(int n_problems, const sw_problem *problems)
{
    size_t total = 0;
    const int rc = guarded([&] {
        PreparedBatch pb;
        const int r = prepare_batch(n_problems, problems, &pb);
        if (r == SW_OK)
            total = pb.total;
        return r;
    });
    return rc == SW_OK ? total : 0;
}

int swept_solve_batch(int n_problems, const sw_problem *problems, void *d_ws, size_t ws_bytes,
                      sw_stream stream)
{
    return guarded([&] {
        return batch_solve(n_problems, problems, nullptr, d_ws, ws_bytes, (hipStream_t)stream);
    });
}

int swept_solve_batch_ex(int n_problems, const sw_problem *problems, const sw_batch_opts *opts,
                         void *d_ws, size_t ws_bytes, sw_stream stream)
{
    return guarded([&] {
        return batch_solve(n_problems, problems, opts, d_ws, ws_bytes, (hipStream_t)stream);
    });
}

static int batch_autotune_impl(int n_problems, sw_problem *problems, int64_t probe_steps,
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
        if (p.eq == SW_KS_F64)
            return fail(SW_ERR_UNSUPPORTED,
                        "problem %d: the batched launch has no Kuramoto-Sivashinsky tile body", i);
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

int sw_batch_autotune(int n_problems, sw_problem *problems, int64_t probe_steps,
                      sw_stream stream, sw_batch_opts *best, double *best_ms_per_update)
{
    return guarded([&] {
        return batch_autotune_impl(n_problems, problems, probe_steps, stream, best,
                                   best_ms_per_update);
    });
}

} // extern "C"
