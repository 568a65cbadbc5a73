// host.h -- helpers shared by the host-side translation units of the
// library (argument checks, sizes, error text, working arrays).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <exception>
#include <new>

#include "../../include/swept.h"
#include "kernels.h"

namespace sw {
namespace host {

int fail(int code, const char *fmt, ...);
int ok();
const char *last_error();

// Run an entry point's body; a C++ exception (host memory or threads
// exhausted) becomes a status code instead of crossing the C boundary.
template <typename F>
int guarded(F f)
{
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return fail(SW_ERR_NOMEM, "host memory exhausted");
    } catch (const std::exception &e) {
        return fail(SW_ERR_NOMEM, "host resources exhausted: %s", e.what());
    }
}

bool valid_eq(int eq);
bool is_euler(int eq);
bool is_heat(int eq);
bool is_flat(int eq);
bool is_f32(int eq);
int substeps(int eq);
int radius(int eq);
int lds_per_cell(int eq);
int struct_bytes(int eq);
int preferred_width(int eq);
int preferred_batch_width(int eq);
int default_threads(int eq, int w);
int max_width(int eq);
bool width_ok(int eq, int64_t n, int64_t w);
// largest valid width up to the preferred one (of the batch kernel if batch)
int default_width(int eq, int64_t n, bool batch);
size_t round_up(size_t x, size_t a);
size_t swept_copy_bytes(int eq, int64_t n);
int check_common(int eq, int64_t n, int64_t steps, double dt, double dx, const void *state,
                 int64_t min_cells);
int check_device_pointer(const void *p, int *dev_out);
int launched(hipError_t e, const char *what);

size_t state_bytes(int eq, int64_t n);

// coefficients of the Kuramoto-Sivashinsky step: a = dt / (2 dx),
// b = dt / dx^2, c = dt / dx^4, in binary64 in this form
void ks_coefficients(double dt, double dx, double *a, double *b, double *c);

// host threads of a shared solve when the caller gives none, and the most
constexpr int kDefaultHostThreads = 8;
constexpr int kMaxHostThreads = 256;

// one swept phase launch of equation id eq (p.tiles tiles from p.offset)
hipError_t swept_phase_launch(int eq, const sw::PhaseLaunch &p, void *state, const void *in,
                              void *out, double dt, double dx, hipStream_t s);

// the swept solve shared between the GPU and host threads (sw_opts.work_factor);
// ws: the device working arrays; synchronises the stream before returning
int run_swept_shared(int eq, int64_t n, int64_t steps, double dt, double dx, void *state,
                     hipStream_t s, int w, int threads, void *ws, int work_factor,
                     int host_threads);

// free the pinned host arrays of shared solves
void release_host_arrays();

// swept_solve runs a heat grid as one persistent launch of the heat-only
// batch kernel (its phases overlap) when its tiles are at least
// kPersistentMinWidth cells wide and more than kPersistentMinTiles in number,
// unless the caller gives a workspace, a workgroup size or a work factor, or
// the autotuner recorded another launch.  Measured on MI355X: with fewer
// tiles than the chip holds resident workgroups (1024 at W = 2048), or with
// narrower tiles (level at W = 1280, behind at 1024), one launch per phase is
// as fast or faster.
constexpr int kPersistentMinWidth = 1792;
constexpr int64_t kPersistentMinTiles = 1024;
bool persistent_route(int eq, int64_t n, int w);

// device workspace of the persistent launch of problem p (0 if p is invalid)
size_t persistent_workspace_bytes(const sw_problem &p);

// one persistent launch of problem p on stream s, then the abort check that
// fills p's state with NaN if a dependency wait of the launch ran out
int run_swept_persistent(const sw_problem &p, void *ws, size_t ws_bytes, hipStream_t s);

// width of a swept solve when the caller gives none: the tuned width of
// (device, eq, n) if sw_autotune recorded one, else default_width; threads
// (if not NULL) receives the tuned workgroup size, else default_threads;
// tuned (if not NULL) tells which of the two it was
int chosen_width(int dev, int eq, int64_t n, int *threads, bool batch, bool *tuned = nullptr);

} // namespace host
} // namespace sw
