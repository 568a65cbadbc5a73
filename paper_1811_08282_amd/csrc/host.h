// host.h -- helpers shared by the host-side translation units of the
// library (argument checks, sizes, error text, working arrays).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/swept.h"

namespace sw {
namespace host {

int fail(int code, const char *fmt, ...);
int ok();
const char *last_error();

bool valid_eq(int eq);
bool is_euler(int eq);
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

// width of a swept solve when the caller gives none: the tuned width of
// (device, eq, n) if sw_autotune recorded one, else default_width; threads
// (if not NULL) receives the tuned workgroup size, else default_threads
int chosen_width(int dev, int eq, int64_t n, int *threads, bool batch);

} // namespace host
} // namespace sw
