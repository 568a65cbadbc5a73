/*
 * swept.h -- C ABI of the swept-rule stencil library (MI355X / gfx950).
 *
 * The library advances a periodic 1D grid of n_cells cells by n_steps
 * explicit time steps, either with the swept time-space decomposition
 * (Magee, Walker & Niemeyer, Sec. 4.1: Up Triangle, Diamond (repeated),
 * Down Triangle, with block edges exchanged between phases) or with the
 * classic one-launch-per-sub-step decomposition the paper compares it with
 * (Sec. 4.1, "Classic").  Both use the same numerical method, so for every
 * valid input they leave bit-identical results in the state buffer.
 *
 * Equations (Sec. 4.2; sub-step layout of Sec. 4.3, Fig. 2b):
 *   heat  : u_t = u_xx, first order forward in time, central in space,
 *           r = dt / (dx * dx); one sub-step per time step.
 *   euler : 1D Euler equations, gamma = 1.4, second-order finite volume with
 *           a minmod limiter driven by a pressure ratio, predictor /
 *           corrector in time; lambda = dt / dx.  Two layouts of the same
 *           arithmetic (Sec. 4.3, Fig. 2): "lengthened" (SW_EULER_F64/F32),
 *           four three-point sub-steps per time step -- Pr(Q0), predictor,
 *           Pr(Q1), corrector -- on a struct of Q0, Q1, Pr; and "flattened"
 *           (SW_EULER_*_FLAT), two five-point sub-steps -- predictor,
 *           corrector, each recomputing the ratio -- on a struct of Q0, Q1.
 *           Both leave bit-identical states after every time step.
 *   ks    : Kuramoto-Sivashinsky u_t + u u_x + u_xx + u_xxxx = 0 (named in
 *           Sec. 2 among the equations the swept rule has been applied to),
 *           binary64, forward Euler with central differences on a five-point
 *           stencil: s_k = (u_{k+1} - u_k) + (u_{k-1} - u_k),
 *           q = (s_{i+1} - s_i) + (s_{i-1} - s_i),
 *           u' = u - ((a (f_{i+1} - f_{i-1}) + b s_i) + c q), f = 0.5 (u u),
 *           a = dt / (2 dx), b = dt / dx^2, c = dt / dx^4.  One sub-step of
 *           radius 2 per time step.  Not available in the batched launch.
 *
 * Precisions:
 *   *_F64 : binary64 throughout.
 *   *_F32 : binary32 state and flux arithmetic; the time update is
 *           accumulated with Kahan compensation whose running compensation is
 *           part of the state; Euler keeps the velocity / pressure /
 *           sound-speed recovery, the pressure ratio and the limiter value in
 *           binary64.  r and lambda are rounded to binary32 once.
 *
 * State layout (d_state, structure of arrays, n = n_cells, one allocation):
 *   SW_HEAT_F64  : double u[n]
 *   SW_HEAT_F32  : float  u[n], c[n]                  (c = Kahan compensation)
 *   SW_EULER_F64, SW_EULER_F64_FLAT : double rho[n], m[n], E[n]
 *                                     (m = rho*u, E = total energy)
 *   SW_EULER_F32, SW_EULER_F32_FLAT : float rho[n], m[n], E[n], c_rho[n], c_m[n], c_E[n]
 *   SW_KS_F64    : double u[n]
 * The buffer is device memory of the current HIP device, at least
 * sw_state_bytes() long and 16-byte aligned.  It is read as the state at step
 * 0 and overwritten in place with the state at step n_steps.  Before the first
 * call of an F32 state the caller zeroes the compensations.  The state buffer
 * alone is a complete checkpoint: solving n1 then n2 steps equals n1 + n2.
 *
 * Ownership: the caller owns d_state; the library never frees caller memory.
 * Working arrays are owned and cached by the library, one set per (device,
 * stream), unless the caller passes one in sw_opts.  A call that needs more
 * than the cached set holds synchronises the device, frees it and allocates
 * a larger one; sw_release() frees every set.  Calls on one stream from
 * several host threads at once must therefore not grow that stream's set or
 * race sw_release(): size it with a first call, or pass workspaces.
 *
 * Asynchrony: calls enqueue on `stream` (a hipStream_t; NULL = null stream)
 * and return without waiting.  A kernel fault surfaces at the caller's next
 * synchronisation; a launch error is reported as SW_ERR_HIP.
 *
 * Errors: every function returns an sw_status.  Argument checks run on the
 * host before any HIP call, so an invalid call touches no device state.
 * sw_last_error() returns a message for the last failure on this thread.
 * Stability (r <= 1/2, CFL <= 1) is not checked.
 */
#ifndef SWEPT_H
#define SWEPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SW_OK = 0,
    SW_ERR_ARG = 1,         /* invalid argument (message in sw_last_error) */
    SW_ERR_UNSUPPORTED = 2, /* no valid triangle width for this grid       */
    SW_ERR_HIP = 3,         /* a HIP runtime call or launch failed          */
    SW_ERR_NOMEM = 4,       /* working-array allocation failed              */
    SW_ERR_CAPTURE = 5      /* stream is capturing and no workspace given   */
} sw_status;

typedef enum {
    SW_HEAT_F64 = 0,
    SW_HEAT_F32 = 1,
    SW_EULER_F64 = 2,       /* lengthened layout: four 3-point sub-steps per step */
    SW_EULER_F32 = 3,
    SW_EULER_F64_FLAT = 4,  /* flattened layout: two 5-point sub-steps per step  */
    SW_EULER_F32_FLAT = 5,
    SW_KS_F64 = 6           /* Kuramoto-Sivashinsky, binary64 (see above)        */
} sw_equation;

typedef enum {
    SW_METHOD_SWEPT = 0, /* Up Triangle / Diamond / Down Triangle in LDS */
    SW_METHOD_NAIVE = 1  /* one kernel launch per sub-step (Classic)     */
} sw_method;

/* A hipStream_t passed through the ABI as an opaque pointer. */
typedef void *sw_stream;

/* Optional launch controls of swept_solve_ex / naive_solve_ex.
 *   width           : triangle width W in cells (swept only).  0 = library
 *                     choice.  Valid W: a multiple of 2R (R = 2 for the
 *                     flattened layout and Kuramoto-Sivashinsky, else 1),
 *                     W divides n_cells,
 *                     n_cells / W >= 2, W <= sw_max_width(eq).
 *   threads         : workgroup size of the swept phase kernels: 64, 128,
 *                     256 or 512 (0 = library choice, sw_default_threads).
 *   d_workspace     : device working arrays supplied by the caller (at least
 *                     sw_workspace_bytes() long, 256-byte aligned), or NULL
 *                     for the library's cached arrays.  Required when the
 *                     stream is being captured into a graph.
 *   workspace_bytes : size of d_workspace.
 *   work_factor     : swept only.  0 = the GPU takes every tile.  WF >= 1
 *                     shares the grid with host threads as the paper's GPU
 *                     work factor (Sec. 4.2, Eq. 1): each of the
 *                     host_threads threads takes k = floor(T / (WF + P))
 *                     consecutive tiles (T = n_cells / W tiles, P host
 *                     threads) and the GPU the remaining T - P k, at least
 *                     WF times a thread's share.  Host threads advance their
 *                     tiles with host-compiled copies of the kernels' cell
 *                     arithmetic (same results bit for bit); once per phase
 *                     the two sides exchange the W/2 + R seam structs they
 *                     need from each other through pinned host memory.  The
 *                     call then runs on the calling thread until the solve
 *                     is complete (it synchronises `stream`); it cannot be
 *                     captured (SW_ERR_CAPTURE) and needs at least two
 *                     phases (one heat step runs on the GPU alone).
 *                     SW_ERR_ARG when k would be 0.
 *   host_threads    : host threads of a shared solve, 0 = 8.               */
typedef struct {
    int width;
    int threads;
    void *d_workspace;
    size_t workspace_bytes;
    int work_factor;
    int host_threads;
} sw_opts;

/* Bytes of the state buffer for `eq` and n_cells (0 for an invalid eq). */
size_t sw_state_bytes(int eq, int64_t n_cells);

/* Bytes of working arrays a call needs: the swept method holds two copies of
 * the per-cell working struct (heat F64 16 B, heat F32 12 B, Euler F64 56 B,
 * Euler F32 44 B, flattened Euler F64 48 B, F32 36 B, Kuramoto-Sivashinsky
 * 16 B per cell); the naive
 * method holds the second time level (heat) or the predictor state (and, for
 * the lengthened layout, the pressure ratio).  `width` is
 * unused by either method and may be 0.  0 for invalid arguments. */
size_t sw_workspace_bytes(int eq, int64_t n_cells, int width, int method);

/* Largest triangle width the swept kernels accept for `eq` (set by the LDS
 * a tile needs: W + 2R cells of working struct plus scratch, within the
 * 160 KiB of LDS of one gfx950 compute unit), at most 8192.  0 for an
 * invalid eq. */
int sw_max_width(int eq);

/* The width swept_solve picks when none is given and the autotuner has
 * recorded none (see sw_tuned_width): the largest valid width (a multiple of
 * 2R dividing n_cells with n_cells / W >= 2) not above the preferred width
 * of `eq` -- heat and Kuramoto-Sivashinsky 2048, Euler 1024 (flattened
 * binary32 2048), measured on
 * MI355X.  0 when there is none. */
int sw_default_width(int eq, int64_t n_cells);

/* The workgroup size swept_solve uses for tile width `width` when none is
 * given and the autotuner has recorded none: 512 for Euler tiles of 1000
 * cells or more and Kuramoto-Sivashinsky tiles of 2048 or more (twice the
 * resident waves per compute unit at the same LDS), else the width rounded
 * up to whole 64-lane waves, at most 256.
 * 0 for an invalid eq or width. */
int sw_default_threads(int eq, int width);

/* Swept-rule solve (Sec. 4.1).  Advances d_state by n_steps time steps.
 * dt, dx: finite and > 0.  n_steps >= 0 (0 is a no-op).  n_cells >= 4.
 * One phase is one launch of n_cells / W workgroups, which HIP bounds at
 * 2^32 - 1 work-items: SW_ERR_ARG when (n_cells / W) * workgroup size
 * exceeds that (a wider tile fixes it).
 * A heat grid of more than 1024 tiles of W >= 1792 cells (more than 2^21
 * cells at W = 2048), with 2 to 2^31 - 2 phases, runs instead as one
 * persistent launch (the batch kernel holding this one problem, whose
 * tiles start as soon as the tiles under them are done), when the caller
 * passes no workspace, workgroup size or work factor and the autotuner has
 * recorded no launch for it, or recorded this one (workgroup size 0); the
 * result is the same bit for bit.  Its
 * library-held working arrays are sw_batch_workspace_bytes() of the problem.
 * A dependency wait of that launch is bounded (10 s, or SW_WAIT_LIMIT_US
 * microseconds from the environment); if one runs out, which takes other
 * work holding the GPU's compute units that long, the call, being
 * asynchronous, cannot return an error: d_state is filled with NaN instead. */
int swept_solve(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx,
                void *d_state, sw_stream stream);

/* Classic decomposition: one kernel launch per sub-step (Sec. 4.1, Fig. 2b).
 * Same arguments and result as swept_solve.  3 <= n_cells <= 2^32 - 256
 * (at most one work-item per cell in one launch), else SW_ERR_ARG. */
int naive_solve(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx,
                void *d_state, sw_stream stream);

/* As swept_solve / naive_solve with launch controls (opts may be NULL). */
int swept_solve_ex(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx,
                   void *d_state, sw_stream stream, const sw_opts *opts);
int naive_solve_ex(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx,
                   void *d_state, sw_stream stream, const sw_opts *opts);

/* ---- schedule queries (host only, no HIP call) ------------------------
 * The swept schedule for a final sub-step level F (F = n_steps for heat,
 * 4 * n_steps for lengthened Euler, 2 * n_steps for flattened Euler), width W
 * and stencil radius R of one sub-step (1, or 2 for flattened Euler) has
 * H = W / (2R) levels per half phase and
 *   K = 0 if F == 0, else ceil((F - 1) / H) + 1
 * phases.  Phase k (1-based) tiles the grid from cell offset
 * ((k - 1) % 2) * W/2 in tiles of W cells.  At level (k-1)H + j it computes
 * the cells [R|j - 1|, W - R|j - 1|) of each tile, for j from 1 (k = 1) or
 * 2 - H (k > 1) up to min(H, F - (k-1)H).  Phase 1 is the Up Triangle,
 * phase K the Down Triangle, the others Diamonds (the last ones cut flat at
 * F when F is not a multiple of H).                                       */

/* Number of phases K; -1 for invalid arguments. */
int64_t sw_phase_count(int64_t final_level, int width, int radius);

/* For phase k: the cell offset of its tiling and its first and last
 * sub-step level (first > last when the phase computes nothing).
 * SW_ERR_ARG for invalid arguments. */
int sw_phase_info(int64_t k, int64_t final_level, int width, int radius, int64_t *offset,
                  int64_t *first_level, int64_t *last_level);

/* Active cells of a tile of phase k at sub-step `level`: [*lo, *hi) in tile
 * coordinates (empty when *lo >= *hi).  SW_ERR_ARG for invalid arguments. */
int sw_phase_interval(int64_t k, int64_t final_level, int width, int radius, int64_t level,
                      int *lo, int *hi);

/* ---- autotuner ---------------------------------------------------------------
 * The paper recommends tuning the block width on a limited number of time
 * steps before a long run, starting from wide blocks (Sec. 6).  sw_autotune
 * times short swept solves on a scratch state (allocated and freed here) over
 * every valid width that is a multiple of 64 (every valid width if there is
 * none) and workgroup sizes 64/128/256/512 (at widths where swept_solve
 * takes its one persistent launch, that launch too, recorded as workgroup
 * size 0), and records the fastest for (device architecture, eq, n_cells).
 * swept_solve and the batch use a recorded width whenever the caller gives
 * none.  probe_steps = 0 picks
 * enough steps for four phases at the widest candidate.  If the environment
 * variable SWEPT_TUNE_CACHE names a file, recorded widths are appended to it
 * and read back by later processes.  Not allowed during stream capture
 * (SW_ERR_CAPTURE); synchronises `stream`. */
int sw_autotune(int eq, int64_t n_cells, int64_t probe_steps, sw_stream stream, sw_opts *best,
                double *best_ms_per_update);

/* The width (and workgroup size; 0 = the persistent launch) recorded for
 * exactly (current device, eq, n_cells); SW_ERR_UNSUPPORTED when none is.  A cell count without a record
 * of its own takes, in swept_solve and sw_batch_create, the latest record of
 * its size class floor(log2 n_cells) for the same device and eq when that
 * width is valid for it. */
int sw_tuned_width(int eq, int64_t n_cells, int *width, int *threads);

/* Forget every recorded width of this process (the cache file is kept). */
void sw_tune_clear(void);

/* ---- batched persistent launch -------------------------------------------------
 * Many independent problems advanced by ONE launch of a persistent kernel,
 * captured once into a hipGraph.  Work items (problem, phase, tile) are
 * handed out in phase order by a global ticket; an item waits for the two
 * tiles of the previous phase of its problem that overlap it (per-tile
 * completion flags in device memory), runs the same tile-phase code as
 * swept_solve, and publishes its flag.  Each problem ends bit-identical to
 * swept_solve of that problem with the same width.  Every wait is bounded in
 * time: a wait that exceeds the bound aborts the whole launch, which then
 * reports SW_ERR_HIP from sw_batch_wait.  The persistent kernel runs
 * 256-thread workgroups unless sw_batch_opts asks for 512 (the batch
 * autotuner tries both); a problem without a width and without a tuned one
 * takes the largest valid width up to 2048 for heat, 1024 for flattened
 * Euler and 512 for lengthened Euler, and the LDS of the widest tile sets
 * the resident workgroups per CU of the whole batch.  A batch whose problems
 * are all heat of one precision runs a kernel compiled with that tile body
 * alone (fewer registers, twice the resident workgroups); a single heat
 * problem in such a batch is one launch that overlaps the phases. */
typedef struct {
    int eq;          /* sw_equation                                          */
    int width;       /* triangle width, 0 = tuned width, else library choice */
    int64_t n_cells; /* >= 4; n_cells / width <= 2^31 - 1                     */
    int64_t n_steps; /* >= 0; at most 2^31 - 2 swept phases (K above)        */
    double dt, dx;   /* finite, > 0                                          */
    void *d_state;   /* device state buffer laid out as for swept_solve; the
                        problems' buffers must not overlap                   */
} sw_problem;

typedef struct {
    int blocks_per_cu;     /* resident workgroups per CU, 0 = occupancy limit */
    int threads;           /* workgroup size: 256 or 512, 0 = 256              */
    int64_t wait_limit_us; /* bound of one dependency wait, 0 = 10 s           */
} sw_batch_opts;

typedef struct sw_batch_impl *sw_batch;

/* Bytes of device workspace swept_solve_batch needs for this problem list
 * (host only; no HIP call): a 256-byte header (ticket and status word), the
 * problem table (one entry per problem), one 32-bit completion flag per tile
 * and every problem's two copies of its working arrays (sw_workspace_bytes
 * of the swept method).  A problem given with width 0 takes its tuned or
 * default width here exactly as in swept_solve_batch, so both calls must see
 * the same recorded widths.  0 for an invalid list (message in
 * sw_last_error). */
size_t sw_batch_workspace_bytes(int n_problems, const sw_problem *problems);

/* Advance every problem of the list by its n_steps in ONE persistent launch
 * (Sec. 4.1 applied to many grids at once) in a workspace the caller owns:
 * d_ws is device memory of the current device, 256-byte aligned, at least
 * sw_batch_workspace_bytes() long, not used by any other call in flight.
 * The call plans the batch on the host and enqueues on `stream` the upload
 * of the problem table (kernels carrying it in their launch arguments), a
 * reset kernel and the persistent kernel.  It allocates nothing, does not
 * wait for the device, and may be captured into a graph: each replay
 * recomputes the batch from the states as they are then.  The problems'
 * state buffers are read and written as by swept_solve; their contents after
 * the launch equal swept_solve of each problem with the same width.
 * SW_ERR_ARG for an invalid list, a NULL or misaligned d_ws, or ws_bytes
 * below what the list needs (all checked before any HIP call).  A dependency
 * wait that exceeds its bound (10 s) aborts the launch; sw_batch_check
 * reports it.  swept_solve_batch_ex takes the launch options of
 * sw_batch_opts (NULL = defaults: 256-thread workgroups, occupancy limit). */
int swept_solve_batch(int n_problems, const sw_problem *problems, void *d_ws, size_t ws_bytes,
                      sw_stream stream);
int swept_solve_batch_ex(int n_problems, const sw_problem *problems, const sw_batch_opts *opts,
                         void *d_ws, size_t ws_bytes, sw_stream stream);

/* Synchronise `stream` and report whether the last launch that used the
 * workspace d_ws completed (SW_ERR_HIP if a dependency wait exceeded its
 * bound).  Reads the status word of the workspace header. */
int sw_batch_check(const void *d_ws, sw_stream stream);

/* Validate the problems, allocate one workspace on the current device (as
 * laid out for swept_solve_batch), upload the table once and capture the
 * reset and persistent kernels into a graph.  Synchronous; must not be
 * called during stream capture.  opts may be NULL. */
int sw_batch_create(int n_problems, const sw_problem *problems, const sw_batch_opts *opts,
                    sw_batch *out);

/* Launch the batch graph on `stream` (asynchronous, allocates nothing). */
int sw_batch_run(sw_batch batch, sw_stream stream);

/* Synchronise `stream` and report whether the last run completed
 * (SW_ERR_HIP if a dependency wait exceeded its bound; SW_OK before any
 * run). */
int sw_batch_wait(sw_batch batch, sw_stream stream);

/* Work items, resident workgroups and working-array bytes of a batch. */
int sw_batch_info(sw_batch batch, int64_t *items, int *blocks, size_t *array_bytes);

/* Width chosen for problem i (0 for an invalid index). */
int sw_batch_width(sw_batch batch, int problem);

/* Synchronise the device and free everything the batch owns. */
void sw_batch_destroy(sw_batch batch);

/* Autotuner of the batched launch (the paper's advice to tune the block
 * width on a few steps before a long run, Sec. 6, applied to a batch).  The
 * batch is timed on scratch copies of the problem states (allocated, copied
 * and freed here; the caller's states are only read), every probe running
 * the same steps per problem: min(n_steps, probe_steps), or with
 * probe_steps = 0 enough steps for four phases at the widest power-of-two
 * width of the problem's equation.
 * For each workgroup size, 256 and 512 threads (only best->threads if it
 * is nonzero on input):
 *  1. widths, one equation at a time: every problem of that equation given
 *     with width 0 takes the largest valid width not above a cap, for caps
 *     64, 128, ... up to the widest tile (512, 1024, ... for 512 threads,
 *     starting from the widths chosen for 256); the fastest cap is kept;
 *  2. resident workgroups per CU: 1, 2, ... up to the occupancy limit.
 * The fastest combination wins.  On success its widths are written into
 * problems[i].width for every problem given with width 0, best->threads and
 * best->blocks_per_cu are set (0 = the occupancy limit was fastest;
 * wait_limit_us = 0) and *best_ms_per_update (may be NULL) gets the fastest
 * probe's time per cell-update.  Synchronous; not
 * allowed during stream capture (SW_ERR_CAPTURE); needs device memory for
 * one copy of every state plus one batch's working arrays (SW_ERR_NOMEM
 * otherwise).  Other errors as sw_batch_create. */
int sw_batch_autotune(int n_problems, sw_problem *problems, int64_t probe_steps,
                      sw_stream stream, sw_batch_opts *best, double *best_ms_per_update);

/* Previous-phase tiles that work item (phase, tile) of a batched problem
 * with `tiles` tiles waits for (host mirror of the device rule, no HIP call):
 * writes up to 3 tile indices to deps and returns their count. */
int sw_batch_item_deps(int phase, int tile, int tiles, int single_phase, int *deps);

/* ---- allocation-free solve -------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * swept_solve_noalloc is swept_solve (same arguments, same result bit for
 * bit, library-chosen width and workgroup size) with its working arrays in
 * a static array of SW_NOALLOC_SCRATCH_BYTES bytes that the library's code
 * object holds on each GPU until the process ends, instead of arrays the
 * library allocates: it calls no hipMalloc, hipFree or other allocating
 * routine.  The swept working arrays take 2 x 16 B per cell for heat
 * binary64 (so at most 2^21 cells), 2 x 12 B for heat binary32, 2 x 56 B /
 * 44 B for lengthened Euler and 2 x 48 B / 36 B for flattened Euler (each
 * copy rounded up to 256 B); a larger problem is refused with SW_ERR_ARG
 * before any HIP call.  Every call on one GPU shares that GPU's array and
 * leaves it holding the last call's arrays: calls whose execution overlaps
 * on the same GPU (several streams or host threads) race and corrupt each
 * other's results; order them on one stream.  The first call on a device
 * looks up the array's device address (hipGetSymbolAddress) and keeps it. */
#define SW_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int swept_solve_noalloc(int eq, int64_t n_cells, int64_t n_steps, double dt, double dx,
                        void *d_state, sw_stream stream);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next library call on the same thread. */
const char *sw_last_error(void);

/* Free the library's cached working arrays on every device (synchronises
 * each device that holds one). */
void sw_release(void);

#ifdef __cplusplus
}
#endif

#endif /* SWEPT_H */
