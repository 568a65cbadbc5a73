// host_share.cpp -- a swept solve shared between the GPU and host threads,
// the heterogeneous decomposition of Sec. 4.2 reduced to one GPU and the
// cores of its host.
//
// Tiles are split by the GPU work factor of Eq. 1: each of P host threads
// takes k consecutive tiles, k = floor(T / (WF + P)) for T tiles, and the GPU
// the first T - P k (at least WF times a thread's share).  In every phase the
// GPU launch covers its tiles of that phase's tiling and the host threads
// step theirs; a tile of either side is the same tile-phase (same level
// window, same two-slot working struct, same cell arithmetic -- the cell
// functions are compiled for host and device from one source), so the
// result equals swept_solve bit for bit.
//
// Ownership and exchange.  In phase k the GPU writes cells
// [o_k, G + o_k) and the host [G + o_k, n + o_k) (mod n), where o_k = 0 or W/2
// is the tiling's offset and G = W (T - P k).  Phase k + 1 reads, besides the
// cells its own side wrote, the W/2 + R cells next to the seam that the other
// side wrote (R halo cells; the paper's W/2 + 1 for a three-point stencil):
// after each phase those cells of every working array are copied between
// the device arrays and pinned host arrays (hipHostMalloc), the device-to-host
// copy waited for by an event before the host starts the next phase.  The
// first phase reads the caller's state: the host's cells are copied down
// once; the last phase's host cells are copied back into the state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/swept.h"
#include "geom.h"
#include "host.h"
#include "kernels.h"
#include "tile_euler.h"
#include "tile_heat.h"
#include "tile_job.h"
#include "tile_ks.h"

namespace sw {
namespace host {
namespace {

// ---- tile-phase bodies on the host ---------------------------------------------
// Each mirrors the GPU tile body of the same equation id: load the W + 2R
// cells of the tile into a local copy of the working struct, sweep the
// phase's levels in the same order with the same cell functions, write the
// W owned cells back.

template <typename T, bool KAHAN>
void host_heat_tile(const TileJob &jb, std::vector<T> &buf)
{
    const int w = jb.w;
    const int wp = w + 2;
    const int64_t n = jb.n;
    buf.resize(3 * (size_t)wp);
    T *s0 = buf.data();
    T *s1 = s0 + wp;
    T *cc = s1 + wp;
    T *state = (T *)jb.state;
    const T *ws_in = (const T *)jb.ws_in;
    T *ws_out = (T *)jb.ws_out;
    for (int i = 0; i < wp; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            s0[i] = state[g];
            if (KAHAN)
                cc[i] = state[n + g];
        } else {
            s0[i] = ws_in[g];
            s1[i] = ws_in[n + g];
            if (KAHAN)
                cc[i] = ws_in[2 * n + g];
        }
    }
    const T r = (T)jb.coef;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j);
        const int64_t m = jb.base + j;
        const T *src = (m & 1) ? s0 : s1;
        T *dst = (m & 1) ? s1 : s0;
        for (int i = a + 1; i <= w - a; ++i) {
            if constexpr (KAHAN)
                dst[i] = heat_update_kahan(src[i - 1], src[i], src[i + 1], r, cc[i]);
            else
                dst[i] = heat_update(src[i - 1], src[i], src[i + 1], r);
        }
    }
    const bool top_odd = ((jb.base + jb.j_last) & 1) != 0;
    for (int i = 1; i <= w; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            state[g] = top_odd ? s1[i] : s0[i];
            if (KAHAN)
                state[n + g] = cc[i];
        } else {
            ws_out[g] = s0[i];
            ws_out[n + g] = s1[i];
            if (KAHAN)
                ws_out[2 * n + g] = cc[i];
        }
    }
}

// Lengthened Euler, binary64: struct Q0[3], Q1[3], Pr, plus the pressure of
// the state the next ratio sub-step reads (as in the GPU body).
void host_euler_f64_tile(const TileJob &jb, std::vector<double> &buf)
{
    const int w = jb.w;
    const int wp = w + 2;
    const int64_t n = jb.n;
    buf.resize(11 * (size_t)wp);
    double *q0 = buf.data();
    double *q1 = q0 + 3 * wp;
    double *pr = q0 + 6 * wp;
    double *pp = q0 + 7 * wp;
    double *face = q0 + 8 * wp;  // [3][wp]: face between cells i - 1 and i
    double *state = (double *)jb.state;
    const double *ws_in = (const double *)jb.ws_in;
    double *ws_out = (double *)jb.ws_out;
    for (int i = 0; i < wp; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            for (int k = 0; k < 3; ++k)
                q0[k * wp + i] = state[k * n + g];
            pp[i] = pressure64(q0[i], q0[wp + i], q0[2 * wp + i]);
        } else {
            for (int k = 0; k < 7; ++k)
                q0[k * wp + i] = ws_in[k * n + g];
            const double *q = ((entry_level(jb, i, w) & 2) == 0) ? q0 : q1;
            pp[i] = pressure64(q[i], q[wp + i], q[2 * wp + i]);
        }
    }
    const double lam = jb.coef;
    const double half_lam = 0.5 * lam;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j);
        const int lo = a + 1, hi = w - a + 1;
        const int t = (int)((jb.base + j - 1) & 3);
        if ((t & 1) == 0) {
            for (int i = lo; i < hi; ++i)
                pr[i] = ratio(pp[i - 1], pp[i], pp[i + 1]);
            continue;
        }
        const double *q = (t == 1) ? q0 : q1;
        double *dst = (t == 1) ? q1 : q0;
        const double c = (t == 1) ? half_lam : lam;
        for (int i = lo; i <= hi; ++i)
            face64(q[i - 1], q[wp + i - 1], q[2 * wp + i - 1], q[i], q[wp + i], q[2 * wp + i],
                   pr[i - 1], pr[i], face[i], face[wp + i], face[2 * wp + i]);
        for (int i = lo; i < hi; ++i) {
            const double n0 = q0[i] + c * (face[i] - face[i + 1]);
            const double n1 = q0[wp + i] + c * (face[wp + i] - face[wp + i + 1]);
            const double n2 = q0[2 * wp + i] + c * (face[2 * wp + i] - face[2 * wp + i + 1]);
            dst[i] = n0;
            dst[wp + i] = n1;
            dst[2 * wp + i] = n2;
            pp[i] = pressure64(n0, n1, n2);
        }
    }
    for (int i = 1; i <= w; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            for (int k = 0; k < 3; ++k)
                state[k * n + g] = q0[k * wp + i];
        } else {
            for (int k = 0; k < 7; ++k)
                ws_out[k * n + g] = q0[k * wp + i];
        }
    }
}

// Lengthened Euler, binary32 + Kahan with binary64 islands.
void host_euler_f32_tile(const TileJob &jb, std::vector<double> &dbuf, std::vector<float> &fbuf)
{
    const int w = jb.w;
    const int wp = w + 2;
    const int64_t n = jb.n;
    dbuf.resize(2 * (size_t)wp);
    fbuf.resize(12 * (size_t)wp);
    double *pr = dbuf.data();
    double *pp = pr + wp;
    float *fst = fbuf.data();  // q0[3], c[3], q1[3], face[3]
    float *q0 = fst;
    float *cc = fst + 3 * wp;
    float *q1 = fst + 6 * wp;
    float *face = fst + 9 * wp;
    float *state = (float *)jb.state;
    const float *win = (const float *)jb.ws_in;
    const double *win_pr = (const double *)((const char *)jb.ws_in + 36 * n);
    float *wout = (float *)jb.ws_out;
    double *wout_pr = (double *)((char *)jb.ws_out + 36 * n);
    for (int i = 0; i < wp; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            for (int k = 0; k < 6; ++k)
                fst[k * wp + i] = state[k * n + g];
            pp[i] = pressure32(q0[i], q0[wp + i], q0[2 * wp + i]);
        } else {
            for (int k = 0; k < 9; ++k)
                fst[k * wp + i] = win[k * n + g];
            pr[i] = win_pr[g];
            const float *q = ((entry_level(jb, i, w) & 2) == 0) ? q0 : q1;
            pp[i] = pressure32(q[i], q[wp + i], q[2 * wp + i]);
        }
    }
    const float lam = (float)jb.coef;
    const float half_lam = 0.5f * lam;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j);
        const int lo = a + 1, hi = w - a + 1;
        const int t = (int)((jb.base + j - 1) & 3);
        if ((t & 1) == 0) {
            for (int i = lo; i < hi; ++i)
                pr[i] = ratio(pp[i - 1], pp[i], pp[i + 1]);
            continue;
        }
        const float *q = (t == 1) ? q0 : q1;
        for (int i = lo; i <= hi; ++i)
            face32(q[i - 1], q[wp + i - 1], q[2 * wp + i - 1], q[i], q[wp + i], q[2 * wp + i],
                   pr[i - 1], pr[i], face[i], face[wp + i], face[2 * wp + i]);
        for (int i = lo; i < hi; ++i) {
            float nq[3];
            if (t == 1) {
                for (int m = 0; m < 3; ++m) {
                    nq[m] = q0[m * wp + i] + half_lam * (face[m * wp + i] - face[m * wp + i + 1]);
                    q1[m * wp + i] = nq[m];
                }
            } else {
                for (int m = 0; m < 3; ++m) {
                    float comp = cc[m * wp + i];
                    nq[m] = kahan_add(q0[m * wp + i],
                                      lam * (face[m * wp + i] - face[m * wp + i + 1]), comp);
                    cc[m * wp + i] = comp;
                    q0[m * wp + i] = nq[m];
                }
            }
            pp[i] = pressure32(nq[0], nq[1], nq[2]);
        }
    }
    for (int i = 1; i <= w; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            for (int k = 0; k < 6; ++k)
                state[k * n + g] = fst[k * wp + i];
        } else {
            for (int k = 0; k < 9; ++k)
                wout[k * n + g] = fst[k * wp + i];
            wout_pr[g] = pr[i];
        }
    }
}

// Flattened Euler (two five-point sub-steps, struct Q0[3], Q1[3]).  Per
// sub-step: the pressure of every cell of [lo - 2, hi + 1], the ratio of
// [lo - 1, hi], the face between x - 1 and x for x in [lo, hi], the update of
// [lo, hi) -- the values the GPU body's lanes exchange.
template <typename T, bool KAHAN>
void host_flat_tile(const TileJob &jb, std::vector<double> &dbuf, std::vector<T> &fbuf)
{
    constexpr int R = 2;
    const int w = jb.w;
    const int wp = w + 2 * R;
    const int64_t n = jb.n;
    const int narr = KAHAN ? 9 : 6;  // q0[3], (c[3]), q1[3]
    dbuf.resize(2 * (size_t)wp);
    fbuf.resize((size_t)(narr + 3) * wp);
    double *p = dbuf.data();
    double *rt = p + wp;
    T *fst = fbuf.data();
    T *q0 = fst;
    T *cc = fst + 3 * wp;                  // KAHAN only
    T *q1 = fst + (KAHAN ? 6 : 3) * wp;
    T *face = fst + narr * wp;
    T *state = (T *)jb.state;
    const T *win = (const T *)jb.ws_in;
    T *wout = (T *)jb.ws_out;
    for (int i = 0; i < wp; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            for (int k = 0; k < (KAHAN ? 6 : 3); ++k)
                fst[k * wp + i] = state[k * n + g];
        } else {
            for (int k = 0; k < narr; ++k)
                fst[k * wp + i] = win[k * n + g];
        }
    }
    const T lam = (T)jb.coef;
    const T half_lam = (T)0.5 * lam;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j, R);
        const int lo = a + R, hi = w - a + R;
        const int t = (int)((jb.base + j - 1) & 1);
        const T *q = (t == 0) ? q0 : q1;
        for (int x = lo - 2; x <= hi + 1; ++x) {
            if constexpr (KAHAN)
                p[x] = pressure32(q[x], q[wp + x], q[2 * wp + x]);
            else
                p[x] = pressure64(q[x], q[wp + x], q[2 * wp + x]);
        }
        for (int x = lo - 1; x <= hi; ++x)
            rt[x] = ratio(p[x - 1], p[x], p[x + 1]);
        for (int x = lo; x <= hi; ++x) {
            if constexpr (KAHAN)
                face32(q[x - 1], q[wp + x - 1], q[2 * wp + x - 1], q[x], q[wp + x], q[2 * wp + x],
                       rt[x - 1], rt[x], face[x], face[wp + x], face[2 * wp + x]);
            else
                face64(q[x - 1], q[wp + x - 1], q[2 * wp + x - 1], q[x], q[wp + x], q[2 * wp + x],
                       rt[x - 1], rt[x], face[x], face[wp + x], face[2 * wp + x]);
        }
        for (int x = lo; x < hi; ++x) {
            for (int m = 0; m < 3; ++m) {
                const T d = face[m * wp + x] - face[m * wp + x + 1];
                if (t == 0) {
                    q1[m * wp + x] = q0[m * wp + x] + half_lam * d;
                } else if constexpr (KAHAN) {
                    float comp = cc[m * wp + x];
                    q0[m * wp + x] = kahan_add(q0[m * wp + x], lam * d, comp);
                    cc[m * wp + x] = comp;
                } else {
                    q0[m * wp + x] = q0[m * wp + x] + lam * d;
                }
            }
        }
    }
    for (int i = R; i < w + R; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            for (int k = 0; k < (KAHAN ? 6 : 3); ++k)
                state[k * n + g] = fst[k * wp + i];
        } else {
            for (int k = 0; k < narr; ++k)
                wout[k * n + g] = fst[k * wp + i];
        }
    }
}

// Kuramoto-Sivashinsky (radius 2, two level slots), coefficients a, b, c.
void host_ks_tile(const TileJob &jb, std::vector<double> &buf, const double abc[3])
{
    constexpr int R = kKsRadius;
    const int w = jb.w;
    const int wp = w + 2 * R;
    const int64_t n = jb.n;
    buf.resize(2 * (size_t)wp);
    double *s0 = buf.data();
    double *s1 = s0 + wp;
    double *state = (double *)jb.state;
    const double *ws_in = (const double *)jb.ws_in;
    double *ws_out = (double *)jb.ws_out;
    for (int i = 0; i < wp; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            s0[i] = state[g];
        } else {
            s0[i] = ws_in[g];
            s1[i] = ws_in[n + g];
        }
    }
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int m = window_margin(j, R);
        const int64_t lv = jb.base + j;
        const double *src = (lv & 1) ? s0 : s1;
        double *dst = (lv & 1) ? s1 : s0;
        for (int i = m + R; i < w - m + R; ++i)
            dst[i] = ks_update(src[i - 2], src[i - 1], src[i], src[i + 1], src[i + 2], abc[0],
                               abc[1], abc[2]);
    }
    const bool top_odd = ((jb.base + jb.j_last) & 1) != 0;
    for (int i = R; i < w + R; ++i) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            state[g] = top_odd ? s1[i] : s0[i];
        } else {
            ws_out[g] = s0[i];
            ws_out[n + g] = s1[i];
        }
    }
}

struct HostScratch {
    std::vector<double> d, d2;
    std::vector<float> f;
};

void host_tile(int eq, const TileJob &jb, HostScratch &sc, const double ks_abc[3])
{
    switch (eq) {
    case SW_KS_F64: host_ks_tile(jb, sc.d, ks_abc); break;
    case SW_HEAT_F64: host_heat_tile<double, false>(jb, sc.d); break;
    case SW_HEAT_F32: host_heat_tile<float, true>(jb, sc.f); break;
    case SW_EULER_F64: host_euler_f64_tile(jb, sc.d); break;
    case SW_EULER_F32: host_euler_f32_tile(jb, sc.d, sc.f); break;
    case SW_EULER_F64_FLAT: host_flat_tile<double, false>(jb, sc.d, sc.d2); break;
    default: host_flat_tile<float, true>(jb, sc.d, sc.f); break;
    }
}

// ---- array layouts (byte offset per cell count, element size) -------------------

struct Arr {
    size_t per_cell_offset;  // array starts at per_cell_offset * n bytes
    size_t elem;
};

std::vector<Arr> state_arrays(int eq)
{
    switch (eq) {
    case SW_HEAT_F64:
    case SW_KS_F64: return {{0, 8}};
    case SW_HEAT_F32: return {{0, 4}, {4, 4}};
    case SW_EULER_F64:
    case SW_EULER_F64_FLAT: return {{0, 8}, {8, 8}, {16, 8}};
    default: return {{0, 4}, {4, 4}, {8, 4}, {12, 4}, {16, 4}, {20, 4}};
    }
}

std::vector<Arr> work_arrays(int eq)
{
    std::vector<Arr> a;
    switch (eq) {
    case SW_HEAT_F64:
    case SW_KS_F64: return {{0, 8}, {8, 8}};
    case SW_HEAT_F32: return {{0, 4}, {4, 4}, {8, 4}};
    case SW_EULER_F64:
        for (int k = 0; k < 7; ++k)
            a.push_back({(size_t)8 * k, 8});
        return a;
    case SW_EULER_F32:
        for (int k = 0; k < 9; ++k)
            a.push_back({(size_t)4 * k, 4});
        a.push_back({36, 8});
        return a;
    case SW_EULER_F64_FLAT:
        for (int k = 0; k < 6; ++k)
            a.push_back({(size_t)8 * k, 8});
        return a;
    default:
        for (int k = 0; k < 9; ++k)
            a.push_back({(size_t)4 * k, 4});
        return a;
    }
}

// a cyclic interval of cells: start (any integer, taken mod n) and length
struct Cyc {
    int64_t start, len;
};

// [lo, hi) pieces of a cyclic interval within [0, n)
int pieces(Cyc c, int64_t n, int64_t out[2][2])
{
    int64_t s = ((c.start % n) + n) % n;
    const int64_t len = c.len < n ? c.len : n;
    if (len <= 0)
        return 0;
    if (s + len <= n) {
        out[0][0] = s;
        out[0][1] = s + len;
        return 1;
    }
    out[0][0] = s;
    out[0][1] = n;
    out[1][0] = 0;
    out[1][1] = s + len - n;
    return 2;
}

// linear [lo, hi) ranges of the intersection of two cyclic intervals
std::vector<std::pair<int64_t, int64_t>> intersect(Cyc a, Cyc b, int64_t n)
{
    int64_t pa[2][2], pb[2][2];
    const int na = pieces(a, n, pa), nb = pieces(b, n, pb);
    std::vector<std::pair<int64_t, int64_t>> r;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
            const int64_t lo = std::max(pa[i][0], pb[j][0]);
            const int64_t hi = std::min(pa[i][1], pb[j][1]);
            if (lo < hi)
                r.push_back({lo, hi});
        }
    return r;
}

hipError_t copy_cells(const std::vector<std::pair<int64_t, int64_t>> &ranges,
                      const std::vector<Arr> &arrays, int64_t n, char *dst, const char *src,
                      hipMemcpyKind kind, hipStream_t s)
{
    for (const auto &r : ranges)
        for (const Arr &a : arrays) {
            const size_t off = a.per_cell_offset * (size_t)n + (size_t)r.first * a.elem;
            const hipError_t e = hipMemcpyAsync(dst + off, src + off,
                                                (size_t)(r.second - r.first) * a.elem, kind, s);
            if (e != hipSuccess)
                return e;
        }
    return hipSuccess;
}

// pinned host copies of the state and of the two working-array copies,
// kept for later calls and freed by sw_release
std::mutex g_host_mutex;
void *g_host_ptr = nullptr;
size_t g_host_bytes = 0;

} // namespace

void release_host_arrays()
{
    std::lock_guard<std::mutex> lock(g_host_mutex);
    if (g_host_ptr)
        (void)hipHostFree(g_host_ptr);
    g_host_ptr = nullptr;
    g_host_bytes = 0;
    (void)hipGetLastError();
}

int run_swept_shared(int eq, int64_t n, int64_t steps, double dt, double dx, void *state,
                     hipStream_t s, int w, int threads, void *ws, int work_factor,
                     int host_threads)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "hipStreamIsCapturing failed");
    }
    if (cs != hipStreamCaptureStatusNone)
        return fail(SW_ERR_CAPTURE, "a solve shared with host threads cannot be captured");
    const int P = host_threads > 0 ? host_threads : kDefaultHostThreads;
    const int64_t T = n / w;
    const int64_t kt = T / ((int64_t)work_factor + P);
    if (kt < 1)
        return fail(SW_ERR_ARG, "work_factor %d leaves no tile for the host", work_factor);
    const int64_t gt = T - (int64_t)P * kt;  // GPU tiles: [0, gt) of every phase's tiling
    const int64_t G = gt * w;
    const int R = radius(eq);
    const int64_t final_level = steps * substeps(eq);
    const int64_t half = w / (2 * R);
    const int64_t phases = sw::phase_count(final_level, half);
    const size_t copy = swept_copy_bytes(eq, n);
    const size_t sbytes = round_up(state_bytes(eq, n), 256);

    std::lock_guard<std::mutex> lock(g_host_mutex);
    const size_t need = sbytes + 2 * copy;
    if (g_host_bytes < need) {
        if (g_host_ptr) {
            if (hipStreamSynchronize(s) != hipSuccess || hipHostFree(g_host_ptr) != hipSuccess) {
                (void)hipGetLastError();
                return fail(SW_ERR_HIP, "releasing the pinned host arrays failed");
            }
            g_host_ptr = nullptr;
            g_host_bytes = 0;
        }
        if (hipHostMalloc(&g_host_ptr, need, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            g_host_ptr = nullptr;
            return fail(SW_ERR_NOMEM, "hipHostMalloc of %zu bytes of host arrays failed", need);
        }
        g_host_bytes = need;
    }
    char *h_state = (char *)g_host_ptr;
    char *h_a = h_state + sbytes;
    char *h_b = h_a + copy;
    char *d_a = (char *)ws;
    char *d_b = d_a + copy;
    const std::vector<Arr> st_arr = state_arrays(eq), ws_arr = work_arrays(eq);
    std::vector<HostScratch> scratch(P);
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_ERR_HIP, "hipEventCreate failed");
    }
    int rc = SW_OK;
    hipError_t e = hipSuccess;
    // the host's tiles of phase 1 read the state cells [G - R, n + R)
    e = copy_cells(intersect({G - R, n - G + 2 * R}, {0, n}, n), st_arr, n, h_state,
                   (const char *)state, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    const double coef = is_euler(eq) ? dt / dx : dt / (dx * dx);
    double ks_abc[3];
    ks_coefficients(dt, dx, &ks_abc[0], &ks_abc[1], &ks_abc[2]);
    const double coef_t = is_f32(eq) ? (double)(float)coef : coef;
    for (int64_t k = 1; k <= phases && e == hipSuccess; ++k) {
        const sw::PhaseRange pr = sw::phase_range(k, final_level, half, R);
        const bool first = (k == 1), last = (k == phases);
        sw::PhaseLaunch p;
        p.n = n;
        p.w = w;
        p.offset = pr.offset;
        p.tiles = gt;
        p.base = pr.base;
        p.j_first = pr.j_first;
        p.j_last = pr.j_last;
        p.threads = threads;
        p.first = first;
        p.last = last;
        char *d_in = (k % 2 == 0) ? d_a : d_b, *d_out = (k % 2 == 1) ? d_a : d_b;
        char *h_in = (k % 2 == 0) ? h_a : h_b, *h_out = (k % 2 == 1) ? h_a : h_b;
        e = swept_phase_launch(eq, p, state, d_in, d_out, dt, dx, s);
        if (e != hipSuccess)
            break;
        // the host tiles of this phase, kt consecutive tiles per thread; a
        // thread that cannot be started has its tiles run on this one, and
        // no exception leaves a worker
        std::atomic<bool> worker_failed{false};
        auto work = [&](int th) {
            try {
                for (int64_t t = gt + (int64_t)th * kt; t < gt + (int64_t)(th + 1) * kt; ++t) {
                    TileJob jb;
                    jb.state = h_state;
                    jb.ws_in = h_in;
                    jb.ws_out = h_out;
                    jb.n = n;
                    jb.g0 = pr.offset + t * w - R;
                    jb.base = pr.base;
                    jb.coef = coef_t;
                    jb.w = w;
                    jb.j_first = pr.j_first;
                    jb.j_last = pr.j_last;
                    jb.first = first;
                    jb.last = last;
                    jb.final_level = pr.base + pr.j_last;
                    host_tile(eq, jb, scratch[th], ks_abc);
                }
            } catch (...) {
                worker_failed = true;
            }
        };
        std::vector<std::thread> pool;
        int started = 0;
        try {
            pool.reserve(P);
            for (; started < P; ++started)
                pool.emplace_back(work, started);
        } catch (...) {
        }
        for (int th = started; th < P; ++th)
            work(th);
        for (auto &t : pool)
            t.join();
        if (worker_failed) {
            (void)hipStreamSynchronize(s);
            (void)hipGetLastError();
            (void)hipEventDestroy(ev);
            return fail(SW_ERR_NOMEM, "host memory exhausted in a host tile");
        }
        const Cyc gpu_wrote = {pr.offset, G}, host_wrote = {G + pr.offset, n - G};
        if (last) {
            e = copy_cells(intersect(host_wrote, {0, n}, n), st_arr, n, (char *)state, h_state,
                           hipMemcpyHostToDevice, s);
            break;
        }
        // what each side reads in phase k + 1 that the other side wrote in phase k
        const int64_t o_next = sw::phase_range(k + 1, final_level, half, R).offset;
        const Cyc gpu_reads = {o_next - R, G + 2 * R}, host_reads = {G + o_next - R, n - G + 2 * R};
        e = copy_cells(intersect(host_reads, gpu_wrote, n), ws_arr, n, h_out, d_out,
                       hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = copy_cells(intersect(gpu_reads, host_wrote, n), ws_arr, n, d_out, h_out,
                           hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipEventRecord(ev, s);
        if (e == hipSuccess)
            e = hipEventSynchronize(ev);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(SW_ERR_HIP, "shared swept solve: %s", hipGetErrorString(e));
    }
    (void)hipEventDestroy(ev);
    return rc;
}

} // namespace host
} // namespace sw
