// C-ABI entry points: argument validation on the host, derived geometry,
// workspace layout and the step loop that sequences the kernels.

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <utility>

#include "md_internal.h"

namespace md {

static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

static int hip_fail(hipError_t e, const char* where)
{
    return fail(MD_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define MD_HIP(expr, where)                        \
    do {                                           \
        hipError_t e__ = (expr);                   \
        if (e__ != hipSuccess) return hip_fail(e__, where); \
    } while (0)

static int check_params(const md_params* p, int32_t nc[3])
{
    if (!p) return fail(MD_ERR_ARG, "params is NULL");
    if (p->n <= 0 || p->n >= MD_MAX_N) return fail(MD_ERR_ARG, "n = %lld outside [1, 2^27)", (long long)p->n);
    for (int k = 0; k < 3; ++k)
        if (!(p->box[k] > 0.0) || !std::isfinite(p->box[k])) return fail(MD_ERR_ARG, "box[%d] must be > 0", k);
    if (!(p->eps > 0.0) || !(p->sigma > 0.0)) return fail(MD_ERR_ARG, "eps and sigma must be > 0");
    if (!(p->rc > 0.0) || !(p->rs >= p->rc)) return fail(MD_ERR_ARG, "need 0 < rc <= rs");
    if (p->precision != MD_FP64 && p->precision != MD_MIXED) return fail(MD_ERR_ARG, "precision must be 0 or 1");
    if (p->resort_every < 0) return fail(MD_ERR_ARG, "resort_every must be >= 0");
    if (p->rebuild_rule != MD_REBUILD_HALF_SKIN && p->rebuild_rule != MD_REBUILD_DUTC_LDC)
        return fail(MD_ERR_ARG, "rebuild_rule must be 0 or 1");
    if (p->ldc_max < 0 || p->ldc_max > (1 << 22)) return fail(MD_ERR_ARG, "ldc_max must be in [0, 2^22]");
    if (p->list_layout != MD_LIST_AUTO && p->list_layout != MD_LIST_SLOTS && p->list_layout != MD_LIST_HALF)
        return fail(MD_ERR_ARG, "list_layout must be 0, 1 or 2");
    if (p->tile_cells < 0 || p->tile_cells > 1023) return fail(MD_ERR_ARG, "tile_cells must be in [0, 1023]");
    if (p->step_run < 0 || p->step_run > MD_STEP_RUN_MAX)
        return fail(MD_ERR_ARG, "step_run must be in [0, %d]", MD_STEP_RUN_MAX);
    if (p->build_waves < MD_BUILD_AUTO || p->build_waves > MD_BUILD_TILE_WAVES)
        return fail(MD_ERR_ARG, "build_waves must be 0, 1 or 2");
    for (int k = 0; k < 3; ++k) {
        const double m = std::floor(p->box[k] / p->rs);
        if (m < 3.0) return fail(MD_ERR_BOX, "axis %d has %.0f cells (< 3): box too small for rs", k, m);
        if (m > 1023.0) return fail(MD_ERR_BOX, "axis %d has %.0f cells (> 1023)", k, m);
        nc[k] = (int32_t)m;
    }
    if ((int64_t)nc[0] * nc[1] * nc[2] >= ((int64_t)1 << 31)) return fail(MD_ERR_BOX, "too many cells");
    return MD_OK;
}

Geo make_geo(const md_params& p, const int32_t nc[3])
{
    Geo g;
    g.n = p.n;
    g.ncell = (int64_t)nc[0] * nc[1] * nc[2];
    g.exact_all = 0;
    for (int k = 0; k < 3; ++k) {
        g.nc[k] = nc[k];
        g.L[k] = p.box[k];
        g.invL[k] = 1.0 / p.box[k];
        g.inv[k] = (double)nc[k] / p.box[k];
        g.cs[k] = p.box[k] / (double)nc[k];
        if (nc[k] < 5) g.exact_all = 1;
    }
    g.force_minimg_all = g.exact_all || p.rebuild_rule == MD_REBUILD_DUTC_LDC;
    // tiles: about kTileKeys keys each at the mean density, at most nz - 2
    // cells long so that a tile's runs wrap at most once
    const int nz = nc[2];
    int tc = p.tile_cells;
    if (tc == 0) {
        const double mean = (double)p.n / (double)g.ncell;
        const int keys = p.precision == MD_MIXED ? kTileKeys : kTileKeys64;
        tc = (int)std::lround((double)keys / (mean > 1e-9 ? mean : 1e-9));
    }
    tc = std::max(1, std::min(tc, nz - 2));
    const bool tiles = p.list_layout == MD_LIST_AUTO;
    g.tc = tiles ? tc : 0;
    g.nt = tiles ? (int32_t)ceil_div(nz, tc) : 0;
    g.ntile = tiles ? (int64_t)nc[0] * nc[1] * g.nt : 0;
    return g;
}

LJ make_lj(const md_params& p)
{
    LJ lj;
    const double e = p.eps, s = p.sigma, rc = p.rc;
    const double x = s / rc;
    const double x2 = x * x, x6 = x2 * x2 * x2, x8 = x6 * x2, x12 = x6 * x6, x14 = x12 * x2;
    const double c2 = 6.0 * x14 - 3.0 * x8;   // V'(rc) = 0
    const double c0 = -7.0 * x12 + 4.0 * x6;  // V(rc) = 0
    const double s2 = s * s, s6 = s2 * s2 * s2, s12 = s6 * s6;
    lj.rc2 = rc * rc;
    lj.A = 48.0 * e * s12;
    lj.B = 24.0 * e * s6;
    lj.C8 = 8.0 * e * c2 / s2;
    lj.A4 = 4.0 * e * s12;
    lj.B4 = 4.0 * e * s6;
    lj.C2 = 4.0 * e * c2 / s2;
    lj.C0 = 4.0 * e * c0;
    lj.eps = e;
    lj.sigma = s;
    const double rc2 = rc * rc, rc6 = rc2 * rc2 * rc2, rc8 = rc6 * rc2, rc12 = rc6 * rc6, rc14 = rc12 * rc2;
    lj.rc6i = 1.0 / rc6;
    lj.rc8i = 1.0 / rc8;
    lj.rc12i = 1.0 / rc12;
    lj.rc14i = 1.0 / rc14;
    // C8 = 48 eps s^12 rc^-14 - 24 eps s^6 rc^-8, so sigma dC8/dsigma:
    lj.Cs = 12.0 * 48.0 * e * s12 / rc14 - 6.0 * 24.0 * e * s6 / rc8;
    return lj;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Small device scalars in the workspace (int64 words):
//   [0], [1]  cell-grid error flags         [2]  md_forces non-finite flag
//   [4]       large-displacement members    [5]  large-displacement violation
//   [6]       largest squared displacement (md_ldc_check)
//   [8]       gate of a run of queued steps (int32; md_step)
//   [16..31]  flags gathered for one read-back (layout in k_gather_flags)
constexpr int kScalOut = 16;

WsLayout ws_layout(const Geo& g, int64_t ldc_max, int precision)
{
    const int64_t n = g.n, ncell = g.ncell;
    WsLayout L;
    L.nbs = ceil_div(ncell, kScanItems);
    L.nbf = ceil_div(n, kKeysPerBlock);
    const int64_t np = std::max(pair_blocks(g), g.ntile);
    L.nbi = ceil_div(n, kStreamBlock);
    size_t off = 0;
    L.rank = off;      off = align256(off + sizeof(int32_t) * (size_t)n);
    L.bsum = off;      off = align256(off + sizeof(int32_t) * (size_t)(L.nbs + 1));
    L.cell_rows = off; off = align256(off + sizeof(int32_t) * (size_t)ncell);
    // (PE, W) partials of the adjoint kernels (nbf blocks) or of a force pass
    // (one per block or tile)
    L.part_a = off;    off = align256(off + sizeof(double) * 2 * (size_t)std::max(L.nbf, np));
    L.part_b = off;    off = align256(off + sizeof(double) * (size_t)(np > L.nbi ? np : L.nbi));
    // local coordinates of md_forces in mixed precision only
    L.pos32 = off;     off = align256(off + (precision == MD_MIXED ? 16 * (size_t)n : 0));
    L.red = off;       off = align256(off + sizeof(int64_t) * 2 * 1024);
    L.ldc = off;       off = align256(off + sizeof(int32_t) * (size_t)(ldc_max > 0 ? ldc_max : 1));
    L.scal = off;      off = align256(off + sizeof(int64_t) * 32);
    L.tmax = off;      off = align256(off + sizeof(int64_t) * kTileMaxSlots);
    L.mx = off;        off = align256(off + sizeof(int64_t) * 2 * kMaxSlots * kMaxSlotStride);
    L.tile_used = off; off = align256(off + sizeof(int32_t) * (size_t)(g.ntile > 0 ? g.ntile : 1));
    L.total = off;
    return L;
}

struct Ctx {
    int32_t nc[3];
    Geo g;
    LJ lj;
    WsLayout W;
};

static int setup(const md_params* p, Ctx& c)
{
    int rc = check_params(p, c.nc);
    if (rc != MD_OK) return rc;
    c.g = make_geo(*p, c.nc);
    c.lj = make_lj(*p);
    c.W = ws_layout(c.g, p->ldc_max, p->precision);
    return MD_OK;
}

static int check_ws(const Ctx& c, const void* ws, size_t ws_bytes)
{
    if (!ws) return fail(MD_ERR_ARG, "workspace is NULL");
    if (ws_bytes < c.W.total)
        return fail(MD_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, c.W.total);
    return MD_OK;
}

static int check_cells(const Ctx& c, const md_cells* cells)
{
    if (!cells || !cells->cell_of || !cells->cell_xyz || !cells->count || !cells->start || !cells->order)
        return fail(MD_ERR_ARG, "cells has a NULL array");
    return MD_OK;
}

// 32-bit words of nbr that a list of cell_stride entries per cell takes:
// 32-bit slot entries, or the 16-bit entries of a state's tiled layout.
static int64_t list_words(const Ctx& c, const md_pairlist* list, bool tiled)
{
    const int64_t entries = c.g.ncell * list->cell_stride;
    return tiled ? (entries + 1) / 2 : entries;
}

// slot_entries: the call reads or writes 32-bit slot entries, so nbr must
// hold them all; a state's list only needs the room of its tiled layout here
// (build_list checks the layout it is about to write).
static int check_list(const Ctx& c, const md_pairlist* list, bool slot_entries = true)
{
    if (!list || !list->offsets || !list->counts || !list->nbr || !list->status)
        return fail(MD_ERR_ARG, "pair list has a NULL array");
    if (list->cell_stride <= 0 || list->cell_stride > ((int64_t)1 << 29))
        return fail(MD_ERR_ARG, "cell_stride must be in [1, 2^29]");
    const int64_t need = list_words(c, list, !slot_entries);
    if (list->capacity < need)
        return fail(MD_ERR_ARG, "capacity %lld < %lld words (ncell * cell_stride = %lld entries of %d bits)",
                    (long long)list->capacity, (long long)need, (long long)(c.g.ncell * list->cell_stride),
                    slot_entries ? 32 : 16);
    return MD_OK;
}

// The standalone force, Hessian and adjoint passes decode slot entries; a
// state's tiled list holds offsets into staged tiles instead.  Only the force
// pass also takes a half list (each pair once).
static int check_slot_list(const Ctx& c, const md_pairlist* list, bool allow_half)
{
    int rc = check_list(c, list);
    if (rc != MD_OK) return rc;
    if (list->tiled)
        return fail(MD_ERR_ARG, "pair list holds the tiled layout of a state; build one with md_build_pairlist");
    if (list->half && !allow_half)
        return fail(MD_ERR_ARG, "this pass needs a full list (each pair in both rows), not a half list");
    return MD_OK;
}

// ---------------------------------------------------------------------------
// timers
// ---------------------------------------------------------------------------
// Up to kTimerSlots launches of each kernel class are timed between two host
// waits (md_step waits at least once per run of steps, and a run is at most
// kTimerSlots steps long, so every launch is covered).
constexpr int kTimerSlots = 64;

struct Timer {
    md_timers* t;
    bool ok;
    int n[MD_T_COUNT];
};

static hipEvent_t g_ev[MD_T_COUNT][kTimerSlots][2];
static bool g_ev_made = false;

static void timer_begin(Timer& T, md_timers* t)
{
    T.t = t;
    T.ok = t != nullptr;
    for (int k = 0; k < MD_T_COUNT; ++k) T.n[k] = 0;
    if (!T.ok || g_ev_made) return;
    for (int a = 0; a < MD_T_COUNT; ++a)
        for (int b = 0; b < kTimerSlots; ++b)
            for (int e = 0; e < 2; ++e)
                if (hipEventCreate(&g_ev[a][b][e]) != hipSuccess) {
                    T.ok = false;
                    return;
                }
    g_ev_made = true;
}

static void tick(Timer& T, int cls, int which, hipStream_t s)
{
    if (!T.ok) return;
    const int k = T.n[cls];
    if (k >= kTimerSlots) return;
    (void)hipEventRecord(g_ev[cls][k][which], s);
    if (which == 1) T.n[cls] = k + 1;
}

// drop all but the first keep timed launches of a class (launches that a
// gate turned into no-ops)
static void timer_keep(Timer& T, int cls, int64_t keep)
{
    if (T.ok && keep < T.n[cls]) T.n[cls] = (int)keep;
}

// call after the stream has been synchronised
static void timer_collect(Timer& T)
{
    if (!T.ok) return;
    for (int c = 0; c < MD_T_COUNT; ++c) {
        for (int k = 0; k < T.n[c]; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, g_ev[c][k][0], g_ev[c][k][1]) == hipSuccess) {
                T.t->ms[c] += ms;
                T.t->launches[c] += 1;
            }
        }
        T.n[c] = 0;
    }
}

}  // namespace md

using namespace md;

extern "C" {

const char* md_last_error(void) { return g_err; }

int md_cell_dims(const md_params* p, int32_t ncell[3])
{
    if (!ncell) return fail(MD_ERR_ARG, "ncell is NULL");
    int32_t nc[3];
    int rc = check_params(p, nc);
    if (rc != MD_OK) return rc;
    for (int k = 0; k < 3; ++k) ncell[k] = nc[k];
    return MD_OK;
}

size_t md_workspace_bytes(const md_params* p)
{
    int32_t nc[3];
    if (check_params(p, nc) != MD_OK) return 0;
    return ws_layout(make_geo(*p, nc), p->ldc_max, p->precision).total;
}

int md_pack_positions(const md_params* p, const double* q, double* pos, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!q || !pos) return fail(MD_ERR_ARG, "q or pos is NULL");
    if ((const void*)q == (const void*)pos) return fail(MD_ERR_ARG, "q and pos must not alias");
    MD_HIP(launch_pack(c.g, q, pos, stream), "md_pack_positions");
    return MD_OK;
}

int md_bin_cells(const md_params* p, const double* pos, md_cells* cells, void* ws, size_t ws_bytes,
                 hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!pos) return fail(MD_ERR_ARG, "pos is NULL");
    if ((rc = check_cells(c, cells)) != MD_OK) return rc;
    if ((rc = check_ws(c, ws, ws_bytes)) != MD_OK) return rc;
    for (int k = 0; k < 3; ++k) cells->ncell[k] = c.nc[k];
    int64_t* err = (int64_t*)((char*)ws + c.W.scal);
    MD_HIP(launch_fill_i32((int32_t*)err, 0, 2, stream), "md_bin_cells/clear");
    MD_HIP(launch_bin(c.g, pos, *cells, ws, c.W, err, stream), "md_bin_cells");
    cells->sorted = 0;
    return MD_OK;
}

int md_build_pairlist(const md_params* p, const double* pos, const md_cells* cells, md_pairlist* list,
                      void* ws, size_t ws_bytes, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!pos) return fail(MD_ERR_ARG, "pos is NULL");
    if ((rc = check_cells(c, cells)) != MD_OK) return rc;
    if ((rc = check_list(c, list)) != MD_OK) return rc;
    if ((rc = check_ws(c, ws, ws_bytes)) != MD_OK) return rc;
    const bool half = p->list_layout == MD_LIST_HALF;
    MD_HIP(launch_build(c.g, p->rs, pos, *cells, *list, ws, c.W, false, half, nullptr, MD_BUILD_AUTO, stream),
           "md_build_pairlist");
    list->tiled = 0;
    list->half = half ? 1 : 0;
    return MD_OK;
}

// The force pass of md_forces and md_forces_noalloc, with its scratch given:
// pos32 (mixed precision: float4 per particle), part (2 doubles per block of
// the pass) and one flag word (cleared here).
static int forces_with(const Ctx& c, const md_params* p, const double* pos, const md_cells* cells,
                       const md_pairlist* list, void* force, double* pe_w, float* pos32, double* part,
                       int64_t* flags, hipStream_t stream)
{
    MD_HIP(launch_fill_i32((int32_t*)flags, 0, 2, stream), "md_forces/flags");
    if (p->precision == MD_MIXED)
        MD_HIP(launch_ref_copy(c.g, pos, cells->cell_xyz, nullptr, pos32, stream), "md_forces/pos32");
    else
        pos32 = nullptr;
    ForceOut out;
    out.force = force;
    out.part = pe_w ? part : nullptr;
    out.flags = flags;
    MD_HIP(launch_forces(c.g, c.lj, p->precision, pos, pos32, cells->cell_xyz, *list, out, stream),
           "md_forces");
    if (pe_w)
        MD_HIP(launch_reduce_pair(out.part, force_blocks(c.g, false), 1.0, 1.0, pe_w, stream), "md_forces/reduce");
    return MD_OK;
}

int md_forces(const md_params* p, const double* pos, const md_cells* cells, const md_pairlist* list,
              void* force, double* pe_w, void* ws, size_t ws_bytes, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!pos || !force) return fail(MD_ERR_ARG, "pos or force is NULL");
    if ((rc = check_cells(c, cells)) != MD_OK) return rc;
    if ((rc = check_slot_list(c, list, true)) != MD_OK) return rc;
    if ((rc = check_ws(c, ws, ws_bytes)) != MD_OK) return rc;
    char* w = (char*)ws;
    return forces_with(c, p, pos, cells, list, force, pe_w, (float*)(w + c.W.pos32), (double*)(w + c.W.part_a),
                       (int64_t*)(w + c.W.scal) + 2, stream);
}

// ---------------------------------------------------------------------------
// md_forces_noalloc: the scratch of md_forces in a file-scope device array.
// Layout: local coordinates (16 bytes per particle, mixed precision), then
// the per-block (PE, W) partials, then the flag words.  Host code reaches the
// array only through the address hipGetSymbolAddress gives on each device.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxN = MD_NOALLOC_MAX_N;
constexpr size_t kNoAllocPos32 = 16 * (size_t)kNoAllocMaxN;
constexpr size_t kNoAllocPart = sizeof(double) * 2 * (size_t)((kNoAllocMaxN + kForceBlock - 1) / kForceBlock);
constexpr size_t kNoAllocFlags = 256;
constexpr size_t kNoAllocBytes = kNoAllocPos32 + kNoAllocPart + kNoAllocFlags;
static_assert(kNoAllocPos32 % 256 == 0 && kNoAllocPart % 256 == 0, "scratch regions stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocDevices] = {};

// Device address of the current device's copy of scratch, looked up once per
// device (with that device current) and kept.
static int scratch_address(void** out)
{
    int dev = -1;
    MD_HIP(hipGetDevice(&dev), "md_forces_noalloc/device");
    if (dev < 0 || dev >= kNoAllocDevices) return fail(MD_ERR_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        MD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "md_forces_noalloc/scratch address");
        if (!ptr) return fail(MD_ERR_HIP, "md_forces_noalloc: no address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MD_OK;
}

int md_forces_noalloc(const md_params* p, const double* pos, const md_cells* cells, const md_pairlist* list,
                      void* force, double* pe_w, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!pos || !force) return fail(MD_ERR_ARG, "pos or force is NULL");
    if (p->n > kNoAllocMaxN)
        return fail(MD_ERR_ARG, "md_forces_noalloc takes at most %lld particles (n = %lld); use md_forces",
                    (long long)kNoAllocMaxN, (long long)p->n);
    if ((rc = check_cells(c, cells)) != MD_OK) return rc;
    if ((rc = check_slot_list(c, list, true)) != MD_OK) return rc;
    void* base = nullptr;
    if ((rc = scratch_address(&base)) != MD_OK) return rc;
    char* w = (char*)base;
    return forces_with(c, p, pos, cells, list, force, pe_w, (float*)w, (double*)(w + kNoAllocPos32),
                       (int64_t*)(w + kNoAllocPos32 + kNoAllocPart), stream);
}

int md_hvp(const md_params* p, const double* pos, const md_cells* cells, const md_pairlist* list,
           const double* u, double* Hu, double* dparam, void* ws, size_t ws_bytes, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!pos || !u || !Hu) return fail(MD_ERR_ARG, "pos, u or Hu is NULL");
    if ((rc = check_cells(c, cells)) != MD_OK) return rc;
    if ((rc = check_slot_list(c, list, false)) != MD_OK) return rc;
    if ((rc = check_ws(c, ws, ws_bytes)) != MD_OK) return rc;
    double* part = dparam ? (double*)((char*)ws + c.W.part_a) : nullptr;
    MD_HIP(launch_hvp(c.g, c.lj, pos, cells->cell_xyz, *list, u, Hu, part, stream), "md_hvp");
    if (dparam) MD_HIP(launch_reduce_pair(part, c.W.nbf, 1.0, 1.0, dparam, stream), "md_hvp/reduce");
    return MD_OK;
}

int md_param_grad(const md_params* p, const double* pos, const md_cells* cells, const md_pairlist* list,
                  double* dU, void* ws, size_t ws_bytes, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!pos || !dU) return fail(MD_ERR_ARG, "pos or dU is NULL");
    if ((rc = check_cells(c, cells)) != MD_OK) return rc;
    if ((rc = check_slot_list(c, list, false)) != MD_OK) return rc;
    if ((rc = check_ws(c, ws, ws_bytes)) != MD_OK) return rc;
    double* part = (double*)((char*)ws + c.W.part_a);
    MD_HIP(launch_param_grad(c.g, c.lj, pos, cells->cell_xyz, *list, part, stream), "md_param_grad");
    MD_HIP(launch_reduce_pair(part, c.W.nbf, 1.0, 1.0, dU, stream), "md_param_grad/reduce");
    return MD_OK;
}

int md_adjoint_kick(const md_params* p, const double* pos, const md_cells* cells, const md_pairlist* list,
                    const double* u, double* out, double* u_out, const double coef[5], double* acc, void* ws,
                    size_t ws_bytes, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!pos || !u || !out || !coef || !acc) return fail(MD_ERR_ARG, "pos, u, out, coef or acc is NULL");
    if (u_out && (u_out == u || u_out == out)) return fail(MD_ERR_ARG, "u_out must not alias u or out");
    if (out == u) return fail(MD_ERR_ARG, "out must not alias u");
    if ((rc = check_cells(c, cells)) != MD_OK) return rc;
    if ((rc = check_slot_list(c, list, false)) != MD_OK) return rc;
    if ((rc = check_ws(c, ws, ws_bytes)) != MD_OK) return rc;
    AdjCoef k;
    k.alpha = coef[0];
    k.beta = coef[1];
    k.gamma = coef[2];
    k.cu = coef[3];
    k.cU = coef[4];
    k.dt = p->dt;
    double* part = (double*)((char*)ws + c.W.part_a);
    MD_HIP(launch_adjoint_kick(c.g, c.lj, pos, cells->cell_xyz, *list, u, out, u_out, k, part, stream),
           "md_adjoint_kick");
    MD_HIP(launch_reduce_pair(part, c.W.nbf, 1.0, 1.0, acc, stream, true), "md_adjoint_kick/reduce");
    return MD_OK;
}

// ---------------------------------------------------------------------------
// state-level calls
// ---------------------------------------------------------------------------
static int check_state(const Ctx& c, const md_params* p, md_state* st)
{
    if (!st) return fail(MD_ERR_ARG, "state is NULL");
    if (!st->pos || !st->vel || !st->force || !st->pos_ref || !st->id || !st->energy || !st->flags)
        return fail(MD_ERR_ARG, "state has a NULL array");
    if (p->precision == MD_MIXED && (!st->pos32 || !st->pos32_alt))
        return fail(MD_ERR_ARG, "mixed precision needs pos32 and pos32_alt");
    if (p->precision == MD_FP64 && !st->pos_alt) return fail(MD_ERR_ARG, "FP64 needs pos_alt");
    if (p->resort_every > 0 && (!st->pos_alt || !st->vel_alt || !st->id_alt))
        return fail(MD_ERR_ARG, "re-sorting needs pos_alt, vel_alt and id_alt");
    int rc = check_cells(c, &st->cells);
    if (rc != MD_OK) return rc;
    if ((rc = check_list(c, &st->list, false)) != MD_OK) return rc;
    return check_ws(c, st->ws, st->ws_bytes);
}

// bin + optional re-sort + reference copy + list build (no wait)
static int read_flags(const Ctx& c, md_state* st, hipStream_t s, int64_t out[16]);

// slot arrays of the block maxima of d2 (which = 0) and v2 (which = 1)
static unsigned long long* mx_slots(const Ctx& c, md_state* st, int which)
{
    return (unsigned long long*)((char*)st->ws + c.W.mx) + (size_t)which * kMaxSlots * kMaxSlotStride;
}

static hipError_t clear_maxima(const Ctx& c, md_state* st, hipStream_t s)
{
    return launch_fill_i32((int32_t*)mx_slots(c, st, 0), 0, 2 * 2 * kMaxSlots * kMaxSlotStride, s);
}

// Pair list of the state: tiled (16-bit entries into each tile's staged
// neighbourhood) when the geometry has tiles and the slots are in cell order,
// else slot entries.
static int build_list(const Ctx& c, const md_params* p, md_state* st, bool tiled, Timer& T, hipStream_t s)
{
    if (st->list.capacity < list_words(c, &st->list, tiled)) {
        // the caller gave room for 16-bit entries only; slot entries need twice
        // as much (the list is left invalid; status[2] stays clear)
        st->list_valid = 0;
        return fail(MD_ERR_CAPACITY, "slot entries need %lld words of nbr, capacity is %lld",
                    (long long)list_words(c, &st->list, tiled), (long long)st->list.capacity);
    }
    int64_t* tmax = (int64_t*)((char*)st->ws + c.W.tmax);
    if (tiled) MD_HIP(launch_fill_i32((int32_t*)tmax, 0, 2 * kTileMaxSlots, s), "rebuild/tile-max");
    tick(T, MD_T_BUILD, 0, s);
    const bool half = p->list_layout == MD_LIST_HALF;
    MD_HIP(launch_build(c.g, p->rs, st->pos, st->cells, st->list, st->ws, c.W, tiled, half,
                        (unsigned long long*)tmax, p->build_waves, s),
           "rebuild/build");
    tick(T, MD_T_BUILD, 1, s);
    st->list_tiled = tiled ? 1 : 0;
    st->list.tiled = st->list_tiled;
    st->list.half = half ? 1 : 0;
    st->tile_stage = 0;
    st->tile_cells = tiled ? c.g.tc : 0;
    return MD_OK;
}

// Bin, re-sort (every resort_every-th build), build the list, and read the
// flags back into f.  A tiled list whose largest tile neighbourhood exceeds
// what the force pass can stage is rebuilt with slot entries.
static int rebuild(const Ctx& c, const md_params* p, md_state* st, bool allow_resort, Timer& T,
                   hipStream_t s, int64_t f[16])
{
    int64_t* err = (int64_t*)((char*)st->ws + c.W.scal);
    tick(T, MD_T_BIN, 0, s);
    MD_HIP(launch_bin(c.g, st->pos, st->cells, st->ws, c.W, err, s), "rebuild/bin");
    tick(T, MD_T_BIN, 1, s);
    for (int k = 0; k < 3; ++k) st->cells.ncell[k] = c.nc[k];
    st->cells.sorted = 0;
    const bool resort = allow_resort && p->resort_every > 0 && (st->rebuilds % p->resort_every) == 0;
    if (resort) {
        tick(T, MD_T_RESORT, 0, s);
        MD_HIP(launch_resort(c.g, st->cells.order, st->pos, st->vel, st->id, st->pos_alt, st->vel_alt,
                             st->id_alt, st->pos_ref, p->precision == MD_MIXED ? st->pos32 : nullptr,
                             st->cells.cell_of, st->cells.cell_xyz, s),
               "rebuild/resort");
        tick(T, MD_T_RESORT, 1, s);
        std::swap(st->pos, st->pos_alt);
        std::swap(st->vel, st->vel_alt);
        std::swap(st->id, st->id_alt);
        st->cells.sorted = 1;
        st->resorts += 1;
    } else {
        MD_HIP(launch_ref_copy(c.g, st->pos, st->cells.cell_xyz, st->pos_ref,
                               p->precision == MD_MIXED ? st->pos32 : nullptr, s),
               "rebuild/ref");
    }
    // tiled rows start at even entries of 4-byte aligned cell blocks
    const bool tiled = c.g.tc > 0 && st->cells.sorted && (st->list.cell_stride & 1) == 0;
    int rc = build_list(c, p, st, tiled, T, s);
    if (rc != MD_OK) return rc;
    if ((rc = read_flags(c, st, s, f)) != MD_OK) return rc;
    if (st->list_tiled) {
        if (f[11] > tile_stage_cap(p->precision)) {
            timer_collect(T);
            if ((rc = build_list(c, p, st, false, T, s)) != MD_OK) return rc;
            if ((rc = read_flags(c, st, s, f)) != MD_OK) return rc;
        } else {
            st->tile_stage = (int32_t)f[11];
        }
    }
    return MD_OK;
}

static TileIo tile_io(const md_state* st)
{
    TileIo t;
    if (st->list_tiled) {
        t.start = st->cells.start;
        t.count = st->cells.count;
        t.stage = st->tile_stage;
    }
    return t;
}

// wait for the stream and read, in one copy: list status [0..3], cell-grid
// error flags [4..5], force flags [6], max squared displacement bits [7]
static int read_flags(const Ctx& c, md_state* st, hipStream_t s, int64_t out[16])
{
    int64_t* scal = (int64_t*)((char*)st->ws + c.W.scal);
    MD_HIP(launch_gather_flags(st->list.status, scal, st->flags, st->energy, (const int64_t*)((char*)st->ws + c.W.tmax),
                               mx_slots(c, st, 0), scal + kScalOut, s),
           "flags/gather");
    int64_t local[16];
    int64_t* dst = st->host_scratch ? st->host_scratch : local;
    MD_HIP(hipMemcpyAsync(dst, scal + kScalOut, 16 * sizeof(int64_t), hipMemcpyDeviceToHost, s), "flags/copy");
    MD_HIP(hipStreamSynchronize(s), "flags/sync");
    for (int k = 0; k < 16; ++k) out[k] = dst[k];
    return MD_OK;
}

static int force_eval(const Ctx& c, const md_params* p, md_state* st, bool energy, Timer& T, hipStream_t s)
{
    ForceOut out;
    out.force = st->force;
    out.part = energy ? (double*)((char*)st->ws + c.W.part_a) : nullptr;
    out.flags = st->flags;
    tick(T, MD_T_FORCE, 0, s);
    MD_HIP(launch_forces(c.g, c.lj, p->precision, st->pos, p->precision == MD_MIXED ? st->pos32 : nullptr,
                         st->cells.cell_xyz, st->list, out, s, tile_io(st)),
           "forces");
    tick(T, MD_T_FORCE, 1, s);
    return MD_OK;
}

static IntArgs int_args(const Ctx& c, const md_params* p, md_state* st, bool ke)
{
    IntArgs a;
    a.pos = st->pos;
    a.vel = st->vel;
    a.force = st->force;
    a.pos_ref = st->pos_ref;
    a.pos32 = st->pos32;
    a.cell_xyz = st->cells.cell_xyz;
    a.part_ke = ke ? (double*)((char*)st->ws + c.W.part_b) : nullptr;
    a.max_d2 = mx_slots(c, st, 0);
    a.max_v2 = mx_slots(c, st, 1);
    a.dt = p->dt;
    a.precision = p->precision;
    return a;
}

static int check_status(const int64_t f[16], const md_state* st)
{
    if (f[2] != 0)
        return fail(MD_ERR_CAPACITY, "pair list overflow: the list needs a cell_stride of %lld, it is %lld",
                    (long long)f[1], (long long)st->list.cell_stride);
    if (f[4] & 2) return fail(MD_ERR_ARG, "positions outside [0, L) given to the cell grid");
    if (f[6] & 1) return fail(MD_ERR_NONFINITE, "non-finite force");
    return MD_OK;
}

// Threshold of the large-displacement check from the largest squared
// displacement: members have displacement > t (lowered by 1e-12 so that
// rounding can only add members).
static double ldc_threshold(const md_params* p, double dmax2)
{
    return (p->rs - p->rc) - std::sqrt(dmax2) - 1e-12;
}

// One large-displacement check inside md_step (positions after the drift).
static int ldc_step(const Ctx& c, const md_params* p, md_state* st, double dmax2, Timer& T, hipStream_t s,
                    bool* keep)
{
    st->ldc_checks += 1;
    // Two outcomes need no kernel and give the same decision: t >= 0 with
    // max d2 <= t^2, so there are no members (kept); or t < 0, so everyone is a
    // member, more than ldc_max (expired).
    const double t = ldc_threshold(p, dmax2);
    if (t >= 0.0 && dmax2 <= t * t) {
        *keep = true;
        st->ldc_kept += 1;
        return MD_OK;
    }
    if (t < 0.0 && c.g.n > (int64_t)p->ldc_max) {
        *keep = false;
        return MD_OK;
    }
    int64_t* scal = (int64_t*)((char*)st->ws + c.W.scal);
    tick(T, MD_T_CHECK, 0, s);
    MD_HIP(launch_fill_i32((int32_t*)(scal + 4), 0, 4, s), "ldc/clear");
    MD_HIP(launch_ldc_check(c.g, st->pos, st->pos_ref, p->rc, p->rs, t, p->ldc_max,
                            (int32_t*)((char*)st->ws + c.W.ldc), (unsigned long long*)(scal + 4),
                            (unsigned long long*)(scal + 5), s),
           "ldc/check");
    tick(T, MD_T_CHECK, 1, s);
    int64_t f[16];
    int rc = read_flags(c, st, s, f);
    if (rc != MD_OK) return rc;
    timer_collect(T);
    *keep = f[9] <= (int64_t)p->ldc_max && f[10] == 0;
    st->ldc_kept += *keep ? 1 : 0;
    return MD_OK;
}

int md_ldc_check(const md_params* p, const double* pos, const double* pos_ref, int32_t* valid,
                 int64_t* members, double* dmax2, void* ws, size_t ws_bytes, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if (!pos || !pos_ref || !valid || !members || !dmax2) return fail(MD_ERR_ARG, "NULL argument");
    if ((rc = check_ws(c, ws, ws_bytes)) != MD_OK) return rc;
    int64_t* scal = (int64_t*)((char*)ws + c.W.scal);
    MD_HIP(launch_fill_i32((int32_t*)(scal + 4), 0, 6, stream), "md_ldc_check/clear");
    MD_HIP(launch_ldc_disp(c.g, pos, pos_ref, (unsigned long long*)(scal + 6), stream), "md_ldc_check/disp");
    int64_t h[3];
    MD_HIP(hipMemcpyAsync(h, scal + 4, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, stream), "md_ldc_check/copy");
    MD_HIP(hipStreamSynchronize(stream), "md_ldc_check/sync");
    double m2;
    std::memcpy(&m2, &h[2], sizeof(double));
    MD_HIP(launch_ldc_check(c.g, pos, pos_ref, p->rc, p->rs, ldc_threshold(p, m2), p->ldc_max,
                            (int32_t*)((char*)ws + c.W.ldc), (unsigned long long*)(scal + 4),
                            (unsigned long long*)(scal + 5), stream),
           "md_ldc_check/check");
    MD_HIP(hipMemcpyAsync(h, scal + 4, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, stream), "md_ldc_check/copy");
    MD_HIP(hipStreamSynchronize(stream), "md_ldc_check/sync");
    *members = h[0];
    *valid = (h[0] <= (int64_t)p->ldc_max && h[1] == 0) ? 1 : 0;
    *dmax2 = m2;
    return MD_OK;
}

int md_resort(const md_params* p, md_state* st, hipStream_t stream)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if ((rc = check_state(c, p, st)) != MD_OK) return rc;
    if (!st->pos_alt || !st->vel_alt || !st->id_alt) return fail(MD_ERR_ARG, "re-sort needs *_alt arrays");
    MD_HIP(launch_resort(c.g, st->cells.order, st->pos, st->vel, st->id, st->pos_alt, st->vel_alt, st->id_alt,
                         st->pos_ref, p->precision == MD_MIXED ? st->pos32 : nullptr, st->cells.cell_of,
                         st->cells.cell_xyz, stream),
           "md_resort");
    std::swap(st->pos, st->pos_alt);
    std::swap(st->vel, st->vel_alt);
    std::swap(st->id, st->id_alt);
    st->cells.sorted = 1;
    st->resorts += 1;
    st->list_valid = 0;
    st->phase = 2;  // forces now belong to the old slot order: md_prepare must run
    return MD_OK;
}

int md_prepare(const md_params* p, md_state* st, hipStream_t s)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if ((rc = check_state(c, p, st)) != MD_OK) return rc;
    Timer T;
    timer_begin(T, nullptr);
    MD_HIP(launch_fill_i32((int32_t*)st->flags, 0, 2, s), "prepare/flags");
    MD_HIP(launch_fill_i32((int32_t*)((char*)st->ws + c.W.scal), 0, 4, s), "prepare/err");
    MD_HIP(clear_maxima(c, st, s), "prepare/maxima");
    int64_t f[16];
    if ((rc = rebuild(c, p, st, true, T, s, f)) != MD_OK) return rc;
    st->rebuilds += 1;
    st->dutc_buffer = p->rs - p->rc;
    if ((rc = check_status(f, st)) != MD_OK) {
        st->list_valid = 0;
        return rc;
    }
    st->list_valid = 1;
    if ((rc = force_eval(c, p, st, true, T, s)) != MD_OK) return rc;
    IntArgs a = int_args(c, p, st, true);
    MD_HIP(launch_integrate(c.g, INT_KE, a, s), "prepare/ke");
    MD_HIP(launch_reduce_energy((double*)((char*)st->ws + c.W.part_a), force_blocks(c.g, st->list_tiled),
                                (double*)((char*)st->ws + c.W.part_b), c.W.nbi, st->energy, nullptr,
                                (double*)((char*)st->ws + c.W.red), s),
           "prepare/reduce");
    if ((rc = read_flags(c, st, s, f)) != MD_OK) return rc;
    if ((rc = check_status(f, st)) != MD_OK) return rc;
    st->phase = 0;
    return MD_OK;
}

int md_energy(const md_params* p, md_state* st, double* out, hipStream_t s)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if ((rc = check_state(c, p, st)) != MD_OK) return rc;
    if (!out) return fail(MD_ERR_ARG, "out is NULL");
    if (!st->list_valid) return fail(MD_ERR_ARG, "state has no valid pair list (call md_prepare)");
    Timer T;
    timer_begin(T, nullptr);
    if ((rc = force_eval(c, p, st, true, T, s)) != MD_OK) return rc;
    IntArgs a = int_args(c, p, st, true);
    MD_HIP(launch_integrate(c.g, INT_KE, a, s), "energy/ke");
    MD_HIP(launch_reduce_energy((double*)((char*)st->ws + c.W.part_a), force_blocks(c.g, st->list_tiled),
                                (double*)((char*)st->ws + c.W.part_b), c.W.nbi, st->energy, out,
                                (double*)((char*)st->ws + c.W.red), s),
           "energy/reduce");
    return MD_OK;
}

// Steps of the half-skin rule with a full list, queued in runs without a host
// wait per step.  The gather after each step decides on the device whether
// the next one must rebuild first (Sec. 2.3: largest displacement since the
// build beyond half the skin); once one must, it sets the gate and the passes
// of the rest of the run do nothing.  The host waits once per run, learns how
// many steps ran, rebuilds when the run stopped for it, and resumes there: the
// steps taken, the lists and the results are those of one wait per step.
static_assert(MD_STEP_RUN_MAX <= kTimerSlots, "a run's launches must fit the timer slots");
constexpr int64_t kRunFirst = 4;   // run length while the list's age is unknown

static int step_runs(const Ctx& c, const md_params* p, md_state* st, int64_t nsteps, int64_t sample_every,
                     double* energy_log, double* traj, int32_t* built, Timer& T, hipStream_t s)
{
    const double half_skin = 0.5 * (p->rs - p->rc);
    const double thr2 = half_skin * half_skin;
    const bool mixed = p->precision == MD_MIXED;
    int64_t* scal = (int64_t*)((char*)st->ws + c.W.scal);
    int32_t* gate = (int32_t*)(scal + 8);
    double* part_pw = (double*)((char*)st->ws + c.W.part_a);
    double* part_ke = (double*)((char*)st->ws + c.W.part_b);
    int rc;
    int64_t f[16];
    if (st->phase == 0) {
        // first half kick and drift of the first step
        MD_HIP(clear_maxima(c, st, s), "step/maxd2");
        tick(T, MD_T_INTEGRATE, 0, s);
        MD_HIP(launch_integrate(c.g, INT_KD, int_args(c, p, st, false), s), "step/kd");
        tick(T, MD_T_INTEGRATE, 1, s);
        st->phase = 1;
    }
    if ((rc = read_flags(c, st, s, f)) != MD_OK) return rc;
    timer_collect(T);
    double maxd2;
    std::memcpy(&maxd2, &f[7], sizeof(double));
    bool expired = !st->list_valid || maxd2 > thr2;
    bool dirty = true;        // slots may hold maxima no gather of a run cleared
    int64_t age = -1;         // steps since the last build (-1: built before this call)
    int64_t cycle = 0;        // steps between the last two builds of this call
    double rate = 0.0;        // growth of the largest displacement per step (age unknown)
    int64_t done = 0, k_log = 0;
    while (done < nsteps) {
        const bool rebuilt = expired;
        if (expired) {
            if ((rc = rebuild(c, p, st, true, T, s, f)) != MD_OK) return rc;
            st->rebuilds += 1;
            st->dutc_buffer = p->rs - p->rc;
            timer_collect(T);
            if (f[2] != 0) {
                st->list_valid = 0;
                return check_status(f, st);
            }
            st->list_valid = 1;
            if (age > 0) cycle = age;
            age = 0;
        }
        if (dirty) {
            MD_HIP(clear_maxima(c, st, s), "step/maxd2");
            dirty = false;
        }
        // run length: the steps left until the largest displacement, growing
        // in proportion to the list's age (or as it did over the last run),
        // passes half the skin, and one more
        const double d0 = rebuilt ? 0.0 : std::sqrt(maxd2);
        double left = (double)kRunFirst;
        if (age > 0 && d0 > 0.0) left = (double)age * (half_skin / d0 - 1.0);
        else if (age == 0 && cycle > 0) left = (double)cycle;
        else if (age < 0 && rate > 0.0) left = (half_skin - d0) / rate;
        int64_t run = p->step_run;
        if (run == 0) run = (int64_t)std::ceil(std::min(std::max(left, 0.0), (double)MD_STEP_RUN_MAX)) + 1;
        run = std::min(std::min(run, (int64_t)MD_STEP_RUN_MAX), nsteps - done);
        // queue the run; the first step needs no gate
        double* P = st->pos;
        double* Palt = st->pos_alt;
        float* P32 = st->pos32;
        float* P32alt = st->pos32_alt;
        const int64_t nfb = force_blocks(c.g, st->list_tiled);
        int64_t k_run = k_log;
        for (int64_t b = 0; b < run; ++b) {
            const int64_t step_no = st->step + 1 + b;
            const bool sample = sample_every > 0 && (step_no % sample_every) == 0;
            const bool last = done + b + 1 == nsteps;
            const int32_t* g = b > 0 ? gate : nullptr;
            if (traj)
                MD_HIP(launch_record(c.g, P, st->id, traj + 4 * c.g.n * (done + b), s, g), "step/record");
            StepIo io;
            io.pos = P;
            io.pos32 = mixed ? P32 : nullptr;
            io.cell_xyz = st->cells.cell_xyz;
            io.list = st->list;
            io.force = st->force;
            io.part_pw = sample ? part_pw : nullptr;
            io.part_ke = sample ? part_ke : nullptr;
            io.flags = st->flags;
            io.vel = st->vel;
            io.pos_ref = st->pos_ref;
            io.pos_out = mixed ? P : Palt;
            io.pos32_out = mixed ? P32alt : nullptr;
            io.max_d2 = mx_slots(c, st, 0);
            io.max_v2 = mx_slots(c, st, 1);
            io.dt = p->dt;
            io.drift = !last;
            io.track_speed = false;
            io.tile = tile_io(st);
            io.gate = g;
            tick(T, MD_T_FORCE, 0, s);
            MD_HIP(launch_force_step(c.g, c.lj, p->precision, io, s), "step/force");
            tick(T, MD_T_FORCE, 1, s);
            if (!last) {
                if (mixed) std::swap(P32, P32alt);
                else std::swap(P, Palt);
            }
            if (sample) {
                tick(T, MD_T_REDUCE, 0, s);
                MD_HIP(launch_reduce_energy(part_pw, nfb, part_ke, nfb, st->energy,
                                            energy_log ? energy_log + 4 * k_run : nullptr,
                                            (double*)((char*)st->ws + c.W.red), s, g),
                       "step/reduce");
                tick(T, MD_T_REDUCE, 1, s);
                ++k_run;
            }
            FlagGate fg;
            fg.gate = gate;
            fg.thr2 = thr2;
            fg.idx = (int32_t)(b + 1);
            fg.fold = !last;     // the last step of a call has no drift
            fg.clear = !last;
            MD_HIP(launch_gather_flags(st->list.status, scal, st->flags, st->energy,
                                       (const int64_t*)((char*)st->ws + c.W.tmax), mx_slots(c, st, 0),
                                       scal + kScalOut, s, fg),
                   "step/gather");
        }
        int64_t* dst = st->host_scratch ? st->host_scratch : f;
        MD_HIP(hipMemcpyAsync(dst, scal + kScalOut, 16 * sizeof(int64_t), hipMemcpyDeviceToHost, s), "step/copy");
        MD_HIP(hipStreamSynchronize(s), "step/sync");
        if (dst != f)
            for (int k = 0; k < 16; ++k) f[k] = dst[k];
        const int64_t ran = f[12];
        if (ran < 1 || ran > run) return fail(MD_ERR_HIP, "step run: gather reported %lld of %lld steps",
                                              (long long)ran, (long long)run);
        // the state after the steps that ran
        int64_t samples = 0;
        for (int64_t b = 0; b < ran; ++b) {
            const int64_t step_no = st->step + 1 + b;
            if (sample_every > 0 && (step_no % sample_every) == 0) ++samples;
            if (built) built[done + b] = (b == 0 && expired) ? 1 : 0;
            if (done + b + 1 != nsteps) {
                if (mixed) std::swap(st->pos32, st->pos32_alt);
                else std::swap(st->pos, st->pos_alt);
            }
        }
        timer_keep(T, MD_T_FORCE, ran);
        timer_keep(T, MD_T_REDUCE, samples);
        timer_collect(T);
        k_log += samples;
        st->step += ran;
        done += ran;
        if (age >= 0) age += ran;
        st->phase = done == nsteps ? 0 : 1;
        std::memcpy(&maxd2, &f[7], sizeof(double));
        if (age < 0 && std::sqrt(maxd2) > d0) rate = (std::sqrt(maxd2) - d0) / (double)ran;
        if (f[6] & 1) return check_status(f, st);
        expired = f[13] != 0;
    }
    return check_status(f, st);
}

// The step loop of md_step and md_step_record (traj / built may be NULL).
static int step_loop(const md_params* p, md_state* st, int64_t nsteps, int64_t sample_every, double* energy_log,
                     double* traj, int32_t* built, hipStream_t s)
{
    Ctx c;
    int rc = setup(p, c);
    if (rc != MD_OK) return rc;
    if ((rc = check_state(c, p, st)) != MD_OK) return rc;
    if (!(p->dt > 0.0)) return fail(MD_ERR_ARG, "dt must be > 0");
    if (nsteps < 0) return fail(MD_ERR_ARG, "nsteps must be >= 0");
    // forces must exist for the current positions (md_prepare); a list that
    // was invalidated since (re-sized by the caller) is rebuilt before use
    if (st->rebuilds == 0 || st->phase == 2)
        return fail(MD_ERR_ARG, "state not prepared (call md_prepare)");
    if (nsteps == 0) return MD_OK;
    const double half_skin = 0.5 * (p->rs - p->rc);
    const double thr2 = half_skin * half_skin;
    Timer T;
    timer_begin(T, st->timers);
    if (p->rebuild_rule == MD_REBUILD_HALF_SKIN && p->list_layout != MD_LIST_HALF)
        return step_runs(c, p, st, nsteps, sample_every, energy_log, traj, built, T, s);
    double* part_pw = (double*)((char*)st->ws + c.W.part_a);
    double* part_ke = (double*)((char*)st->ws + c.W.part_b);
    int64_t k_log = 0;
    int64_t done = 0;
    bool need_drift = st->phase == 0;
    while (done < nsteps) {
        const int64_t step_no = st->step + 1;
        const bool sample = sample_every > 0 && (step_no % sample_every) == 0;
        if (need_drift) {
            // first half kick and drift of this step (the previous step ended
            // with a completed kick, or this is the first step of the call)
            MD_HIP(clear_maxima(c, st, s), "step/maxd2");
            tick(T, MD_T_INTEGRATE, 0, s);
            MD_HIP(launch_integrate(c.g, INT_KD, int_args(c, p, st, false), s), "step/kd");
            tick(T, MD_T_INTEGRATE, 1, s);
            st->phase = 1;
        }
        int64_t f[16];
        if ((rc = read_flags(c, st, s, f)) != MD_OK) return rc;
        timer_collect(T);
        double maxd2, maxv2;
        std::memcpy(&maxd2, &f[7], sizeof(double));
        std::memcpy(&maxv2, &f[8], sizeof(double));
        bool expired = !st->list_valid;
        if (!expired && p->rebuild_rule == MD_REBUILD_HALF_SKIN) {
            expired = maxd2 > thr2;
        } else if (!expired) {
            // DUTC: the buffer shrinks by twice the distance the fastest
            // particle drifted; once it is used up, the large-displacement
            // check decides
            st->dutc_buffer -= 2.0 * std::sqrt(maxv2) * p->dt;
            if (!(st->dutc_buffer > 0.0)) {
                bool keep = false;
                if ((rc = ldc_step(c, p, st, maxd2, T, s, &keep)) != MD_OK) return rc;
                expired = !keep;
            }
        }
        if (expired) {
            if ((rc = rebuild(c, p, st, true, T, s, f)) != MD_OK) return rc;
            st->rebuilds += 1;
            st->dutc_buffer = p->rs - p->rc;
            timer_collect(T);
            if (f[2] != 0) {
                st->list_valid = 0;
                return check_status(f, st);
            }
            st->list_valid = 1;
        }
        if (built) built[done] = expired ? 1 : 0;
        if (traj)
            MD_HIP(launch_record(c.g, st->pos, st->id, traj + 4 * c.g.n * done, s), "step/record");
        // force pass with the second half kick of this step, fused with the
        // next step's first half kick and drift unless this is the last step
        // of the call (then the force is stored for the next call)
        const bool last = done + 1 == nsteps;
        const bool mixed = p->precision == MD_MIXED;
        StepIo io;
        io.pos = st->pos;
        io.pos32 = mixed ? st->pos32 : nullptr;
        io.cell_xyz = st->cells.cell_xyz;
        io.list = st->list;
        io.force = st->force;
        io.part_pw = sample ? part_pw : nullptr;
        io.part_ke = sample ? part_ke : nullptr;
        io.flags = st->flags;
        io.vel = st->vel;
        io.pos_ref = st->pos_ref;
        io.pos_out = mixed ? st->pos : st->pos_alt;
        io.pos32_out = mixed ? st->pos32_alt : nullptr;
        io.max_d2 = mx_slots(c, st, 0);
        io.max_v2 = mx_slots(c, st, 1);
        io.dt = p->dt;
        io.drift = !last;
        io.track_speed = p->rebuild_rule == MD_REBUILD_DUTC_LDC;
        io.tile = tile_io(st);
        if (!last) MD_HIP(clear_maxima(c, st, s), "step/maxd2");
        tick(T, MD_T_FORCE, 0, s);
        MD_HIP(launch_force_step(c.g, c.lj, p->precision, io, s), "step/force");
        tick(T, MD_T_FORCE, 1, s);
        if (!last) {
            if (mixed) std::swap(st->pos32, st->pos32_alt);
            else std::swap(st->pos, st->pos_alt);
        }
        if (sample) {
            tick(T, MD_T_REDUCE, 0, s);
            const int64_t nfb = force_blocks(c.g, st->list_tiled);
            MD_HIP(launch_reduce_energy(part_pw, nfb, part_ke, nfb, st->energy,
                                        energy_log ? energy_log + 4 * k_log : nullptr,
                                        (double*)((char*)st->ws + c.W.red), s),
                   "step/reduce");
            tick(T, MD_T_REDUCE, 1, s);
            ++k_log;
        }
        st->step += 1;
        ++done;
        st->phase = last ? 0 : 1;
        need_drift = false;
        if (last) {
            if ((rc = read_flags(c, st, s, f)) != MD_OK) return rc;
            timer_collect(T);
            if ((rc = check_status(f, st)) != MD_OK) return rc;
        } else if (f[6] & 1) {
            return check_status(f, st);
        }
    }
    return MD_OK;
}

int md_step(const md_params* p, md_state* st, int64_t nsteps, int64_t sample_every, double* energy_log,
            hipStream_t s)
{
    return step_loop(p, st, nsteps, sample_every, energy_log, nullptr, nullptr, s);
}

int md_step_record(const md_params* p, md_state* st, int64_t nsteps, int64_t sample_every, double* energy_log,
                   double* traj, int32_t* built, hipStream_t s)
{
    if (!traj || !built) return fail(MD_ERR_ARG, "traj or built is NULL");
    return step_loop(p, st, nsteps, sample_every, energy_log, traj, built, s);
}

}  // extern "C"
