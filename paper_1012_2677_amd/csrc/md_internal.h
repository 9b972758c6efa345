// Internal declarations of the gfx950 LJ hot path: launch geometry, workspace
// layout, kernel argument blocks and the launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "md.h"

namespace md {

// ---------------------------------------------------------------------------
// Launch configuration
// ---------------------------------------------------------------------------
constexpr int kStreamBlock = 256;        // streaming kernels (label, integrate, ...)
constexpr int kScanItems = 1024;         // items per block of the three-phase scan
constexpr int kForceBlock = 256;         // force / adjoint kernels
#ifndef MD_LANES_PER_KEY
#define MD_LANES_PER_KEY 8
#endif
#ifndef MD_FORCE_UNROLL
#define MD_FORCE_UNROLL 8
#endif
#ifndef MD_FORCE_UNROLL_FP64
#define MD_FORCE_UNROLL_FP64 4
#endif
#ifndef MD_PAIR_MIN_BLOCKS
#define MD_PAIR_MIN_BLOCKS 1
#endif
constexpr int kLanesPerKey = MD_LANES_PER_KEY;   // lanes cooperating on one key's row (adjoint kernels)
constexpr int kForceUnroll = MD_FORCE_UNROLL;    // row entries in flight per lane (FP32 pair terms)
constexpr int kForceUnroll64 = MD_FORCE_UNROLL_FP64;  // same for FP64 pair terms (register bound)
constexpr int kKeysPerBlock = kForceBlock / kLanesPerKey;
#ifndef MD_BUILD_NCH
#define MD_BUILD_NCH 8
#endif
constexpr int kBuildChunks = MD_BUILD_NCH;   // candidates held in registers: kBuildChunks x 64
constexpr int kBuildChunksSmall = 6;          // the same where neighbourhoods are small (fewer registers)
constexpr int kReduceBlock = 1024;

constexpr uint32_t kSlotMask = (1u << 27) - 1u;
constexpr int kCodeShift = 27;
#ifndef MD_TILE_BLOCK
#define MD_TILE_BLOCK 256
#endif
#ifndef MD_TILE_KEYS
#define MD_TILE_KEYS 200
#endif
constexpr int kTileBlock = MD_TILE_BLOCK;     // threads of the tiled force kernel (one block per tile)
constexpr int kTileKeys = MD_TILE_KEYS;       // target keys per tile (automatic tile length)
#ifndef MD_TILE_KEYS_FP64
#define MD_TILE_KEYS_FP64 146
#endif
constexpr int kTileKeys64 = MD_TILE_KEYS_FP64;  // same for FP64 (24-byte staged particles; 13 cells at rho = 0.5)
constexpr int kTileMaxStage = 3500;      // staged particles per tile: 16-bit byte offsets, under 64 KB of LDS
constexpr int kTileMaxStage64 = 1950;    // FP64: 32 bytes per staged particle, under 64 KB of LDS
static_assert((kTileMaxStage + 1) * 16 < 65536, "tiled entries are 16-bit byte offsets");
__host__ __device__ inline int tile_stage_cap(int precision)
{
    return precision == MD_MIXED ? kTileMaxStage : kTileMaxStage64;
}
constexpr int kTileMaxSlots = 256;
// Block maxima (squared displacement, squared drift speed) go to one of
// kMaxSlots slots by block index, each on its own 64-byte line, so that the
// atomics of many blocks do not meet at one address; the flag read-back takes
// the maximum over the slots.
constexpr int kMaxSlots = 256;
constexpr int kMaxSlotStride = 8;   // int64 words between slots
__host__ __device__ inline unsigned long long* max_slot(unsigned long long* base, int64_t blk)
{
    return base + (blk & (kMaxSlots - 1)) * kMaxSlotStride;
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Division of 0 <= x < 2^31 by a divisor d >= 1 fixed at launch, by a
// multiply-high and a shift (division by invariant integers): with
// s = ceil(log2 d) and m = floor(2^32 (2^s - d) / d) + 1, x / d equals
// (umulhi(x, m) + x) >> s.
struct FastDiv {
    uint32_t d, m, s;
};
inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    f.s = 0;
    while ((1ull << f.s) < d) ++f.s;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << f.s) - d)) / d) + 1);
    return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f)
{
    return (__umulhi(x, f.m) + x) >> f.s;
}

// ---------------------------------------------------------------------------
// Geometry derived on the host from md_params (FP64, computed once)
// ---------------------------------------------------------------------------
struct Geo {
    int64_t n;
    int32_t nc[3];
    int64_t ncell;
    double L[3];
    double invL[3];   // 1 / L
    double inv[3];    // nc / L   (cell label scale)
    double cs[3];     // L / nc   (cell side)
    int32_t exact_all;  // some axis has fewer than 5 cells: always take minimum images
    // force passes take minimum images for every pair: under the DUTC + LDC
    // rule a kept list can outlive displacements of more than (cell side -
    // rc), after which a partner that crossed the box boundary can come within
    // rc of a key whose build-time cell is interior
    int32_t force_minimg_all;
    // tiles of the LDS-staged force pass: runs of tc cells along z in one
    // (x, y) column, nt per column, ntile in all (tc = 0: no tiled layout)
    int32_t tc, nt;
    int64_t ntile;
};

// LJ coefficients in the form the kernels evaluate:
//   g(r)  = r^-2 r^-6 (A r^-6 - B) - C8                 (= -V'(r)/r)
//   V(r)  = r^-6 (A4 r^-6 - B4) + C2 r^2 + C0
//   g'(s) = dg/d(r^2) = r^-4 r^-6 (-7 A r^-6 + 4 B)
// with A = 48 eps sig^12, B = 24 eps sig^6, C8 = 8 eps c2 / sig^2,
//      A4 = 4 eps sig^12, B4 = 4 eps sig^6, C2 = 4 eps c2 / sig^2, C0 = 4 eps c0.
struct LJ {
    double rc2;
    double A, B, C8;
    double A4, B4, C2, C0;
    double eps, sigma;
    double Cs;        // sigma * dC8/dsigma
    double rc6i, rc8i, rc12i, rc14i;  // rc^-6, rc^-8, rc^-12, rc^-14
};

Geo make_geo(const md_params& p, const int32_t nc[3]);
// Records msg as the message of md_last_error() and returns code.
int set_error(int code, const char* msg);
LJ make_lj(const md_params& p);

// ---------------------------------------------------------------------------
// Workspace layout (all offsets 256-byte aligned)
// ---------------------------------------------------------------------------
struct WsLayout {
    size_t rank;       // int32[n]       atomic ranks during binning
    size_t bsum;       // int32[nbs+1]   scan block sums
    size_t cell_rows;  // int32[ncell]   entries per cell block (pair list)
    size_t part_a;     // double[2*nbf]  per-block partial sums (force kernels)
    size_t part_b;     // double[nbi]    per-block partial sums (streaming kernels)
    size_t pos32;      // float4[n]      mixed-mode local coordinates (md_forces; empty in FP64)
    size_t red;        // int64[2*1024]  partials of the list statistics
    size_t ldc;        // int32[ldc_max] members of the large-displacement check
    size_t scal;       // int64[32]      small device scalars (layout in md_api.hip)
    size_t tmax;       // int64[kTileMaxSlots]  largest staged tile neighbourhood, spread over slots
    size_t mx;         // int64[2][kMaxSlots * kMaxSlotStride]  block maxima of d2 and v2
    size_t tile_used;  // int32[ntile]   entries taken in each tile's pooled block (tiled list build)
    size_t total;
    int64_t nbs;       // scan blocks
    int64_t nbf;       // adjoint-kernel blocks (kKeysPerBlock keys each)
    int64_t nbi;       // streaming-kernel blocks
};
WsLayout ws_layout(const Geo& g, int64_t ldc_max, int precision);

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
// Blocks are dispatched round-robin over the 8 XCDs; give each XCD one
// contiguous range of logical blocks so neighbouring tiles share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t q = nb >> 3, r = nb & 7;
    const int64_t x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int cell_coord(double x, double inv, int n)
{
    int c = (int)(x * inv);
    c = c > n - 1 ? n - 1 : c;
    return c < 0 ? 0 : c;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// ---------------------------------------------------------------------------
// Tiles (list layout MD_LIST_TILED).  Tile t = (cx * ny + cy) * nt + tz holds
// the cells z0 = tz * tc .. z1 - 1 (z1 = min(z0 + tc, nz)) of column (cx, cy);
// its keys are those cells' slots, contiguous once the slots are in cell order.
// Its partners lie in the runs of cells z0 - 1 .. z1 (periodic in z) of the
// 9 columns (cx + sx, cy + sy), column index col = (sx + 1) * 3 + (sy + 1).
// Run position j = 0 .. R - 1 (R = z1 - z0 + 2) is cell z0 - 1 + j.  With
// tc <= nz - 2 a run wraps at most once: at jw = 1 (z0 = 0) or jw = R - 1
// (z1 = nz), otherwise jw = R; piece A = positions [0, jw) and piece B =
// [jw, R) are contiguous slot ranges.  The staged copy of a tile lists the
// runs column after column, each run in position order, so a particle's
// index in it is base[col] + (its slot - sA) in piece A and
// base[col] + lenA + (its slot - sB) in piece B; base[col] sums the earlier
// runs' lengths.  The list build and the force pass both derive this layout
// from the cell starts and counts.
// ---------------------------------------------------------------------------
struct TileRun {
    int32_t sA, lenA, sB, lenB;
};

__device__ __forceinline__ int wrap_cell(int z, int n) { return z < 0 ? z + n : (z >= n ? z - n : z); }

__device__ __forceinline__ int tile_jw(int z0, int z1, int nz)
{
    const int R = z1 - z0 + 2;
    return z0 == 0 ? 1 : (z1 == nz ? R - 1 : R);
}

// The same run in two steps, so that a caller can issue its loads together with
// others: the cells whose start / count give the run's ends (cell 0 where
// `use` is false or there is no second segment), then the loads.
struct TileCells {
    int64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    bool two = false;
};
__device__ __forceinline__ TileCells tile_run_cells(int X, int Y, int ny, int nz, int z0, int z1, bool use)
{
    const int R = z1 - z0 + 2, jw = tile_jw(z0, z1, nz);
    const int64_t col = ((int64_t)X * ny + Y) * nz;
    TileCells t;
    t.two = use && jw < R;
    if (use) {
        t.a0 = col + wrap_cell(z0 - 1, nz);
        t.a1 = col + wrap_cell(z0 - 2 + jw, nz);
    }
    if (t.two) {
        t.b0 = col + wrap_cell(z0 - 1 + jw, nz);
        t.b1 = col + wrap_cell(z1, nz);
    }
    return t;
}
__device__ __forceinline__ TileRun tile_run_load(const int32_t* start, const int32_t* count, const TileCells& t)
{
    const int sa = start[t.a0], ea = start[t.a1], ca = count[t.a1];
    const int sb = start[t.b0], eb = start[t.b1], cb = count[t.b1];
    TileRun r;
    r.sA = sa;
    r.lenA = ea + ca - sa;
    r.sB = t.two ? sb : 0;
    r.lenB = t.two ? eb + cb - sb : 0;
    return r;
}

// Run of column (X, Y) (already wrapped) for the tile cells [z0, z1).
__device__ __forceinline__ TileRun tile_run(const int32_t* start, const int32_t* count, int X, int Y, int ny,
                                            int nz, int z0, int z1)
{
    const int R = z1 - z0 + 2, jw = tile_jw(z0, z1, nz);
    const int64_t col = ((int64_t)X * ny + Y) * nz;
    const int64_t a0 = col + wrap_cell(z0 - 1, nz), a1 = col + wrap_cell(z0 - 2 + jw, nz);
    TileRun r;
    r.sA = start[a0];
    r.lenA = start[a1] + count[a1] - r.sA;
    r.sB = 0;
    r.lenB = 0;
    if (jw < R) {
        const int64_t b0 = col + wrap_cell(z0 - 1 + jw, nz), b1 = col + wrap_cell(z1, nz);
        r.sB = start[b0];
        r.lenB = start[b1] + count[b1] - r.sB;
    }
    return r;
}

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// 1/x in FP64 from the hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}

// 1/x from the estimate and one Newton step, for the force passes: the
// estimate's relative error is below 2^-24 on gfx950, one step squares it,
// leaving at most ~1e-14 relative (10 ulp; 2.2e-15 measured over 2^22 values of
// r^2 in [1e-3, 1e3]), far inside the force passes' 1e-12 bound, for two fewer
// FMAs in the pair's dependent chain.
__device__ __forceinline__ double rcp64_1(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    return __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
}

// ---------------------------------------------------------------------------
// Launchers (each returns hipGetLastError() of its launches)
// ---------------------------------------------------------------------------
// md_cells.hip
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s);
hipError_t launch_bin(const Geo& g, const double* pos, const md_cells& cells, void* ws,
                      const WsLayout& L, int64_t* err_flags, hipStream_t s);
hipError_t launch_resort(const Geo& g, const int32_t* order, const double* pos, const double* vel,
                         const int32_t* id, double* pos_alt, double* vel_alt, int32_t* id_alt,
                         double* pos_ref, float* pos32, int32_t* cell_of, int32_t* cell_xyz,
                         hipStream_t s);
hipError_t launch_pack(const Geo& g, const double* q, double* pos, hipStream_t s);
// frame[id[slot]] = pos[slot] (double4, w = 0): positions in the original order
// (nothing when gate is given and *gate != 0)
hipError_t launch_record(const Geo& g, const double* pos, const int32_t* id, double* frame, hipStream_t s,
                         const int32_t* gate = nullptr);
hipError_t launch_ref_copy(const Geo& g, const double* pos, const int32_t* cell_xyz, double* pos_ref,
                           float* pos32, hipStream_t s);

// md_pairlist.hip
// tiled: write 16-bit entries that index the staged copy of the key's tile
// (slots must be in cell order); the largest staged count of any tile goes to
// tile_max[0 .. kTileMaxSlots) (atomic max into slot tile % kTileMaxSlots, so
// that the atomics do not all meet at one address).  waves: MD_BUILD_* (tiled
// builds only).
hipError_t launch_build(const Geo& g, double rs, const double* pos, const md_cells& cells,
                        const md_pairlist& list, void* ws, const WsLayout& L, bool tiled, bool half,
                        unsigned long long* tile_max, int waves, hipStream_t s);

// md_forces.hip
struct ForceOut {
    void* force;        // [3][n] double or float
    double* part;       // per-block (PE, W) partials, or nullptr
    int64_t* flags;     // [0] |= 1 on a non-finite force
};
// Tiled lists (mixed only) need cells (start / count) and the largest staged
// count (tile_stage); tile_stage = 0 selects the list of slot entries.
struct TileIo {
    const int32_t* start = nullptr;
    const int32_t* count = nullptr;
    int32_t stage = 0;
};
hipError_t launch_forces(const Geo& g, const LJ& lj, int precision, const double* pos,
                         const float* pos32, const int32_t* cell_xyz, const md_pairlist& list,
                         const ForceOut& out, hipStream_t s, const TileIo& tio = TileIo());
// Force evaluation fused with the integrator: the second half kick (drift =
// false: also writes the force) or second kick + next first kick + drift
// (drift = true: writes positions to pos_out and, in mixed mode, local
// coordinates to pos32_out; the force is not stored).
struct StepIo {
    const double* pos;
    const float* pos32;
    const int32_t* cell_xyz;
    md_pairlist list;
    void* force;
    double* part_pw;              // per-block (PE, W) partials, or nullptr
    double* part_ke;              // per-block KE partials (with part_pw)
    int64_t* flags;
    double* vel;
    const double* pos_ref;
    double* pos_out;
    float* pos32_out;
    unsigned long long* max_d2;
    unsigned long long* max_v2;   // with track_speed
    double dt;
    bool drift;
    bool track_speed;             // also record the largest squared drift speed
    TileIo tile;                  // tiled list (tile.stage > 0)
    const int32_t* gate = nullptr;  // full list: the pass does nothing when *gate != 0
};
hipError_t launch_force_step(const Geo& g, const LJ& lj, int precision, const StepIo& io, hipStream_t s);
int64_t pair_blocks(const Geo& g);   // blocks (and energy partials) of one pair-kernel launch
int64_t force_blocks(const Geo& g, bool tiled);   // same for either list layout

// md_integrate.hip
enum IntMode { INT_KD = 0, INT_KE = 1 };
struct IntArgs {
    double* pos;
    double* vel;
    const void* force;
    const double* pos_ref;
    float* pos32;
    const int32_t* cell_xyz;
    double* part_ke;                // per-block KE partials (or nullptr)
    unsigned long long* max_d2;     // atomic max of squared displacement bits
    unsigned long long* max_v2;     // atomic max of squared drift speed bits
    double dt;
    int precision;
};

// Pinned squared length fma(z, z, fma(y, y, x * x)) (displacements, speeds).
__device__ __forceinline__ double pinned_len2(double x, double y, double z)
{
    return __builtin_fma(z, z, __builtin_fma(y, y, __dmul_rn(x, x)));
}
hipError_t launch_integrate(const Geo& g, IntMode mode, const IntArgs& a, hipStream_t s);
// scratch: device double[3 * 256] (block partials)
hipError_t launch_reduce_energy(const double* part_pw, int64_t nbf, const double* part_ke,
                                int64_t nbi, double* energy, double* log_row, double* scratch, hipStream_t s,
                                const int32_t* gate = nullptr);
hipError_t launch_reduce_pair(const double* part, int64_t nb, double scale0, double scale1,
                              double* out2, hipStream_t s, bool accumulate = false);
// The step decision of a run of steps queued without reading flags back
// (half-skin rule): the gather that follows step idx - 1 of the run sets *gate
// when step idx must rebuild first (largest squared displacement > thr2) or a
// non-finite force was seen; the passes of later steps, given the gate, then
// do nothing, and the gathers after it keep out as the stopping one wrote it.
// out[12] = idx and out[13] = 1 when it stopped the run.
struct FlagGate {
    int32_t* gate = nullptr;      // nullptr: a plain gather
    double thr2 = 0.0;
    int32_t idx = 0;
    bool fold = true;             // fold the slot maxima into energy[4], energy[5]
    bool clear = false;           // and clear the slots after reading them
};
// Also folds the slot maxima of d2 and v2 (mx) into energy[4] and energy[5].
hipError_t launch_gather_flags(const int64_t* status, const int64_t* err, const int64_t* flags, double* energy,
                               const int64_t* tmax, unsigned long long* mx, int64_t* out, hipStream_t s,
                               const FlagGate& gate = FlagGate());
hipError_t launch_list_stats(const int32_t* cell_rows, int64_t ncell, int64_t* status, long long* part,
                             hipStream_t s);

// md_validity.hip
hipError_t launch_ldc_disp(const Geo& g, const double* pos, const double* pos_ref, unsigned long long* max_d2,
                           hipStream_t s);
hipError_t launch_ldc_check(const Geo& g, const double* pos, const double* pos_ref, double rc, double rs,
                            double t, int64_t cap, int32_t* list, unsigned long long* count,
                            unsigned long long* flag, hipStream_t s);

// md_adjoint.hip
hipError_t launch_hvp(const Geo& g, const LJ& lj, const double* pos, const int32_t* cell_xyz,
                      const md_pairlist& list, const double* u, double* Hu, double* part,
                      hipStream_t s);
struct AdjCoef {
    double alpha, beta, gamma, cu, cU, dt;
};
hipError_t launch_adjoint_kick(const Geo& g, const LJ& lj, const double* pos, const int32_t* cell_xyz,
                               const md_pairlist& list, const double* u, double* out, double* u_out,
                               const AdjCoef& k, double* part, hipStream_t s);
hipError_t launch_param_grad(const Geo& g, const LJ& lj, const double* pos,
                             const int32_t* cell_xyz, const md_pairlist& list, double* part,
                             hipStream_t s);

}  // namespace md
