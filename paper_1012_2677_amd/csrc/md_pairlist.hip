// Pair-list construction (Sec. 2.3 bookkeeping with search length rs; Sec. 2.4
// key-sorted list), one 64-lane wavefront per cell (or, for the tiled list of
// a large grid, per tile of cells built one after another).
//
// The wave stages the particles of the 27 surrounding cells (~300 at
// rho = 0.5) in its registers, one candidate per lane per 64-chunk.  It then
// walks the keys of its own cell: each lane tests its candidates against the
// key with the exact FP64 predicate, a ballot gives the passing lanes, and the
// prefix popcount below each lane gives its output position, so every row is
// written compactly in candidate order (the key's own cell first, then the
// neighbour cells of stencil codes 14 .. 26 and 0 .. 12, each in ascending
// slot) with no atomics.  Rows of one cell are packed one after another into the
// cell's block of the list; the block base is the cell id times a fixed stride,
// so cells never have to wait for each other (tiled lists pool the blocks of a
// tile's cells, below).
//
// The work is ALU bound (about 300 FP64 distance tests per particle).

#include <cmath>
#include <type_traits>

#include "md_internal.h"

namespace md {

struct BuildArgs {
    const double4* pos;
    const int32_t* start;
    const int32_t* count;
    const int32_t* order;   // nullptr when the slots are already in cell order
    int32_t nc[3];
    int64_t ncell;
    double L[3], invL[3];
    double rs2;
    int32_t exact_all;
    int64_t stride;
    uint32_t* nbr;
    int64_t* offsets;
    int32_t* counts;
    int32_t* cell_rows;
    int64_t* status;
    int32_t tc;                       // tiled: cells per tile along z
    unsigned long long* tile_max;     // tiled: atomic max of the staged count per tile
    FastDiv div_nz;                   // division by nz and by kBuildStrip * ny (cell order decode)
    FastDiv div_strip;
    FastDiv div_tc;                   // tiled: division by tc
    int32_t nt;                       // tiled: tiles per column
    int32_t* tile_used;               // tiled: entries taken so far in each tile's pooled block
    int64_t ntile;                    // tiled: tiles in all
    FastDiv div_nt;                   // tiled: division by nt (tile order decode)
};

// r^2 of the pinned predicate: d = q_j - q_i, optional minimum image,
// r2 = fma(dz, dz, fma(dy, dy, dx * dx)).
template <bool MINIMG>
__device__ __forceinline__ double pair_r2(const BuildArgs& a, double xj, double yj, double zj, double xi,
                                          double yi, double zi)
{
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    if (MINIMG) {
        // one component after another (scheduling barriers): interleaved,
        // their temporaries would set the kernel's register count
        dx = dx - a.L[0] * rint(dx * a.invL[0]);
        __builtin_amdgcn_sched_barrier(0);
        dy = dy - a.L[1] * rint(dy * a.invL[1]);
        __builtin_amdgcn_sched_barrier(0);
        dz = dz - a.L[2] * rint(dz * a.invL[2]);
    }
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, __dmul_rn(dx, dx)));
}

// Inclusive prefix sums by DPP lane moves (no LDS round trips): over each row
// of 16 lanes (Hillis-Steele shifts by 1, 2, 4, 8; lanes shifted in from
// outside the row read 0), and over lanes 0 .. 31 (row 1 then adds lane 15).
constexpr int kDppRowShr = 0x110;     // row_shr:n is kDppRowShr + n
constexpr int kDppRowBcast15 = 0x142;
__device__ __forceinline__ int scan_row16(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 1, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 2, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 4, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 8, 0xF, 0xF, true);
    return v;
}
__device__ __forceinline__ int scan_lanes32(int v)
{
    v = scan_row16(v);
    // rows 1 and 3 take lane 15 of the row below; rows 0 and 2 add nothing
    return v + __builtin_amdgcn_update_dpp(0, v, kDppRowBcast15, 0xA, 0xF, false);
}

// Row header of one key.  When the cell block overflows, the row is clipped to
// the entries actually stored, so an invalid (overflowed) list still only
// references written, in-range entries.
__device__ __forceinline__ void write_row(const BuildArgs& a, int32_t kslot, int64_t base, int64_t used,
                                          int64_t wpos, int64_t cap)
{
    const int64_t start = used < cap ? used : cap;
    const int64_t room = cap - start;
    a.offsets[kslot] = base + start;
    a.counts[kslot] = (int32_t)(wpos < room ? wpos : room);
}

constexpr int kMaxOwn = 64;     // own-cell particles kept in LDS for the key loop (all in the first chunk)

// The neighbour cells in candidate order: rank 0 is the own cell (stencil code
// 13), ranks 1 .. 13 codes 14 .. 26, ranks 14 .. 26 codes 0 .. 12, so that the
// candidates of a half row (own cell, codes 14 .. 26) are the first 14 ranks.
// Code (sx+1)*9 + (sy+1)*3 + (sz+1) for the offsets s in {-1, 0, 1}^3.
__device__ __forceinline__ int code_of_rank(int r) { return r < 14 ? r + 13 : r - 14; }
#ifndef MD_BUILD_STRIP
#define MD_BUILD_STRIP 8
#endif
constexpr int kBuildStrip = MD_BUILD_STRIP;   // x-columns per strip of the cell order

// Tiled (16-bit) rows start at even entries, so the force pass can read two
// entries with one 32-bit load; the entry after a row of odd length holds the
// tile's stand-in partner.  Slot-entry rows are packed.
template <typename E>
__device__ __forceinline__ uint32_t row_start(uint32_t end)
{
    return sizeof(E) == 2 ? (end + 1u) & ~1u : end;
}

#ifndef MD_BUILD_ROWBUF
#define MD_BUILD_ROWBUF 768
#endif
constexpr int kRowBuf = MD_BUILD_ROWBUF;   // entries of one cell's rows staged in LDS before the block is written

template <typename E>
__device__ __forceinline__ void pad_row(E* blk, uint32_t stride, uint32_t* s_rows, uint32_t end, uint32_t pad)
{
    if (sizeof(E) == 2 && (end & 1u) && lane_id() == 0) {
        if (end < (uint32_t)kRowBuf) s_rows[end] = pad;
        else if (end < stride) blk[end] = (E)pad;
    }
}

// Keys of one cell against candidates held in registers: NACT chunks of 64
// (the cell's neighbourhood rounded up; the key loop is instantiated per
// chunk count, so the unrolled chunk sequence carries no branch).  Empty
// candidate slots carry a NaN x coordinate, so r2 < rs2 fails for them in
// both the plain and the minimum-image form of the test.  The own cell's
// particles come first among the candidates, so the key itself is candidate
// self_t < 64 of the first chunk, and only that chunk needs the test that
// drops it.  Output positions come from mbcnt of the row mask, counted on from
// the row's start.
//
// Half rows (HALF): the candidates are the own cell (ascending slots), then
// the cells of codes 14 .. 26, so "partner slot > key slot in the own cell" is
// "candidate number > self_t"; candidates up to self_t are dropped.
//
// Fast form (the key's row surely fits in the LDS row buffer): the row mask is
// the ballot of the distance test (minus the key's own lane in the first
// chunk), and the lanes in it store under that mask as the execution mask, at
// byte offsets formed by one shift-add from mbcnt (the mask moves to the
// scalar unit, which has room here, while the vector unit, which bounds the
// build, saves the select of a spare address per chunk).  The drop test is
// one vector compare of the lane against the key's place (a scalar mask built
// from that place would cost several scalar instructions).
template <bool MINIMG, int NACT, bool HALF>
__device__ __forceinline__ uint32_t row_chunks_lds(const BuildArgs& a, const double4& kp, int self_t,
                                                   uint32_t w0, const double* cx, const double* cy,
                                                   const double* cz, const uint32_t* meta, uint32_t* s_rows)
{
    const int lane = (int)lane_id();
    uint32_t wpos = w0;
#pragma unroll
    for (int ch = 0; ch < NACT; ++ch) {
        const double r2 = pair_r2<MINIMG>(a, cx[ch], cy[ch], cz[ch], kp.x, kp.y, kp.z);
        const bool in = r2 < a.rs2;
        uint64_t m = __builtin_amdgcn_ballot_w64(in);
        if (ch == 0) m &= ~__builtin_amdgcn_ballot_w64(HALF ? lane <= self_t : lane == self_t);
        if (__builtin_amdgcn_inverse_ballot_w64(m))
            *(uint32_t*)((char*)s_rows + ((mbcnt64(m) << 2) + 4u * wpos)) = meta[ch];
        wpos += (uint32_t)__popcll(m);
    }
    return wpos;
}

// General form: entries go to the LDS row buffer while they fit in it, past
// that straight to the cell block with a capacity test.
template <bool MINIMG, int NACT, typename E, bool HALF>
__device__ __forceinline__ uint32_t row_chunks(const BuildArgs& a, E* blk, uint32_t stride, const double4& kp,
                                               int self_t, uint32_t w0, const double* cx, const double* cy,
                                               const double* cz, const uint32_t* meta, uint32_t* s_rows)
{
    const int lane = (int)lane_id();
    uint32_t wpos = w0;
#pragma unroll
    for (int ch = 0; ch < NACT; ++ch) {
        const double r2 = pair_r2<MINIMG>(a, cx[ch], cy[ch], cz[ch], kp.x, kp.y, kp.z);
        const bool drop = ch == 0 && (HALF ? lane <= self_t : lane == self_t);
        const bool in = r2 < a.rs2 && !drop;
        const uint64_t m = __builtin_amdgcn_ballot_w64(in);
        const uint32_t w = mbcnt64(m) + wpos;
        if (in) {
            if (w < (uint32_t)kRowBuf) s_rows[w] = meta[ch];
            else if (w < stride) blk[w] = (E)meta[ch];
        }
        wpos += (uint32_t)__popcll(m);
    }
    return wpos;
}

template <bool MINIMG, int NACT, typename E, bool HALF>
__device__ __forceinline__ uint32_t rows_from_registers(const BuildArgs& a, E* blk, uint32_t stride,
                                                       int T, int own_pref, int own_cnt, const double4* s_key,
                                                       const double* cx, const double* cy, const double* cz,
                                                       const uint32_t* meta, uint32_t* s_rows, uint32_t* s_rowend,
                                                       uint32_t pad)
{
    uint32_t used = 0;
    for (int kk = 0; kk < own_cnt; ++kk) {
        if (used + (uint32_t)T <= (uint32_t)kRowBuf)
            used = row_chunks_lds<MINIMG, NACT, HALF>(a, s_key[kk], own_pref + kk, used, cx, cy, cz, meta, s_rows);
        else
            used = row_chunks<MINIMG, NACT, E, HALF>(a, blk, stride, s_key[kk], own_pref + kk, used, cx, cy, cz,
                                                     meta, s_rows);
        if (lane_id() == 0) s_rowend[kk] = used;
        pad_row<E>(blk, stride, s_rows, used, pad);
        used = row_start<E>(used);
    }
    __syncthreads();
    // the staged part of the block, then the row headers, with full-wave stores
    const uint32_t staged = min(min(used, (uint32_t)kRowBuf), stride);
    if (sizeof(E) == 2) {
        // two 16-bit entries per 32-bit store (rows start at even entries, the
        // block base is 4-byte aligned and staged is even)
        uint32_t* blk2 = (uint32_t*)blk;
        for (uint32_t t = lane_id(); 2 * t < staged; t += 64) {
            const uint2 v = *(const uint2*)(s_rows + 2 * t);
            blk2[t] = (v.x & 0xFFFFu) | (v.y << 16);
        }
    } else {
        for (uint32_t t = lane_id(); t < staged; t += 64) blk[t] = (E)s_rows[t];
    }
    const int kk = (int)lane_id();
    if (kk < own_cnt) {
        const uint32_t end = s_rowend[kk], beg = kk > 0 ? row_start<E>(s_rowend[kk - 1]) : 0u;
        write_row(a, (int32_t)__double_as_longlong(s_key[kk].w), (int64_t)(blk - (E*)a.nbr), beg, end - beg,
                  a.stride);
    }
    return used;
}

// Tiled rows.  The cells of a tile share one pooled block of tile_cells *
// cell_stride 16-bit entries (the first cell's block and those after it): a
// cell stages its rows in LDS as 16-bit entries, then takes its slice of the
// pool (one atomic add, or in cell order when one wave builds the tile) and
// writes it with full-wave 32-bit stores, so the pool has to hold the tile's
// total rather than every cell the largest cell's rows.  With a wave per cell
// the order of the slices inside a pool follows the order in which the cells
// finish.  A cell whose rows outgrow the LDS buffer counts the rest,
// takes its slice, and computes those rows again straight into it.

// 16-bit entries of one tiled cell staged in LDS (the row buffer, which first
// holds the candidate table): with the smaller register set of candidates,
// sized so that the block's LDS stays within 5 KB (32 blocks, 8 waves per SIMD)
template <int NCH>
constexpr int tiled_rowbuf_words()
{
    return NCH <= kBuildChunksSmall ? 608 : kRowBuf;
}
template <int NCH>
constexpr int rowbuf16()
{
    return 2 * tiled_rowbuf_words<NCH>();
}

// A cell's slice of its tile's pool: one atomic add on the tile's counter when
// every cell has a wave of its own; when one wave builds the tile's cells one
// after another (SEQ), the slices follow in cell order and the wave keeps the
// running offset itself.
template <bool SEQ>
__device__ __forceinline__ uint32_t reserve_slice(int lane, int32_t* tile_used, uint32_t seq_base, uint32_t used)
{
    if (SEQ) return seq_base;
    uint32_t base = 0;
    if (lane == 0) base = (uint32_t)atomicAdd(tile_used, (int32_t)used);
    return __builtin_amdgcn_readfirstlane(base);
}

template <bool MINIMG, int NACT, int NCH>
__device__ __forceinline__ uint32_t tiled_row_lds(const BuildArgs& a, int lane, const double4& kp, int self_t,
                                                  uint32_t w0, const double* cx, const double* cy, const double* cz,
                                                  const uint32_t* meta, uint16_t* s_rows16)
{
    uint32_t wpos = w0;
#pragma unroll
    for (int ch = 0; ch < NACT; ++ch) {
        const double r2 = pair_r2<MINIMG>(a, cx[ch], cy[ch], cz[ch], kp.x, kp.y, kp.z);
        const bool in = r2 < a.rs2;
        uint64_t m = __builtin_amdgcn_ballot_w64(in);
        if (ch == 0) m &= ~__builtin_amdgcn_ballot_w64(lane == self_t);
        if (__builtin_amdgcn_inverse_ballot_w64(m))
            *(uint16_t*)((char*)s_rows16 + ((mbcnt64(m) << 1) + 2u * wpos)) = (uint16_t)meta[ch];
        wpos += (uint32_t)__popcll(m);
    }
    return wpos;
}

// the same row, counted only (STORE = false) or written to dst[w0 ..]
template <bool MINIMG, int NACT, bool STORE>
__device__ __forceinline__ uint32_t tiled_row_direct(const BuildArgs& a, int lane, const double4& kp, int self_t,
                                                     uint32_t w0, const double* cx, const double* cy,
                                                     const double* cz, const uint32_t* meta, uint16_t* dst)
{
    uint32_t wpos = w0;
#pragma unroll
    for (int ch = 0; ch < NACT; ++ch) {
        const double r2 = pair_r2<MINIMG>(a, cx[ch], cy[ch], cz[ch], kp.x, kp.y, kp.z);
        const bool in = r2 < a.rs2 && (ch != 0 || lane != self_t);
        const uint64_t m = __builtin_amdgcn_ballot_w64(in);
        if (STORE && in) dst[mbcnt64(m) + wpos] = (uint16_t)meta[ch];
        wpos += (uint32_t)__popcll(m);
    }
    return wpos;
}

// One tiled cell: rows, its slice of the tile's pool and the row headers.
// Returns the entries the cell takes (even).
template <bool MINIMG, int NACT, int NCH, bool SEQ>
__device__ __forceinline__ uint32_t tiled_rows_from_registers(const BuildArgs& a, int lane, uint16_t* tblk,
                                                             uint64_t tcap, int32_t* tile_used, uint32_t seq_base,
                                                             int T, int own_pref, int own_cnt, const double4* s_key,
                                                             const double* cx, const double* cy, const double* cz,
                                                             const uint32_t* meta, uint16_t* s_rows16,
                                                             uint32_t* s_rowend, uint32_t pad)
{
    uint32_t used = 0;
    int kk = 0;
    // rows staged while they surely fit: a row adds at most T - 1 entries
    for (; kk < own_cnt && used + (uint32_t)T <= (uint32_t)rowbuf16<NCH>(); ++kk) {
        used = tiled_row_lds<MINIMG, NACT, NCH>(a, lane, s_key[kk], own_pref + kk, used, cx, cy, cz, meta, s_rows16);
        if (lane == 0) {
            s_rowend[kk] = used;
            if (used & 1u) s_rows16[used] = (uint16_t)pad;
        }
        used = (used + 1u) & ~1u;
    }
    const int ks = kk;
    const uint32_t staged = used;
    // the rest counted, then computed again into the slice below
    for (int k2 = ks; k2 < own_cnt; ++k2) {
        used = tiled_row_direct<MINIMG, NACT, false>(a, lane, s_key[k2], own_pref + k2, used, cx, cy, cz, meta, nullptr);
        if (lane == 0) s_rowend[k2] = used;
        used = (used + 1u) & ~1u;
    }
    const uint32_t base = reserve_slice<SEQ>(lane, tile_used, seq_base, used);
    const bool fits = (uint64_t)base + used <= tcap;
    if (!fits && lane == 0) atomicOr((unsigned long long*)&a.status[2], 1ull);
    __syncthreads();
    uint16_t* dst = tblk + base;
    if (fits) {
        // base and staged are even and the pool starts 4-byte aligned
        uint32_t* dst2 = (uint32_t*)dst;
        const uint32_t* src2 = (const uint32_t*)s_rows16;
        for (uint32_t t = lane; 2 * t < staged; t += 64) dst2[t] = src2[t];
        uint32_t w = staged;
        for (int k2 = ks; k2 < own_cnt; ++k2) {
            w = tiled_row_direct<MINIMG, NACT, true>(a, lane, s_key[k2], own_pref + k2, w, cx, cy, cz, meta, dst);
            if (lane == 0 && (w & 1u)) dst[w] = (uint16_t)pad;
            w = (w + 1u) & ~1u;
        }
    }
    if (lane < own_cnt) {
        const uint32_t end = s_rowend[lane], beg = lane > 0 ? (s_rowend[lane - 1] + 1u) & ~1u : 0u;
        const int32_t kslot = (int32_t)__double_as_longlong(s_key[lane].w);
        // an overflowed cell (list invalid) keeps in-range, empty rows
        a.offsets[kslot] = (int64_t)((fits ? dst : tblk) - (uint16_t*)a.nbr) + (fits ? beg : 0u);
        a.counts[kslot] = fits ? (int32_t)(end - beg) : 0;
    }
    return used;
}

template <bool MINIMG, int NCH, bool SEQ>
__device__ __forceinline__ uint32_t tiled_rows_for_chunks(int nact, const BuildArgs& a, int lane, uint16_t* tblk,
                                                         uint64_t tcap, int32_t* tile_used, uint32_t seq_base, int T,
                                                         int own_pref, int own_cnt, const double4* s_key,
                                                         const double* cx, const double* cy, const double* cz,
                                                         const uint32_t* meta, uint16_t* s_rows16, uint32_t* s_rowend,
                                                         uint32_t pad)
{
    static_assert(NCH >= 2 && NCH <= 8, "one case per chunk count");
#define MD_TROWS_CASE(N)                                                                                              \
    case N:                                                                                                           \
        if constexpr (N < NCH)                                                                                        \
            return tiled_rows_from_registers<MINIMG, N, NCH, SEQ>(a, lane, tblk, tcap, tile_used, seq_base, T, own_pref,  \
                                                             own_cnt, s_key, cx, cy, cz, meta, s_rows16, s_rowend, pad); \
        break;
    switch (nact) {
        MD_TROWS_CASE(1)
        MD_TROWS_CASE(2)
        MD_TROWS_CASE(3)
        MD_TROWS_CASE(4)
        MD_TROWS_CASE(5)
        MD_TROWS_CASE(6)
        MD_TROWS_CASE(7)
        default:
            break;
    }
#undef MD_TROWS_CASE
    return tiled_rows_from_registers<MINIMG, NCH, NCH, SEQ>(a, lane, tblk, tcap, tile_used, seq_base, T, own_pref, own_cnt, s_key,
                                                       cx, cy, cz, meta, s_rows16, s_rowend, pad);
}

// The key loop for the cell's chunk count nact in [1, NCH].
template <bool MINIMG, int NCH, typename E, bool HALF>
__device__ __forceinline__ uint32_t rows_for_chunks(int nact, const BuildArgs& a, E* blk, uint32_t stride, int T,
                                                   int own_pref, int own_cnt, const double4* s_key, const double* cx,
                                                   const double* cy, const double* cz, const uint32_t* meta,
                                                   uint32_t* s_rows, uint32_t* s_rowend, uint32_t pad)
{
    static_assert(NCH >= 2 && NCH <= 8, "one case per chunk count");
#define MD_ROWS_CASE(N)                                                                                             \
    case N:                                                                                                         \
        if constexpr (N < NCH)                                                                                      \
            return rows_from_registers<MINIMG, N, E, HALF>(a, blk, stride, T, own_pref, own_cnt, s_key, cx, cy, cz, \
                                                            meta, s_rows, s_rowend, pad);                           \
        break;
    switch (nact) {
        MD_ROWS_CASE(1)
        MD_ROWS_CASE(2)
        MD_ROWS_CASE(3)
        MD_ROWS_CASE(4)
        MD_ROWS_CASE(5)
        MD_ROWS_CASE(6)
        MD_ROWS_CASE(7)
        default:
            break;
    }
#undef MD_ROWS_CASE
    return rows_from_registers<MINIMG, NCH, E, HALF>(a, blk, stride, T, own_pref, own_cnt, s_key, cx, cy, cz, meta,
                                                     s_rows, s_rowend, pad);
}

// Same rows, candidates re-read from memory for every key (neighbourhoods with
// more than NCH*64 particles or cells with more than 64 particles: never at
// liquid densities, kept for generality).
// COUNT: only the rows' total (with the even starts of 16-bit rows) is
// returned, nothing is written.
template <bool MINIMG, typename E, bool HALF, bool COUNT = false>
__device__ uint32_t rows_from_memory(const BuildArgs& a, E* blk, uint32_t stride, int T, int own_start,
                                     int own_cnt, const int* s_pref, const int* s_nstart, const int* s_lbase,
                                     uint32_t pad)
{
    uint32_t used = 0;
    for (int kk = 0; kk < own_cnt; ++kk) {
        const int kidx = own_start + kk;
        const int32_t kslot = a.order ? a.order[kidx] : kidx;
        const double4 kp = a.pos[kslot];
        uint32_t wpos = 0;
        for (int t0 = 0; t0 < T; t0 += 64) {
            const int t = t0 + (int)lane_id();
            bool pass = false;
            uint32_t meta = 0;
            if (t < T) {
                int q = 0;
                while (s_pref[q + 1] <= t) ++q;
                const int idx = s_nstart[q] + (t - s_pref[q]);
                const int32_t slot = a.order ? a.order[idx] : idx;
                const double4 p = a.pos[slot];
                const double r2 = pair_r2<MINIMG>(a, p.x, p.y, p.z, kp.x, kp.y, kp.z);
                // q ranks the neighbour cells (rank 0 the own cell)
                pass = r2 < a.rs2 && (HALF ? (q > 0 || slot > kslot) : slot != kslot);
                meta = s_lbase ? (uint32_t)(s_lbase[q] + (t - s_pref[q])) << 4
                               : (uint32_t)slot | ((uint32_t)code_of_rank(q) << kCodeShift);
            }
            const uint64_t m = __ballot(pass);
            const uint32_t w = used + wpos + mbcnt64(m);
            if (!COUNT && pass && w < stride) blk[w] = (E)meta;
            wpos += (uint32_t)__popcll(m);
        }
        if (!COUNT && lane_id() == 0) {
            write_row(a, kslot, (int64_t)(blk - (E*)a.nbr), used, wpos, stride);
            if (sizeof(E) == 2 && ((used + wpos) & 1u) && used + wpos < stride) blk[used + wpos] = (E)pad;
        }
        used = row_start<E>(used + wpos);
    }
    return used;
}

// What a tiled build takes from the cell's tile: its z range, the pooled block
// of its list (the first cell's block and the blocks after it) and, for lane
// q < 27 (neighbour cell q, in column q / 3 of the tile's 3 x 3 columns), the
// two offsets that turn the start of that neighbour cell into the staged index
// of its first particle in the tile's neighbourhood: the staged layout is the 9
// column runs one after another (exclusive prefix of the run lengths), and a
// run that wraps around the box has a second segment.
struct TileCtx {
    int z0 = 0, z1 = 0, jw = 0;
    int offA = 0, offB = 0;
    uint32_t pad = 0;            // the stand-in partner of the force pass (staged total << 4)
    uint32_t total = 0;          // staged particles of the tile's neighbourhood
    uint16_t* tblk = nullptr;
    uint64_t tcap = 0;
    int32_t* tused = nullptr;    // entries taken so far in the tile's pool
    int64_t tile = 0;
};

// Lanes 0..8 hold the run of column `lane` as tile_run_load gives it.
__device__ __forceinline__ TileCtx tile_ctx(const BuildArgs& a, int cx, int cy, int tz, int z0, int z1,
                                            const TileRun& run)
{
    const int lane = (int)lane_id();
    TileCtx t;
    t.z0 = z0;
    t.z1 = z1;
    t.jw = tile_jw(z0, z1, a.nc[2]);
    const int len = lane < 9 ? run.lenA + run.lenB : 0;
    const int inc = scan_row16(len);
    t.total = (uint32_t)__builtin_amdgcn_readlane(inc, 8);
    const int col = lane < 27 ? code_of_rank(lane) / 3 : 0;
    const int cbase = __shfl(inc - len, col, 64);
    const int sA = __shfl(run.sA, col, 64), lenA = __shfl(run.lenA, col, 64), sB = __shfl(run.sB, col, 64);
    t.offA = cbase - sA;
    t.offB = cbase + lenA - sB;
    t.pad = t.total << 4;
    const int64_t colc = (int64_t)cx * a.nc[1] + cy;
    t.tblk = (uint16_t*)a.nbr + (colc * a.nc[2] + z0) * a.stride;
    t.tcap = (uint64_t)(z1 - z0) * (uint64_t)a.stride;
    t.tile = colc * a.nt + tz;
    t.tused = a.tile_used + t.tile;
    return t;
}

// The rows of one cell (cx, cy, cz), from the starts and counts of its 27
// neighbour cells (lane q < 27 holds those of cell q; half rows use q >= 13
// only).  Tiled: the cell's slice of the tile's pool is reserved by an atomic
// add or, SEQ, starts at seq_base.  Returns the entries the cell takes.
template <int NCH, bool TILED, bool HALF, bool SEQ>
__device__ __forceinline__ uint32_t build_cell(const BuildArgs& a, int cx, int cy, int cz, int st_l, int cnt_l,
                                               const TileCtx& tx, uint32_t seq_base)
{
    using E = typename std::conditional<TILED, uint16_t, uint32_t>::type;
    int lane = (int)lane_id();
    // opaque to the compiler when a wave builds several cells: the per-lane
    // addresses below are then formed per cell instead of being hoisted out of
    // the cell loop into registers that stay live across it
    if (SEQ) asm volatile("" : "+v"(lane));
    const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
    const int64_t c = ((int64_t)cx * ny + cy) * nz + cz;

    __shared__ int s_nstart[27];
    __shared__ int s_pref[28];
    __shared__ double4 s_key[kMaxOwn];
    // rows of the cell's keys before the block is written (and two words of
    // margin); before that, the candidate table
    constexpr int kRows = TILED ? tiled_rowbuf_words<NCH>() : kRowBuf;
    __shared__ __align__(8) uint32_t s_rows[kRows + 2];
    __shared__ uint32_t s_rowend[kMaxOwn];
    __shared__ int s_lbase[27];
    const bool has_nb = lane < 27 && (!HALF || lane <= 13);
    const int st = has_nb ? st_l : 0, cnt = has_nb ? cnt_l : 0;
    const int incl = scan_lanes32(cnt);
    if (lane < 27) {
        s_nstart[lane] = st;
        s_pref[lane + 1] = incl;
    }
    if (lane == 0) s_pref[0] = 0;
    int lb = 0;   // tiled: staged index of the first particle of this lane's cell
    if (TILED && lane < 27) {
        const int j = cz + code_of_rank(lane) % 3 - tx.z0;   // place of the neighbour cell in its column run
        lb = st + (j < tx.jw ? tx.offA : tx.offB);
        s_lbase[lane] = lb;
    }
    __syncthreads();

    const int T = s_pref[27];
    const uint32_t pad = TILED ? tx.pad : 0u;
    const int own_pref = 0;   // the own cell's particles are the first candidates
    const int own_start = s_nstart[0];
    const int own_cnt = s_pref[1];
    const bool minimg = a.exact_all || cx == 0 || cx == nx - 1 || cy == 0 || cy == ny - 1 || cz == 0 ||
                        cz == nz - 1;
    E* blk = (E*)a.nbr + c * a.stride;
    // capped so that byte offsets (entries << 2) fit in 32 bits
    const uint32_t stride = (uint32_t)(a.stride < (1 << 29) ? a.stride : (1 << 29));
    uint32_t used = 0;

    if (own_cnt > 0 && T <= NCH * 64 && own_cnt <= kMaxOwn) {
        // candidate table: for entry t, the candidate's position in the cell
        // order and (16 bits) its staged index in the tile's neighbourhood
        // (tiled) or its stencil code, written by the lane of its cell; it
        // lives in the row buffer, which is free until the rows are made
        static_assert(NCH * 64 * (sizeof(uint32_t) + sizeof(uint16_t)) <= sizeof(uint32_t) * (kRows + 2),
                      "table fits the row buffer");
        uint32_t* s_tpos = s_rows;
        uint16_t* s_tcode = reinterpret_cast<uint16_t*>(s_rows + NCH * 64);
        // two lanes per neighbour cell (lanes q and q + 32 for q < 27), each
        // writing every other entry of it
        {
            const int q = lane & 31;
            const int t0 = __shfl(incl - cnt, q, 64), stq = __shfl(st, q, 64), cq = __shfl(cnt, q, 64);
            const int eq = TILED ? __shfl(lb, q, 64) : code_of_rank(q);
            if (q < 27) {
                for (int i = lane >> 5; i < cq; i += 2) {
                    s_tpos[t0 + i] = (uint32_t)(stq + i);
                    s_tcode[t0 + i] = (uint16_t)(TILED ? eq + i : eq);
                }
            }
        }
        __syncthreads();
        double px[NCH], py[NCH], pz[NCH];
        uint32_t meta[NCH];
        const double qnan = __longlong_as_double(0x7FF8000000000000LL);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            px[ch] = py[ch] = pz[ch] = qnan;
            meta[ch] = 0;
            if (ch * 64 >= T) continue;          // uniform: chunk beyond the neighbourhood
            const int tq = ch * 64 + lane;
            const bool ok = tq < T;
            const int te = ok ? tq : T - 1;   // in-range entry; discarded if tq >= T
            const uint32_t ex = s_tpos[te], ey = s_tcode[te];
            const int32_t slot = a.order ? a.order[ex] : (int32_t)ex;
            const double4 p = a.pos[slot];
            // a NaN x alone fails the distance test in both forms of it
            px[ch] = ok ? p.x : qnan;
            py[ch] = p.y;
            pz[ch] = p.z;
            meta[ch] = TILED ? ey << 4 : ((uint32_t)slot | (ey << kCodeShift));
            if (ch == 0 && tq < own_cnt) s_key[tq] = make_double4(p.x, p.y, p.z, __longlong_as_double((long long)slot));
        }
        __syncthreads();
        const int nact = (T + 63) >> 6;
        if constexpr (TILED) {
            uint16_t* s_rows16 = reinterpret_cast<uint16_t*>(s_rows);
            used = minimg ? tiled_rows_for_chunks<true, NCH, SEQ>(nact, a, lane, tx.tblk, tx.tcap, tx.tused, seq_base, T,
                                                                  own_pref, own_cnt, s_key, px, py, pz, meta,
                                                                  s_rows16, s_rowend, pad)
                          : tiled_rows_for_chunks<false, NCH, SEQ>(nact, a, lane, tx.tblk, tx.tcap, tx.tused, seq_base, T,
                                                                   own_pref, own_cnt, s_key, px, py, pz, meta,
                                                                   s_rows16, s_rowend, pad);
        } else {
            used = minimg ? rows_for_chunks<true, NCH, E, HALF>(nact, a, blk, stride, T, own_pref, own_cnt, s_key,
                                                                px, py, pz, meta, s_rows, s_rowend, pad)
                          : rows_for_chunks<false, NCH, E, HALF>(nact, a, blk, stride, T, own_pref, own_cnt, s_key,
                                                                 px, py, pz, meta, s_rows, s_rowend, pad);
        }
    } else if (own_cnt > 0) {
        if constexpr (TILED) {
            // count the rows, take the cell's slice of the tile's pool, write
            const uint32_t total =
                minimg ? rows_from_memory<true, E, false, true>(a, nullptr, 0, T, own_start, own_cnt, s_pref,
                                                                s_nstart, s_lbase, pad)
                       : rows_from_memory<false, E, false, true>(a, nullptr, 0, T, own_start, own_cnt, s_pref,
                                                                 s_nstart, s_lbase, pad);
            const uint32_t base = reserve_slice<SEQ>(lane, tx.tused, seq_base, total);
            const bool fits = (uint64_t)base + total <= tx.tcap;
            if (!fits && lane == 0) atomicOr((unsigned long long*)&a.status[2], 1ull);
            // an overflowed cell writes empty rows (capacity 0)
            E* cblk = (E*)(fits ? tx.tblk + base : tx.tblk);
            const uint32_t cap = fits ? total : 0u;
            if (minimg)
                rows_from_memory<true, E, false>(a, cblk, cap, T, own_start, own_cnt, s_pref, s_nstart, s_lbase, pad);
            else
                rows_from_memory<false, E, false>(a, cblk, cap, T, own_start, own_cnt, s_pref, s_nstart, s_lbase, pad);
            used = total;
        } else {
            used = minimg ? rows_from_memory<true, E, HALF>(a, blk, stride, T, own_start, own_cnt, s_pref, s_nstart,
                                                            nullptr, pad)
                          : rows_from_memory<false, E, HALF>(a, blk, stride, T, own_start, own_cnt, s_pref,
                                                             s_nstart, nullptr, pad);
        }
    }
    if (lane == 0) {
        a.cell_rows[c] = used > 0x7FFFFFFFu ? 0x7FFFFFFF : (int32_t)used;
        if (!TILED && used > stride) atomicOr((unsigned long long*)&a.status[2], 1ull);
    }
    return used;
}

// One wave per cell, or (SEQ, tiled lists of large grids) one wave per tile
// that builds the tile's cells one after another along z: the cells' slices
// of the tile's pool then follow in cell order with no atomic, the tile's runs
// and staged layout are worked out once, and the next cell's neighbour starts
// and counts load while a cell is built.
template <int NCH, bool TILED, bool HALF, bool SEQ>
__global__ __launch_bounds__(64) void k_build(BuildArgs a)
{
    static_assert(!SEQ || (TILED && !HALF), "tile-sequential builds write tiled full rows");
    const int64_t tb = xcd_remap(blockIdx.x, gridDim.x);
    if (tb >= (SEQ ? a.ntile : a.ncell)) return;
    const int lane = (int)threadIdx.x;
    const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
    // cells (tiles) in strips of kBuildStrip x-columns walked along y (a
    // column's cells consecutive), so that cells built close in time share
    // their neighbour cells in L2 (ids < 2^31: 32-bit arithmetic, divisions
    // by the launch's multiply-shift divisors)
    const uint32_t t = (uint32_t)tb;
    const uint32_t seq = fdiv(t, SEQ ? a.div_nt : a.div_nz);
    const int zi = (int)(t - seq * (uint32_t)(SEQ ? a.nt : nz));   // the tile along z (SEQ), else the cell's z
    const uint32_t strip = fdiv(seq, a.div_strip);
    const uint32_t in = seq - strip * (uint32_t)(kBuildStrip * ny);
    const int sw = min(kBuildStrip, nx - (int)strip * kBuildStrip);
    uint32_t cyu;
    if (sw == kBuildStrip) cyu = in / (uint32_t)kBuildStrip;   // a power of two
    else cyu = in / (uint32_t)sw;                              // the last, narrower strip
    const int cy = (int)cyu, cx = (int)(strip * kBuildStrip + (in - cyu * (uint32_t)sw));

    // Every lane issues its loads before any result is used (a wait inside a
    // branch would serialise them): the neighbour cell of lanes 0..26, and,
    // tiled, the cells at the ends of the tile's column runs (lanes 0..8);
    // lanes without one load cell 0.  Half rows take candidates from the own
    // cell (code 13) and codes 14 .. 26 only: the other 13 cells count as empty.
    const bool has_nb = lane < 27 && (!HALF || lane <= 13);
    const int code = code_of_rank(lane);   // lanes 0 .. 26: the neighbour cells in candidate order
    int colb = 0;                          // first cell of the lane's neighbour column
    if (lane < 27) {
        const int ax = wrap_cell(cx + code / 9 - 1, nx), ay = wrap_cell(cy + (code / 3) % 3 - 1, ny);
        colb = (ax * ny + ay) * nz;
    }
    const int dz = code % 3 - 1;
    const int tz = SEQ ? zi : (TILED ? (int)fdiv((uint32_t)zi, a.div_tc) : 0);
    const int z0 = tz * a.tc, z1 = TILED ? min(z0 + a.tc, nz) : 0;
    const int cz0 = SEQ ? z0 : zi;   // the (first) cell built
    const int nb = has_nb ? colb + wrap_cell(cz0 + dz, nz) : 0;
    TileCells tcl;
    if (TILED) tcl = tile_run_cells(wrap_cell(cx + lane / 3 - 1, nx), wrap_cell(cy + lane % 3 - 1, ny), ny, nz, z0, z1,
                                    lane < 9);
    int st_l = a.start[nb], cnt_l = a.count[nb];
    TileRun run = {0, 0, 0, 0};
    if (TILED) run = tile_run_load(a.start, a.count, tcl);
    TileCtx tx;
    if (TILED) {
        tx = tile_ctx(a, cx, cy, tz, z0, z1, run);
        if (lane == 0 && cz0 == z0)
            atomicMax(a.tile_max + (tx.tile & (kTileMaxSlots - 1)), (unsigned long long)tx.total);
    }
    if constexpr (!SEQ) {
        build_cell<NCH, TILED, HALF, false>(a, cx, cy, cz0, st_l, cnt_l, tx, 0u);
    } else {
        uint32_t off = 0;
        for (int cz = z0; cz < z1; ++cz) {
            // the next cell's neighbour starts and counts, loaded while this
            // cell is built
            int st_n = 0, cnt_n = 0;
            if (cz + 1 < z1) {
                const int nbn = has_nb ? colb + wrap_cell(cz + 1 + dz, nz) : 0;
                st_n = a.start[nbn];
                cnt_n = a.count[nbn];
            }
            off += build_cell<NCH, true, false, true>(a, cx, cy, cz, st_l, cnt_l, tx, off);
            st_l = st_n;
            cnt_l = cnt_n;
            __syncthreads();
        }
        if (lane == 0) tx.tused[0] = (int32_t)off;
    }
}

// Stride a tiled list needs: the largest ceil(tile total / cells of the tile)
// over the tiles (block maxima, then one block), into status[1].  Tile totals
// and counts stay below 2^31.
constexpr int kNeedBlocks = 1024;
__device__ __forceinline__ int block_max_256(int m)
{
    __shared__ int s_m[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    return max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
}
__global__ __launch_bounds__(256) void k_tile_need(const int32_t* __restrict__ tile_used, int32_t ntile, int32_t nt,
                                                   int32_t tc, int32_t last_cells, int32_t* __restrict__ part)
{
    int m = 0;
    for (int t = blockIdx.x * 256 + threadIdx.x; t < ntile; t += gridDim.x * 256) {
        const int cells = (t % nt) == nt - 1 ? last_cells : tc;
        m = max(m, (tile_used[t] + cells - 1) / cells);
    }
    m = block_max_256(m);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}
__global__ __launch_bounds__(256) void k_tile_need_final(const int32_t* __restrict__ part, int nb,
                                                         int64_t* __restrict__ status)
{
    int m = 0;
    for (int b = threadIdx.x; b < nb; b += 256) m = max(m, part[b]);
    m = block_max_256(m);
    if (threadIdx.x == 0) status[1] = m;
}

hipError_t launch_build(const Geo& g, double rs, const double* pos, const md_cells& cells,
                        const md_pairlist& list, void* ws, const WsLayout& L, bool tiled, bool half,
                        unsigned long long* tile_max, int waves, hipStream_t s)
{
    int32_t* tile_used = (int32_t*)((char*)ws + L.tile_used);
    BuildArgs a;
    a.pos = (const double4*)pos;
    a.start = cells.start;
    a.count = cells.count;
    a.order = cells.sorted ? nullptr : cells.order;
    for (int k = 0; k < 3; ++k) {
        a.nc[k] = g.nc[k];
        a.L[k] = g.L[k];
        a.invL[k] = g.invL[k];
    }
    a.ncell = g.ncell;
    a.rs2 = rs * rs;
    a.exact_all = g.exact_all;
    a.stride = list.cell_stride;
    a.nbr = list.nbr;
    a.offsets = list.offsets;
    a.counts = list.counts;
    a.cell_rows = (int32_t*)((char*)ws + L.cell_rows);
    a.status = list.status;
    a.tc = g.tc;
    a.tile_max = tile_max;
    a.div_nz = make_fastdiv((uint32_t)g.nc[2]);
    a.div_strip = make_fastdiv((uint32_t)(kBuildStrip * g.nc[1]));
    a.div_tc = make_fastdiv((uint32_t)(g.tc > 0 ? g.tc : 1));
    a.nt = g.nt;
    a.tile_used = tile_used;
    a.ntile = g.ntile;
    a.div_nt = make_fastdiv((uint32_t)(g.nt > 0 ? g.nt : 1));
    if (tiled && (half || !cells.sorted || g.tc <= 0 || !tile_max)) return hipErrorInvalidValue;
    // one wave per tile where the tiles alone fill the GPU several times over
    // (below that, the cells' own waves keep more of it busy)
    const bool seq =
        tiled && (waves == MD_BUILD_TILE_WAVES || (waves == MD_BUILD_AUTO && g.ntile >= MD_BUILD_TILE_MIN));
    // status[2] (overflow) is cleared by the statistics kernel of the previous
    // build or by the caller; clear it here on the stream before the build.
    hipError_t e = launch_fill_i32((int32_t*)list.status, 0, 8, s);
    if (e != hipSuccess) return e;
    if (tiled && !seq && (e = launch_fill_i32(tile_used, 0, g.ntile, s)) != hipSuccess) return e;
    const dim3 grid((unsigned)(seq ? g.ntile : g.ncell));
    // candidates held in registers: 6 chunks of 64 (fewer registers, more
    // waves per SIMD) when a neighbourhood that large is far in the tail at
    // the mean density (4 standard deviations of a Poisson count above the
    // mean), else 8; larger neighbourhoods take the path that re-reads
    // memory for every key
    const double mean_t = (half ? 14.0 : 27.0) * (double)g.n / (double)g.ncell;
    const bool small = mean_t + 4.0 * std::sqrt(mean_t) <= (double)(kBuildChunksSmall * 64);
    if (seq) {
        if (small) hipLaunchKernelGGL((k_build<kBuildChunksSmall, true, false, true>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_build<kBuildChunks, true, false, true>), grid, dim3(64), 0, s, a);
    } else if (tiled) {
        if (small) hipLaunchKernelGGL((k_build<kBuildChunksSmall, true, false, false>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_build<kBuildChunks, true, false, false>), grid, dim3(64), 0, s, a);
    } else if (half) {
        if (small) hipLaunchKernelGGL((k_build<kBuildChunksSmall, false, true, false>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_build<kBuildChunks, false, true, false>), grid, dim3(64), 0, s, a);
    } else {
        if (small) hipLaunchKernelGGL((k_build<kBuildChunksSmall, false, false, false>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_build<kBuildChunks, false, false, false>), grid, dim3(64), 0, s, a);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_list_stats(a.cell_rows, g.ncell, list.status, (long long*)((char*)ws + L.red), s);
    if (e != hipSuccess || !tiled) return e;
    // the statistics are read: their scratch takes the tiles' block maxima
    int32_t* part = (int32_t*)((char*)ws + L.red);
    const int nb = (int)std::min<int64_t>(ceil_div(g.ntile, 256), kNeedBlocks);
    const int last_cells = g.nc[2] - (g.nt - 1) * g.tc;
    hipLaunchKernelGGL(k_tile_need, dim3(nb), dim3(256), 0, s, tile_used, (int32_t)g.ntile, g.nt, g.tc, last_cells,
                       part);
    hipLaunchKernelGGL(k_tile_need_final, dim3(1), dim3(256), 0, s, (const int32_t*)part, nb, list.status);
    return hipGetLastError();
}

}  // namespace md
