// Pair-list construction (Sec. 2.3 bookkeeping with search length rs; Sec. 2.4
// key-sorted list), one 64-lane wavefront per cell.
//
// The wave stages the particles of the 27 surrounding cells (~300 at
// rho = 0.5) in its registers, one candidate per lane per 64-chunk.  It then
// walks the keys of its own cell: each lane tests its candidates against the
// key with the exact FP64 predicate, a ballot gives the passing lanes, and the
// prefix popcount below each lane gives its output position, so every row is
// written compactly in candidate order (stencil code, then ascending slot)
// with no atomics.  Rows of one cell are packed one after another into the
// cell's block of the list; the block base is the cell id times a fixed stride,
// so cells never have to wait for each other.
//
// The work is ALU bound (about 300 FP64 distance tests per particle).

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
};

// r^2 of the pinned predicate: d = q_j - q_i, optional minimum image,
// r2 = fma(dz, dz, fma(dy, dy, dx * dx)).
template <bool MINIMG>
__device__ __forceinline__ double pair_r2(const BuildArgs& a, double xj, double yj, double zj, double xi,
                                          double yi, double zi)
{
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    if (MINIMG) {
        dx = dx - a.L[0] * rint(dx * a.invL[0]);
        dy = dy - a.L[1] * rint(dy * a.invL[1]);
        dz = dz - a.L[2] * rint(dz * a.invL[2]);
    }
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, __dmul_rn(dx, dx)));
}

// Row header of one key.  When the cell block overflows, the row is clipped to
// the entries actually stored, so an invalid (overflowed) list still only
// references written, in-range entries.
__device__ __forceinline__ void write_row(const BuildArgs& a, int32_t kslot, int64_t base, int64_t used,
                                          int64_t wpos)
{
    const int64_t start = used < a.stride ? used : a.stride;
    const int64_t room = a.stride - start;
    a.offsets[kslot] = base + start;
    a.counts[kslot] = (int32_t)(wpos < room ? wpos : room);
}

constexpr int kMaxOwn = 64;     // own-cell particles kept in LDS for the key loop
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

constexpr int kRowBuf = 1024;   // entries of one cell's rows staged in LDS before the block is written

template <typename E>
__device__ __forceinline__ void pad_row(E* blk, uint32_t stride, uint32_t* s_rows, uint32_t end, uint32_t pad)
{
    if (sizeof(E) == 2 && (end & 1u) && lane_id() == 0) {
        if (end < (uint32_t)kRowBuf) s_rows[end] = pad;
        else if (end < stride) blk[end] = (E)pad;
    }
}

// Keys of one cell against candidates held in registers (at most NCH*64).
// Empty candidate slots carry NaN coordinates, so r2 < rs2 fails for them in
// both the plain and the minimum-image form of the test.  The key itself is
// candidate number self_t.  Output positions come from mbcnt of the row mask,
// counted on from the row's start.
//
// Half rows (HALF): the candidates are the own cell first (ascending slots),
// then the cells of codes 14 .. 26, so "partner slot > key slot in the own
// cell" is "candidate number > self_t"; candidates up to self_t are dropped.
//
// Fast form (the key's row surely fits in the LDS row buffer): the row mask is
// the ballot of the distance test minus the key's own lane; every lane stores,
// those outside the mask into a spare LDS word, so there is no branch and no
// exec-mask change per chunk.
template <bool MINIMG, int NCH, bool HALF>
__device__ __forceinline__ uint32_t row_chunks_lds(const BuildArgs& a, int T, const double4& kp, int self_t,
                                                   uint32_t w0, const double* cx, const double* cy,
                                                   const double* cz, const uint32_t* meta, uint32_t* s_rows)
{
    const int lane = (int)lane_id();
    uint32_t wpos = w0;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        if (ch * 64 < T) {
            const double r2 = pair_r2<MINIMG>(a, cx[ch], cy[ch], cz[ch], kp.x, kp.y, kp.z);
            const bool in = r2 < a.rs2;
            const bool self = HALF ? ch * 64 + lane <= self_t : lane == self_t - ch * 64;
            const uint64_t m = __builtin_amdgcn_ballot_w64(in) & ~__builtin_amdgcn_ballot_w64(self);
            const uint32_t wb = (mbcnt64(m) + wpos) << 2;   // byte offset in the row buffer
            *(uint32_t*)((char*)s_rows + (__builtin_amdgcn_inverse_ballot_w64(m) ? wb : 4u * kRowBuf)) = meta[ch];
            wpos += (uint32_t)__popcll(m);
        }
    }
    return wpos;
}

// General form: entries go to the LDS row buffer while they fit in it, past
// that straight to the cell block with a capacity test.
template <bool MINIMG, int NCH, typename E, bool HALF>
__device__ __forceinline__ uint32_t row_chunks(const BuildArgs& a, E* blk, uint32_t stride, int T,
                                               const double4& kp, int self_t, uint32_t w0, const double* cx,
                                               const double* cy, const double* cz, const uint32_t* meta,
                                               uint32_t* s_rows)
{
    const int lane = (int)lane_id();
    uint32_t wpos = w0;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        if (ch * 64 < T) {
            const double r2 = pair_r2<MINIMG>(a, cx[ch], cy[ch], cz[ch], kp.x, kp.y, kp.z);
            const bool in = r2 < a.rs2;
            uint64_t m = __builtin_amdgcn_ballot_w64(in);
            const int sl = self_t - ch * 64;          // the key's own lane in this chunk, if any
            const bool drop = HALF ? lane <= sl : lane == sl;
            if (HALF) m &= ~__builtin_amdgcn_ballot_w64(drop);
            else if (sl >= 0 && sl < 64) m &= ~(1ull << sl);
            const uint32_t w = mbcnt64(m) + wpos;
            if (in && !drop) {
                if (w < (uint32_t)kRowBuf) s_rows[w] = meta[ch];
                else if (w < stride) blk[w] = (E)meta[ch];
            }
            wpos += (uint32_t)__popcll(m);
        }
    }
    return wpos;
}

template <bool MINIMG, int NCH, typename E, bool HALF>
__device__ __forceinline__ uint32_t rows_from_registers(const BuildArgs& a, E* blk, uint32_t stride,
                                                       int T, int own_pref, int own_cnt, const double4* s_key,
                                                       const double* cx, const double* cy, const double* cz,
                                                       const uint32_t* meta, uint32_t* s_rows, uint32_t* s_rowend,
                                                       uint32_t pad)
{
    uint32_t used = 0;
    for (int kk = 0; kk < own_cnt; ++kk) {
        if (used + (uint32_t)T <= (uint32_t)kRowBuf)
            used = row_chunks_lds<MINIMG, NCH, HALF>(a, T, s_key[kk], own_pref + kk, used, cx, cy, cz, meta,
                                                     s_rows);
        else
            used = row_chunks<MINIMG, NCH, E, HALF>(a, blk, stride, T, s_key[kk], own_pref + kk, used, cx, cy, cz,
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
        write_row(a, (int32_t)__double_as_longlong(s_key[kk].w), (int64_t)(blk - (E*)a.nbr), beg, end - beg);
    }
    return used;
}

// Same rows, candidates re-read from memory for every key (neighbourhoods with
// more than NCH*64 particles or cells with more than 64 particles: never at
// liquid densities, kept for generality).
template <bool MINIMG, typename E, bool HALF>
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
                pass = r2 < a.rs2 && (HALF ? (q > 13 || slot > kslot) : slot != kslot);
                meta = s_lbase ? (uint32_t)(s_lbase[q] + (t - s_pref[q])) << 4
                               : (uint32_t)slot | ((uint32_t)q << kCodeShift);
            }
            const uint64_t m = __ballot(pass);
            const uint32_t w = used + wpos + mbcnt64(m);
            if (pass && w < stride) blk[w] = (E)meta;
            wpos += (uint32_t)__popcll(m);
        }
        if (lane_id() == 0) {
            write_row(a, kslot, (int64_t)(blk - (E*)a.nbr), used, wpos);
            if (sizeof(E) == 2 && ((used + wpos) & 1u) && used + wpos < stride) blk[used + wpos] = (E)pad;
        }
        used = row_start<E>(used + wpos);
    }
    return used;
}

template <int NCH, bool TILED, bool HALF>
__global__ __launch_bounds__(64) void k_build(BuildArgs a)
{
    using E = typename std::conditional<TILED, uint16_t, uint32_t>::type;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    if (t >= a.ncell) return;
    const int lane = (int)threadIdx.x;
    const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
    // cells in strips of kBuildStrip x-columns walked along y (a column's
    // cells consecutive), so that cells built close in time share their
    // neighbour cells in L2
    const int cz = (int)(t % nz);
    const int64_t seq = t / nz;
    const int64_t strip = seq / ((int64_t)kBuildStrip * ny);
    const int sw = (int)min((int64_t)kBuildStrip, (int64_t)nx - strip * kBuildStrip);
    const int64_t in = seq - strip * kBuildStrip * ny;
    const int cy = (int)(in / sw), cx = (int)(strip * kBuildStrip + in % sw);
    const int64_t c = ((int64_t)cx * ny + cy) * nz + cz;

    __shared__ int s_nstart[27];
    __shared__ int s_pref[28];
    __shared__ double4 s_key[kMaxOwn];
    __shared__ __align__(8) uint32_t s_rows[kRowBuf + 2];   // + a spare word for lanes that store nothing
    __shared__ uint32_t s_rowend[kMaxOwn];
    __shared__ int s_lbase[27];
    __shared__ uint32_t s_pad;
    // tiled: the tile's 9 column runs (lanes 0..8), loaded together with the
    // neighbour cells below
    const int z0 = TILED ? (cz / a.tc) * a.tc : 0, z1 = TILED ? min(z0 + a.tc, nz) : 0;
    TileRun run = {0, 0, 0, 0};
    if (TILED && lane < 9)
        run = tile_run(a.start, a.count, wrap_cell(cx + lane / 3 - 1, nx), wrap_cell(cy + lane % 3 - 1, ny), ny, nz,
                       z0, z1);
    // half rows take candidates from the own cell (code 13) and codes 14 .. 26
    // only: the other 13 cells count as empty
    int cnt = 0, st = 0;
    if (lane < 27 && (!HALF || lane >= 13)) {
        int ax = cx + lane / 9 - 1, ay = cy + (lane / 3) % 3 - 1, az = cz + lane % 3 - 1;
        ax += ax < 0 ? nx : 0;
        ax -= ax >= nx ? nx : 0;
        ay += ay < 0 ? ny : 0;
        ay -= ay >= ny ? ny : 0;
        az += az < 0 ? nz : 0;
        az -= az >= nz ? nz : 0;
        const int64_t nb = ((int64_t)ax * ny + ay) * nz + az;
        st = a.start[nb];
        cnt = a.count[nb];
    }
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane < 27) {
        s_nstart[lane] = st;
        s_pref[lane + 1] = incl;
    }
    if (lane == 0) s_pref[0] = 0;
    if (TILED) {
        // the tile's staged layout: the bases of the 9 column runs (exclusive
        // prefix of the run lengths), then the staged index of
        // the first particle of each neighbour cell q (lanes 0..26; q / 3 is
        // the column of q)
        const int jw = tile_jw(z0, z1, nz);
        const int len = lane < 9 ? run.lenA + run.lenB : 0;
        int inc = len;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        const int total = __shfl(inc, 8, 64);
        const int col = lane < 27 ? lane / 3 : 0;
        const int cbase = __shfl(inc - len, col, 64);
        const int sA = __shfl(run.sA, col, 64), lenA = __shfl(run.lenA, col, 64), sB = __shfl(run.sB, col, 64);
        if (lane < 27) {
            const int j = cz + lane % 3 - 1 - z0 + 1;
            s_lbase[lane] = cbase + (j < jw ? st - sA : lenA + st - sB);
        }
        if (lane == 0) {
            s_pad = (uint32_t)total << 4;   // the stand-in partner of the force pass
            if (cz == z0) {
                const int64_t tile = ((int64_t)cx * ny + cy) * ((nz + a.tc - 1) / a.tc) + cz / a.tc;
                atomicMax(a.tile_max + (tile & (kTileMaxSlots - 1)), (unsigned long long)total);
            }
        }
    }
    __syncthreads();

    const int T = s_pref[27];
    const uint32_t pad = TILED ? s_pad : 0u;
    const int own_pref = s_pref[13];
    const int own_start = s_nstart[13];
    const int own_cnt = s_pref[14] - own_pref;
    const bool minimg = a.exact_all || cx == 0 || cx == nx - 1 || cy == 0 || cy == ny - 1 || cz == 0 ||
                        cz == nz - 1;
    E* blk = (E*)a.nbr + c * a.stride;
    // capped so that byte offsets (entries << 2) fit in 32 bits
    const uint32_t stride = (uint32_t)(a.stride < (1 << 29) ? a.stride : (1 << 29));
    uint32_t used = 0;

    if (own_cnt > 0 && T <= NCH * 64 && own_cnt <= kMaxOwn) {
        double px[NCH], py[NCH], pz[NCH];
        uint32_t meta[NCH];
        const double qnan = __longlong_as_double(0x7FF8000000000000LL);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            px[ch] = py[ch] = pz[ch] = qnan;
            meta[ch] = 0;
            if (ch * 64 >= T) continue;          // uniform: chunk beyond the neighbourhood
            const int t = ch * 64 + lane;
            const int tt = t < T ? t : T - 1;   // in-range index; the result is discarded if t >= T
            // neighbour cell holding candidate tt: binary search in the prefix
            int lo = 0, hi = 27;
#pragma unroll
            for (int it = 0; it < 5; ++it) {
                const int mid = (lo + hi) >> 1;
                const bool le = s_pref[mid] <= tt;
                lo = le ? mid : lo;
                hi = le ? hi : mid;
            }
            const int idx = s_nstart[lo] + (tt - s_pref[lo]);
            const int32_t slot = a.order ? a.order[idx] : idx;
            const double4 p = a.pos[slot];
            const bool ok = t < T;
            px[ch] = ok ? p.x : qnan;
            py[ch] = ok ? p.y : qnan;
            pz[ch] = ok ? p.z : qnan;
            meta[ch] = TILED ? (uint32_t)(s_lbase[lo] + (tt - s_pref[lo])) << 4
                             : (uint32_t)slot | ((uint32_t)lo << kCodeShift);
            const int k = t - own_pref;
            if (ok && k >= 0 && k < own_cnt) s_key[k] = make_double4(p.x, p.y, p.z, __longlong_as_double((long long)slot));
        }
        __syncthreads();
        used = minimg ? rows_from_registers<true, NCH, E, HALF>(a, blk, stride, T, own_pref, own_cnt, s_key, px,
                                                                py, pz, meta, s_rows, s_rowend, pad)
                      : rows_from_registers<false, NCH, E, HALF>(a, blk, stride, T, own_pref, own_cnt, s_key, px,
                                                                 py, pz, meta, s_rows, s_rowend, pad);
    } else if (own_cnt > 0) {
        const int* lb = TILED ? s_lbase : nullptr;
        used = minimg ? rows_from_memory<true, E, HALF>(a, blk, stride, T, own_start, own_cnt, s_pref, s_nstart,
                                                        lb, pad)
                      : rows_from_memory<false, E, HALF>(a, blk, stride, T, own_start, own_cnt, s_pref, s_nstart,
                                                         lb, pad);
    }
    if (lane == 0) {
        a.cell_rows[c] = used > 0x7FFFFFFFu ? 0x7FFFFFFF : (int32_t)used;
        if (used > stride) atomicOr((unsigned long long*)&a.status[2], 1ull);
    }
}

hipError_t launch_build(const Geo& g, double rs, const double* pos, const md_cells& cells,
                        const md_pairlist& list, void* ws, const WsLayout& L, bool tiled, bool half,
                        unsigned long long* tile_max, hipStream_t s)
{
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
    if (tiled && (half || !cells.sorted || g.tc <= 0 || !tile_max)) return hipErrorInvalidValue;
    // status[2] (overflow) is cleared by the statistics kernel of the previous
    // build or by the caller; clear it here on the stream before the build.
    hipError_t e = launch_fill_i32((int32_t*)list.status, 0, 8, s);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)g.ncell);
    if (tiled) hipLaunchKernelGGL((k_build<kBuildChunks, true, false>), grid, dim3(64), 0, s, a);
    else if (half) hipLaunchKernelGGL((k_build<kBuildChunks, false, true>), grid, dim3(64), 0, s, a);
    else hipLaunchKernelGGL((k_build<kBuildChunks, false, false>), grid, dim3(64), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_list_stats(a.cell_rows, g.ncell, list.status, (long long*)((char*)ws + L.red), s);
}

}  // namespace md
