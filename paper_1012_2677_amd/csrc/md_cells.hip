// Cell grid and re-sort kernels (Sec. 2.2 GridList, Sec. 3.3 re-sort).
//
// GridList on the GPU: a thread per slot labels it with its cell and takes a
// rank inside the cell with an integer atomic; a three-phase scan turns the
// per-cell counts into pointers; ranks place the slots; finally every cell's
// segment is sorted by slot, which makes the result identical to the
// sequential counting sort that visits particles in index order (stable).
// All passes are integer work and read/write each array once, so they are
// bound by HBM bandwidth.

#include "md_internal.h"

namespace md {

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(count, kStreamBlock)), dim3(kStreamBlock),
                       0, s, p, v, count);
    return hipGetLastError();
}

// ---- label + count ---------------------------------------------------------
__global__ __launch_bounds__(kStreamBlock) void k_label(Geo g, const double4* __restrict__ pos,
                                                        int32_t* __restrict__ cell_of,
                                                        int32_t* __restrict__ cell_xyz,
                                                        int32_t* __restrict__ count,
                                                        int32_t* __restrict__ rank,
                                                        int64_t* __restrict__ err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const double4 p = pos[i];
    const bool inside = p.x >= 0.0 && p.x < g.L[0] && p.y >= 0.0 && p.y < g.L[1] && p.z >= 0.0 &&
                        p.z < g.L[2];
    if (!inside) atomicOr((unsigned long long*)err, 2ull);
    const int cx = cell_coord(p.x, g.inv[0], g.nc[0]);
    const int cy = cell_coord(p.y, g.inv[1], g.nc[1]);
    const int cz = cell_coord(p.z, g.inv[2], g.nc[2]);
    const int32_t c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
    cell_of[i] = c;
    cell_xyz[i] = cx | (cy << 10) | (cz << 20);
    // Slots in cell order (after a re-sort) put runs of equal cells in one
    // wave: the lanes are grouped by cell first, then the first lane of each
    // group adds the group's size with one atomic, all groups' atomics issued
    // together; ranks follow lane order inside a group (the order within a
    // cell is made stable afterwards by k_sort_cells).
    uint64_t todo = __ballot(1);
    int leader_of = 0;
    uint64_t group = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t cl = __shfl(c, leader, 64);
        const uint64_t same = __ballot(c == cl);
        if (c == cl) {
            leader_of = leader;
            group = same;
        }
        todo &= ~same;
    }
    int32_t base = 0;
    if ((int)lane_id() == leader_of) base = atomicAdd(&count[c], (int32_t)__popcll(group));
    base = __shfl(base, leader_of, 64);
    rank[i] = base + (int32_t)mbcnt64(group);
}

// ---- three-phase exclusive scan of int32 (block: 256 threads x 4 items) -----
__device__ __forceinline__ int32_t block_excl_scan_256(int32_t v, int32_t* total)
{
    // inclusive wave scan
    __shared__ int32_t s_wave[kStreamBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int32_t wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kStreamBlock / 64; ++w) {
        const int32_t t = s_wave[w];
        if (w < wave) wbase += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

__global__ __launch_bounds__(kStreamBlock) void k_scan_partial(const int32_t* __restrict__ in, int64_t m,
                                                               int32_t* __restrict__ bsum)
{
    const int64_t base = (int64_t)blockIdx.x * kScanItems + threadIdx.x * 4;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < m) s += in[base + k];
    int32_t tot;
    block_excl_scan_256(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// one block: exclusive scan of the block sums in place, total into bsum[nb]
__global__ __launch_bounds__(kStreamBlock) void k_scan_bsums(int32_t* __restrict__ bsum, int64_t nb)
{
    const int64_t per = ceil_div(nb, kStreamBlock);
    const int64_t b0 = threadIdx.x * per;
    int32_t s = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) s += bsum[b0 + k];
    int32_t tot;
    int32_t run = block_excl_scan_256(s, &tot);
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) {
            const int32_t v = bsum[b0 + k];
            bsum[b0 + k] = run;
            run += v;
        }
    if (threadIdx.x == 0) bsum[nb] = tot;
}

__global__ __launch_bounds__(kStreamBlock) void k_scan_final(const int32_t* __restrict__ in, int64_t m,
                                                             const int32_t* __restrict__ bsum,
                                                             int64_t nb, int32_t* __restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanItems + threadIdx.x * 4;
    int32_t v[4];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < m) ? in[base + k] : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t run = block_excl_scan_256(s, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[m] = bsum[nb];
}

// ---- place + per-cell sort ---------------------------------------------------
__global__ __launch_bounds__(kStreamBlock) void k_scatter(int64_t n, const int32_t* __restrict__ cell_of,
                                                          const int32_t* __restrict__ rank,
                                                          const int32_t* __restrict__ start,
                                                          int32_t* __restrict__ order)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    order[start[cell_of[i]] + rank[i]] = (int32_t)i;
}

// Insertion sort of each cell's segment by slot (segments hold ~11 slots at
// rho = 0.5; any length is handled).
// Insertion sort of each cell's slots (the scatter leaves the groups of
// different waves in atomic order).  A block's cells are contiguous in
// `order`: when their slots fit, they are loaded into LDS with coalesced
// loads, sorted there (one thread per cell) and written back; otherwise each
// thread sorts its cell in place in global memory.
constexpr int kSortLds = 4096;   // slots of one block's cells sorted in LDS

__device__ __forceinline__ void insertion_sort(int32_t* v, int32_t len)
{
    for (int32_t k = 1; k < len; ++k) {
        const int32_t x = v[k];
        int32_t p = k - 1;
        while (p >= 0 && v[p] > x) {
            v[p + 1] = v[p];
            --p;
        }
        v[p + 1] = x;
    }
}

__global__ __launch_bounds__(kStreamBlock) void k_sort_cells(int64_t ncell, const int32_t* __restrict__ start,
                                                             int32_t* __restrict__ order)
{
    __shared__ int32_t s_o[kSortLds];
    const int64_t c0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t c1 = c0 + blockDim.x < ncell ? c0 + blockDim.x : ncell;
    const int64_t c = c0 + threadIdx.x;
    const int32_t b0 = start[c0], b1 = start[c1];
    if (b1 - b0 <= kSortLds) {
        for (int32_t t = threadIdx.x; t < b1 - b0; t += blockDim.x) s_o[t] = order[b0 + t];
        __syncthreads();
        if (c < c1) insertion_sort(s_o + (start[c] - b0), start[c + 1] - start[c]);
        __syncthreads();
        for (int32_t t = threadIdx.x; t < b1 - b0; t += blockDim.x) order[b0 + t] = s_o[t];
    } else if (c < c1) {
        insertion_sort(order + start[c], start[c + 1] - start[c]);
    }
}

// ---- the same for small systems in one block --------------------------------
// Label, count (LDS atomics), exclusive scan, place and per-cell sort in one
// launch of one block: the same count, start, cell_of, cell_xyz and (sorted)
// order as the kernels above, without their seven launches, which dominate
// a rebuild of a few thousand particles.
constexpr int kBinSmallThreads = 1024;
constexpr int64_t kBinSmallN = 65536;
constexpr int64_t kBinSmallCells = 4096;

__global__ __launch_bounds__(kBinSmallThreads) void k_bin_small(Geo g, const double4* __restrict__ pos,
                                                                int32_t* __restrict__ cell_of,
                                                                int32_t* __restrict__ cell_xyz,
                                                                int32_t* __restrict__ count,
                                                                int32_t* __restrict__ start,
                                                                int32_t* __restrict__ order,
                                                                int32_t* __restrict__ rank,
                                                                int64_t* __restrict__ err)
{
    __shared__ int32_t s_cnt[kBinSmallCells];
    __shared__ int32_t s_wave[kBinSmallThreads / 64];
    const int tid = threadIdx.x;
    const int nc = (int)g.ncell;
    const int n = (int)g.n;
    for (int c = tid; c < nc; c += kBinSmallThreads) s_cnt[c] = 0;
    __syncthreads();
    bool outside = false;
    for (int i = tid; i < n; i += kBinSmallThreads) {
        const double4 p = pos[i];
        outside |= !(p.x >= 0.0 && p.x < g.L[0] && p.y >= 0.0 && p.y < g.L[1] && p.z >= 0.0 && p.z < g.L[2]);
        const int cx = cell_coord(p.x, g.inv[0], g.nc[0]);
        const int cy = cell_coord(p.y, g.inv[1], g.nc[1]);
        const int cz = cell_coord(p.z, g.inv[2], g.nc[2]);
        const int32_t c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
        cell_of[i] = c;
        cell_xyz[i] = cx | (cy << 10) | (cz << 20);
        rank[i] = atomicAdd(&s_cnt[c], 1);
    }
    if (outside) atomicOr((unsigned long long*)err, 2ull);
    __syncthreads();
    // exclusive scan of the counts: each thread takes a contiguous run of
    // cells, then a scan of the runs' totals over the block
    const int per = (nc + kBinSmallThreads - 1) / kBinSmallThreads;
    const int c0 = min(tid * per, nc), c1 = min(c0 + per, nc);
    int32_t run = 0;
    for (int c = c0; c < c1; ++c) run += s_cnt[c];
    const int lane = tid & 63, wave = tid >> 6;
    int32_t x = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int32_t base = x - run;
    for (int w2 = 0; w2 < wave; ++w2) base += s_wave[w2];
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
        const int32_t v = s_cnt[c];
        count[c] = v;
        start[c] = base;
        s_cnt[c] = base;
        base += v;
    }
    if (tid == 0) start[nc] = n;
    __syncthreads();
    for (int i = tid; i < n; i += kBinSmallThreads) order[s_cnt[cell_of[i]] + rank[i]] = i;
    __syncthreads();
    for (int c = tid; c < nc; c += kBinSmallThreads) insertion_sort(order + start[c], count[c]);
}

hipError_t launch_bin(const Geo& g, const double* pos, const md_cells& cells, void* ws,
                      const WsLayout& L, int64_t* err_flags, hipStream_t s)
{
    char* w = (char*)ws;
    int32_t* rank = (int32_t*)(w + L.rank);
    int32_t* bsum = (int32_t*)(w + L.bsum);
    if (g.n <= kBinSmallN && g.ncell <= kBinSmallCells) {
        hipLaunchKernelGGL(k_bin_small, dim3(1), dim3(kBinSmallThreads), 0, s, g, (const double4*)pos,
                           cells.cell_of, cells.cell_xyz, cells.count, cells.start, cells.order, rank, err_flags);
        return hipGetLastError();
    }
    hipError_t e = launch_fill_i32(cells.count, 0, g.ncell, s);
    if (e != hipSuccess) return e;
    const unsigned nbn = (unsigned)ceil_div(g.n, kStreamBlock);
    hipLaunchKernelGGL(k_label, dim3(nbn), dim3(kStreamBlock), 0, s, g, (const double4*)pos,
                       cells.cell_of, cells.cell_xyz, cells.count, rank, err_flags);
    const int64_t nbs = ceil_div(g.ncell, kScanItems);
    hipLaunchKernelGGL(k_scan_partial, dim3((unsigned)nbs), dim3(kStreamBlock), 0, s,
                       (const int32_t*)cells.count, g.ncell, bsum);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kStreamBlock), 0, s, bsum, nbs);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nbs), dim3(kStreamBlock), 0, s,
                       (const int32_t*)cells.count, g.ncell, (const int32_t*)bsum, nbs, cells.start);
    hipLaunchKernelGGL(k_scatter, dim3(nbn), dim3(kStreamBlock), 0, s, g.n,
                       (const int32_t*)cells.cell_of, (const int32_t*)rank,
                       (const int32_t*)cells.start, cells.order);
    hipLaunchKernelGGL(k_sort_cells, dim3((unsigned)ceil_div(g.ncell, kStreamBlock)), dim3(kStreamBlock),
                       0, s, g.ncell, (const int32_t*)cells.start, cells.order);
    return hipGetLastError();
}

// ---- local (cell-corner) coordinates for the mixed-precision force -----------
// l = x - c * cs, taken as the periodic image nearest the cell, rounded to FP32.
__device__ __forceinline__ float local_coord(double x, int c, double cs, double L, double invL)
{
    double l = x - (double)c * cs;
    l -= L * rint((l - 0.5 * cs) * invL);
    return (float)l;
}

// ---- re-sort: gather every per-particle array into cell order ---------------
__global__ __launch_bounds__(kStreamBlock) void k_resort(Geo g, const int32_t* __restrict__ order,
                                                         const double4* __restrict__ pos,
                                                         const double* __restrict__ vel,
                                                         const int32_t* __restrict__ id,
                                                         double4* __restrict__ pos_alt,
                                                         double* __restrict__ vel_alt,
                                                         int32_t* __restrict__ id_alt,
                                                         double* __restrict__ pos_ref,
                                                         float4* __restrict__ pos32,
                                                         int32_t* __restrict__ cell_of,
                                                         int32_t* __restrict__ cell_xyz)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.n) return;
    const int64_t n = g.n;
    const int64_t src = order[k];
    const double4 p = pos[src];
    pos_alt[k] = p;
    vel_alt[k] = vel[src];
    vel_alt[n + k] = vel[n + src];
    vel_alt[2 * n + k] = vel[2 * n + src];
    id_alt[k] = id[src];
    pos_ref[k] = p.x;
    pos_ref[n + k] = p.y;
    pos_ref[2 * n + k] = p.z;
    const int cx = cell_coord(p.x, g.inv[0], g.nc[0]);
    const int cy = cell_coord(p.y, g.inv[1], g.nc[1]);
    const int cz = cell_coord(p.z, g.inv[2], g.nc[2]);
    cell_of[k] = (cx * g.nc[1] + cy) * g.nc[2] + cz;
    cell_xyz[k] = cx | (cy << 10) | (cz << 20);
    if (pos32) {
        pos32[k] = make_float4(local_coord(p.x, cx, g.cs[0], g.L[0], g.invL[0]),
                               local_coord(p.y, cy, g.cs[1], g.L[1], g.invL[1]),
                               local_coord(p.z, cz, g.cs[2], g.L[2], g.invL[2]),
                               __int_as_float(cx | (cy << 10) | (cz << 20)));
    }
}

hipError_t launch_resort(const Geo& g, const int32_t* order, const double* pos, const double* vel,
                         const int32_t* id, double* pos_alt, double* vel_alt, int32_t* id_alt,
                         double* pos_ref, float* pos32, int32_t* cell_of, int32_t* cell_xyz,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_resort, dim3((unsigned)ceil_div(g.n, kStreamBlock)), dim3(kStreamBlock), 0, s, g,
                       order, (const double4*)pos, vel, id, (double4*)pos_alt, vel_alt, id_alt, pos_ref,
                       (float4*)pos32, cell_of, cell_xyz);
    return hipGetLastError();
}

// ---- user [n][3] coordinates -> [n][4] slots, folded into the box ------------
__device__ __forceinline__ double fold(double x, double L, double invL)
{
    double y = x - L * floor(x * invL);
    if (y >= L) y -= L;
    if (y < 0.0) y += L;
    return y;
}

__global__ __launch_bounds__(kStreamBlock) void k_pack(Geo g, const double* __restrict__ q,
                                                       double4* __restrict__ pos)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    pos[i] = make_double4(fold(q[3 * i], g.L[0], g.invL[0]), fold(q[3 * i + 1], g.L[1], g.invL[1]),
                          fold(q[3 * i + 2], g.L[2], g.invL[2]), 0.0);
}

hipError_t launch_pack(const Geo& g, const double* q, double* pos, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack, dim3((unsigned)ceil_div(g.n, kStreamBlock)), dim3(kStreamBlock), 0, s, g, q,
                       (double4*)pos);
    return hipGetLastError();
}

// ---- reference positions (and local coordinates) without a re-sort ----------
__global__ __launch_bounds__(kStreamBlock) void k_ref_copy(Geo g, const double4* __restrict__ pos,
                                                           const int32_t* __restrict__ cell_xyz,
                                                           double* __restrict__ pos_ref,
                                                           float4* __restrict__ pos32)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.n) return;
    const int64_t n = g.n;
    const double4 p = pos[k];
    if (pos_ref) {
        pos_ref[k] = p.x;
        pos_ref[n + k] = p.y;
        pos_ref[2 * n + k] = p.z;
    }
    if (pos32) {
        const int32_t c = cell_xyz[k];
        pos32[k] = make_float4(local_coord(p.x, c & 1023, g.cs[0], g.L[0], g.invL[0]),
                               local_coord(p.y, (c >> 10) & 1023, g.cs[1], g.L[1], g.invL[1]),
                               local_coord(p.z, (c >> 20) & 1023, g.cs[2], g.L[2], g.invL[2]), __int_as_float(c));
    }
}

// Positions of the current slots into a trajectory frame in the particles'
// original order: frame[id[s]] = pos[s] (x, y, z, 0).
__global__ __launch_bounds__(kStreamBlock) void k_record(int64_t n, const double4* __restrict__ pos,
                                                         const int32_t* __restrict__ id, double4* __restrict__ frame,
                                                         const int32_t* __restrict__ gate)
{
    const int64_t s = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    if (s >= n || (gate && gate[0])) return;
    const double4 p = pos[s];
    frame[id[s]] = make_double4(p.x, p.y, p.z, 0.0);
}

hipError_t launch_record(const Geo& g, const double* pos, const int32_t* id, double* frame, hipStream_t s,
                         const int32_t* gate)
{
    hipLaunchKernelGGL(k_record, dim3((unsigned)ceil_div(g.n, kStreamBlock)), dim3(kStreamBlock), 0, s, g.n,
                       (const double4*)pos, id, (double4*)frame, gate);
    return hipGetLastError();
}

hipError_t launch_ref_copy(const Geo& g, const double* pos, const int32_t* cell_xyz, double* pos_ref,
                           float* pos32, hipStream_t s)
{
    hipLaunchKernelGGL(k_ref_copy, dim3((unsigned)ceil_div(g.n, kStreamBlock)), dim3(kStreamBlock), 0, s,
                       g, (const double4*)pos, cell_xyz, pos_ref, (float4*)pos32);
    return hipGetLastError();
}

}  // namespace md
