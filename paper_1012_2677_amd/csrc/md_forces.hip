// Force / energy / virial kernel (Sec. 3.1-3.2 force loop over a key-sorted
// list; Sec. 2.4: the key particle's position and force stay in registers).
//
// kLanesPerKey lanes share one key's row: lane t of the group takes entries
// t, t + G, t + 2G, ... of the row, so the group reads the row as one
// contiguous run and the rows of consecutive keys (consecutive slots, hence
// neighbouring cells after the re-sort) follow each other in memory.  Every
// listed pair is evaluated; pairs with r >= rc are zeroed by a select rather
// than a branch (Sec. 3.1).  Per-lane partial sums are combined with
// cross-lane shuffles inside the group, and one lane writes the force.
//
// FP64 mode: displacements from absolute FP64 positions, with the minimum
// image taken only for keys in boundary cells (elsewhere no partner can wrap).
// Mixed mode: each slot carries FP32 coordinates relative to its cell corner;
// d = (l_j - l_i) + s * cs with s the stencil offset stored in the entry, so
// the FP32 displacement never suffers the cancellation of absolute FP32
// coordinates.  Forces are accumulated per key in FP32; PE and W in FP64.
//
// The kernel is bound by HBM bandwidth (list indices dominate the traffic)
// with the FP64 arithmetic close behind.

#include "md_internal.h"

namespace md {

struct ForceArgs {
    const double4* pos;
    const float4* pos32;
    const int32_t* cell_xyz;
    const int64_t* offsets;
    const int32_t* counts;
    const uint32_t* nbr;
    int64_t n;
    int64_t nblocks;
    double L[3], invL[3];
    int32_t nc[3];
    int32_t exact_all;
    LJ lj;
    float shift[27][4];   // s * cs per stencil code (mixed mode)
    void* force;
    double* part;
    int64_t* flags;
};

__device__ __forceinline__ bool boundary_cell(int32_t c, const int32_t* nc)
{
    const int x = c & 1023, y = (c >> 10) & 1023, z = (c >> 20) & 1023;
    return x == 0 || x == nc[0] - 1 || y == 0 || y == nc[1] - 1 || z == 0 || z == nc[2] - 1;
}

// block-wide sum of (a, b) into part[2*block]
template <int BLOCK>
__device__ __forceinline__ void block_partial2(double a, double b, double* part, int64_t blk)
{
    __shared__ double s_a[BLOCK / 64], s_b[BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_a[wave] = a;
        s_b[wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) {
            sa += s_a[w];
            sb += s_b[w];
        }
        part[2 * blk] = sa;
        part[2 * blk + 1] = sb;
    }
}

// Row walk shared by both precisions.  Lane `sub` of a key's group handles
// entries sub, sub + G, ... of the row.  The wave walks the rows of its keys
// in lockstep up to the longest one (a wave-uniform bound), U entries per lane
// at a time: the U index loads are issued, then the U position gathers, then
// the U pair terms are evaluated.  Unroll slots that no lane of the wave needs
// are skipped by a uniform branch; inside a slot, lanes past the end of their
// row load nothing and use a stand-in partner placed beyond the cutoff.
// maximum over the wave, returned as a wave-uniform (scalar) value
__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

template <int G, int U, bool ENERGY>
__global__ __launch_bounds__(kForceBlock) void k_forces_fp64(ForceArgs a)
{
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t key = blk * (kForceBlock / G) + threadIdx.x / G;
    const int sub = threadIdx.x % G;
    const bool valid = key < a.n;
    int64_t off = 0;
    int cnt = 0;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    bool minimg = false;
    if (valid) {
        off = a.offsets[key];
        cnt = a.counts[key];
        const double4 p = a.pos[key];
        xi = p.x;
        yi = p.y;
        zi = p.z;
        minimg = a.exact_all || boundary_cell(a.cell_xyz[key], a.nc);
    }
    const double rc2 = a.lj.rc2, A = a.lj.A, B = a.lj.B, C8 = a.lj.C8;
    double fx = 0.0, fy = 0.0, fz = 0.0, pe = 0.0, w = 0.0;
    const uint32_t* row = a.nbr + off;
    const int cmax = wave_max_i32(cnt);
    for (int t0 = sub; t0 - sub < cmax; t0 += G * U) {
        uint32_t e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * G;
            e[u] = t < cnt ? row[t] : 0xFFFFFFFFu;
        }
        double4 pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (t0 - sub + u * G < cmax) {
                // stand-in for masked slots: half a box away along x, which the
                // minimum image leaves in place (rint(1/2) = 0) and which is
                // beyond rs because every axis has at least three cells
                if (e[u] != 0xFFFFFFFFu) pj[u] = a.pos[e[u] & kSlotMask];
                else pj[u] = make_double4(xi + 0.5 * a.L[0], yi, zi, 0.0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (t0 - sub + u * G < cmax) {
                double dx = pj[u].x - xi, dy = pj[u].y - yi, dz = pj[u].z - zi;
                if (minimg) {
                    dx -= a.L[0] * rint(dx * a.invL[0]);
                    dy -= a.L[1] * rint(dy * a.invL[1]);
                    dz -= a.L[2] * rint(dz * a.invL[2]);
                }
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double r2i = rcp64(r2);
                const double r6i = r2i * r2i * r2i;
                double g = r2i * r6i * (A * r6i - B) - C8;
                const bool in = r2 < rc2;
                g = in ? g : 0.0;
                fx -= g * dx;
                fy -= g * dy;
                fz -= g * dz;
                if (ENERGY) {
                    const double V = r6i * (a.lj.A4 * r6i - a.lj.B4) + a.lj.C2 * r2 + a.lj.C0;
                    pe += in ? V : 0.0;
                    w += g * r2;
                }
            }
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, G);
        fy += __shfl_xor(fy, o, G);
        fz += __shfl_xor(fz, o, G);
    }
    if (valid && sub == 0) {
        double* F = (double*)a.force;
        F[key] = fx;
        F[a.n + key] = fy;
        F[2 * a.n + key] = fz;
        if (!isfinite(fx + fy + fz)) atomicOr((unsigned long long*)a.flags, 1ull);
    }
    if (ENERGY) block_partial2<kForceBlock>(0.5 * pe, 0.5 * w, a.part, blk);
}

template <int G, int U, bool ENERGY>
__global__ __launch_bounds__(kForceBlock) void k_forces_mixed(ForceArgs a)
{
    __shared__ float4 s_shift[32];
    if (threadIdx.x < 32) {
        // code 27 never occurs in an entry: it is the stand-in used for
        // masked slots, displaced far beyond the cutoff
        s_shift[threadIdx.x] = threadIdx.x < 27 ? make_float4(a.shift[threadIdx.x][0], a.shift[threadIdx.x][1],
                                                              a.shift[threadIdx.x][2], 0.0f)
                                                : make_float4(1.0e3f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t key = blk * (kForceBlock / G) + threadIdx.x / G;
    const int sub = threadIdx.x % G;
    const bool valid = key < a.n;
    int64_t off = 0;
    int cnt = 0;
    float4 li = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
        off = a.offsets[key];
        cnt = a.counts[key];
        li = a.pos32[key];
    }
    const float rc2 = (float)a.lj.rc2, A = (float)a.lj.A, B = (float)a.lj.B, C8 = (float)a.lj.C8;
    float fx = 0.f, fy = 0.f, fz = 0.f;
    double pe = 0.0, w = 0.0;
    const uint32_t* row = a.nbr + off;
    const uint32_t dummy = (uint32_t)(valid ? key : 0) | (27u << kCodeShift);
    const int cmax = wave_max_i32(cnt);
    for (int t0 = sub; t0 - sub < cmax; t0 += G * U) {
        uint32_t e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * G;
            e[u] = t < cnt ? row[t] : dummy;
        }
        float4 pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 - sub + u * G < cmax) pj[u] = a.pos32[e[u] & kSlotMask];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (t0 - sub + u * G < cmax) {
                const float4 sh = s_shift[e[u] >> kCodeShift];
                const float dx = (pj[u].x - li.x) + sh.x;
                const float dy = (pj[u].y - li.y) + sh.y;
                const float dz = (pj[u].z - li.z) + sh.z;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float r2i = __builtin_amdgcn_rcpf(r2);
                const float r6i = r2i * r2i * r2i;
                float g = r2i * r6i * (A * r6i - B) - C8;
                const bool in = r2 < rc2;
                g = in ? g : 0.0f;
                fx -= g * dx;
                fy -= g * dy;
                fz -= g * dz;
                if (ENERGY) {
                    const float V = r6i * ((float)a.lj.A4 * r6i - (float)a.lj.B4) + (float)a.lj.C2 * r2 +
                                    (float)a.lj.C0;
                    pe += in ? (double)V : 0.0;
                    w += (double)(g * r2);
                }
            }
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, G);
        fy += __shfl_xor(fy, o, G);
        fz += __shfl_xor(fz, o, G);
    }
    if (valid && sub == 0) {
        float* F = (float*)a.force;
        F[key] = fx;
        F[a.n + key] = fy;
        F[2 * a.n + key] = fz;
        if (!isfinite(fx + fy + fz)) atomicOr((unsigned long long*)a.flags, 1ull);
    }
    if (ENERGY) block_partial2<kForceBlock>(0.5 * pe, 0.5 * w, a.part, blk);
}

hipError_t launch_forces(const Geo& g, const LJ& lj, int precision, const double* pos,
                         const float* pos32, const int32_t* cell_xyz, const md_pairlist& list,
                         const ForceOut& out, hipStream_t s)
{
    ForceArgs a;
    a.pos = (const double4*)pos;
    a.pos32 = (const float4*)pos32;
    a.cell_xyz = cell_xyz;
    a.offsets = list.offsets;
    a.counts = list.counts;
    a.nbr = list.nbr;
    a.n = g.n;
    a.nblocks = ceil_div(g.n, kKeysPerBlock);
    for (int k = 0; k < 3; ++k) {
        a.L[k] = g.L[k];
        a.invL[k] = g.invL[k];
        a.nc[k] = g.nc[k];
    }
    a.exact_all = g.exact_all;
    a.lj = lj;
    for (int code = 0; code < 27; ++code) {
        const int sx = code / 9 - 1, sy = (code / 3) % 3 - 1, sz = code % 3 - 1;
        a.shift[code][0] = (float)(sx * g.cs[0]);
        a.shift[code][1] = (float)(sy * g.cs[1]);
        a.shift[code][2] = (float)(sz * g.cs[2]);
        a.shift[code][3] = 0.0f;
    }
    a.force = out.force;
    a.part = out.part;
    a.flags = out.flags;
    const dim3 grid((unsigned)a.nblocks), block(kForceBlock);
    const bool energy = out.part != nullptr;
    constexpr int G = kLanesPerKey, U = kForceUnroll, U64 = kForceUnroll64;
    if (precision == MD_MIXED) {
        if (energy)
            hipLaunchKernelGGL((k_forces_mixed<G, U, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((k_forces_mixed<G, U, false>), grid, block, 0, s, a);
    } else {
        if (energy)
            hipLaunchKernelGGL((k_forces_fp64<G, U64, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((k_forces_fp64<G, U64, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace md
