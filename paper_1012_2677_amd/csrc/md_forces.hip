// Pair-force kernels: force / energy / virial over the key-sorted list
// (Sec. 3.1-3.2 force loop; Sec. 2.4: the key's position and force stay in
// registers while its row is walked), optionally fused with the velocity-Verlet
// kicks and drift that consume the force (Sec. 4.5 integrator).
//
// Work layout.  A wave owns 64 consecutive keys: lane L owns key base + L for
// everything that is per key (row bounds, own coordinates, the force it ends
// with and the integrator epilogue, all coalesced).  The pair work runs in
// 8 rounds: in round r the 8 lanes of group q (lanes 8q .. 8q+7) walk the row of
// key base + 8r + q together, lane j of the group taking entries j, j+8, ...
// so each group reads its row as one contiguous run and a round covers 8
// consecutive keys (consecutive rows; partners in the same few cells).  The wave walks the 8 rows
// of a round in lockstep up to the longest (a wave-uniform bound), U entries
// per lane at a time: U index loads, then U position gathers, then U pair terms.
// Unroll slots no lane needs are skipped by a uniform branch; lanes past the
// end of their row use a stand-in partner beyond the cutoff.  Every listed pair
// is evaluated and pairs with r >= rc are zeroed by a select, not a branch
// (Sec. 3.1).  A group's partial sums are combined with DPP lane moves, leaving
// the key's force in every lane of the group; lane 8r + q fetches it with one
// cross-lane permute, so after the rounds lane L holds the force of key base + L.
//
// FP64 mode: displacements from absolute FP64 positions, with the minimum
// image taken only for keys in boundary cells: elsewhere no listed partner can
// be a wrapped image while no particle has moved more than (cell side - rc)
// since the build, which the half-skin rule guarantees.  Under the DUTC + LDC
// rule (no such bound) every key takes minimum images (exact_all).
// Mixed mode: each slot carries FP32 coordinates relative to its cell corner;
// d = (l_j - l_i) + s * cs with s the stencil offset stored in the entry, so
// the FP32 displacement never suffers the cancellation of absolute FP32
// coordinates.  Forces are accumulated per key in FP32; PE and W in FP64.
//
// Integrator epilogue (MODE_KICK: second half kick; MODE_KKD: second half kick,
// next step's first half kick and drift, as two separate roundings): positions
// move only after every wave has read them, so the drifted coordinates the
// other waves still gather go to a second buffer (FP64 positions in FP64 mode,
// local coordinates in mixed mode) that the caller swaps in afterwards.

#include "md_internal.h"

namespace md {

enum PairMode { MODE_FORCE = 0, MODE_KICK = 1, MODE_KKD = 2 };

struct PairArgs {
    const double4* pos;        // positions (partners and keys)
    const float4* pos32;       // mixed: local coordinates (partners and keys)
    const int32_t* cell_xyz;
    const int64_t* offsets;
    const int32_t* counts;
    const uint32_t* nbr;
    int64_t nbr_entries;       // 16-bit entries the list buffer holds (tiled: bound of the row prefetch)
    int64_t n;
    double L[3], invL[3], cs[3];
    int32_t nc[3];
    int32_t exact_all;
    LJ lj;
    float shift[27][4];        // s * cs per stencil code (mixed mode)
    void* force;               // [3][n]; written unless MODE_KKD
    double* part_pw;           // per-block (PE, W) partials (ENERGY)
    double* part_ke;           // per-block KE partials (ENERGY, MODE_KICK / MODE_KKD)
    int64_t* flags;            // [0] |= 1 on a non-finite force
    double* vel;               // [3][n], updated in place (MODE_KICK / MODE_KKD)
    const double* pos_ref;     // [3][n], positions at the last build (MODE_KKD)
    double4* pos_out;          // positions after the drift (MODE_KKD; FP64: other buffer)
    float4* pos32_out;         // mixed: local coordinates after the drift (other buffer)
    unsigned long long* max_d2;  // atomic max of squared displacement bits (MODE_KKD)
    unsigned long long* max_v2;  // atomic max of squared drift speed bits (MODE_KKD)
    double dt;
    const int32_t* start;      // tiled: cell starts and counts (slots in cell order)
    const int32_t* count;
    int32_t tc, nt;            // tiled: cells per tile along z, tiles per column
    const int32_t* gate;       // step passes: nothing to do when *gate != 0
};

// Keys [kb, ke) of logical block b: a chunk of kForceBlock consecutive slots.
__device__ __forceinline__ void block_keys(const PairArgs& a, int64_t b, int64_t& kb, int64_t& ke)
{
    kb = b * kForceBlock;
    ke = kb + kForceBlock < a.n ? kb + kForceBlock : a.n;
}

__device__ __forceinline__ bool boundary_cell(int32_t c, const int32_t* nc)
{
    const int x = c & 1023, y = (c >> 10) & 1023, z = (c >> 20) & 1023;
    return x == 0 || x == nc[0] - 1 || y == 0 || y == nc[1] - 1 || z == 0 || z == nc[2] - 1;
}

// DPP lane moves inside each group of 8 lanes: mirror (lane j <-> 7 - j), then
// swap pairs of pairs, then neighbours.  Summing over the three moves gives
// every lane of the group the same, bitwise identical total (each step adds
// two values that the partner lane adds in the other order).
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppXor2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int kDppXor1 = 0xB1;   // quad_perm [1, 0, 3, 2]

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ float group8_sum(float v)
{
    v += dpp_f32<kDppHalfMirror>(v);
    v += dpp_f32<kDppXor2>(v);
    return v + dpp_f32<kDppXor1>(v);
}

__device__ __forceinline__ double group8_sum(double v)
{
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppXor2>(v);
    return v + dpp_f64<kDppXor1>(v);
}

__device__ __forceinline__ int group8_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kDppHalfMirror, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kDppXor2, 0xF, 0xF, false));
    return max(v, __builtin_amdgcn_update_dpp(0, v, kDppXor1, 0xF, 0xF, false));
}

// Sums over groups of G = 4 or 8 lanes (every lane of a group gets the same,
// bitwise identical total) and maxima over groups of K = 8 or 16 lanes.
constexpr int kDppRowMirror = 0x140;   // lane j <-> 15 - j inside each row of 16
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v)
{
    if constexpr (G == 8) return group8_sum(v);
    static_assert(G == 8 || G == 4, "groups of 4 or 8 lanes");
    if constexpr (sizeof(T) == 4) {
        v += dpp_f32<kDppXor2>(v);
        return v + dpp_f32<kDppXor1>(v);
    } else {
        v += dpp_f64<kDppXor2>(v);
        return v + dpp_f64<kDppXor1>(v);
    }
}
template <int K>
__device__ __forceinline__ int group_max(int v)
{
    static_assert(K == 8 || K == 16, "groups of 8 or 16 lanes");
    if constexpr (K == 16) v = max(v, __builtin_amdgcn_update_dpp(0, v, kDppRowMirror, 0xF, 0xF, false));
    return group8_max(v);
}

__device__ __forceinline__ double wrap_coord(double x, double L, double invL)
{
    double y = x - L * floor(x * invL);
    if (y >= L) y -= L;
    if (y < 0.0) y += L;
    return y;
}

__device__ __forceinline__ float local_coord(double x, int c, double cs, double L, double invL)
{
    double l = x - (double)c * cs;
    l -= L * rint((l - 0.5 * cs) * invL);
    return (float)l;
}

// Block-level epilogue: (PE, W) and KE partials, displacement maximum.  A
// full list meets every pair twice, so PE and W are halved (pscale = 1/2); a
// half list passes pscale = 1.
template <bool ENERGY, int MODE, bool VMAX, int NW = kForceBlock / 64>
__device__ __forceinline__ void block_epilogue(const PairArgs& a, int64_t blk, double pe, double w, double ke,
                                               double d2, double v2, double pscale = 0.5)
{
    __shared__ double s_r[5][NW];
    const int wave = threadIdx.x >> 6;
    if (ENERGY) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            pe += __shfl_xor(pe, o, 64);
            w += __shfl_xor(w, o, 64);
            if (MODE != MODE_FORCE) ke += __shfl_xor(ke, o, 64);
        }
    }
    if (MODE == MODE_KKD) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            d2 = fmax(d2, __shfl_xor(d2, o, 64));
            if (VMAX) v2 = fmax(v2, __shfl_xor(v2, o, 64));
        }
    }
    if ((threadIdx.x & 63) == 0) {
        s_r[0][wave] = pe;
        s_r[1][wave] = w;
        s_r[2][wave] = ke;
        s_r[3][wave] = d2;
        s_r[4][wave] = v2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double spe = 0.0, sw = 0.0, ske = 0.0, m = 0.0, mv = 0.0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            spe += s_r[0][k];
            sw += s_r[1][k];
            ske += s_r[2][k];
            m = fmax(m, s_r[3][k]);
            mv = fmax(mv, s_r[4][k]);
        }
        if (ENERGY) {
            a.part_pw[2 * blk] = pscale * spe;
            a.part_pw[2 * blk + 1] = pscale * sw;
            if (MODE != MODE_FORCE) a.part_ke[blk] = 0.5 * ske;
        }
        if (MODE == MODE_KKD) {
            atomicMax(max_slot(a.max_d2, blk), (unsigned long long)__double_as_longlong(m));
            if (VMAX) atomicMax(max_slot(a.max_v2, blk), (unsigned long long)__double_as_longlong(mv));
        }
    }
}

// Integrator epilogue of one key (lane): kicks, drift, wrap, displacement since
// the last build.  Same arithmetic as the stand-alone integrator.  The loads
// (load_key) and the arithmetic and stores (integrate_loaded) are separate so
// that a kernel can issue the loads early.
struct KeyIn {
    double vx, vy, vz;
    double4 p;
    double rx, ry, rz;
    int32_t c;
};

template <int MODE, bool MIXED>
__device__ __forceinline__ KeyIn load_key(const PairArgs& a, int64_t k)
{
    const int64_t n = a.n;
    KeyIn in;
    in.vx = a.vel[k];
    in.vy = a.vel[n + k];
    in.vz = a.vel[2 * n + k];
    in.p = make_double4(0.0, 0.0, 0.0, 0.0);
    in.rx = in.ry = in.rz = 0.0;
    in.c = 0;
    if (MODE == MODE_KKD) {
        in.p = a.pos[k];
        in.rx = a.pos_ref[k];
        in.ry = a.pos_ref[n + k];
        in.rz = a.pos_ref[2 * n + k];
        if (MIXED) in.c = a.cell_xyz[k];
    }
    return in;
}

template <int MODE, bool MIXED, bool VMAX>
__device__ __forceinline__ void integrate_loaded(const PairArgs& a, int64_t k, const KeyIn& in, double fx,
                                                 double fy, double fz, double& ke, double& d2, double& v2)
{
    const int64_t n = a.n;
    const double h = 0.5 * a.dt;
    double* __restrict__ vel = a.vel;
    double vx = in.vx, vy = in.vy, vz = in.vz;
    double4 p = in.p;
    const int32_t c = in.c;
    vx = vx + h * fx;
    vy = vy + h * fy;
    vz = vz + h * fz;
    ke = vx * vx + vy * vy + vz * vz;
    if (MODE == MODE_KKD) {
        vx = vx + h * fx;
        vy = vy + h * fy;
        vz = vz + h * fz;
        if (VMAX) v2 = pinned_len2(vx, vy, vz);
        p.x = wrap_coord(p.x + a.dt * vx, a.L[0], a.invL[0]);
        p.y = wrap_coord(p.y + a.dt * vy, a.L[1], a.invL[1]);
        p.z = wrap_coord(p.z + a.dt * vz, a.L[2], a.invL[2]);
        double ex = p.x - in.rx, ey = p.y - in.ry, ez = p.z - in.rz;
        ex -= a.L[0] * rint(ex * a.invL[0]);
        ey -= a.L[1] * rint(ey * a.invL[1]);
        ez -= a.L[2] * rint(ez * a.invL[2]);
        d2 = pinned_len2(ex, ey, ez);
        a.pos_out[k] = p;
        if (MIXED)
            a.pos32_out[k] = make_float4(local_coord(p.x, c & 1023, a.cs[0], a.L[0], a.invL[0]),
                                         local_coord(p.y, (c >> 10) & 1023, a.cs[1], a.L[1], a.invL[1]),
                                         local_coord(p.z, (c >> 20) & 1023, a.cs[2], a.L[2], a.invL[2]),
                                         __int_as_float(c));
    }
    vel[k] = vx;
    vel[n + k] = vy;
    vel[2 * n + k] = vz;
}

template <int MODE, bool MIXED, bool VMAX>
__device__ __forceinline__ void integrate_key(const PairArgs& a, int64_t k, double fx, double fy, double fz,
                                              double& ke, double& d2, double& v2)
{
    integrate_loaded<MODE, MIXED, VMAX>(a, k, load_key<MODE, MIXED>(a, k), fx, fy, fz, ke, d2, v2);
}

template <int U, bool ENERGY, int MODE, bool VMAX>
__global__ __launch_bounds__(kForceBlock, MD_PAIR_MIN_BLOCKS) void k_pairs_fp64(PairArgs a)
{
    constexpr int NW = kForceBlock / 64;
    __shared__ double4 s_p[NW][64];     // own position, .w = 1 if the key needs minimum images
    __shared__ int64_t s_off[NW][64];
    __shared__ int32_t s_cnt[NW][64];
    if (a.gate && a.gate[0]) return;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, sub = lane & 7, grp = lane >> 3;
    int64_t kb, kend;
    block_keys(a, blk, kb, kend);
    const double rc2 = a.lj.rc2, A = a.lj.A, B = a.lj.B, C8 = a.lj.C8;
    double pe = 0.0, w = 0.0, ke = 0.0, d2 = 0.0, v2 = 0.0;
    // each wave takes 64-key chunks of the block's range (a wave-uniform loop;
    // the LDS rows below are private to the wave, so no block barrier inside;
    // written as a loop, which also schedules better than a straight pass)
    for (int64_t base = kb + wave * 64; base < kend; base += NW * 64) {
    const int64_t mykey = base + lane;
    const bool myvalid = mykey < kend;
    {
        // lanes past the end load the last key (no branch) and get an empty row
        const int64_t k = myvalid ? mykey : kend - 1;
        double4 p = a.pos[k];
        p.w = (a.exact_all || boundary_cell(a.cell_xyz[k], a.nc)) ? 1.0 : 0.0;
        s_p[wave][lane] = p;
        s_off[wave][lane] = a.offsets[k];
        s_cnt[wave][lane] = myvalid ? a.counts[k] : 0;
    }
    __builtin_amdgcn_wave_barrier();
    double kfx = 0.0, kfy = 0.0, kfz = 0.0;
    for (int r = 0; r < 8; ++r) {
        const int ks = (r << 3) | grp;           // key base + 8 r + grp
        const int cmax = __builtin_amdgcn_readfirstlane(group8_max(s_cnt[wave][(r << 3) | sub]));
        const int cnt = s_cnt[wave][ks];
        const uint32_t* row = a.nbr + s_off[wave][ks];
        const double4 pi = s_p[wave][ks];
        const double xi = pi.x, yi = pi.y, zi = pi.z;
        const bool minimg = pi.w != 0.0;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int t0 = sub; t0 - sub < cmax; t0 += 8 * U) {
            uint32_t e[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * 8;
                e[u] = t < cnt ? row[t] : 0xFFFFFFFFu;
            }
            double4 pj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t0 - sub + u * 8 < cmax) {
                    // stand-in for masked slots: half a box away along x, which
                    // the minimum image leaves in place (rint(1/2) = 0) and which
                    // is beyond rs because every axis has at least three cells
                    if (e[u] != 0xFFFFFFFFu) pj[u] = a.pos[e[u] & kSlotMask];
                    else pj[u] = make_double4(xi + 0.5 * a.L[0], yi, zi, 0.0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t0 - sub + u * 8 < cmax) {
                    double dx = pj[u].x - xi, dy = pj[u].y - yi, dz = pj[u].z - zi;
                    if (minimg) {
                        dx -= a.L[0] * rint(dx * a.invL[0]);
                        dy -= a.L[1] * rint(dy * a.invL[1]);
                        dz -= a.L[2] * rint(dz * a.invL[2]);
                    }
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double r2i = rcp64_1(r2);
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
        fx = __shfl(group8_sum(fx), sub << 3, 64);
        fy = __shfl(group8_sum(fy), sub << 3, 64);
        fz = __shfl(group8_sum(fz), sub << 3, 64);
        if (grp == r) {
            kfx = fx;
            kfy = fy;
            kfz = fz;
        }
    }
    if (myvalid) {
        if (!isfinite(kfx + kfy + kfz)) atomicOr((unsigned long long*)a.flags, 1ull);
        if (MODE != MODE_KKD) {
            double* F = (double*)a.force;
            F[mykey] = kfx;
            F[a.n + mykey] = kfy;
            F[2 * a.n + mykey] = kfz;
        }
        if (MODE != MODE_FORCE) {
            double kk = 0.0, dd = 0.0, vv = 0.0;
            integrate_key<MODE, false, VMAX>(a, mykey, kfx, kfy, kfz, kk, dd, vv);
            ke += kk;
            d2 = fmax(d2, dd);
            v2 = fmax(v2, vv);
        }
    }
    __builtin_amdgcn_wave_barrier();
    }
    if (ENERGY || MODE == MODE_KKD) block_epilogue<ENERGY, MODE, VMAX>(a, blk, pe, w, ke, d2, v2);
}

template <int U, bool ENERGY, int MODE, bool VMAX>
__global__ __launch_bounds__(kForceBlock, MD_PAIR_MIN_BLOCKS) void k_pairs_mixed(PairArgs a)
{
    constexpr int NW = kForceBlock / 64;
    __shared__ float4 s_shift[32];
    __shared__ float4 s_l[NW][64];
    __shared__ int64_t s_off[NW][64];
    __shared__ int32_t s_cnt[NW][64];
    if (a.gate && a.gate[0]) return;
    if (threadIdx.x < 32) {
        // code 27 never occurs in an entry: it is the stand-in used for
        // masked slots, displaced far beyond the cutoff
        s_shift[threadIdx.x] = threadIdx.x < 27 ? make_float4(a.shift[threadIdx.x][0], a.shift[threadIdx.x][1],
                                                              a.shift[threadIdx.x][2], 0.0f)
                                                : make_float4(1.0e3f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, sub = lane & 7, grp = lane >> 3;
    int64_t kb, kend;
    block_keys(a, blk, kb, kend);
    const float rc2 = (float)a.lj.rc2, A = (float)a.lj.A, B = (float)a.lj.B, C8 = (float)a.lj.C8;
    double pe = 0.0, w = 0.0, ke = 0.0, d2 = 0.0, v2 = 0.0;
    // each wave takes 64-key chunks of the block's range (a wave-uniform loop;
    // the LDS rows below are private to the wave, so no block barrier inside;
    // written as a loop, which also schedules better than a straight pass)
    for (int64_t base = kb + wave * 64; base < kend; base += NW * 64) {
    const int64_t mykey = base + lane;
    const bool myvalid = mykey < kend;
    {
        // lanes past the end load the last key (no branch) and get an empty row
        const int64_t k = myvalid ? mykey : kend - 1;
        float4 l = a.pos32[k];
        l.w = __int_as_float((int)k);   // the key's own slot (stand-in partner)
        s_l[wave][lane] = l;
        s_off[wave][lane] = a.offsets[k];
        s_cnt[wave][lane] = myvalid ? a.counts[k] : 0;
    }
    __builtin_amdgcn_wave_barrier();
    float kfx = 0.f, kfy = 0.f, kfz = 0.f;
    for (int r = 0; r < 8; ++r) {
        const int ks = (r << 3) | grp;           // key base + 8 r + grp
        const int cmax = __builtin_amdgcn_readfirstlane(group8_max(s_cnt[wave][(r << 3) | sub]));
        const int cnt = s_cnt[wave][ks];
        const uint32_t* row = a.nbr + s_off[wave][ks];
        const float4 li = s_l[wave][ks];
        const uint32_t dummy = (uint32_t)__float_as_int(li.w) | (27u << kCodeShift);
        float fx = 0.f, fy = 0.f, fz = 0.f;
        for (int t0 = sub; t0 - sub < cmax; t0 += 8 * U) {
            uint32_t e[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * 8;
                e[u] = t < cnt ? row[t] : dummy;
            }
            float4 pj[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (t0 - sub + u * 8 < cmax) pj[u] = a.pos32[e[u] & kSlotMask];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t0 - sub + u * 8 < cmax) {
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
        fx = __shfl(group8_sum(fx), sub << 3, 64);
        fy = __shfl(group8_sum(fy), sub << 3, 64);
        fz = __shfl(group8_sum(fz), sub << 3, 64);
        if (grp == r) {
            kfx = fx;
            kfy = fy;
            kfz = fz;
        }
    }
    if (myvalid) {
        if (!isfinite(kfx + kfy + kfz)) atomicOr((unsigned long long*)a.flags, 1ull);
        if (MODE != MODE_KKD) {
            float* F = (float*)a.force;
            F[mykey] = kfx;
            F[a.n + mykey] = kfy;
            F[2 * a.n + mykey] = kfz;
        }
        if (MODE != MODE_FORCE) {
            double kk = 0.0, dd = 0.0, vv = 0.0;
            integrate_key<MODE, true, VMAX>(a, mykey, kfx, kfy, kfz, kk, dd, vv);
            ke += kk;
            d2 = fmax(d2, dd);
            v2 = fmax(v2, vv);
        }
    }
    __builtin_amdgcn_wave_barrier();
    }
    if (ENERGY || MODE == MODE_KKD) block_epilogue<ENERGY, MODE, VMAX>(a, blk, pe, w, ke, d2, v2);
}

// Half list (Sec. 2.4 with Newton's third law): each pair is listed once, in
// the row of one of its particles.  The rows are walked as in k_pairs_fp64 /
// k_pairs_mixed (8 lanes per key, 8 rounds per 64-key chunk, the same pair
// arithmetic); the key's share -g d is summed in registers, the partner's
// share +g d goes to the force array with one device atomic per component
// (pairs beyond the cutoff and stand-ins add nothing), and the key's sum is
// added with atomics at the end.  The caller clears the force array first.
// PE and W count each pair once.
template <int U, bool ENERGY, bool MIXED>
__global__ __launch_bounds__(kForceBlock, MD_PAIR_MIN_BLOCKS) void k_pairs_half(PairArgs a)
{
    using R = typename std::conditional<MIXED, float, double>::type;
    using P = typename std::conditional<MIXED, float4, double4>::type;
    constexpr int NW = kForceBlock / 64;
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    __shared__ float4 s_shift[32];
    __shared__ P s_p[NW][64];           // own coordinates; .w: mixed, the key's slot; FP64, 1 if minimum images
    __shared__ int64_t s_off[NW][64];
    __shared__ int32_t s_cnt[NW][64];
    if (MIXED) {
        // code 27 is the stand-in of masked slots, displaced far beyond the cutoff
        if (threadIdx.x < 32)
            s_shift[threadIdx.x] = threadIdx.x < 27 ? make_float4(a.shift[threadIdx.x][0], a.shift[threadIdx.x][1],
                                                                  a.shift[threadIdx.x][2], 0.0f)
                                                    : make_float4(1.0e3f, 0.0f, 0.0f, 0.0f);
        __syncthreads();
    }
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, sub = lane & 7, grp = lane >> 3;
    int64_t kb, kend;
    block_keys(a, blk, kb, kend);
    const R rc2 = (R)a.lj.rc2, A = (R)a.lj.A, B = (R)a.lj.B, C8 = (R)a.lj.C8;
    const R A4 = (R)a.lj.A4, B4 = (R)a.lj.B4, C2 = (R)a.lj.C2, C0 = (R)a.lj.C0;
    R* __restrict__ F = (R*)a.force;
    const int64_t n = a.n;
    double pe = 0.0, w = 0.0;
    for (int64_t base = kb + wave * 64; base < kend; base += NW * 64) {
    const int64_t mykey = base + lane;
    const bool myvalid = mykey < kend;
    {
        const int64_t k = myvalid ? mykey : kend - 1;
        P p;
        if constexpr (MIXED) {
            p = a.pos32[k];
            p.w = __int_as_float((int)k);
        } else {
            p = a.pos[k];
            p.w = (a.exact_all || boundary_cell(a.cell_xyz[k], a.nc)) ? 1.0 : 0.0;
        }
        s_p[wave][lane] = p;
        s_off[wave][lane] = a.offsets[k];
        s_cnt[wave][lane] = myvalid ? a.counts[k] : 0;
    }
    __builtin_amdgcn_wave_barrier();
    R kfx = 0, kfy = 0, kfz = 0;
    for (int r = 0; r < 8; ++r) {
        const int ks = (r << 3) | grp;
        const int cmax = __builtin_amdgcn_readfirstlane(group8_max(s_cnt[wave][(r << 3) | sub]));
        const int cnt = s_cnt[wave][ks];
        const uint32_t* row = a.nbr + s_off[wave][ks];
        const P pi = s_p[wave][ks];
        R fx = 0, fy = 0, fz = 0;
        for (int t0 = sub; t0 - sub < cmax; t0 += 8 * U) {
            uint32_t e[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * 8;
                e[u] = t < cnt ? row[t] : kNone;
            }
            P pj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t0 - sub + u * 8 < cmax) {
                    if constexpr (MIXED) {
                        // masked slots read the key itself, moved by the stand-in shift
                        pj[u] = a.pos32[e[u] != kNone ? (e[u] & kSlotMask) : (uint32_t)__float_as_int(pi.w)];
                    } else {
                        // half a box away along x: beyond rs, left in place by the minimum image
                        if (e[u] != kNone) pj[u] = a.pos[e[u] & kSlotMask];
                        else pj[u] = make_double4(pi.x + 0.5 * a.L[0], pi.y, pi.z, 0.0);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t0 - sub + u * 8 < cmax) {
                    R dx, dy, dz;
                    if constexpr (MIXED) {
                        const float4 sh = s_shift[e[u] != kNone ? (e[u] >> kCodeShift) : 27u];
                        dx = (pj[u].x - pi.x) + sh.x;
                        dy = (pj[u].y - pi.y) + sh.y;
                        dz = (pj[u].z - pi.z) + sh.z;
                    } else {
                        dx = pj[u].x - pi.x;
                        dy = pj[u].y - pi.y;
                        dz = pj[u].z - pi.z;
                        if (pi.w != 0.0) {
                            dx -= a.L[0] * rint(dx * a.invL[0]);
                            dy -= a.L[1] * rint(dy * a.invL[1]);
                            dz -= a.L[2] * rint(dz * a.invL[2]);
                        }
                    }
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    R r2i;
                    if constexpr (MIXED) r2i = __builtin_amdgcn_rcpf(r2);
                    else r2i = rcp64_1(r2);
                    const R r6i = r2i * r2i * r2i;
                    R g = r2i * r6i * (A * r6i - B) - C8;
                    const bool in = r2 < rc2;
                    g = in ? g : (R)0;
                    const R gx = g * dx, gy = g * dy, gz = g * dz;
                    fx -= gx;
                    fy -= gy;
                    fz -= gz;
                    if (ENERGY) {
                        const R V = r6i * (A4 * r6i - B4) + C2 * r2 + C0;
                        pe += in ? (double)V : 0.0;
                        w += (double)(g * r2);
                    }
                    if (in && e[u] != kNone) {
                        const int64_t j = e[u] & kSlotMask;
                        unsafeAtomicAdd(F + j, gx);
                        unsafeAtomicAdd(F + n + j, gy);
                        unsafeAtomicAdd(F + 2 * n + j, gz);
                    }
                }
            }
        }
        fx = __shfl(group8_sum(fx), sub << 3, 64);
        fy = __shfl(group8_sum(fy), sub << 3, 64);
        fz = __shfl(group8_sum(fz), sub << 3, 64);
        if (grp == r) {
            kfx = fx;
            kfy = fy;
            kfz = fz;
        }
    }
    if (myvalid) {
        if (!isfinite(kfx + kfy + kfz)) atomicOr((unsigned long long*)a.flags, 1ull);
        unsafeAtomicAdd(F + mykey, kfx);
        unsafeAtomicAdd(F + n + mykey, kfy);
        unsafeAtomicAdd(F + 2 * n + mykey, kfz);
    }
    __builtin_amdgcn_wave_barrier();
    }
    if (ENERGY) block_epilogue<true, MODE_FORCE, false>(a, blk, pe, w, 0.0, 0.0, 0.0, 1.0);
}

// Integrator of a half-list step: the force of a particle is complete only
// when the whole pair pass has run, so the kicks and the drift (the fused
// epilogue's arithmetic) run here as a pass of their own, one lane per slot,
// in the same blocks of kForceBlock slots as the pair pass (KE partials).
template <int MODE, bool MIXED, bool VMAX, bool ENERGY>
__global__ __launch_bounds__(kForceBlock) void k_integrate_half(PairArgs a)
{
    constexpr int NW = kForceBlock / 64;
    __shared__ double s_r[3][NW];
    const int64_t blk = blockIdx.x;
    const int64_t k = blk * kForceBlock + threadIdx.x;
    double ke = 0.0, d2 = 0.0, v2 = 0.0;
    if (k < a.n) {
        double fx, fy, fz;
        if constexpr (MIXED) {
            const float* F = (const float*)a.force;
            fx = F[k];
            fy = F[a.n + k];
            fz = F[2 * a.n + k];
        } else {
            const double* F = (const double*)a.force;
            fx = F[k];
            fy = F[a.n + k];
            fz = F[2 * a.n + k];
        }
        if (!isfinite(fx + fy + fz)) atomicOr((unsigned long long*)a.flags, 1ull);
        integrate_key<MODE, MIXED, VMAX>(a, k, fx, fy, fz, ke, d2, v2);
    }
    if (!ENERGY && MODE != MODE_KKD) return;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        if (ENERGY) ke += __shfl_xor(ke, o, 64);
        if (MODE == MODE_KKD) d2 = fmax(d2, __shfl_xor(d2, o, 64));
        if (VMAX) v2 = fmax(v2, __shfl_xor(v2, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        s_r[0][wave] = ke;
        s_r[1][wave] = d2;
        s_r[2][wave] = v2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ske = 0.0, m = 0.0, mv = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            ske += s_r[0][q];
            m = fmax(m, s_r[1][q]);
            mv = fmax(mv, s_r[2][q]);
        }
        if (ENERGY) a.part_ke[blk] = 0.5 * ske;
        if (MODE == MODE_KKD) {
            atomicMax(max_slot(a.max_d2, blk), (unsigned long long)__double_as_longlong(m));
            if (VMAX) atomicMax(max_slot(a.max_v2, blk), (unsigned long long)__double_as_longlong(mv));
        }
    }
}

// Tiled force pass: one block per tile of tc cells along z.  The block first
// copies the tile's neighbourhood (the runs of cells z0-1 .. z1 of the 9
// columns around it, in the order of the list build) into LDS; entries are
// 16 x the partner's index in that copy (its byte offset at 16 bytes per
// particle) and a row of odd length ends with a stand-in partner beyond the
// cutoff.
//   Mixed: each particle is staged from its local coordinates as
//   (x + sx cs_x, y + sy cs_y, z, j) with (sx, sy) its column offset and j its
//   position in the run.  With the key's (x, y, z) local and its own run
//   position jk, d = (x_j - x_i, y_j - y_i, (z_j - z_i) + (j - jk) cs_z), the
//   last term exact ((j - jk) is -1, 0 or 1).
//   FP64: particles are staged as their FP64 positions (24 bytes, so the
//   byte offset is 1.5 x the entry: a copy of ~1600 particles leaves room for
//   4 blocks per CU, which 32-byte records would cut to 3), and
//   displacements take the minimum image in tiles that touch the box
//   boundary (a no-op for pairs that do not wrap), as in k_pairs_fp64.
// The tile's keys are split evenly over the waves.  In each 64-key chunk the
// rows are walked in rounds of 64 / G keys grouped by row length (G = 4 lanes
// per row), the first kPrefetch (mixed) or kPrefetch64 (FP64) entries of all G
// rounds loaded up front, two per 32-bit load.  Key
// data reach the round's lanes by shuffles; group sums and the integrator
// epilogue are those of the other pair kernels.
#ifndef MD_TILE_STRIP
#define MD_TILE_STRIP 8
#endif
constexpr int kTileStrip = MD_TILE_STRIP;       // x-columns per strip of the tile order
#ifndef MD_TILE_PREFETCH
#define MD_TILE_PREFETCH 64
#endif
constexpr int kPrefetch = MD_TILE_PREFETCH;     // row entries per key loaded up front (multiple of 16)
#ifndef MD_TILE_PREFETCH_FP64
#define MD_TILE_PREFETCH_FP64 56
#endif
// the same in FP64 (a multiple of 2 x its lanes per row), short enough that the
// pass stays within 128 registers (4 waves per SIMD); 48 in its energy variant
constexpr int kPrefetch64 = MD_TILE_PREFETCH_FP64;
#ifndef MD_TILE_LANES_MIXED
#define MD_TILE_LANES_MIXED 4
#endif
#ifndef MD_TILE_LANES_FP64
#define MD_TILE_LANES_FP64 4
#endif
// lanes that walk one row (4 or 8): fewer lanes spread a round's fixed costs
// (key data, group sums) over more entries per lane
constexpr int kTileLanesMixed = MD_TILE_LANES_MIXED;
constexpr int kTileLanes64 = MD_TILE_LANES_FP64;

template <bool MIXED>
struct TileT;
// A staged FP64 particle is its position alone (24 bytes, no padding), so a
// tile's neighbourhood takes three quarters of the LDS a double4 copy would.
struct D3 {
    double x, y, z;
};
template <>
struct TileT<true> {
    using R = float;
    using V4 = float4;
    using S = float4;                   // staged particle: 16 bytes, byte offset = entry
    __device__ static uint32_t off(uint32_t e) { return e; }
};
template <>
struct TileT<false> {
    using R = double;
    using V4 = double4;
    using S = D3;                       // 24 bytes: byte offset = 1.5 x entry
    __device__ static uint32_t off(uint32_t e) { return e + (e >> 1); }
};

template <int U, bool ENERGY, int MODE, bool VMAX, bool MIXED>
__global__ __launch_bounds__(kTileBlock, MD_PAIR_MIN_BLOCKS) void k_pairs_tiled(PairArgs a)
{
    using R = typename TileT<MIXED>::R;
    using V4 = typename TileT<MIXED>::V4;
    using S = typename TileT<MIXED>::S;
    constexpr int NW = kTileBlock / 64;
    extern __shared__ float4 s_lds[];     // staged neighbourhood, then one stand-in
    S* s_nb = (S*)s_lds;
    __shared__ uint8_t s_perm[NW][64];
    __shared__ int32_t s_run[9][4];
    __shared__ int32_t s_base[10];
    if (a.gate && a.gate[0]) return;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
    const int tz = (int)(blk % a.nt);
    // columns in strips of kTileStrip x-columns walked along y, so that the
    // tiles an XCD runs close in time share their neighbour columns in L2
    const int64_t seq = blk / a.nt;
    const int64_t strip = seq / ((int64_t)kTileStrip * ny);
    const int sw = (int)min((int64_t)kTileStrip, (int64_t)nx - strip * kTileStrip);
    const int64_t in = seq - strip * kTileStrip * ny;
    const int cy = (int)(in / sw), cx = (int)(strip * kTileStrip + in % sw);
    const int z0 = tz * a.tc, z1 = min(z0 + a.tc, nz);
    const int tid = threadIdx.x;
    // FP64: the tile's pairs need minimum images only when it touches the box
    // boundary (or when some axis has fewer than 5 cells)
    const bool minimg = !MIXED && (a.exact_all || cx == 0 || cx == nx - 1 || cy == 0 || cy == ny - 1 || z0 == 0 ||
                                   z1 == nz);
    if (tid < 9) {
        const TileRun r = tile_run(a.start, a.count, wrap_cell(cx + tid / 3 - 1, nx), wrap_cell(cy + tid % 3 - 1, ny),
                                   ny, nz, z0, z1);
        s_run[tid][0] = r.sA;
        s_run[tid][1] = r.lenA;
        s_run[tid][2] = r.sB;
        s_run[tid][3] = r.lenB;
    }
    __syncthreads();
    if (tid == 0) {
        int b = 0;
        for (int col = 0; col < 9; ++col) {
            s_base[col] = b;
            b += s_run[col][1] + s_run[col][3];
        }
        s_base[9] = b;
        // stand-in partner beyond the cutoff of every key of the tile: in mixed
        // mode far outside the cell frame; in FP64 half a box away from the
        // tile's column in x, which the minimum image leaves at least
        // L/2 - cs/2 >= cs >= rs away
        if constexpr (MIXED) {
            s_nb[b] = make_float4(1.0e3f, 0.0f, 0.0f, 0.0f);
        } else {
            double x = ((double)cx + 0.5) * a.cs[0] + 0.5 * a.L[0];
            x -= x >= a.L[0] ? a.L[0] : 0.0;
            s_nb[b] = D3{x, ((double)cy + 0.5) * a.cs[1], ((double)z0 + 0.5) * a.cs[2]};
        }
    }
    __syncthreads();
    const float csx = (float)a.cs[0], csy = (float)a.cs[1];
    const R csz = (R)a.cs[2];
    {
        // every thread takes elements tid, tid + kTileBlock, ... (SB of them) of
        // each column run (the loads of all 9 columns in flight together),
        // then writes them (mixed: shifted by the column offset and tagged
        // with their run position); longer runs finish in a plain loop.  FP64
        // takes one element per column (its runs are shorter, and 18 double4
        // would hold 144 registers)
        constexpr int SB = MIXED ? 2 : 1;
        V4 p[9][SB];
        auto src_of = [&](int col, int i) {
            const int lenA = s_run[col][1];
            return i < lenA ? s_run[col][0] + i : s_run[col][2] + (i - lenA);
        };
        auto load = [&](int slot) -> V4 {
            if constexpr (MIXED) return a.pos32[slot];
            else return a.pos[slot];
        };
        auto put = [&](const V4& q, int col, int i) {
            if constexpr (MIXED) {
                int j = ((__float_as_int(q.w) >> 20) & 1023) - z0 + 1;
                j += j < 0 ? nz : 0;
                j -= j >= nz ? nz : 0;
                s_nb[s_base[col] + i] = make_float4(q.x + (float)(col / 3 - 1) * csx, q.y + (float)(col % 3 - 1) * csy,
                                                    q.z, (float)j);
            } else {
                s_nb[s_base[col] + i] = D3{q.x, q.y, q.z};
            }
        };
#pragma unroll
        for (int col = 0; col < 9; ++col) {
            const int len = s_run[col][1] + s_run[col][3];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                // unconditional loads (slot 0 past the run's end, result unused)
                const int i = tid + u * kTileBlock;
                p[col][u] = load(i < len ? src_of(col, i) : 0);
            }
        }
#pragma unroll
        for (int col = 0; col < 9; ++col) {
            const int len = s_run[col][1] + s_run[col][3];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int i = tid + u * kTileBlock;
                if (i < len) put(p[col][u], col, i);
            }
        }
        for (int col = 0; col < 9; ++col) {
            const int len = s_run[col][1] + s_run[col][3];
            for (int i = tid + SB * kTileBlock; i < len; i += kTileBlock) put(load(src_of(col, i)), col, i);
        }
    }
    __syncthreads();
    // G lanes walk each row; a round takes K = 64 / G keys, a chunk of 64
    // keys G rounds
    constexpr int G = MIXED ? kTileLanesMixed : kTileLanes64, K = 64 / G;
    const uint32_t dummy = (uint32_t)s_base[9] << 4;   // entry of the stand-in partner
    const int64_t colc = ((int64_t)cx * ny + cy) * nz;
    const int64_t kb = a.start[colc + z0];
    const int64_t kend = (int64_t)a.start[colc + z1 - 1] + a.count[colc + z1 - 1];
    const int wave = tid >> 6, lane = tid & 63, sub = lane & (G - 1), grp = lane / G;
    const R rc2 = (R)a.lj.rc2, A = (R)a.lj.A, B = (R)a.lj.B, C8 = (R)a.lj.C8;
    double pe = 0.0, w = 0.0, ke = 0.0, d2 = 0.0, v2 = 0.0;
    auto nb = [&](uint32_t e) { return *(const S*)((const char*)s_nb + TileT<MIXED>::off(e)); };
    auto pair = [&](const auto& pj, const V4& li, R& fx, R& fy, R& fz) {
        R dx = pj.x - li.x;
        R dy = pj.y - li.y;
        R dz;
        if constexpr (MIXED) {
            dz = __builtin_fmaf(pj.w - li.w, csz, pj.z - li.z);
        } else {
            dz = pj.z - li.z;
            if (minimg) {
                dx -= a.L[0] * rint(dx * a.invL[0]);
                dy -= a.L[1] * rint(dy * a.invL[1]);
                dz -= a.L[2] * rint(dz * a.invL[2]);
            }
        }
        const R r2 = dx * dx + dy * dy + dz * dz;
        R r2i;
        if constexpr (MIXED) r2i = __builtin_amdgcn_rcpf(r2);
        else r2i = rcp64_1(r2);
        const R r6i = r2i * r2i * r2i;
        R g = r2i * r6i * (A * r6i - B) - C8;
        const bool in = r2 < rc2;
        g = in ? g : (R)0;
        fx -= g * dx;
        fy -= g * dy;
        fz -= g * dz;
        if (ENERGY) {
            const R V = r6i * ((R)a.lj.A4 * r6i - (R)a.lj.B4) + (R)a.lj.C2 * r2 + (R)a.lj.C0;
            pe += in ? (double)V : 0.0;
            w += (double)(g * r2);
        }
    };
    // the tile's keys split evenly over the waves, in chunks of at most 64
    // keys and a whole number of rounds (a multiple of K, so that only a
    // wave's last chunk has a round with empty key slots): nr rounds per
    // chunk instead of always G
    const int64_t nk = kend - kb;
    // the tile's keys are cells z0 .. z1 - 1 of the centre column (run 4), in
    // slot order: key slot k is staged at key0 + (k - kb); the run's first part
    // starts at cell z0 - 1, or, when the tile starts the column, is the
    // wrapped cell nz - 1 alone and the keys open its second part
    const int key0 = s_base[4] + (z0 == 0 ? s_run[4][1] + (int)(kb - s_run[4][2]) : (int)(kb - s_run[4][0]));
    const int csz_k = nk >= NW * 64 ? 64 : (int)((((nk + NW - 1) / NW) + K - 1) / K * K);
    for (int64_t base = kb + wave * csz_k; base < kend; base += NW * csz_k) {
    const int64_t cend = base + csz_k < kend ? base + csz_k : kend;
    const int nr = (int)((cend - base + K - 1) / K);
    const int64_t mykey = base + lane;
    const bool myvalid = mykey < cend;
    // the lane's own key: row offset and length (mixed: also its local
    // coordinates with its run position in w); rounds fetch them from the
    // owner lane.  FP64 rounds read the key's coordinates from its staged
    // copy instead (two LDS reads against six cross-lane permutes; in mixed
    // precision that takes the pass past 128 VGPRs)
    float4 own;
    int64_t own_off;
    int own_cnt;
    {
        const int64_t k = myvalid ? mykey : kend - 1;
        if constexpr (MIXED) {
            own = a.pos32[k];
            own.w = (float)(((__float_as_int(own.w) >> 20) & 1023) - z0 + 1);
        }
        own_off = a.offsets[k];
        own_cnt = myvalid ? a.counts[k] : 0;
    }
    // round order: the chunk's keys grouped by row length in steps of 2G
    // entries (longest first), so that the K rows a round walks to a common
    // bound have similar lengths; lane L's key is walked in round pr / K by
    // group pr % K
    int pr;
    {
        const int b = min((own_cnt + 2 * G - 1) / (2 * G), 7);
        int off = 0;
        pr = 0;
#pragma unroll
        for (int v = 7; v >= 0; --v) {
            const uint64_t m = __ballot(b == v);
            if (b == v) pr = off + (int)mbcnt64(m);
            off += __popcll(m);
        }
        s_perm[wave][pr] = (uint8_t)lane;
    }
    __builtin_amdgcn_wave_barrier();
    // the first kPrefetch entries of the rows each lane walks, two per 32-bit
    // load: lane j of a group takes entries 2j + 2Gu and 2j + 2Gu + 1; all
    // loads of the chunk go out at once (48 entries in the energy variants and
    // when the drift speed is tracked, to stay within 128 VGPRs)
    constexpr int PF = (VMAX || ENERGY) ? 48 : (MIXED ? kPrefetch : kPrefetch64);
    constexpr int UP = PF / (2 * G);
    const uint32_t dummy2 = dummy | (dummy << 16);
    uint32_t E[G][UP];
#pragma unroll
    for (int r = 0; r < G; ++r) {
        if (r >= nr) break;
        const int ks = s_perm[wave][r * K + grp];
        const int cnt = __shfl(own_cnt, ks, 64);
        const int64_t roff = __shfl(own_off, ks, 64);
        const uint32_t* row2 = (const uint32_t*)((const uint16_t*)a.nbr + roff);
        if (__all(roff + PF <= a.nbr_entries)) {
            // every lane's window of PF entries lies in the buffer: plain loads
            // at constant offsets (entries past the row are replaced by the
            // stand-in where they are used)
            const uint32_t* rp = row2 + sub;
#pragma unroll
            for (int u = 0; u < UP; ++u) E[r][u] = rp[G * u];
        } else {
#pragma unroll
            for (int u = 0; u < UP; ++u) {
                const int t = 2 * sub + 2 * G * u;
                E[r][u] = t < cnt ? row2[t >> 1] : dummy2;
            }
        }
    }
    R kfx = 0, kfy = 0, kfz = 0;
#pragma unroll
    for (int r = 0; r < G; ++r) {
        if (r >= nr) break;
        const int ks = s_perm[wave][r * K + grp];
        const int cmax =
            __builtin_amdgcn_readfirstlane(group_max<K>(__shfl(own_cnt, s_perm[wave][r * K + (lane & (K - 1))], 64)));
        const int cnt = __shfl(own_cnt, ks, 64);
        const int lim = cnt - 2 * sub;   // entries 2 G u + 2 sub + (0, 1) are the row's where 2 G u < lim
        V4 li;
        if constexpr (MIXED) {
            li.x = __shfl(own.x, ks, 64);
            li.y = __shfl(own.y, ks, 64);
            li.z = __shfl(own.z, ks, 64);
            li.w = __shfl(own.w, ks, 64);
        } else {
            // empty key slots read the tile's last key
            const S lk = s_nb[key0 + (int)(min(base + ks, kend - 1) - kb)];
            li.x = lk.x;
            li.y = lk.y;
            li.z = lk.z;
        }
        R fx = 0, fy = 0, fz = 0;
        // mixed: four partners (two words) per step where the round's bound
        // allows, so that four LDS reads and pair chains overlap (FP64 stays at
        // two: four take it past 128 VGPRs, 3.24 -> 3.79 ms)
        constexpr bool QUAD = MIXED && !(ENERGY && VMAX);
#pragma unroll
        for (int u = 0; u < UP; u += QUAD ? 2 : 1) {
            if (QUAD && u + 1 < UP && 2 * G * (u + 1) < cmax) {
                const uint32_t e2 = 2 * G * u < lim ? E[r][u] : dummy2;
                const uint32_t e3 = 2 * G * (u + 1) < lim ? E[r][u + 1] : dummy2;
                const S p0 = nb(e2 & 0xFFFFu), p1 = nb(e2 >> 16), p2 = nb(e3 & 0xFFFFu), p3 = nb(e3 >> 16);
                pair(p0, li, fx, fy, fz);
                pair(p1, li, fx, fy, fz);
                pair(p2, li, fx, fy, fz);
                pair(p3, li, fx, fy, fz);
            } else if (2 * G * u < cmax) {
                const uint32_t e2 = 2 * G * u < lim ? E[r][u] : dummy2;
                const S p0 = nb(e2 & 0xFFFFu), p1 = nb(e2 >> 16);
                pair(p0, li, fx, fy, fz);
                pair(p1, li, fx, fy, fz);
            }
        }
        if (cmax > PF) {
            // the rest of rows longer than the prefetched part
            const uint16_t* row = (const uint16_t*)a.nbr + __shfl(own_off, ks, 64);
            for (int t0 = PF + sub; t0 - sub < cmax; t0 += G * U) {
                uint32_t e[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int t = t0 + u * G;
                    e[u] = t < cnt ? (uint32_t)row[t] : dummy;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (t0 - sub + u * G < cmax) pair(nb(e[u]), li, fx, fy, fz);
            }
        }
        const int src = (pr % K) * G;
        fx = __shfl(group_sum<G>(fx), src, 64);
        fy = __shfl(group_sum<G>(fy), src, 64);
        fz = __shfl(group_sum<G>(fz), src, 64);
        if (pr / K == r) {
            kfx = fx;
            kfy = fy;
            kfz = fz;
        }
    }
    if (myvalid) {
        if (!isfinite(kfx + kfy + kfz)) atomicOr((unsigned long long*)a.flags, 1ull);
        if (MODE != MODE_KKD) {
            R* F = (R*)a.force;
            F[mykey] = kfx;
            F[a.n + mykey] = kfy;
            F[2 * a.n + mykey] = kfz;
        }
        if (MODE != MODE_FORCE) {
            double kk = 0.0, dd = 0.0, vv = 0.0;
            integrate_key<MODE, MIXED, VMAX>(a, mykey, kfx, kfy, kfz, kk, dd, vv);
            ke += kk;
            d2 = fmax(d2, dd);
            v2 = fmax(v2, vv);
        }
    }
    __builtin_amdgcn_wave_barrier();
    }
    if (ENERGY || MODE == MODE_KKD) block_epilogue<ENERGY, MODE, VMAX, NW>(a, blk, pe, w, ke, d2, v2);
}

int64_t pair_blocks(const Geo& g) { return ceil_div(g.n, kForceBlock); }

int64_t force_blocks(const Geo& g, bool tiled) { return tiled ? g.ntile : pair_blocks(g); }

static PairArgs make_pair_args(const Geo& g, const LJ& lj, const double* pos, const float* pos32,
                               const int32_t* cell_xyz, const md_pairlist& list)
{
    PairArgs a = {};
    a.pos = (const double4*)pos;
    a.pos32 = (const float4*)pos32;
    a.cell_xyz = cell_xyz;
    a.offsets = list.offsets;
    a.counts = list.counts;
    a.nbr = list.nbr;
    a.nbr_entries = 2 * list.capacity;
    a.n = g.n;
    for (int k = 0; k < 3; ++k) {
        a.L[k] = g.L[k];
        a.invL[k] = g.invL[k];
        a.cs[k] = g.cs[k];
        a.nc[k] = g.nc[k];
    }
    a.exact_all = g.force_minimg_all;
    a.tc = g.tc;
    a.nt = g.nt;
    a.lj = lj;
    for (int code = 0; code < 27; ++code) {
        const int sx = code / 9 - 1, sy = (code / 3) % 3 - 1, sz = code % 3 - 1;
        a.shift[code][0] = (float)(sx * g.cs[0]);
        a.shift[code][1] = (float)(sy * g.cs[1]);
        a.shift[code][2] = (float)(sz * g.cs[2]);
        a.shift[code][3] = 0.0f;
    }
    return a;
}

template <bool ENERGY, int MODE, bool VMAX = false>
static void launch_pairs_mode(const Geo& g, int precision, const PairArgs& a, hipStream_t s, int stage)
{
    if (stage > 0) {
        if (precision == MD_MIXED)
            hipLaunchKernelGGL((k_pairs_tiled<kForceUnroll, ENERGY, MODE, VMAX, true>), dim3((unsigned)g.ntile),
                               dim3(kTileBlock), sizeof(float4) * (size_t)(stage + 1), s, a);
        else
            hipLaunchKernelGGL((k_pairs_tiled<kForceUnroll64, ENERGY, MODE, VMAX, false>), dim3((unsigned)g.ntile),
                               dim3(kTileBlock), sizeof(D3) * (size_t)(stage + 1), s, a);
        return;
    }
    const dim3 grid((unsigned)pair_blocks(g)), block(kForceBlock);
    if (precision == MD_MIXED)
        hipLaunchKernelGGL((k_pairs_mixed<kForceUnroll, ENERGY, MODE, VMAX>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_pairs_fp64<kForceUnroll64, ENERGY, MODE, VMAX>), grid, block, 0, s, a);
}

// Half list: clear the force array, then the pair pass with atomics.
template <bool ENERGY>
static hipError_t launch_pairs_half(const Geo& g, int precision, const PairArgs& a, hipStream_t s)
{
    const int64_t words = (precision == MD_MIXED ? 3 : 6) * g.n;
    if (hipError_t e = launch_fill_i32((int32_t*)a.force, 0, words, s)) return e;
    const dim3 grid((unsigned)pair_blocks(g)), block(kForceBlock);
    if (precision == MD_MIXED)
        hipLaunchKernelGGL((k_pairs_half<kForceUnroll, ENERGY, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_pairs_half<kForceUnroll64, ENERGY, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int MODE, bool VMAX, bool ENERGY>
static void launch_integrate_half(const Geo& g, int precision, const PairArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)pair_blocks(g)), block(kForceBlock);
    if (precision == MD_MIXED)
        hipLaunchKernelGGL((k_integrate_half<MODE, true, VMAX, ENERGY>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_integrate_half<MODE, false, VMAX, ENERGY>), grid, block, 0, s, a);
}

static hipError_t check_tiles(const Geo& g, int precision, const TileIo& t)
{
    if (t.stage <= 0) return hipSuccess;
    if (g.tc <= 0 || !t.start || !t.count || t.stage > tile_stage_cap(precision)) return hipErrorInvalidValue;
    return hipSuccess;
}

hipError_t launch_forces(const Geo& g, const LJ& lj, int precision, const double* pos,
                         const float* pos32, const int32_t* cell_xyz, const md_pairlist& list,
                         const ForceOut& out, hipStream_t s, const TileIo& tio)
{
    if (hipError_t e = check_tiles(g, precision, tio)) return e;
    PairArgs a = make_pair_args(g, lj, pos, pos32, cell_xyz, list);
    a.start = tio.start;
    a.count = tio.count;
    a.force = out.force;
    a.part_pw = out.part;
    a.flags = out.flags;
    if (list.half) {
        if (tio.stage > 0 || !out.force) return hipErrorInvalidValue;
        return out.part ? launch_pairs_half<true>(g, precision, a, s) : launch_pairs_half<false>(g, precision, a, s);
    }
    if (out.part)
        launch_pairs_mode<true, MODE_FORCE>(g, precision, a, s, tio.stage);
    else
        launch_pairs_mode<false, MODE_FORCE>(g, precision, a, s, tio.stage);
    return hipGetLastError();
}

hipError_t launch_force_step(const Geo& g, const LJ& lj, int precision, const StepIo& io, hipStream_t s)
{
    if (hipError_t e = check_tiles(g, precision, io.tile)) return e;
    PairArgs a = make_pair_args(g, lj, io.pos, io.pos32, io.cell_xyz, io.list);
    a.start = io.tile.start;
    a.count = io.tile.count;
    a.force = io.force;
    a.part_pw = io.part_pw;
    a.part_ke = io.part_ke;
    a.flags = io.flags;
    a.vel = io.vel;
    a.pos_ref = io.pos_ref;
    a.pos_out = (double4*)io.pos_out;
    a.pos32_out = (float4*)io.pos32_out;
    a.max_d2 = io.max_d2;
    a.max_v2 = io.max_v2;
    a.dt = io.dt;
    const bool energy = io.part_pw != nullptr;
    if (io.list.half) {
        if (io.gate) return hipErrorInvalidValue;   // the half-list passes take no gate
        // pair pass into the cleared force array, then the integrator
        if (io.tile.stage > 0 || !io.force) return hipErrorInvalidValue;
        hipError_t e = energy ? launch_pairs_half<true>(g, precision, a, s)
                              : launch_pairs_half<false>(g, precision, a, s);
        if (e != hipSuccess) return e;
        if (io.drift && io.track_speed) {
            if (energy) launch_integrate_half<MODE_KKD, true, true>(g, precision, a, s);
            else launch_integrate_half<MODE_KKD, true, false>(g, precision, a, s);
        } else if (io.drift) {
            if (energy) launch_integrate_half<MODE_KKD, false, true>(g, precision, a, s);
            else launch_integrate_half<MODE_KKD, false, false>(g, precision, a, s);
        } else {
            if (energy) launch_integrate_half<MODE_KICK, false, true>(g, precision, a, s);
            else launch_integrate_half<MODE_KICK, false, false>(g, precision, a, s);
        }
        return hipGetLastError();
    }
    a.gate = io.gate;
    if (io.drift && io.track_speed) {
        // the largest drift speed is needed by the DUTC rule only
        if (energy) launch_pairs_mode<true, MODE_KKD, true>(g, precision, a, s, io.tile.stage);
        else launch_pairs_mode<false, MODE_KKD, true>(g, precision, a, s, io.tile.stage);
    } else if (io.drift) {
        if (energy) launch_pairs_mode<true, MODE_KKD>(g, precision, a, s, io.tile.stage);
        else launch_pairs_mode<false, MODE_KKD>(g, precision, a, s, io.tile.stage);
    } else {
        if (energy) launch_pairs_mode<true, MODE_KICK>(g, precision, a, s, io.tile.stage);
        else launch_pairs_mode<false, MODE_KICK>(g, precision, a, s, io.tile.stage);
    }
    return hipGetLastError();
}

}  // namespace md
