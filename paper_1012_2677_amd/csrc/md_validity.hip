// Large-displacement check of a pair list (Sec. 2.3, Alg. alg_validity_check).
//
// The list built at positions q_ref holds every pair whose pinned squared
// distance was below rs^2.  It expires only if some pair not listed (old
// squared distance >= rs^2) now interacts (squared distance < rc^2), which
// needs both partners to have moved: only particles with displacement greater
// than t = (rs - rc) - (largest displacement) can take part.  The host derives
// t from the largest displacement and passes t^2 (or "everyone" when t < 0);
//   k_ldc_collect  gathers the members into a list of at most `cap` slots and
//                  counts all of them (one atomic per block: the member order
//                  is arbitrary, the count exact);
//   k_ldc_pairs    tests every pair of listed members, 64 x 64 tiles with the
//                  partners staged in LDS, and raises a flag on a violation.
// Distances use the pinned form d = x_j - x_i, minimum image,
// r^2 = fma(dz, dz, fma(dy, dy, dx * dx)) in FP64, so the decision depends on
// the positions alone.  One more kernel, k_ldc_disp, takes the largest pinned
// squared displacement for the stand-alone call.

#include "md_internal.h"

namespace md {

struct LdcArgs {
    const double4* pos;
    const double* ref;        // [3][n]
    int64_t n;
    double L[3], invL[3];
    double t2;                // member iff d2 > t2 (or all)
    int32_t all;
    int64_t cap;
    int32_t* list;
    unsigned long long* count;
    unsigned long long* flag;
    unsigned long long* max_d2;
    double rs2, rc2;
};

__device__ __forceinline__ double pinned_r2(double dx, double dy, double dz, const double* L, const double* invL)
{
    dx = dx - L[0] * rint(dx * invL[0]);
    dy = dy - L[1] * rint(dy * invL[1]);
    dz = dz - L[2] * rint(dz * invL[2]);
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, __dmul_rn(dx, dx)));
}

__device__ __forceinline__ double disp2(const LdcArgs& a, int64_t i)
{
    const double4 p = a.pos[i];
    return pinned_r2(p.x - a.ref[i], p.y - a.ref[a.n + i], p.z - a.ref[2 * a.n + i], a.L, a.invL);
}

__global__ __launch_bounds__(kStreamBlock) void k_ldc_disp(LdcArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double d2 = i < a.n ? disp2(a, i) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d2 = fmax(d2, __shfl_xor(d2, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(a.max_d2, (unsigned long long)__double_as_longlong(d2));
}

// Members are counted per block first, so the counter sees one atomic per
// block that has any.
__global__ __launch_bounds__(kStreamBlock) void k_ldc_collect(LdcArgs a)
{
    constexpr int NW = kStreamBlock / 64;
    __shared__ unsigned s_cnt[NW];
    __shared__ unsigned long long s_base;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool member = i < a.n && (a.all || disp2(a, i) > a.t2);
    const uint64_t m = __ballot(member);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_cnt[wave] = (unsigned)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int w = 0; w < NW; ++w) {
            const unsigned c = s_cnt[w];
            s_cnt[w] = tot;   // exclusive offset of the wave inside the block
            tot += c;
        }
        s_base = tot ? atomicAdd(a.count, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    const unsigned long long k = s_base + s_cnt[wave] + mbcnt64(m);
    if (member && k < (unsigned long long)a.cap) a.list[k] = (int32_t)i;
}

__global__ __launch_bounds__(64) void k_ldc_pairs(LdcArgs a)
{
    const int ta = (int)blockIdx.x, tb = (int)blockIdx.y;
    if (tb < ta) return;
    const unsigned long long total = *a.count;
    if (total > (unsigned long long)a.cap) return;   // too many members: expired outright
    const int cnt = (int)total;
    if (ta * 64 >= cnt || tb * 64 >= cnt) return;
    __shared__ double s_q[64][3], s_r[64][3];
    const int lane = (int)threadIdx.x;
    const int b = tb * 64 + lane;
    if (b < cnt) {
        const int64_t j = a.list[b];
        const double4 p = a.pos[j];
        s_q[lane][0] = p.x;
        s_q[lane][1] = p.y;
        s_q[lane][2] = p.z;
        s_r[lane][0] = a.ref[j];
        s_r[lane][1] = a.ref[a.n + j];
        s_r[lane][2] = a.ref[2 * a.n + j];
    }
    __syncthreads();
    const int ia = ta * 64 + lane;
    if (ia >= cnt) return;
    const int64_t i = a.list[ia];
    const double4 pi = a.pos[i];
    const double rx = a.ref[i], ry = a.ref[a.n + i], rz = a.ref[2 * a.n + i];
    const int kend = cnt - tb * 64 < 64 ? cnt - tb * 64 : 64;
    bool bad = false;
    for (int k = 0; k < kend; ++k) {
        if (tb == ta && k <= lane) continue;   // each unordered pair once
        const double ro = pinned_r2(s_r[k][0] - rx, s_r[k][1] - ry, s_r[k][2] - rz, a.L, a.invL);
        const double rn = pinned_r2(s_q[k][0] - pi.x, s_q[k][1] - pi.y, s_q[k][2] - pi.z, a.L, a.invL);
        bad = bad || (ro >= a.rs2 && rn < a.rc2);
    }
    if (bad) atomicOr(a.flag, 1ull);
}

static LdcArgs ldc_args(const Geo& g, const double* pos, const double* pos_ref, double rc, double rs)
{
    LdcArgs a = {};
    a.pos = (const double4*)pos;
    a.ref = pos_ref;
    a.n = g.n;
    for (int k = 0; k < 3; ++k) {
        a.L[k] = g.L[k];
        a.invL[k] = g.invL[k];
    }
    a.rs2 = rs * rs;
    a.rc2 = rc * rc;
    return a;
}

hipError_t launch_ldc_disp(const Geo& g, const double* pos, const double* pos_ref, unsigned long long* max_d2,
                           hipStream_t s)
{
    LdcArgs a = ldc_args(g, pos, pos_ref, 0.0, 0.0);
    a.max_d2 = max_d2;
    hipLaunchKernelGGL(k_ldc_disp, dim3((unsigned)ceil_div(g.n, kStreamBlock)), dim3(kStreamBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ldc_check(const Geo& g, const double* pos, const double* pos_ref, double rc, double rs,
                            double t, int64_t cap, int32_t* list, unsigned long long* count,
                            unsigned long long* flag, hipStream_t s)
{
    LdcArgs a = ldc_args(g, pos, pos_ref, rc, rs);
    a.all = t < 0.0;
    a.t2 = t * t;
    a.cap = cap;
    a.list = list;
    a.count = count;
    a.flag = flag;
    hipLaunchKernelGGL(k_ldc_collect, dim3((unsigned)ceil_div(g.n, kStreamBlock)), dim3(kStreamBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || cap <= 0) return e;
    const unsigned tiles = (unsigned)ceil_div(cap, 64);
    hipLaunchKernelGGL(k_ldc_pairs, dim3(tiles, tiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace md
