// Adjoint kernels of the LJ force field (FP64), same row layout and lane
// grouping as the force kernel.
//
// Hessian-vector product.  With s = r^2, d = q_j - q_i, du = u_j - u_i and
// g(s) = -V'(r)/r, the force on i is F_i = -sum_j g d, so
//   (H u)_i = -dF_i[u] = sum_j [ 2 g'(s) (d . du) d + g du ],
// summed over listed partners with r < rc.  Each lane keeps its partial
// (H u)_i in registers; the group reduces it with shuffles.  The parameter
// derivative u . dF/dtheta = sum_pairs (dg/dtheta) d . du is accumulated over
// the full list and halved (each pair appears twice).
//
// Parameter gradient of U: dU/deps = U/eps and dU/dsigma = sum_pairs dV/dsigma
// with V = 4 eps [sigma^12 a(r) - sigma^6 b(r)],
//   a = r^-12 + 6 r^2 rc^-14 - 7 rc^-12,  b = r^-6 + 3 r^2 rc^-8 - 4 rc^-6,
// dV/dsigma = (48 eps sigma^12 a - 24 eps sigma^6 b) / sigma.

#include "md_internal.h"

namespace md {

struct AdjArgs {
    const double4* pos;
    const int32_t* cell_xyz;
    const int64_t* offsets;
    const int32_t* counts;
    const uint32_t* nbr;
    const double* u;
    double* out;
    double* u_out;
    double* part;
    double alpha, beta, gamma, cu, cU, dt;
    double inv_eps, inv_sigma;   // 1/eps and 1/sigma, computed on the host
    int64_t n;
    double L[3], invL[3];
    int32_t nc[3];
    int32_t exact_all;
    LJ lj;
};

__device__ __forceinline__ bool boundary_cell_a(int32_t c, const int32_t* nc)
{
    const int x = c & 1023, y = (c >> 10) & 1023, z = (c >> 20) & 1023;
    return x == 0 || x == nc[0] - 1 || y == 0 || y == nc[1] - 1 || z == 0 || z == nc[2] - 1;
}

template <int BLOCK>
__device__ __forceinline__ void block_partial2_a(double a, double b, double* part, int64_t blk)
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

// One pass over the list for the key's partners with r < rc, accumulating
//   Hu_i  = sum_j [2 g'(s) (d . du) d + g du]        (if HAS_U; du = u_j - u_i)
//   F_i   = -sum_j g d
//   t_e   = sum (dg/deps) d . du,   t_s = sum (dg/dsigma) d . du   (if HAS_U)
//   v_e   = sum V / eps,            v_s = sum dV/dsigma
// then out_i = alpha out_i + beta Hu_i + gamma F_i (when out != nullptr),
// u_out_i = u_i + dt out_i (when u_out != nullptr), and the block partials
// (cu t_e + cU v_e, cu t_s + cU v_s) / 2 (each pair is visited twice).
template <int G, int U, bool HAS_U>
__global__ __launch_bounds__(kForceBlock) void k_adjoint(AdjArgs a)
{
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t key = blk * (kForceBlock / G) + threadIdx.x / G;
    const int sub = threadIdx.x % G;
    const bool valid = key < a.n;
    const int64_t n = a.n;
    int64_t off = 0;
    int cnt = 0;
    double xi = 0.0, yi = 0.0, zi = 0.0, uxi = 0.0, uyi = 0.0, uzi = 0.0;
    bool minimg = false;
    if (valid) {
        off = a.offsets[key];
        cnt = a.counts[key];
        const double4 p = a.pos[key];
        xi = p.x;
        yi = p.y;
        zi = p.z;
        if (HAS_U) {
            uxi = a.u[key];
            uyi = a.u[n + key];
            uzi = a.u[2 * n + key];
        }
        minimg = a.exact_all || boundary_cell_a(a.cell_xyz[key], a.nc);
    }
    const LJ& lj = a.lj;
    double hx = 0.0, hy = 0.0, hz = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    double te = 0.0, ts = 0.0, ve = 0.0, vs = 0.0;
    // U row entries per lane at a time: their loads, then the partners'
    // positions and u, then the pair terms, so that several gathers are in
    // flight per lane (slots past the row's end read the key itself and are
    // skipped)
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    for (int t0 = sub; t0 < cnt; t0 += G * U) {
        uint32_t e[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int t = t0 + q * G;
            e[q] = t < cnt ? a.nbr[off + t] : kNone;
        }
        double4 pj[U];
        double ujx[U], ujy[U], ujz[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t j = e[q] != kNone ? (int64_t)(e[q] & kSlotMask) : key;
            pj[q] = a.pos[j];
            if (HAS_U) {
                ujx[q] = a.u[j];
                ujy[q] = a.u[n + j];
                ujz[q] = a.u[2 * n + j];
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (e[q] == kNone) continue;
            double dx = pj[q].x - xi, dy = pj[q].y - yi, dz = pj[q].z - zi;
            if (minimg) {
                dx -= a.L[0] * rint(dx * a.invL[0]);
                dy -= a.L[1] * rint(dy * a.invL[1]);
                dz -= a.L[2] * rint(dz * a.invL[2]);
            }
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < lj.rc2)) continue;
            const double r2i = rcp64(r2);
            const double r6i = r2i * r2i * r2i;
            const double g = r2i * r6i * (lj.A * r6i - lj.B) - lj.C8;
            fx -= g * dx;
            fy -= g * dy;
            fz -= g * dz;
            if (HAS_U) {
                const double gp = r2i * r2i * r6i * (-7.0 * lj.A * r6i + 4.0 * lj.B);
                const double dux = ujx[q] - uxi, duy = ujy[q] - uyi, duz = ujz[q] - uzi;
                const double ddu = dx * dux + dy * duy + dz * duz;
                const double c = 2.0 * gp * ddu;
                hx += c * dx + g * dux;
                hy += c * dy + g * duy;
                hz += c * dz + g * duz;
                // dg/deps = g/eps;  dg/dsigma = (12 A s^-7 - 6 B s^-4 - Cs) / sigma
                te += g * a.inv_eps * ddu;
                ts += ((12.0 * lj.A * r6i - 6.0 * lj.B) * r6i * r2i - lj.Cs) * a.inv_sigma * ddu;
            }
            const double V = r6i * (lj.A4 * r6i - lj.B4) + lj.C2 * r2 + lj.C0;
            const double sa = r6i * r6i + 6.0 * r2 * lj.rc14i - 7.0 * lj.rc12i;
            const double sb = r6i + 3.0 * r2 * lj.rc8i - 4.0 * lj.rc6i;
            ve += V * a.inv_eps;
            vs += (12.0 * lj.A4 * sa - 6.0 * lj.B4 * sb) * a.inv_sigma;
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, G);
        fy += __shfl_xor(fy, o, G);
        fz += __shfl_xor(fz, o, G);
        if (HAS_U) {
            hx += __shfl_xor(hx, o, G);
            hy += __shfl_xor(hy, o, G);
            hz += __shfl_xor(hz, o, G);
        }
    }
    if (valid && sub == 0 && a.out) {
        double ox = a.beta * hx + a.gamma * fx;
        double oy = a.beta * hy + a.gamma * fy;
        double oz = a.beta * hz + a.gamma * fz;
        if (a.alpha != 0.0) {
            ox += a.alpha * a.out[key];
            oy += a.alpha * a.out[n + key];
            oz += a.alpha * a.out[2 * n + key];
        }
        a.out[key] = ox;
        a.out[n + key] = oy;
        a.out[2 * n + key] = oz;
        if (a.u_out) {
            a.u_out[key] = uxi + a.dt * ox;
            a.u_out[n + key] = uyi + a.dt * oy;
            a.u_out[2 * n + key] = uzi + a.dt * oz;
        }
    }
    if (a.part)
        block_partial2_a<kForceBlock>(0.5 * (a.cu * te + a.cU * ve), 0.5 * (a.cu * ts + a.cU * vs), a.part, blk);
}

#ifndef MD_ADJ_UNROLL
#define MD_ADJ_UNROLL 2
#endif
constexpr int kAdjUnroll = MD_ADJ_UNROLL;   // row entries in flight per lane

static AdjArgs make_args(const Geo& g, const LJ& lj, const double* pos, const int32_t* cell_xyz,
                         const md_pairlist& list)
{
    AdjArgs a;
    a.pos = (const double4*)pos;
    a.cell_xyz = cell_xyz;
    a.offsets = list.offsets;
    a.counts = list.counts;
    a.nbr = list.nbr;
    a.u = nullptr;
    a.out = nullptr;
    a.u_out = nullptr;
    a.part = nullptr;
    a.alpha = a.beta = a.gamma = a.cu = a.cU = a.dt = 0.0;
    a.n = g.n;
    for (int k = 0; k < 3; ++k) {
        a.L[k] = g.L[k];
        a.invL[k] = g.invL[k];
        a.nc[k] = g.nc[k];
    }
    a.exact_all = g.exact_all;
    a.lj = lj;
    a.inv_eps = 1.0 / lj.eps;
    a.inv_sigma = 1.0 / lj.sigma;
    return a;
}

static void launch_adj(const Geo& g, const AdjArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)ceil_div(g.n, kKeysPerBlock)), block(kForceBlock);
    if (a.u)
        hipLaunchKernelGGL((k_adjoint<kLanesPerKey, kAdjUnroll, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint<kLanesPerKey, kAdjUnroll, false>), grid, block, 0, s, a);
}

hipError_t launch_hvp(const Geo& g, const LJ& lj, const double* pos, const int32_t* cell_xyz,
                      const md_pairlist& list, const double* u, double* Hu, double* part, hipStream_t s)
{
    AdjArgs a = make_args(g, lj, pos, cell_xyz, list);
    a.u = u;
    a.out = Hu;
    a.beta = 1.0;
    a.part = part;
    a.cu = 1.0;
    launch_adj(g, a, s);
    return hipGetLastError();
}

hipError_t launch_param_grad(const Geo& g, const LJ& lj, const double* pos, const int32_t* cell_xyz,
                             const md_pairlist& list, double* part, hipStream_t s)
{
    AdjArgs a = make_args(g, lj, pos, cell_xyz, list);
    a.part = part;
    a.cU = 1.0;
    launch_adj(g, a, s);
    return hipGetLastError();
}

hipError_t launch_adjoint_kick(const Geo& g, const LJ& lj, const double* pos, const int32_t* cell_xyz,
                               const md_pairlist& list, const double* u, double* out, double* u_out,
                               const AdjCoef& k, double* part, hipStream_t s)
{
    AdjArgs a = make_args(g, lj, pos, cell_xyz, list);
    a.u = u;
    a.out = out;
    a.u_out = u_out;
    a.alpha = k.alpha;
    a.beta = k.beta;
    a.gamma = k.gamma;
    a.cu = k.cu;
    a.cU = k.cU;
    a.dt = k.dt;
    a.part = part;
    launch_adj(g, a, s);
    return hipGetLastError();
}

}  // namespace md
