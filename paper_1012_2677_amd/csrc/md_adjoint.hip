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
    double* Hu;
    double* part;
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

// mode 0: Hessian-vector product (+ parameter VJP partials); mode 1: dU/dtheta partials
template <int G, int MODE>
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
        if (MODE == 0) {
            uxi = a.u[key];
            uyi = a.u[n + key];
            uzi = a.u[2 * n + key];
        }
        minimg = a.exact_all || boundary_cell_a(a.cell_xyz[key], a.nc);
    }
    const LJ& lj = a.lj;
    double hx = 0.0, hy = 0.0, hz = 0.0, t0 = 0.0, t1 = 0.0;
    for (int t = sub; t < cnt; t += G) {
        const uint32_t e = a.nbr[off + t];
        const int64_t j = e & kSlotMask;
        const double4 pj = a.pos[j];
        double dx = pj.x - xi, dy = pj.y - yi, dz = pj.z - zi;
        if (minimg) {
            dx -= a.L[0] * rint(dx * a.invL[0]);
            dy -= a.L[1] * rint(dy * a.invL[1]);
            dz -= a.L[2] * rint(dz * a.invL[2]);
        }
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < lj.rc2)) continue;
        const double r2i = 1.0 / r2;
        const double r6i = r2i * r2i * r2i;
        if (MODE == 0) {
            const double g = r2i * r6i * (lj.A * r6i - lj.B) - lj.C8;
            const double gp = r2i * r2i * r6i * (-7.0 * lj.A * r6i + 4.0 * lj.B);
            const double dux = a.u[j] - uxi, duy = a.u[n + j] - uyi, duz = a.u[2 * n + j] - uzi;
            const double ddu = dx * dux + dy * duy + dz * duz;
            const double c = 2.0 * gp * ddu;
            hx += c * dx + g * dux;
            hy += c * dy + g * duy;
            hz += c * dz + g * duz;
            // dg/deps = g/eps;  dg/dsigma = (12 A s^-7 - 6 B s^-4 - Cs) / sigma
            t0 += (g / lj.eps) * ddu;
            t1 += ((12.0 * lj.A * r6i - 6.0 * lj.B) * r6i * r2i - lj.Cs) / lj.sigma * ddu;
        } else {
            const double V = r6i * (lj.A4 * r6i - lj.B4) + lj.C2 * r2 + lj.C0;
            const double sa = r6i * r6i + 6.0 * r2 * lj.rc14i - 7.0 * lj.rc12i;
            const double sb = r6i + 3.0 * r2 * lj.rc8i - 4.0 * lj.rc6i;
            t0 += V / lj.eps;
            t1 += (12.0 * lj.A4 * sa - 6.0 * lj.B4 * sb) / lj.sigma;
        }
    }
    if (MODE == 0) {
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            hx += __shfl_xor(hx, o, G);
            hy += __shfl_xor(hy, o, G);
            hz += __shfl_xor(hz, o, G);
        }
        if (valid && sub == 0) {
            a.Hu[key] = hx;
            a.Hu[n + key] = hy;
            a.Hu[2 * n + key] = hz;
        }
    }
    if (a.part) block_partial2_a<kForceBlock>(0.5 * t0, 0.5 * t1, a.part, blk);
}

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
    a.Hu = nullptr;
    a.part = nullptr;
    a.n = g.n;
    for (int k = 0; k < 3; ++k) {
        a.L[k] = g.L[k];
        a.invL[k] = g.invL[k];
        a.nc[k] = g.nc[k];
    }
    a.exact_all = g.exact_all;
    a.lj = lj;
    return a;
}

hipError_t launch_hvp(const Geo& g, const LJ& lj, const double* pos, const int32_t* cell_xyz,
                      const md_pairlist& list, const double* u, double* Hu, double* part, hipStream_t s)
{
    AdjArgs a = make_args(g, lj, pos, cell_xyz, list);
    a.u = u;
    a.Hu = Hu;
    a.part = part;
    hipLaunchKernelGGL((k_adjoint<kLanesPerKey, 0>), dim3((unsigned)ceil_div(g.n, kKeysPerBlock)),
                       dim3(kForceBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_param_grad(const Geo& g, const LJ& lj, const double* pos, const int32_t* cell_xyz,
                             const md_pairlist& list, double* part, hipStream_t s)
{
    AdjArgs a = make_args(g, lj, pos, cell_xyz, list);
    a.part = part;
    hipLaunchKernelGGL((k_adjoint<kLanesPerKey, 1>), dim3((unsigned)ceil_div(g.n, kKeysPerBlock)),
                       dim3(kForceBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace md
