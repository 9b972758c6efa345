// Velocity-Verlet integration (Sec. 4.5: second-order symplectic, periodic on
// all axes) with the half-skin rebuild trigger (Sec. 2.3, search-length figure),
// and the fixed-order FP64 reductions of energy and list statistics.
//
// One thread per slot streams pos, vel, force and pos_ref (SoA, coalesced);
// the kernel is bound by HBM bandwidth.  It runs the first half kick and drift
// at the start of a run and the kinetic energy of a state; inside a run the
// kicks and drift after each force evaluation are fused into the pair kernel.
// Block maxima of the squared displacement since the last build go to one
// atomic max (exact, order independent); kinetic-energy block sums go to a
// partials array reduced later in a fixed order (deterministic).

#include "md_internal.h"

namespace md {

__device__ __forceinline__ double wrap_coord(double x, double L, double invL)
{
    double y = x - L * floor(x * invL);
    if (y >= L) y -= L;
    if (y < 0.0) y += L;
    return y;
}

__device__ __forceinline__ float local_coord_i(double x, int c, double cs, double L, double invL)
{
    double l = x - (double)c * cs;
    l -= L * rint((l - 0.5 * cs) * invL);
    return (float)l;
}

// MODE INT_KD: first half kick and drift of a step (the start of a run, when
// no force evaluation precedes it in the same pass).  MODE INT_KE: kinetic
// energy only.  The kicks that follow a force evaluation run inside the pair
// kernel (launch_force_step).
template <int MODE, bool MIXED>
__global__ __launch_bounds__(kStreamBlock) void k_integrate(Geo g, IntArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = g.n;
    const bool valid = i < n;
    const double h = 0.5 * a.dt;
    constexpr bool DRIFT = MODE == INT_KD;
    constexpr bool KE = MODE == INT_KE;
    double* __restrict__ vel = a.vel;
    double4* __restrict__ P = (double4*)a.pos;
    const double* __restrict__ ref = a.pos_ref;
    double ke = 0.0, d2 = 0.0, v2 = 0.0;
    if (valid) {
        // every input is loaded before anything is stored, so all loads of a
        // thread are in flight together
        double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
        double fx = 0.0, fy = 0.0, fz = 0.0;
        if (DRIFT) {
            if (MIXED) {
                const float* __restrict__ F = (const float*)a.force;
                fx = F[i];
                fy = F[n + i];
                fz = F[2 * n + i];
            } else {
                const double* __restrict__ F = (const double*)a.force;
                fx = F[i];
                fy = F[n + i];
                fz = F[2 * n + i];
            }
        }
        double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
        double rx = 0.0, ry = 0.0, rz = 0.0;
        int32_t c = 0;
        if (DRIFT) {
            p = P[i];
            rx = ref[i];
            ry = ref[n + i];
            rz = ref[2 * n + i];
            if (MIXED) c = a.cell_xyz[i];
        }
        if (KE) ke = vx * vx + vy * vy + vz * vz;
        if (DRIFT) {
            vx = vx + h * fx;
            vy = vy + h * fy;
            vz = vz + h * fz;
            v2 = pinned_len2(vx, vy, vz);
            p.x = wrap_coord(p.x + a.dt * vx, g.L[0], g.invL[0]);
            p.y = wrap_coord(p.y + a.dt * vy, g.L[1], g.invL[1]);
            p.z = wrap_coord(p.z + a.dt * vz, g.L[2], g.invL[2]);
            double ex = p.x - rx, ey = p.y - ry, ez = p.z - rz;
            ex -= g.L[0] * rint(ex * g.invL[0]);
            ey -= g.L[1] * rint(ey * g.invL[1]);
            ez -= g.L[2] * rint(ez * g.invL[2]);
            d2 = pinned_len2(ex, ey, ez);
            P[i] = p;
            if (MIXED) {
                ((float4*)a.pos32)[i] =
                    make_float4(local_coord_i(p.x, c & 1023, g.cs[0], g.L[0], g.invL[0]),
                                local_coord_i(p.y, (c >> 10) & 1023, g.cs[1], g.L[1], g.invL[1]),
                                local_coord_i(p.z, (c >> 20) & 1023, g.cs[2], g.L[2], g.invL[2]),
                                __int_as_float(c));
            }
            vel[i] = vx;
            vel[n + i] = vy;
            vel[2 * n + i] = vz;
        }
    }
    __shared__ double s_v[kStreamBlock / 64], s_u[kStreamBlock / 64];
    if (DRIFT) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            d2 = fmax(d2, __shfl_xor(d2, o, 64));
            v2 = fmax(v2, __shfl_xor(v2, o, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            s_v[threadIdx.x >> 6] = d2;
            s_u[threadIdx.x >> 6] = v2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = 0.0, mv = 0.0;
#pragma unroll
            for (int w = 0; w < kStreamBlock / 64; ++w) {
                m = fmax(m, s_v[w]);
                mv = fmax(mv, s_u[w]);
            }
            atomicMax(max_slot(a.max_d2, blockIdx.x), (unsigned long long)__double_as_longlong(m));
            atomicMax(max_slot(a.max_v2, blockIdx.x), (unsigned long long)__double_as_longlong(mv));
        }
    }
    if (KE) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ke += __shfl_xor(ke, o, 64);
        if ((threadIdx.x & 63) == 0) s_v[threadIdx.x >> 6] = ke;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < kStreamBlock / 64; ++w) s += s_v[w];
            a.part_ke[blockIdx.x] = 0.5 * s;
        }
    }
}

hipError_t launch_integrate(const Geo& g, IntMode mode, const IntArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)ceil_div(g.n, kStreamBlock)), block(kStreamBlock);
    const bool mixed = a.precision == MD_MIXED;
    if (mode == INT_KD) {
        if (mixed) hipLaunchKernelGGL((k_integrate<INT_KD, true>), grid, block, 0, s, g, a);
        else hipLaunchKernelGGL((k_integrate<INT_KD, false>), grid, block, 0, s, g, a);
    } else {
        if (mixed) hipLaunchKernelGGL((k_integrate<INT_KE, true>), grid, block, 0, s, g, a);
        else hipLaunchKernelGGL((k_integrate<INT_KE, false>), grid, block, 0, s, g, a);
    }
    return hipGetLastError();
}

// ---- fixed-order reductions -------------------------------------------------
__device__ __forceinline__ double block_sum_1024(double v)
{
    __shared__ double s_w[kReduceBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kReduceBlock / 64; ++w) t += s_w[w];
    __syncthreads();
    return t;
}

// energy[0..3] = (KE, PE, W, KE + PE); also into log_row when given.  Two
// fixed-order levels: block b sums its contiguous share of the partials into
// part3[3b .. 3b+2], then one block sums those in block order.
constexpr int kEnergyBlocks = 256;
__global__ __launch_bounds__(kReduceBlock) void k_reduce_energy_part(const double* __restrict__ part_pw, int64_t nbf,
                                                                     const double* __restrict__ part_ke, int64_t nbi,
                                                                     double* __restrict__ part3,
                                                                     const int32_t* __restrict__ gate)
{
    if (gate && gate[0]) return;
    const int64_t cf = (nbf + gridDim.x - 1) / gridDim.x, ci = (nbi + gridDim.x - 1) / gridDim.x;
    const int64_t f0 = (int64_t)blockIdx.x * cf, f1 = min(f0 + cf, nbf);
    const int64_t i0 = (int64_t)blockIdx.x * ci, i1 = min(i0 + ci, nbi);
    double pe = 0.0, w = 0.0, ke = 0.0;
    for (int64_t b = f0 + threadIdx.x; b < f1; b += kReduceBlock) {
        pe += part_pw[2 * b];
        w += part_pw[2 * b + 1];
    }
    for (int64_t b = i0 + threadIdx.x; b < i1; b += kReduceBlock) ke += part_ke[b];
    pe = block_sum_1024(pe);
    w = block_sum_1024(w);
    ke = block_sum_1024(ke);
    if (threadIdx.x == 0) {
        part3[3 * blockIdx.x] = pe;
        part3[3 * blockIdx.x + 1] = w;
        part3[3 * blockIdx.x + 2] = ke;
    }
}

__global__ __launch_bounds__(kReduceBlock) void k_reduce_energy(const double* __restrict__ part3, int nb,
                                                                double* __restrict__ energy,
                                                                double* __restrict__ log_row,
                                                                const int32_t* __restrict__ gate)
{
    if (gate && gate[0]) return;
    double pe = 0.0, w = 0.0, ke = 0.0;
    if ((int)threadIdx.x < nb) {
        pe = part3[3 * threadIdx.x];
        w = part3[3 * threadIdx.x + 1];
        ke = part3[3 * threadIdx.x + 2];
    }
    pe = block_sum_1024(pe);
    w = block_sum_1024(w);
    ke = block_sum_1024(ke);
    if (threadIdx.x == 0) {
        energy[0] = ke;
        energy[1] = pe;
        energy[2] = w;
        energy[3] = ke + pe;
        if (log_row) {
            log_row[0] = ke;
            log_row[1] = pe;
            log_row[2] = w;
            log_row[3] = ke + pe;
        }
    }
}

hipError_t launch_reduce_energy(const double* part_pw, int64_t nbf, const double* part_ke, int64_t nbi,
                                double* energy, double* log_row, double* scratch, hipStream_t s,
                                const int32_t* gate)
{
    const int64_t most = nbf > nbi ? nbf : nbi;
    const int nb = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(most, kReduceBlock), 1), kEnergyBlocks);
    hipLaunchKernelGGL(k_reduce_energy_part, dim3(nb), dim3(kReduceBlock), 0, s, part_pw, nbf, part_ke, nbi,
                       scratch, gate);
    hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(kReduceBlock), 0, s, (const double*)scratch, nb, energy,
                       log_row, gate);
    return hipGetLastError();
}

// out2[k] = scale_k * sum_b part[2b + k]   (or += when accumulating)
__global__ __launch_bounds__(kReduceBlock) void k_reduce_pair(const double* __restrict__ part, int64_t nb,
                                                              double s0, double s1, double* __restrict__ out2,
                                                              int accumulate)
{
    double a = 0.0, b = 0.0;
    for (int64_t k = threadIdx.x; k < nb; k += kReduceBlock) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    a = block_sum_1024(a);
    b = block_sum_1024(b);
    if (threadIdx.x == 0) {
        out2[0] = (accumulate ? out2[0] : 0.0) + s0 * a;
        out2[1] = (accumulate ? out2[1] : 0.0) + s1 * b;
    }
}

hipError_t launch_reduce_pair(const double* part, int64_t nb, double scale0, double scale1, double* out2,
                              hipStream_t s, bool accumulate)
{
    hipLaunchKernelGGL(k_reduce_pair, dim3(1), dim3(kReduceBlock), 0, s, part, nb, scale0, scale1, out2,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

// status[0] = total entries, status[1] = largest cell block (stride needed):
// per-block (sum, max) partials, then one block combines them in order.
constexpr int kStatsBlocks = 1024;

__global__ __launch_bounds__(kStreamBlock) void k_rows_partial(const int32_t* __restrict__ rows, int64_t ncell,
                                                               long long* __restrict__ part)
{
    __shared__ long long s_sum[kStreamBlock / 64], s_max[kStreamBlock / 64];
    long long sum = 0, mx = 0;
    for (int64_t c = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * kStreamBlock) {
        const long long r = rows[c];
        sum += r;
        mx = r > mx ? r : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o, 64);
        const long long y = __shfl_xor(mx, o, 64);
        mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        s_sum[threadIdx.x >> 6] = sum;
        s_max[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long ts = 0, tm = 0;
        for (int w = 0; w < kStreamBlock / 64; ++w) {
            ts += s_sum[w];
            tm = s_max[w] > tm ? s_max[w] : tm;
        }
        part[2 * blockIdx.x] = ts;
        part[2 * blockIdx.x + 1] = tm;
    }
}

__global__ __launch_bounds__(kStatsBlocks) void k_rows_final(const long long* __restrict__ part, int nb,
                                                             int64_t* __restrict__ status)
{
    __shared__ long long s_sum[kStatsBlocks / 64], s_max[kStatsBlocks / 64];
    long long sum = 0, mx = 0;
    if ((int)threadIdx.x < nb) {
        sum = part[2 * threadIdx.x];
        mx = part[2 * threadIdx.x + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o, 64);
        const long long y = __shfl_xor(mx, o, 64);
        mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        s_sum[threadIdx.x >> 6] = sum;
        s_max[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long ts = 0, tm = 0;
        for (int w = 0; w < kStatsBlocks / 64; ++w) {
            ts += s_sum[w];
            tm = s_max[w] > tm ? s_max[w] : tm;
        }
        status[0] = ts;
        status[1] = tm;
    }
}

hipError_t launch_list_stats(const int32_t* cell_rows, int64_t ncell, int64_t* status, long long* part,
                             hipStream_t s)
{
    const int nb = (int)(ceil_div(ncell, kStreamBlock) < kStatsBlocks ? ceil_div(ncell, kStreamBlock)
                                                                     : kStatsBlocks);
    hipLaunchKernelGGL(k_rows_partial, dim3(nb), dim3(kStreamBlock), 0, s, cell_rows, ncell, part);
    hipLaunchKernelGGL(k_rows_final, dim3(1), dim3(kStatsBlocks), 0, s, (const long long*)part, nb, status);
    return hipGetLastError();
}

__global__ void k_gather_flags(const int64_t* __restrict__ status, const int64_t* __restrict__ err,
                               const int64_t* __restrict__ flags, double* __restrict__ energy,
                               const int64_t* __restrict__ tmax, unsigned long long* __restrict__ mx,
                               int64_t* __restrict__ out, FlagGate g)
{
    // a run already stopped: leave out (and the slots) as the stopping gather left them
    if (g.gate && g.gate[0] && g.idx > 1) return;
    // wave-wide maxima over the slots: largest staged tile neighbourhood,
    // largest squared displacement and drift speed (bit patterns of
    // non-negative doubles order like the values)
    int64_t m = 0;
    unsigned long long md = 0, mv = 0;
    for (int k = threadIdx.x; k < kTileMaxSlots; k += 64) m = max(m, tmax[k]);
    if (g.fold) {
        for (int k = threadIdx.x; k < kMaxSlots; k += 64) {
            md = max(md, mx[k * kMaxSlotStride]);
            mv = max(mv, mx[(kMaxSlots + k) * kMaxSlotStride]);
            if (g.clear) {
                mx[k * kMaxSlotStride] = 0;
                mx[(kMaxSlots + k) * kMaxSlotStride] = 0;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m = max(m, (int64_t)__shfl_xor((long long)m, o, 64));
        md = max(md, (unsigned long long)__shfl_xor((long long)md, o, 64));
        mv = max(mv, (unsigned long long)__shfl_xor((long long)mv, o, 64));
    }
    if (threadIdx.x != 0) return;
    if (g.fold) {
        energy[4] = __longlong_as_double((long long)md);
        energy[5] = __longlong_as_double((long long)mv);
    }
    out[0] = status[0];
    out[1] = status[1];
    out[2] = status[2];
    out[3] = status[3];
    out[4] = err[0];
    out[5] = err[1];
    out[6] = flags[0];
    out[7] = __double_as_longlong(energy[4]);
    out[8] = __double_as_longlong(energy[5]);
    out[9] = err[4];    // large-displacement check: member count
    out[10] = err[5];   // large-displacement check: violation flag
    out[11] = m;        // tiled list: largest staged neighbourhood of a tile
    int32_t stop = 0;
    if (g.gate) {
        stop = ((flags[0] & 1) != 0 || (g.fold && energy[4] > g.thr2)) ? 1 : 0;
        g.gate[0] = stop;
    }
    out[12] = g.idx;
    out[13] = stop;
}

hipError_t launch_gather_flags(const int64_t* status, const int64_t* err, const int64_t* flags, double* energy,
                               const int64_t* tmax, unsigned long long* mx, int64_t* out, hipStream_t s,
                               const FlagGate& gate)
{
    hipLaunchKernelGGL(k_gather_flags, dim3(1), dim3(64), 0, s, status, err, flags, energy, tmax, mx, out, gate);
    return hipGetLastError();
}

}  // namespace md
