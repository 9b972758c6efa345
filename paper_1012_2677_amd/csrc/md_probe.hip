// Streaming probes of achievable HBM bandwidth (read, copy, triad), the
// yardstick the hot path's kernels are priced against beside the vendor peak.
//
// Each thread moves four 16-byte vectors per launch-grid slot, all loads of
// the slot issued before any store, with consecutive threads on consecutive
// vectors (64-byte runs per lane group, full 64-lane waves); the grid covers
// the array once.  The non-temporal variants mark every access as streaming.

#include <algorithm>

#include "md_internal.h"
#include "md_probe.h"

namespace md {

constexpr int kProbeBlock = 256;
constexpr int kProbeVec = 4;   // 16-byte vectors per thread

template <bool NT>
__device__ __forceinline__ double2 ld(const double2* p)
{
    if constexpr (NT) {
        double2 v;
        v.x = __builtin_nontemporal_load(&p->x);
        v.y = __builtin_nontemporal_load(&p->y);
        return v;
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ void st(double2* p, double2 v)
{
    if constexpr (NT) {
        __builtin_nontemporal_store(v.x, &p->x);
        __builtin_nontemporal_store(v.y, &p->y);
    } else {
        *p = v;
    }
}

template <int OP, bool NT>
__global__ __launch_bounds__(kProbeBlock) void k_probe(const double2* __restrict__ a, double2* __restrict__ b,
                                                     double2* __restrict__ c, int64_t nvec)
{
    const int64_t base = (int64_t)blockIdx.x * (kProbeBlock * kProbeVec) + threadIdx.x;
    double2 x[kProbeVec], y[kProbeVec];
#pragma unroll
    for (int k = 0; k < kProbeVec; ++k) {
        const int64_t i = base + k * kProbeBlock;
        if (i < nvec) {
            x[k] = ld<NT>(a + i);
            if (OP == MD_PROBE_TRIAD) y[k] = ld<NT>(b + i);
        }
    }
    if (OP == MD_PROBE_READ) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kProbeVec; ++k)
            if (base + k * kProbeBlock < nvec) s += x[k].x + x[k].y;
        // never true for the probe's data (finite values); keeps the loads
        if (s == -1.0e300) b[0] = make_double2(s, s);
        return;
    }
#pragma unroll
    for (int k = 0; k < kProbeVec; ++k) {
        const int64_t i = base + k * kProbeBlock;
        if (i < nvec) {
            if (OP == MD_PROBE_COPY) st<NT>(b + i, x[k]);
            else st<NT>(c + i, make_double2(x[k].x + 3.0 * y[k].x, x[k].y + 3.0 * y[k].y));
        }
    }
}

template <int OP>
static void launch_probe(bool nt, const double2* a, double2* b, double2* c, int64_t nvec, hipStream_t s)
{
    const dim3 grid((unsigned)ceil_div(nvec, (int64_t)kProbeBlock * kProbeVec)), block(kProbeBlock);
    if (nt) hipLaunchKernelGGL((k_probe<OP, true>), grid, block, 0, s, a, b, c, nvec);
    else hipLaunchKernelGGL((k_probe<OP, false>), grid, block, 0, s, a, b, c, nvec);
}

}  // namespace md

using namespace md;

extern "C" int md_hbm_probe(int32_t kind, const double* a, double* b, double* c, size_t nbytes, int32_t reps,
                            float* ms_best, hipStream_t stream)
{
    const int op = kind & 3;
    const bool nt = (kind & MD_PROBE_NT) != 0;
    if (kind < 0 || kind > (MD_PROBE_TRIAD | MD_PROBE_NT) || op > MD_PROBE_TRIAD)
        return set_error(MD_ERR_ARG, "md_hbm_probe: unknown kind");
    if (!a || !ms_best || nbytes == 0 || nbytes % 64 != 0 || reps < 1)
        return set_error(MD_ERR_ARG, "md_hbm_probe: need a, ms_best, nbytes > 0 (multiple of 64), reps >= 1");
    if ((op == MD_PROBE_COPY || op == MD_PROBE_READ) && !b)
        return set_error(MD_ERR_ARG, "md_hbm_probe: read and copy need b");
    if (op == MD_PROBE_TRIAD && (!b || !c))
        return set_error(MD_ERR_ARG, "md_hbm_probe: triad needs b and c");
    const int64_t nvec = (int64_t)(nbytes / 16);
    const double2* A2 = (const double2*)a;
    double2* B2 = (double2*)b;
    double2* C2 = (double2*)c;
    auto launch = [&]() {
        if (op == MD_PROBE_READ) launch_probe<MD_PROBE_READ>(nt, A2, B2, C2, nvec, stream);
        else if (op == MD_PROBE_COPY) launch_probe<MD_PROBE_COPY>(nt, A2, B2, C2, nvec, stream);
        else launch_probe<MD_PROBE_TRIAD>(nt, A2, B2, C2, nvec, stream);
        return hipGetLastError();
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(MD_ERR_HIP, "md_hbm_probe: event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(MD_ERR_HIP, "md_hbm_probe: event");
    }
    int rc = MD_OK;
    float best = 1e30f;
    if (launch() != hipSuccess) rc = set_error(MD_ERR_HIP, "md_hbm_probe: launch");
    for (int r = 0; r < reps && rc == MD_OK; ++r) {
        float ms = 0.f;
        if (hipEventRecord(e0, stream) != hipSuccess || launch() != hipSuccess ||
            hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = set_error(MD_ERR_HIP, "md_hbm_probe: timed launch");
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == MD_OK) *ms_best = best;
    return rc;
}
