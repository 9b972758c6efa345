/*
 * md_probe.h -- achievable-HBM-bandwidth probe of the MI355X (gfx950) build.
 *
 * Not a step of the method: the measurement of the hot path prices its
 * kernels against the bandwidth that plain streaming kernels reach on the same
 * GPU in the same job (read, copy and triad over arrays much larger than the
 * 256 MB last-level cache), beside the 8 TB/s vendor peak.
 *
 * Status codes are those of md.h; md_last_error() gives the message.
 */
#ifndef MD355_MD_PROBE_H
#define MD355_MD_PROBE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* probe kernels (md_hbm_probe kind): the operation in the low bits, plus
 * MD_PROBE_NT for non-temporal loads and stores */
#define MD_PROBE_READ  0   /* s += a[i]                 (bytes read: nbytes)            */
#define MD_PROBE_COPY  1   /* b[i] = a[i]               (read nbytes, write nbytes)     */
#define MD_PROBE_TRIAD 2   /* c[i] = a[i] + 3 b[i]      (read 2 nbytes, write nbytes)   */
#define MD_PROBE_NT    4

/* Runs one probe kernel reps times back to back on stream (after one untimed
 * launch) and returns the shortest launch in *ms_best (HIP events around each
 * launch).  a, b, c: device arrays of nbytes each (FP64 elements; b and c may
 * be NULL where the kind does not use them; no aliasing).  nbytes: a positive
 * multiple of 64.  Synchronises the stream.  MD_ERR_ARG for a bad kind, size
 * or missing array; MD_ERR_HIP for launch or event failures. */
int md_hbm_probe(int32_t kind, const double* a, double* b, double* c, size_t nbytes, int32_t reps,
                 float* ms_best, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MD355_MD_PROBE_H */
