/* A STREAM-style device copy, built into its own library
 * (paper_1008_1685_amd/libstreamcopy.so).  It is a measurement aid, not part
 * of the method: its bandwidth is the measured ceiling that the push
 * kernels' achieved HBM bandwidth is read against, beside the published
 * peak of the device. */
#ifndef STREAM_COPY_H
#define STREAM_COPY_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copy `bytes` from src to dst, device memory, on `stream` (a hipStream_t;
 * NULL: the default stream), one 16-byte element per thread.  bytes must be
 * a multiple of 16 and both pointers 16-byte aligned; the ranges must not
 * overlap.  Ownership stays with the caller; asynchronous on the stream.
 * Returns 0, or a HIP error code: hipErrorInvalidValue (1) for a size or
 * alignment it does not take or a copy of more than 2^31 - 1 work-groups,
 * else the launch's error. */
int stream_copy(const void* src, void* dst, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif
