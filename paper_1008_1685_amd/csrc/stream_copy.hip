// A STREAM-style device copy: the measured bandwidth ceiling that the
// roofline of the push kernels is read against, beside the published peak.
// Not part of the method; built into its own library (libstreamcopy.so).
#include <hip/hip_runtime.h>

#include "stream_copy.h"

#include <stddef.h>
#include <stdint.h>

namespace {

constexpr int kCopyThreads = 256;

// one 16-byte element per thread: every wave reads and writes 1 KB
// contiguous, the simplest pattern that keeps the most loads in flight
__global__ __launch_bounds__(kCopyThreads) void k_stream_copy(const uint4* __restrict__ a,
                                                              uint4* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * kCopyThreads + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace

extern "C" {

// (declared in stream_copy.h)
int stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16) return (int)hipErrorInvalidValue;
  const size_t n = bytes / 16;
  if (n == 0) return 0;
  const size_t blocks = (n + kCopyThreads - 1) / kCopyThreads;
  if (blocks > 0x7fffffffull) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kCopyThreads), 0,
                     reinterpret_cast<hipStream_t>(stream), static_cast<const uint4*>(src),
                     static_cast<uint4*>(dst), n);
  return (int)hipGetLastError();
}

}  // extern "C"
