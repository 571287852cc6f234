// Streaming device copy: the achievable HBM bandwidth that the apply's
// passes are measured against (a copy of S bytes reads S and writes S).
//
// Each lane moves 16-byte vectors, four independent loads in flight per
// lane; loads and stores are non-temporal.
#include "common.h"

namespace ls {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Block b copies vectors [1024 b, 1024 b + 1024): four loads per lane in
// flight, then four stores.  Measured on MI355X (2 GiB): 5.99 TB/s with
// non-temporal hints, 5.62 TB/s without, 4.36 TB/s as a grid-stride loop
// over a CU-sized grid; reads alone 6.33 TB/s, writes alone 5.97 TB/s.
__global__ __launch_bounds__(256) void stream_copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                          long nvec) {
  const long b = (long)blockIdx.x * 1024 + threadIdx.x;
  u32x4 v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (b + 256 * u < nvec) v[u] = __builtin_nontemporal_load(src + b + 256 * u);
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (b + 256 * u < nvec) __builtin_nontemporal_store(v[u], dst + b + 256 * u);
}

__global__ void tail_copy_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, long nb) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) dst[i] = src[i];
}

}  // namespace
}  // namespace ls

using namespace ls;

extern "C" ls_status ls_hbm_copy(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream) {
  if (bytes == 0) return LS_OK;
  if (!dst_dev || !src_dev) return LS_EINVAL;
  if ((reinterpret_cast<uintptr_t>(dst_dev) | reinterpret_cast<uintptr_t>(src_dev)) & 15) return LS_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const long nvec = (long)(bytes / 16);
  if (nvec > 0) {
    const long blocks = (nvec + 1023) / 1024;
    if (blocks > 0x7fffffffL) return LS_EINVAL;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const u32x4*>(src_dev), static_cast<u32x4*>(dst_dev), nvec);
    LS_HIP(hipGetLastError());
  }
  const long tail = (long)(bytes - (size_t)nvec * 16);
  if (tail > 0) {
    hipLaunchKernelGGL(tail_copy_kernel, dim3(1), dim3(64), 0, s,
                       static_cast<const unsigned char*>(src_dev) + nvec * 16,
                       static_cast<unsigned char*>(dst_dev) + nvec * 16, tail);
    LS_HIP(hipGetLastError());
  }
  return LS_OK;
}
