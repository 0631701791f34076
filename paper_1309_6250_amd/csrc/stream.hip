// Read-rate probe: a linear stream of 16-byte reads over a device buffer, with no writes but one
// that practically never happens (it keeps the loads alive).  Its rate is the achievable ceiling of
// reading device memory, the figure the gather's algorithmic bandwidth is compared with (a copy
// also writes, so it understates what a read-only kernel can reach).
#include "common.hpp"

namespace pws {

constexpr int STREAM_THREADS = 256;
constexpr int STREAM_BLOCKS = 65536;      // 256 workgroups per compute unit over the pass, grid-strided
constexpr int STREAM_UNROLL = 8;

// Eight independent 16-byte loads in flight per lane, marked nontemporal (the data is read once):
// of the patterns measured on MI355X over 4 GiB (grid-strided or one contiguous chunk per
// workgroup, 4 or 8 loads in flight, 1024 to 65536 workgroups, with and without the nontemporal
// hint) this one read fastest.
__global__ __launch_bounds__(STREAM_THREADS) void k_stream_read(const u4v* __restrict__ p, int64_t n16,
                                                                uint32_t* sink) {
  const int64_t stride = (int64_t)STREAM_BLOCKS * STREAM_THREADS;
  int64_t i = (int64_t)blockIdx.x * STREAM_THREADS + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (STREAM_UNROLL - 1) * stride < n16; i += STREAM_UNROLL * stride) {
    u4v v[STREAM_UNROLL];
#pragma unroll
    for (int u = 0; u < STREAM_UNROLL; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
    for (int u = 0; u < STREAM_UNROLL; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n16; i += stride) {
    const u4v a = __builtin_nontemporal_load(p + i);
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;
}

}  // namespace pws

using namespace pws;

extern "C" int spline_stream_read(const void* buf, int64_t bytes, void* sink, void* stream) {
  clear_error();
  if (bytes < 0) return fail(SPL_EINVAL, "bytes = %lld < 0", (long long)bytes);
  if (bytes % 16) return fail(SPL_EINVAL, "bytes = %lld is not a multiple of 16", (long long)bytes);
  if (bytes == 0) return SPL_OK;
  if (!buf || !sink) return fail(SPL_EINVAL, "buf and sink must be device pointers");
  if ((uintptr_t)buf % 16 || (uintptr_t)sink % 4) return fail(SPL_EINVAL, "buf must be 16-byte and sink 4-byte aligned");
  hipLaunchKernelGGL(k_stream_read, dim3(STREAM_BLOCKS), dim3(STREAM_THREADS), 0, (hipStream_t)stream,
                     static_cast<const u4v*>(buf), bytes / 16, static_cast<uint32_t*>(sink));
  return hip_fail(hipGetLastError(), "stream read launch");
}
