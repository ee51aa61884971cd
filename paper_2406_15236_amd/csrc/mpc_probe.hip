// mpc_probe.hip -- plain HBM streaming kernels that measure the bandwidth a
// kernel can attain on this device (copy: read + write once; read: read
// once), the reference beside which the MPC kernels' byte rates are judged.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpc.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte word
constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;  // 16-byte words in flight per thread and iteration

// Grid-stride copy of n16 16-byte words: each iteration issues kProbeUnroll
// independent loads (one per stride) before their stores.
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const u32x4* __restrict__ src,
                                                              u32x4* __restrict__ dst,
                                                              uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * kProbeThreads;
  uint64_t i = (uint64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n16; i += kProbeUnroll * stride) {
    u32x4 w[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) w[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) __builtin_nontemporal_store(w[u], dst + i + u * stride);
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Grid-stride read of n16 16-byte words, folded by XOR into one word per
// thread and written to out[thread] (so the loads cannot be dropped).
__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const u32x4* __restrict__ src,
                                                              uint64_t n16,
                                                              uint32_t* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * kProbeThreads;
  const uint64_t tid = (uint64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  uint64_t i = tid;
  uint32_t acc = 0;
  for (; i + (kProbeUnroll - 1) * stride < n16; i += kProbeUnroll * stride) {
    u32x4 w[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) w[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc ^= w[u].x ^ w[u].y ^ w[u].z ^ w[u].w;
  }
  for (; i < n16; i += stride) {
    const u32x4 w = src[i];
    acc ^= w.x ^ w.y ^ w.z ^ w.w;
  }
  out[tid] = acc;
}

int probe_grid(int grid) {
  if (grid > 0) return grid;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return 8 * cus;
}

}  // namespace

extern "C" {

int mpc_probe_copy(void* dst, const void* src, size_t bytes, int32_t grid, void* hip_stream) {
  if (!dst || !src || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15) || grid < 0)
    return MPC_EINVAL;
  if (bytes == 0) return MPC_OK;
  hipLaunchKernelGGL(k_probe_copy, dim3(probe_grid(grid)), dim3(kProbeThreads), 0,
                     (hipStream_t)hip_stream, (const u32x4*)src, (u32x4*)dst,
                     (uint64_t)(bytes / 16));
  return hipGetLastError() == hipSuccess ? MPC_OK : MPC_EHIP;
}

int mpc_probe_read(const void* src, size_t bytes, void* out, size_t out_bytes, int32_t grid,
                   void* hip_stream) {
  if (!src || !out || (bytes & 15) || ((uintptr_t)src & 15) || grid < 0) return MPC_EINVAL;
  const int g = probe_grid(grid);
  if (out_bytes < (size_t)g * kProbeThreads * sizeof(uint32_t)) return MPC_EINVAL;
  hipLaunchKernelGGL(k_probe_read, dim3(g), dim3(kProbeThreads), 0, (hipStream_t)hip_stream,
                     (const u32x4*)src, (uint64_t)(bytes / 16), (uint32_t*)out);
  return hipGetLastError() == hipSuccess ? MPC_OK : MPC_EHIP;
}

}  // extern "C"
