// ht_roofline.hip -- microbenchmarks that measure the ceilings the fill and peak kernels run
// against on this GPU: streaming HBM writes and reads, a plain copy (the reference kernel for
// hardware byte counters), no-return 32-bit atomics at random addresses in a buffer the size of
// a vote matrix, and LDS atomics. Each call is one launch on the caller's stream; the caller
// times it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "ht_debug.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;

unsigned grid_for(int64_t items)
{
  const int64_t per_wave = (int64_t)kBlock * 8;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + per_wave - 1) / per_wave, 256 * 64));
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_write(u32x4* dst, int64_t n4, uint32_t value)
{
  const u32x4 v = {value, value, value, value};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  if (MODE == 2) {  // 4-byte stores
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    const int64_t n = 4 * n4;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) d[i] = value;
    return;
  }
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
    if (MODE == 0) __builtin_nontemporal_store(v, dst + i);
    else dst[i] = v;
  }
}

// Stores tile by tile, as the fill writes the matrix: workgroup w writes the 16 KiB tiles w,
// w + G, ... (G workgroups), each as four 4 KiB rows of 16-byte stores, non-temporal (NT) or
// ordinary.
constexpr int64_t kTileVec = 1024;  // 16-byte vectors per 16 KiB tile
template <bool NT>
__global__ __launch_bounds__(kBlock) void k_write_tiles(u32x4* dst, int64_t n4, uint32_t value)
{
  const u32x4 v = {value, value, value, value};
  const int64_t n_tiles = n4 / kTileVec;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    u32x4* d = dst + t * kTileVec;
#pragma unroll
    for (int k = 0; k < (int)(kTileVec / kBlock); ++k) {
      if (NT) __builtin_nontemporal_store(v, d + k * kBlock + threadIdx.x);
      else d[k * kBlock + threadIdx.x] = v;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_read(const u32x4* src, int64_t n4, uint32_t* sink)
{
  uint32_t acc = 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
    const u32x4 v = __builtin_nontemporal_load(src + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads alive; practically never taken
}

__global__ __launch_bounds__(kBlock) void k_copy(u32x4* dst, const u32x4* src, int64_t n4)
{
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(kBlock) void k_atomic_rand(uint32_t* buf, uint32_t n_words, int64_t n_ops)
{
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_ops; i += stride) {
    const uint32_t h = mix32((uint32_t)i ^ (uint32_t)(i >> 32) * 0x9e3779b9u);
    atomicAdd(buf + (uint32_t)(((uint64_t)h * n_words) >> 32), 1u);
  }
}

__global__ __launch_bounds__(kBlock) void k_lds_atomic(int iters, uint32_t* sink)
{
  __shared__ uint32_t s[8192];
  for (int i = threadIdx.x; i < 8192; i += kBlock) s[i] = 0u;
  __syncthreads();
  uint32_t x = mix32(blockIdx.x * kBlock + threadIdx.x);
  for (int it = 0; it < iters; ++it) {
    x = x * 1664525u + 1013904223u;
    atomicAdd(&s[x >> 19], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0 && s[0] == 0xffffffffu) sink[0] = s[1];
}

}  // namespace

extern "C" {

int ht_bench_hbm_write(void* buf, int64_t bytes, int32_t mode, void* stream)
{
  if (!buf || bytes < 16 || bytes % 16 || mode < 0 || mode > 4) return HT_EINVAL;
  if (mode >= 3 && bytes % (16 * kTileVec)) return HT_EINVAL;
  const dim3 grid(grid_for(bytes / 16));
  hipStream_t s = (hipStream_t)stream;
  if (mode == 0) hipLaunchKernelGGL(k_write<0>, grid, dim3(kBlock), 0, s, (u32x4*)buf, bytes / 16, 0u);
  else if (mode == 1) hipLaunchKernelGGL(k_write<1>, grid, dim3(kBlock), 0, s, (u32x4*)buf, bytes / 16, 0u);
  else if (mode == 2) hipLaunchKernelGGL(k_write<2>, grid, dim3(kBlock), 0, s, (u32x4*)buf, bytes / 16, 0u);
  else {
    // one workgroup per tile, as the fill launches on the paper grid (at most 2^20 of them)
    const dim3 tgrid((unsigned)std::min<int64_t>(bytes / (16 * kTileVec), 1 << 20));
    if (mode == 3) hipLaunchKernelGGL(k_write_tiles<true>, tgrid, dim3(kBlock), 0, s, (u32x4*)buf, bytes / 16, 0u);
    else hipLaunchKernelGGL(k_write_tiles<false>, tgrid, dim3(kBlock), 0, s, (u32x4*)buf, bytes / 16, 0u);
  }
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

int ht_bench_hbm_read(const void* buf, int64_t bytes, uint32_t* sink, void* stream)
{
  if (!buf || !sink || bytes < 16 || bytes % 16) return HT_EINVAL;
  hipLaunchKernelGGL(k_read, dim3(grid_for(bytes / 16)), dim3(kBlock), 0, (hipStream_t)stream,
                     (const u32x4*)buf, bytes / 16, sink);
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

int ht_bench_copy(void* dst, const void* src, int64_t bytes, void* stream)
{
  if (!dst || !src || bytes < 16 || bytes % 16) return HT_EINVAL;
  hipLaunchKernelGGL(k_copy, dim3(grid_for(bytes / 16)), dim3(kBlock), 0, (hipStream_t)stream,
                     (u32x4*)dst, (const u32x4*)src, bytes / 16);
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

int ht_bench_atomic_rand(uint32_t* buf, int64_t n_words, int64_t n_ops, void* stream)
{
  if (!buf || n_words < 1 || n_words > 0xffffffffLL || n_ops < 1) return HT_EINVAL;
  hipLaunchKernelGGL(k_atomic_rand, dim3(256 * 32), dim3(kBlock), 0, (hipStream_t)stream, buf,
                     (uint32_t)n_words, n_ops);
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

int ht_bench_lds_atomic(int32_t blocks, int32_t iters, uint32_t* sink, void* stream)
{
  if (blocks < 1 || iters < 1 || !sink) return HT_EINVAL;
  hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(kBlock), 0, (hipStream_t)stream, iters, sink);
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

}  // extern "C"
