// Plain streaming kernels: the practical HBM ceiling that the stencil kernels
// are measured against. Each moves 16-byte words with every lane of a
// wavefront on consecutive addresses (full 64 x 16 B = 1 KiB spans), eight
// independent words in flight per thread, over buffers far larger than the
// 256 MiB Infinity Cache, so that what they reach is what HBM delivers to a
// perfectly coalesced access stream.
#include <hip/hip_runtime.h>

#include "wd_internal.hpp"

namespace wd {

constexpr int kStreamBlock = 256;
constexpr int kStreamUnroll = 8;

// Streaming (non-temporal) 16-byte load and store: a copy with plain accesses
// reached 3.8 TB/s here against 5.3 TB/s with these, the caches otherwise
// holding lines that are never read again.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_nt(const uint4* p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_nt(uint4* p, const uint4& v) {
  const u32x4 u = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(u, reinterpret_cast<u32x4*>(p));
}

__global__ __launch_bounds__(kStreamBlock) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                              size_t n) {
  const size_t stride = (size_t)gridDim.x * kStreamBlock * kStreamUnroll;
  for (size_t base = (size_t)blockIdx.x * kStreamBlock * kStreamUnroll + threadIdx.x; base < n; base += stride) {
    uint4 v[kStreamUnroll];
#pragma unroll
    for (int k = 0; k < kStreamUnroll; ++k) {
      const size_t i = base + (size_t)k * kStreamBlock;
      if (i < n) v[k] = ld_nt(src + i);
    }
#pragma unroll
    for (int k = 0; k < kStreamUnroll; ++k) {
      const size_t i = base + (size_t)k * kStreamBlock;
      if (i < n) st_nt(dst + i, v[k]);
    }
  }
}

// XOR of every word; one 16-byte result per workgroup, combined by a second pass.
__global__ __launch_bounds__(kStreamBlock) void k_stream_read(const uint4* __restrict__ src, size_t n,
                                                              uint4* __restrict__ part) {
  const size_t stride = (size_t)gridDim.x * kStreamBlock * kStreamUnroll;
  uint4 acc = make_uint4(0, 0, 0, 0);
  for (size_t base = (size_t)blockIdx.x * kStreamBlock * kStreamUnroll + threadIdx.x; base < n; base += stride) {
    uint4 v[kStreamUnroll];
#pragma unroll
    for (int k = 0; k < kStreamUnroll; ++k) {
      const size_t i = base + (size_t)k * kStreamBlock;
      v[k] = i < n ? src[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < kStreamUnroll; ++k) {
      acc.x ^= v[k].x;
      acc.y ^= v[k].y;
      acc.z ^= v[k].z;
      acc.w ^= v[k].w;
    }
  }
  __shared__ uint4 red[kStreamBlock];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      uint4 o = red[threadIdx.x + s];
      red[threadIdx.x].x ^= o.x;
      red[threadIdx.x].y ^= o.y;
      red[threadIdx.x].z ^= o.z;
      red[threadIdx.x].w ^= o.w;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kStreamBlock) void k_stream_fill(uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * kStreamBlock * kStreamUnroll;
  for (size_t base = (size_t)blockIdx.x * kStreamBlock * kStreamUnroll + threadIdx.x; base < n; base += stride) {
#pragma unroll
    for (int k = 0; k < kStreamUnroll; ++k) {
      const size_t i = base + (size_t)k * kStreamBlock;
      if (i < n) st_nt(dst + i, make_uint4(0, 0, 0, 0));
    }
  }
}

// Workgroups of a streaming launch: enough to keep every CU busy (8 per CU on
// 256 CUs), fewer for small buffers.
static unsigned stream_grid(size_t n) {
  const size_t per = (size_t)kStreamBlock * kStreamUnroll;
  const size_t want = (n + per - 1) / per;
  return (unsigned)(want < 2048 ? (want ? want : 1) : 2048);
}

unsigned stream_read_partials(size_t bytes) { return stream_grid(bytes / 16); }

void launch_stream(int kind, const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  const unsigned grid = stream_grid(n);
  if (kind == 0)
    k_stream_copy<<<grid, kStreamBlock, 0, s>>>(static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
  else if (kind == 1)
    k_stream_read<<<grid, kStreamBlock, 0, s>>>(static_cast<const uint4*>(src), n, static_cast<uint4*>(dst));
  else
    k_stream_fill<<<grid, kStreamBlock, 0, s>>>(static_cast<uint4*>(dst), n);
}

}  // namespace wd
