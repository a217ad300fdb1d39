// Workgroup reductions and the launch gate shared by the solver kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "wd_common.hpp"
#include "wd_internal.hpp"

namespace wd {

// Sum over a 256-thread workgroup in a fixed order: butterfly within each
// 64-lane wavefront, then the four wavefront sums in index order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double wsum[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  if (lane == 0) wsum[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) t += wsum[i];
  }
  __syncthreads();
  return t;   // valid in thread 0
}

// Per-workgroup partial of a grid-wide sum, written with a plain store; the
// launcher follows the kernel with k_finalize, which adds the partials in
// index order (deterministic) and applies `fin` to the solver state. Keeping
// the cross-workgroup step in its own launch avoids device-scope
// acquire/release per workgroup, which on a multi-XCD part writes back and
// invalidates the XCD's L2 and would throw away the stencil's neighbour reuse.
__device__ __forceinline__ void store_partial(double v, double* partials, int index) {
  const double bs = block_sum(v);
  if (threadIdx.x == 0) partials[index] = bs;
}
__device__ __forceinline__ void store_partial(double v, double* partials) { store_partial(v, partials, blockIdx.x); }

// ---- several systems per launch (Rhs): system k's buffers are offset by
// k * stride bytes.
template <class T>
__device__ __forceinline__ T* rhs_shift(T* p, long long off) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<char*>(p) + off) : p;
}
template <class T>
__device__ __forceinline__ const T* rhs_shift(const T* p, long long off) {
  return p ? reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off) : p;
}
__device__ __forceinline__ SpinorBuf rhs_shift(SpinorBuf b, long long off) {
  b.data = rhs_shift(static_cast<char*>(b.data), off);
  b.scale = rhs_shift(b.scale, off);
  return b;
}
__device__ __forceinline__ RingBuf rhs_shift(RingBuf r, long long off) {
  r.data = rhs_shift(r.data, off);
  r.scale = rhs_shift(r.scale, off);
  return r;
}
// Split a workgroup index L over n systems, system fastest: the n systems
// of one tile run back to back (on one XCD, after xcd_tile), so that the
// tile's links are read from HBM once for all of them.
__device__ __forceinline__ int rhs_split(int L, const Rhs& rb, int& k) {
  if (rb.n == 1) {
    k = 0;
    return L;
  }
  const int T = L / rb.n;
  k = L - T * rb.n;
  return T;
}

__device__ __forceinline__ bool gate_open(const SolverState* st, int gate) {
  if (gate == G_ALWAYS || gate == G_FINAL) return true;
  const int status = st->status;
  if (gate == G_ITER) return status == 0 && st->inner_done == 0;
  if (gate == G_FLUSH) return status == 0 && st->flush_at > 0 && st->npend >= st->flush_at;
  // G_RELIABLE
  return status == 0 && (st->inner_done != 0 || st->iter - st->last_update >= st->interval ||
                         st->rho <= st->delta2 * st->rho_update);
}

}  // namespace wd
