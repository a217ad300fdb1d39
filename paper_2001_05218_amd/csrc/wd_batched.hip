// Batched multi-RHS conjugate gradient in one persistent cooperative launch.
//
// Up to 16 right-hand sides share one gauge field. Inner iterations run in
// FP32 arithmetic on p, r and t stored in FP32, BF16, FP16 (+ per-site scale)
// or int8 fixed point (the template parameter P), with the solution
// increment in FP32; every few iterations (and whenever an inner residual
// has dropped by a fixed factor or reached the target) an FP64 reliable
// update flushes the FP32 solution increment into the FP64 solution and
// recomputes that system's residual exactly -- the two-precision scheme of
// the paper's Sec. 2 / Sec. 3.2 applied per right-hand side.
//
// Work decomposition. A workgroup owns one 64-site block at a time (grid-
// stride over site blocks) and four wavefronts; wavefront w serves the
// right-hand sides k = w, w + 4, w + 8, w + 12. The 8 links a site needs
// (U_mu(x) and U_mu(x - mu), FP32) are staged once in LDS per site block and
// then read by every right-hand side: each link leaves HBM once per operator
// application for all systems together.
//
// Control. All scalars (alpha, beta, residual norms, convergence masks) are
// computed redundantly by every workgroup from the same per-workgroup
// partial sums, in the same order, after a grid barrier; every workgroup
// therefore takes the same branches and reaches the same barriers. The
// iteration loop is bounded by max_iter.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "../../include/wilson.h"
#include "wd_dslash.hpp"
#include "wd_internal.hpp"

namespace cgrp = cooperative_groups;

namespace wd {

constexpr int kMaxRhs = 16;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxGrid = 8192;

struct BatchArgs {
  Geom g;
  int nrhs;
  int max_iter;
  int nsb;            // 64-site blocks
  int pad;
  double diag;        // m + 4
  const float2* U32;  // packed FP32 links
  const double2* U64; // packed FP64 links
  char* p;            // inner-storage vectors, right-hand side k at base + k * strideL
  char* r;
  char* t;
  char* ps;           // their per-site scales (FP16, int8), at base + k * strideS; else null
  char* rs;
  char* ts;
  size_t strideL;
  size_t strideS;
  char* xh;           // FP32 solution increment, right-hand side k at base + k * stride32
  char* x64;          // FP64 vectors, right-hand side k at base + k * stride64
  char* b64;
  char* t64;
  size_t stride32;
  size_t stride64;
  SolverState* st;    // [nrhs]
  double* partA;      // [kMaxGrid][kMaxRhs]
  double* partB;
  double* partC;
};

// Links of the current site block in LDS: [mu * 9 + e][lane].
struct LdsGauge {
  using Real = float;
  const float2 (*fwd)[64];
  const float2 (*bwd)[64];
  int lane;
  __device__ __forceinline__ void load_fwd(int, int mu, float u[18]) const {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      const float2 v = fwd[mu * 9 + e][lane];
      u[2 * e] = v.x;
      u[2 * e + 1] = v.y;
    }
  }
  __device__ __forceinline__ void load_bwd(int, int mu, float u[18]) const {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      const float2 v = bwd[mu * 9 + e][lane];
      u[2 * e] = v.x;
      u[2 * e + 1] = v.y;
    }
  }
};

__device__ __forceinline__ PackedSpinor<P_F32> f32_of(char* base, size_t stride, int k) {
  PackedSpinor<P_F32> s;
  s.data = reinterpret_cast<float4*>(base + (size_t)k * stride);
  s.scale = nullptr;
  return s;
}
// Inner-storage spinors as a stencil source, fenced per direction (see FencedF64).
template <int P>
struct Fenced : PackedSpinor<P> {
  static constexpr bool kFence = true;
};

template <int P>
__device__ __forceinline__ Fenced<P> low_of(char* base, char* sbase, const BatchArgs& a, int k) {
  Fenced<P> s;
  s.data = reinterpret_cast<decltype(s.data)>(base + (size_t)k * a.strideL);
  s.scale = sbase ? reinterpret_cast<float*>(sbase + (size_t)k * a.strideS) : nullptr;
  return s;
}
// FP64 spinors for the reliable update's stencils, with the per-direction
// fence of hop_dir: without it the compiler hoists all eight neighbours' loads
// and the whole kernel needs over 400 registers (one wave per SIMD).
struct FencedF64 : PackedSpinor<P_F64> {
  static constexpr bool kFence = true;
};

__device__ __forceinline__ FencedF64 f64_of(char* base, size_t stride, int k) {
  FencedF64 s;
  s.data = reinterpret_cast<double2*>(base + (size_t)k * stride);
  s.scale = nullptr;
  return s;
}

__device__ __forceinline__ int bwd_of(const Nbrs& nb, int mu) {
  return mu == 0 ? nb.bwd[0] : mu == 1 ? nb.bwd[1] : mu == 2 ? nb.bwd[2] : nb.bwd[3];
}

// Per-RHS scalars, identical in every workgroup.
struct Scal {
  double rho[kMaxRhs], rho_prev[kMaxRhs], alpha[kMaxRhs], beta[kMaxRhs];
  double rho_upd[kMaxRhs], rho_true[kMaxRhs], stop2[kMaxRhs], delta2[kMaxRhs];
  int active[kMaxRhs], iter[kMaxRhs], last[kMaxRhs], nupd[kMaxRhs], flag[kMaxRhs], status[kMaxRhs];
  int interval;
  int any_active;
  int any_flag;
};

// Sum part[b][k] over b = 0 .. G-1 for every k < nrhs, in a fixed order:
// 16 lanes per right-hand side, strided partial sums, then a fixed xor tree.
__device__ void reduce_parts(const double* part, int G, int nrhs, double* out) {
  const int k = threadIdx.x >> 4;   // 0..15
  const int j = threadIdx.x & 15;
  double acc = 0.0;
  if (k < nrhs)
    for (int b = j; b < G; b += 16)
      acc += __hip_atomic_load(&part[(size_t)b * kMaxRhs + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
  if (j == 0 && k < nrhs) out[k] = acc;
  __syncthreads();
}

// One wavefront's per-RHS partial sums -> part[blockIdx][k] (each k belongs to one wavefront).
__device__ void publish_parts(double* part, const double n2[kMaxRhs / kWaves], int nrhs) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kMaxRhs / kWaves; ++j) {
    const int k = wave + kWaves * j;
    double v = n2[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0 && k < nrhs)
      __hip_atomic_store(&part[(size_t)blockIdx.x * kMaxRhs + k], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// n2[j] += v for a runtime j < 4 without indexing a register array (which
// would move it to scratch memory).
__device__ __forceinline__ void add_part(double n2[kMaxRhs / kWaves], int j, double v) {
  n2[0] += (j == 0) ? v : 0.0;
  n2[1] += (j == 1) ? v : 0.0;
  n2[2] += (j == 2) ? v : 0.0;
  n2[3] += (j == 3) ? v : 0.0;
}

// Stage the FP32 links of site block sb into LDS.
__device__ __forceinline__ void stage_links(const BatchArgs& a, int s, bool valid, const Nbrs& nb,
                                            float2 (*fwd)[64], float2 (*bwd)[64]) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  __syncthreads();   // previous readers are done
  for (int w = wave; w < 36; w += kWaves)
    fwd[w][lane] = valid ? a.U32[word_index(s, 36, w)] : make_float2(0.f, 0.f);
  const int sbw = valid ? bwd_of(nb, wave) : 0;
#pragma unroll
  for (int e = 0; e < 9; ++e)
    bwd[wave * 9 + e][lane] = valid ? a.U32[word_index(sbw, 36, wave * 9 + e)] : make_float2(0.f, 0.f);
  __syncthreads();
}

// The reliable update's FP64 stencils, kept out of line: inlined into the
// persistent loop they need over 400 registers (the compiler overlaps them
// with the surrounding loops), which left room for one wave per SIMD.
__device__ __noinline__ void reliable_dx(const BatchArgs& a, int s, const Nbrs& nb, int k) {
  const PackedGauge<P_F64> U64{a.U64};
  double o[24];
  wilson_site<false>(U64, f64_of(a.x64, a.stride64, k), s, nb, a.diag, o);
  f64_of(a.t64, a.stride64, k).store(s, o);
}

// r = low(b - D^+ t) at site s for right-hand side k; returns ||b - D^+ t||^2 there.
template <int P>
__device__ __noinline__ double reliable_res(const BatchArgs& a, int s, const Nbrs& nb, int k) {
  const PackedGauge<P_F64> U64{a.U64};
  double q[24], bv[24];
  float rv[24];
  wilson_site<true>(U64, f64_of(a.t64, a.stride64, k), s, nb, a.diag, q);
  f64_of(a.b64, a.stride64, k).load(s, bv);
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < 24; ++i) {
    const double d = bv[i] - q[i];
    part += d * d;
    rv[i] = (float)d;
  }
  low_of<P>(a.r, a.rs, a, k).store(s, rv);
  return part;
}

// FP16 and int8 storage (whose packing needs a few more registers) are held
// to two waves per SIMD: left alone the compiler takes 258-259 registers
// (256 VGPRs and 2-3 AGPRs) and runs one wave, 17-20 % slower. FP32 and BF16
// fit two waves by themselves.
template <int P>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((P == P_F16 || P == P_I8) ? 2 : 1, 8)))
void k_batched_cg(BatchArgs a) {
  cgrp::grid_group grid = cgrp::this_grid();
  __shared__ float2 lds_fwd[36][64];
  __shared__ float2 lds_bwd[36][64];
  __shared__ Scal sc;
  __shared__ double red[kMaxRhs];

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int nrhs = a.nrhs;
  const int G = gridDim.x;
  const float diag = (float)a.diag;

  if (threadIdx.x < kMaxRhs) {
    const int k = threadIdx.x;
    if (k < nrhs) {
      const SolverState& s = a.st[k];
      sc.rho[k] = s.rho;
      sc.rho_prev[k] = s.rho;
      sc.alpha[k] = 0.0;
      sc.beta[k] = 0.0;
      sc.rho_upd[k] = s.rho_update;
      sc.rho_true[k] = s.rho_true;
      sc.stop2[k] = s.stop2;
      sc.delta2[k] = s.delta2;
      sc.status[k] = s.status;
      sc.active[k] = s.status == 0;
      sc.iter[k] = 0;
      sc.last[k] = 0;
      sc.nupd[k] = 0;
      sc.flag[k] = 0;
    } else {
      sc.active[k] = 0;
      sc.flag[k] = 0;
    }
    if (k == 0) sc.interval = a.st[0].interval;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int any = 0;
    for (int k = 0; k < nrhs; ++k) any |= sc.active[k];
    sc.any_active = any;
  }
  __syncthreads();

  LdsGauge lg{lds_fwd, lds_bwd, lane};

  // FP64 reliable update for the flagged right-hand sides: x += xhat, xhat = 0,
  // r = low(b' - D^+ D x), rho_true = ||b' - D^+ D x||^2.
  auto reliable = [&]() {
    for (int sb = blockIdx.x; sb < a.nsb; sb += G) {
      const int s = sb * 64 + lane;
      if (s < a.g.V) {
        for (int k = wave; k < nrhs; k += kWaves) {
          if (!sc.flag[k]) continue;
          double xv[24];
          float hv[24];
          const auto X = f64_of(a.x64, a.stride64, k);
          const auto H = f32_of(a.xh, a.stride32, k);
          X.load(s, xv);
          H.load(s, hv);
#pragma unroll
          for (int i = 0; i < 24; ++i) {
            xv[i] += (double)hv[i];
            hv[i] = 0.f;
          }
          X.store(s, xv);
          H.store(s, hv);
        }
      }
    }
    grid.sync();
    for (int sb = blockIdx.x; sb < a.nsb; sb += G) {
      const int s = sb * 64 + lane;
      if (s < a.g.V) {
        const Nbrs nb = neighbours(a.g, s);
        for (int k = wave; k < nrhs; k += kWaves) {
          if (!sc.flag[k]) continue;
          reliable_dx(a, s, nb, k);
        }
      }
    }
    grid.sync();
    double n2[kMaxRhs / kWaves] = {0.0, 0.0, 0.0, 0.0};
    for (int sb = blockIdx.x; sb < a.nsb; sb += G) {
      const int s = sb * 64 + lane;
      if (s < a.g.V) {
        const Nbrs nb = neighbours(a.g, s);
#pragma unroll 1
        for (int j = 0; j < kMaxRhs / kWaves; ++j) {
          const int k = wave + kWaves * j;
          if (k >= nrhs || !sc.flag[k]) continue;
          add_part(n2, j, reliable_res<P>(a, s, nb, k));
        }
      }
    }
    publish_parts(a.partC, n2, nrhs);
    grid.sync();
    reduce_parts(a.partC, G, nrhs, red);
  };

  for (int it = 0; it < a.max_iter && sc.any_active; ++it) {
    // ---- phase A: t = D p, ||t||^2
    {
      double n2[kMaxRhs / kWaves] = {0.0, 0.0, 0.0, 0.0};
      for (int sb = blockIdx.x; sb < a.nsb; sb += G) {
        const int s = sb * 64 + lane;
        const bool valid = s < a.g.V;
        Nbrs nb{};
        if (valid) nb = neighbours(a.g, s);
        stage_links(a, s, valid, nb, lds_fwd, lds_bwd);
        if (valid) {
#pragma unroll 1
          for (int j = 0; j < kMaxRhs / kWaves; ++j) {
            const int k = wave + kWaves * j;
            if (k >= nrhs || !sc.active[k]) continue;
            float o[24];
            wilson_site<false>(lg, low_of<P>(a.p, a.ps, a, k), s, nb, diag, o);
            low_of<P>(a.t, a.ts, a, k).store(s, o);
            double part = 0.0;
#pragma unroll
            for (int i = 0; i < 24; ++i) part += (double)o[i] * (double)o[i];
            add_part(n2, j, part);
          }
        }
      }
      publish_parts(a.partA, n2, nrhs);
    }
    grid.sync();
    reduce_parts(a.partA, G, nrhs, red);
    if (threadIdx.x < nrhs) {
      const int k = threadIdx.x;
      if (sc.active[k]) {
        const double tn = red[k];
        if (!(tn - tn == 0.0)) { sc.status[k] = -4; sc.active[k] = 0; }
        else if (tn <= 0.0) { sc.status[k] = -3; sc.active[k] = 0; }
        else sc.alpha[k] = sc.rho[k] / tn;
      }
    }
    __syncthreads();

    // ---- phase B: q = D^+ t; r -= alpha q; xhat += alpha p; ||r||^2
    {
      double n2[kMaxRhs / kWaves] = {0.0, 0.0, 0.0, 0.0};
      for (int sb = blockIdx.x; sb < a.nsb; sb += G) {
        const int s = sb * 64 + lane;
        const bool valid = s < a.g.V;
        Nbrs nb{};
        if (valid) nb = neighbours(a.g, s);
        stage_links(a, s, valid, nb, lds_fwd, lds_bwd);
        if (valid) {
#pragma unroll 1
          for (int j = 0; j < kMaxRhs / kWaves; ++j) {
            const int k = wave + kWaves * j;
            if (k >= nrhs || !sc.active[k]) continue;
            float q[24], rv[24], pv[24], xv[24];
            wilson_site<true>(lg, low_of<P>(a.t, a.ts, a, k), s, nb, diag, q);
            const auto R = low_of<P>(a.r, a.rs, a, k);
            const auto X = f32_of(a.xh, a.stride32, k);
            R.load(s, rv);
            low_of<P>(a.p, a.ps, a, k).load(s, pv);
            X.load(s, xv);
            const float al = (float)sc.alpha[k];
#pragma unroll
            for (int i = 0; i < 24; ++i) {
              rv[i] = fmaf(-al, q[i], rv[i]);
              xv[i] = fmaf(al, pv[i], xv[i]);
            }
            if constexpr (P == P_F32) {
              R.store(s, rv);
            } else {
              // store, then take the norm of what the next iteration reads
              typename SpinorWord<P>::T d[3];
              float scl;
              PackedSpinor<P>::pack(rv, d, scl);
              R.store_raw(s, d, scl);
              PackedSpinor<P>::unpack(d, scl, rv);
            }
            double part = 0.0;
#pragma unroll
            for (int i = 0; i < 24; ++i) part += (double)rv[i] * (double)rv[i];
            add_part(n2, j, part);
            X.store(s, xv);
          }
        }
      }
      publish_parts(a.partB, n2, nrhs);
    }
    grid.sync();
    reduce_parts(a.partB, G, nrhs, red);
    if (threadIdx.x < nrhs) {
      const int k = threadIdx.x;
      sc.flag[k] = 0;
      if (sc.active[k]) {
        const double rn = red[k];
        sc.rho_prev[k] = sc.rho[k];
        sc.rho[k] = rn;
        sc.iter[k] += 1;
        if (!(rn - rn == 0.0)) {
          sc.status[k] = -4;
          sc.active[k] = 0;
        } else {
          sc.beta[k] = rn / sc.rho_prev[k];
          sc.flag[k] = (rn <= sc.stop2[k]) || (sc.iter[k] - sc.last[k] >= sc.interval) ||
                       (rn <= sc.delta2[k] * sc.rho_upd[k]);
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int f = 0;
      for (int k = 0; k < nrhs; ++k) f |= sc.flag[k];
      sc.any_flag = f;
    }
    __syncthreads();

    // ---- FP64 reliable update where due
    if (sc.any_flag) {
      reliable();
      if (threadIdx.x < nrhs) {
        const int k = threadIdx.x;
        if (sc.flag[k]) {
          const double rt = red[k];
          const double iterated = sc.rho[k];
          sc.rho_true[k] = rt;
          sc.rho_upd[k] = rt;
          sc.nupd[k] += 1;
          sc.last[k] = sc.iter[k];
          if (!(rt - rt == 0.0)) { sc.status[k] = -4; sc.active[k] = 0; }
          else if (rt <= sc.stop2[k]) { sc.status[k] = 1; sc.active[k] = 0; }
          else {
            sc.rho[k] = rt;
            sc.beta[k] = (rt > 4.0 * iterated) ? 0.0 : rt / sc.rho_prev[k];
          }
        }
      }
      __syncthreads();
    }

    // ---- phase C: p = r + beta p
    for (int sb = blockIdx.x; sb < a.nsb; sb += G) {
      const int s = sb * 64 + lane;
      if (s >= a.g.V) continue;
      for (int k = wave; k < nrhs; k += kWaves) {
        if (!sc.active[k]) continue;
        float rv[24], pv[24];
        const auto Pk = low_of<P>(a.p, a.ps, a, k);
        low_of<P>(a.r, a.rs, a, k).load(s, rv);
        Pk.load(s, pv);
        const float be = (float)sc.beta[k];
#pragma unroll
        for (int i = 0; i < 24; ++i) pv[i] = fmaf(be, pv[i], rv[i]);
        Pk.store(s, pv);
      }
    }
    if (threadIdx.x == 0) {
      int any = 0;
      for (int k = 0; k < nrhs; ++k) any |= sc.active[k];
      sc.any_active = any;
    }
    grid.sync();
  }

  // Systems still running at max_iter: flush xhat and measure the true residual.
  if (threadIdx.x < kMaxRhs) sc.flag[threadIdx.x] = (threadIdx.x < nrhs) && sc.active[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    int f = 0;
    for (int k = 0; k < nrhs; ++k) f |= sc.flag[k];
    sc.any_flag = f;
  }
  __syncthreads();
  if (sc.any_flag) {
    reliable();
    if (threadIdx.x < nrhs && sc.flag[threadIdx.x]) sc.rho_true[threadIdx.x] = red[threadIdx.x];
    __syncthreads();
  }

  if (blockIdx.x == 0 && threadIdx.x < nrhs) {
    const int k = threadIdx.x;
    SolverState& s = a.st[k];
    s.iter = sc.iter[k];
    s.status = sc.status[k];
    s.rho = sc.rho[k];
    s.rho_true = sc.rho_true[k];
    s.rel_updates = sc.nupd[k];
  }
}

// ------------------------------------------------------------------ host

struct BatchedWorkspace {
  SolverState* st;
  double* partA;
  double* partB;
  double* partC;
  void* U32;
  void* U64;
  char* p;
  char* r;
  char* t;
  char* ps;
  char* rs;
  char* ts;
  char* xh;
  char* x64;
  char* b64;
  char* t64;
  size_t strideL, strideS, stride32, stride64;
  size_t bytes;
};

static size_t al256(size_t n) { return (n + 255) & ~size_t(255); }

static BatchedWorkspace layout_batched(void* base, const Geom& g, int nrhs, int prec) {
  BatchedWorkspace w{};
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t n) -> char* {
    char* p = b ? b + off : nullptr;
    off += al256(n);
    return p;
  };
  w.st = reinterpret_cast<SolverState*>(take(sizeof(SolverState) * kMaxRhs));
  const size_t np = std::max<size_t>((size_t)kMaxGrid * kMaxRhs, (size_t)g.nblocks);
  w.partA = reinterpret_cast<double*>(take(np * sizeof(double)));
  w.partB = reinterpret_cast<double*>(take(np * sizeof(double)));
  w.partC = reinterpret_cast<double*>(take(np * sizeof(double)));
  w.U32 = take(gauge_bytes(P_F32, g.Vpad));
  w.U64 = take(gauge_bytes(P_F64, g.Vpad));
  w.strideL = al256(spinor_bytes(prec, g.Vpad));
  w.strideS = al256(spinor_scale_bytes(prec, g.Vpad));
  w.stride32 = al256(spinor_bytes(P_F32, g.Vpad));
  w.stride64 = al256(spinor_bytes(P_F64, g.Vpad));
  w.p = take(w.strideL * nrhs);
  w.r = take(w.strideL * nrhs);
  w.t = take(w.strideL * nrhs);
  if (w.strideS) {
    w.ps = take(w.strideS * nrhs);
    w.rs = take(w.strideS * nrhs);
    w.ts = take(w.strideS * nrhs);
  }
  w.xh = take(w.stride32 * nrhs);
  w.x64 = take(w.stride64 * nrhs);
  w.b64 = take(w.stride64 * nrhs);
  w.t64 = take(w.stride64 * nrhs);
  w.bytes = off;
  return w;
}

// Inner storage of a batched solve: the caller's precision, FP32 for anything
// the batched kernel does not store (FP64).
static int batched_prec(int inner) {
  return (inner == WD_BF16 || inner == WD_F16 || inner == WD_I8) ? inner : P_F32;
}

size_t batched_workspace_bytes(const Geom& g, int nrhs, int hist_len, int inner_prec) {
  (void)hist_len;
  return layout_batched(nullptr, g, nrhs, batched_prec(inner_prec)).bytes;
}

int batched_solve(const Geom& g, double mass, const void* U, int nrhs, const void* B, void* X,
                  const wd_cg_params* p, wd_cg_result* res, void* ws, hipStream_t s, char* err, size_t errlen) {
  const auto t0 = std::chrono::steady_clock::now();
  const int P = batched_prec(p->inner_prec);
  const BatchedWorkspace w = layout_batched(ws, g, nrhs, P);
  const int interval = p->reliable_interval > 0 ? p->reliable_interval : 50;
  // residual reduction between FP64 recomputations, as for single solves
  double delta = (P == WD_BF16 || P == WD_I8) ? 0.1 : (P == WD_F16) ? 1e-2 : 1e-4;
  if (p->inner_tol > 0.0) delta = p->inner_tol;
  const int c64 = p->io_dtype == WD_C64;
  const size_t io_elem = c64 ? 8 : 16;
  const size_t io_stride = (size_t)g.V * 12 * io_elem;

  launch_pack_gauge(g, U, P_F32, w.U32, s);
  launch_pack_gauge(g, U, P_F64, w.U64, s);
  for (int k = 0; k < nrhs; ++k) {
    SolverState* st = w.st + k;
    SpinorBuf b64{w.b64 + k * w.stride64, nullptr, P_F64};
    SpinorBuf t64{w.t64 + k * w.stride64, nullptr, P_F64};
    SpinorBuf x64{w.x64 + k * w.stride64, nullptr, P_F64};
    SpinorBuf rl{w.r + k * w.strideL, w.rs ? reinterpret_cast<float*>(w.rs + k * w.strideS) : nullptr, P};
    SpinorBuf pl{w.p + k * w.strideL, w.ps ? reinterpret_cast<float*>(w.ps + k * w.strideS) : nullptr, P};
    SpinorBuf x32{w.xh + k * w.stride32, nullptr, P_F32};
    const char* bk = static_cast<const char*>(B) + k * io_stride;
    char* xk = static_cast<char*>(X) + k * io_stride;
    launch_init_state(st, p->tol, interval, delta, nullptr, 0, s);
    if (p->rhs_mode == WD_RHS_SOURCE) {
      launch_pack_spinor(g, bk, c64, t64, s);
      launch_wilson_packed(g, P_F64, w.U64, t64, b64, mass, 1, G_ALWAYS, F_NONE, st, w.partA, s);
    } else {
      launch_pack_spinor(g, bk, c64, b64, s);
    }
    launch_norm2(g, b64, G_ALWAYS, F_BNORM, st, w.partA, s);
    if (p->zero_guess) {
      // x = 0: the initial residual is b' itself, no stencils
      launch_zero(g, x64, G_ALWAYS, st, s);
      launch_norm2(g, b64, G_ALWAYS, F_RHO_INIT, st, w.partA, s);
      launch_convert(g, b64, rl, G_ALWAYS, st, s);
    } else {
      launch_pack_spinor(g, xk, c64, x64, s);
      launch_wilson_packed(g, P_F64, w.U64, x64, t64, mass, 0, G_ALWAYS, F_NONE, st, w.partA, s);
      launch_residual(g, w.U64, t64, b64, rl, mass, G_ALWAYS, F_RHO_INIT, st, w.partA, s);
    }
    launch_convert(g, rl, pl, G_ALWAYS, st, s);
    launch_zero(g, x32, G_ALWAYS, st, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    snprintf(err, errlen, "batched set-up launch: %s", hipGetErrorString(e));
    return WD_ERR_HIP;
  }

  BatchArgs a{};
  a.g = g;
  a.nrhs = nrhs;
  a.max_iter = p->max_iter;
  a.nsb = (g.V + 63) / 64;
  a.diag = mass + 4.0;
  a.U32 = static_cast<const float2*>(w.U32);
  a.U64 = static_cast<const double2*>(w.U64);
  a.p = w.p; a.r = w.r; a.t = w.t; a.xh = w.xh;
  a.ps = w.ps; a.rs = w.rs; a.ts = w.ts;
  a.strideL = w.strideL;
  a.strideS = w.strideS;
  a.x64 = w.x64; a.b64 = w.b64; a.t64 = w.t64;
  a.stride32 = w.stride32;
  a.stride64 = w.stride64;
  a.st = w.st;
  a.partA = w.partA; a.partB = w.partB; a.partC = w.partC;

  const void* kernel = P == WD_BF16 ? reinterpret_cast<const void*>(k_batched_cg<P_BF16>)
                       : P == WD_F16 ? reinterpret_cast<const void*>(k_batched_cg<P_F16>)
                       : P == WD_I8  ? reinterpret_cast<const void*>(k_batched_cg<P_I8>)
                                     : reinterpret_cast<const void*>(k_batched_cg<P_F32>);
  int dev = 0, cus = 0, per_cu = 0, coop = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev)) != hipSuccess ||
      (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0)) != hipSuccess) {
    snprintf(err, errlen, "device query: %s", hipGetErrorString(e));
    return WD_ERR_HIP;
  }
  if (!coop || per_cu < 1) {
    snprintf(err, errlen, "cooperative launch unsupported (coop=%d, blocks/CU=%d)", coop, per_cu);
    return WD_ERR_HIP;
  }
  int grid = std::min(per_cu * cus, kMaxGrid);
  grid = std::max(1, std::min(grid, a.nsb));
  void* args[] = {&a};
  e = hipLaunchCooperativeKernel(kernel, dim3(grid), dim3(kBlock), args, 0, s);
  if (e != hipSuccess) {
    snprintf(err, errlen, "hipLaunchCooperativeKernel(grid=%d): %s", grid, hipGetErrorString(e));
    return WD_ERR_HIP;
  }
  for (int k = 0; k < nrhs; ++k) {
    SpinorBuf x64{w.x64 + k * w.stride64, nullptr, P_F64};
    launch_unpack_spinor(g, x64, static_cast<char*>(X) + k * io_stride, c64, s);
  }
  SolverState host[kMaxRhs];
  if ((e = hipMemcpyAsync(host, w.st, sizeof(SolverState) * nrhs, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    snprintf(err, errlen, "batched solve: %s", hipGetErrorString(e));
    return WD_ERR_HIP;
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int code = WD_OK;
  for (int k = 0; k < nrhs; ++k) {
    const SolverState& st = host[k];
    int ck;
    if (st.status == -4) ck = WD_ERR_NAN;
    else if (st.status == -3) ck = WD_ERR_BREAKDOWN;
    else if (st.status == 1) ck = WD_OK;
    else ck = WD_NOT_CONVERGED;
    if (ck < 0 && (code >= 0 || ck < code)) code = ck;
    else if (ck == WD_NOT_CONVERGED && code == WD_OK) code = WD_NOT_CONVERGED;
    if (res) {
      const double bn = st.bnorm2 > 0 ? st.bnorm2 : 1.0;
      res[k].iterations = st.iter;
      res[k].reliable_updates = st.rel_updates;
      res[k].status = ck;
      res[k].two_row_links = 0;
      res[k].true_rel_res = std::sqrt(st.rho_true / bn);
      res[k].iter_rel_res = std::sqrt(st.rho / bn);
      res[k].seconds = secs;
    }
  }
  if (code == WD_NOT_CONVERGED) snprintf(err, errlen, "at least one system did not converge in %d iterations",
                                         p->max_iter);
  else if (code < 0) snprintf(err, errlen, "a system ended with status %d (NaN/Inf or breakdown)", code);
  return code;
}

}  // namespace wd
