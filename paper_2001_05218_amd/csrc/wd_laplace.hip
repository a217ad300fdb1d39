// HIP kernels of the second operator: the gauge-covariant lattice Laplacian
// on colour vectors (3 complex numbers per site),
//
//   (L psi)(x) = (m2 + 8) psi(x) - sum_mu [ U_mu(x) psi(x + mu) + U_mu(x - mu)^+ psi(x - mu) ],
//
// Hermitian and, for unitary links and m2 > 0, positive definite, so plain CG
// solves L x = b without normal equations. The paper offers its CG design as a
// backbone for further linear operators with the data movement unchanged
// (abstract, Sec. 3.2, Sec. 7); here the solver state, its gates, the
// deterministic reductions and the host loop are the Wilson solver's, and only
// the stencil and the vector updates below are specific to colour vectors.
//
// Packed colour field: FP64, site-blocked like the spinors, 3 words of one
// complex<double> each: word c of site s at word_index(s, 3, c). Links use the
// FP64 packed gauge layout of the Wilson solver.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "wd_internal.hpp"
#include "wd_reduce.hpp"

namespace wd {

namespace {

// One colour vector in registers: re, im of colour 0, 1, 2.
struct CVec {
  double v[6];
};

struct PackedVec {
  double2* data;
  __device__ __forceinline__ CVec load(int s) const {
    CVec r;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 d = data[word_index(s, 3, c)];
      r.v[2 * c] = d.x;
      r.v[2 * c + 1] = d.y;
    }
    return r;
  }
  __device__ __forceinline__ void store(int s, const CVec& r) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) data[word_index(s, 3, c)] = make_double2(r.v[2 * c], r.v[2 * c + 1]);
  }
};

// Canonical colour field (V, 3) complex128, linear site order.
struct CanonVec {
  double2* data;
  __device__ __forceinline__ CVec load(int s) const {
    CVec r;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 d = data[(size_t)s * 3 + c];
      r.v[2 * c] = d.x;
      r.v[2 * c + 1] = d.y;
    }
    return r;
  }
  __device__ __forceinline__ void store(int s, const CVec& r) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) data[(size_t)s * 3 + c] = make_double2(r.v[2 * c], r.v[2 * c + 1]);
  }
};

// acc -= U v
__device__ __forceinline__ void sub_mul(const double u[18], const CVec& v, CVec& acc) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double ar = u[2 * (3 * i + j)], ai = u[2 * (3 * i + j) + 1];
      acc.v[2 * i] -= ar * v.v[2 * j] - ai * v.v[2 * j + 1];
      acc.v[2 * i + 1] -= ar * v.v[2 * j + 1] + ai * v.v[2 * j];
    }
  }
}

// acc -= U^+ v, (U^+)_ij = conj(U_ji)
__device__ __forceinline__ void sub_mul_dag(const double u[18], const CVec& v, CVec& acc) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double ar = u[2 * (3 * j + i)], ai = u[2 * (3 * j + i) + 1];
      acc.v[2 * i] -= ar * v.v[2 * j] + ai * v.v[2 * j + 1];
      acc.v[2 * i + 1] -= ar * v.v[2 * j + 1] - ai * v.v[2 * j];
    }
  }
}

// h = U^+ v
__device__ __forceinline__ CVec mul_dag(const double u[18], const CVec& v) {
  CVec h;
#pragma unroll
  for (int i = 0; i < 6; ++i) h.v[i] = 0.0;
  sub_mul_dag(u, v, h);
#pragma unroll
  for (int i = 0; i < 6; ++i) h.v[i] = -h.v[i];
  return h;
}

// (L in)(s); also returns in(s) in `c` (the caller may need it for <p, L p>).
template <class Gauge, class Vec>
__device__ __forceinline__ CVec lap_site(const Geom& g, const Gauge& U, const Vec& in, int s, double diag, CVec& c) {
  const Nbrs nb = neighbours(g, s);
  c = in.load(s);
  CVec acc;
#pragma unroll
  for (int i = 0; i < 6; ++i) acc.v[i] = diag * c.v[i];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double u[18];
    U.load(s, mu, u);
    sub_mul(u, in.load(nb.fwd[mu]), acc);
    U.load(nb.bwd[mu], mu, u);
    sub_mul_dag(u, in.load(nb.bwd[mu]), acc);
  }
  return acc;
}

// Tiled order: one workgroup per 4^4 tile. The tile's input vectors are
// staged in LDS, and each link is read once: U_mu(x) is loaded by the thread
// at x, which applies it forward for x and, as U_mu(x)^+ in(x), hands the
// backward term of the site x + mu over through LDS. Only at the tile's
// lower faces does a thread load U_mu(x - mu) itself, and only at the faces
// does it read a neighbour's vector from memory.
struct LapTileLds {
  double2 in[3][kBlock];
  double2 up[3][kBlock];   // backward terms for the site above, current direction
};

__device__ __forceinline__ CVec lap_tile(const Geom& g, const PackedGauge<P_F64>& U, const PackedVec& in, int T,
                                         double diag, CVec& c, LapTileLds& lds) {
  const int l = threadIdx.x;
  const int s = T * kBlock + l;
  c = in.load(s);
#pragma unroll
  for (int k = 0; k < 3; ++k) lds.in[k][l] = make_double2(c.v[2 * k], c.v[2 * k + 1]);
  CVec acc;
#pragma unroll
  for (int i = 0; i < 6; ++i) acc.v[i] = diag * c.v[i];
  int b[4];
  tile_coords(g, (uint32_t)T, b);
  __syncthreads();
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int ls = 1 << (2 * mu);
    const int lm = (l >> (2 * mu)) & 3;
    double u[18];
    U.load(s, mu, u);
    CVec f;
    if (lm < 3) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double2 d = lds.in[k][l + ls];
        f.v[2 * k] = d.x;
        f.v[2 * k + 1] = d.y;
      }
    } else {
      f = in.load((tile_step(g, T, b, mu, +1) << 8) + (l - 3 * ls));
    }
    sub_mul(u, f, acc);
    if (lm < 3) {
      const CVec h = mul_dag(u, c);
#pragma unroll
      for (int k = 0; k < 3; ++k) lds.up[k][l + ls] = make_double2(h.v[2 * k], h.v[2 * k + 1]);
    }
    __syncthreads();
    if (lm > 0) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double2 d = lds.up[k][l];
        acc.v[2 * k] -= d.x;
        acc.v[2 * k + 1] -= d.y;
      }
    } else {
      const int sb = (tile_step(g, T, b, mu, -1) << 8) + (l + 3 * ls);
      U.load(sb, mu, u);
      sub_mul_dag(u, in.load(sb), acc);
    }
    __syncthreads();   // lds.up is rewritten for the next direction
  }
  return acc;
}

__device__ __forceinline__ PackedGauge<P_F64> packed_links(const void* U) {
  PackedGauge<P_F64> u;
  u.data = static_cast<const double2*>(U);
  return u;
}

__device__ __forceinline__ double dot_re(const CVec& a, const CVec& b) {
  double d = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) d += a.v[i] * b.v[i];
  return d;
}

}  // namespace

// out = L in on canonical fields (linear order, one thread per site).
__global__ __launch_bounds__(kBlock) void k_lap_canonical(Geom g, const double2* __restrict__ U, const double2* in,
                                                          double2* out, double diag) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  CanonGauge u;
  u.data = U;
  u.V = (size_t)g.V;
  CanonVec vi{const_cast<double2*>(in)};
  CVec c;
  const CVec o = lap_site(g, u, vi, s, diag, c);
  CanonVec{out}.store(s, o);
}

// Canonical (V, 3) colour field (complex128 or complex64) <-> packed FP64.
__global__ __launch_bounds__(kBlock) void k_lap_pack(Geom g, const void* in, int c64, double2* out) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int ci = canonical_index(g, s);
  CVec r;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c64) {
      const float2 f = static_cast<const float2*>(in)[(size_t)ci * 3 + c];
      r.v[2 * c] = f.x;
      r.v[2 * c + 1] = f.y;
    } else {
      const double2 d = static_cast<const double2*>(in)[(size_t)ci * 3 + c];
      r.v[2 * c] = d.x;
      r.v[2 * c + 1] = d.y;
    }
  }
  PackedVec{out}.store(s, r);
}

__global__ __launch_bounds__(kBlock) void k_lap_unpack(Geom g, const double2* in, void* out, int c64) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int ci = canonical_index(g, s);
  const CVec r = PackedVec{const_cast<double2*>(in)}.load(s);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c64) static_cast<float2*>(out)[(size_t)ci * 3 + c] = make_float2((float)r.v[2 * c], (float)r.v[2 * c + 1]);
    else static_cast<double2*>(out)[(size_t)ci * 3 + c] = make_double2(r.v[2 * c], r.v[2 * c + 1]);
  }
}

// t = L p on packed fields; with fin != F_NONE, Re <p, t> per workgroup.
template <bool TILE>
__global__ __launch_bounds__(kBlock) void k_lap_packed(Geom g, const void* U, const double2* p, double2* t,
                                                       double diag, int gate, int fin, SolverState* st,
                                                       double* partials) {
  if (!gate_open(st, gate)) return;
  const int T = xcd_tile(blockIdx.x, gridDim.x);
  const int s = T * kBlock + threadIdx.x;
  double d = 0.0;
  const PackedVec in{const_cast<double2*>(p)};
  if constexpr (TILE) {
    __shared__ LapTileLds lds;
    CVec c;
    const CVec o = lap_tile(g, packed_links(U), in, T, diag, c, lds);
    PackedVec{t}.store(s, o);
    d = dot_re(c, o);
  } else if (s < g.V) {
    CVec c;
    const CVec o = lap_site(g, packed_links(U), in, s, diag, c);
    PackedVec{t}.store(s, o);
    d = dot_re(c, o);
  }
  if (fin != F_NONE) store_partial(d, partials);
}

// r = b - L x; |r|^2 per workgroup.
template <bool TILE>
__global__ __launch_bounds__(kBlock) void k_lap_residual(Geom g, const void* U, const double2* x, const double2* b,
                                                         double2* r, double diag, int gate, SolverState* st,
                                                         double* partials) {
  if (!gate_open(st, gate)) return;
  const int T = xcd_tile(blockIdx.x, gridDim.x);
  const int s = T * kBlock + threadIdx.x;
  double n2 = 0.0;
  const PackedVec in{const_cast<double2*>(x)};
  CVec lx, c;
  bool have = true;
  if constexpr (TILE) {
    __shared__ LapTileLds lds;
    lx = lap_tile(g, packed_links(U), in, T, diag, c, lds);
  } else {
    have = s < g.V;
    if (have) lx = lap_site(g, packed_links(U), in, s, diag, c);
  }
  if (have) {
    CVec o = PackedVec{const_cast<double2*>(b)}.load(s);
#pragma unroll
    for (int i = 0; i < 6; ++i) o.v[i] -= lx.v[i];
    PackedVec{r}.store(s, o);
    n2 = dot_re(o, o);
  }
  store_partial(n2, partials);
}

// x += alpha p; r -= alpha t; |r|^2 per workgroup (a CG iteration's vector step).
__global__ __launch_bounds__(kBlock) void k_lap_update(Geom g, const double2* t, double2* r, const double2* p,
                                                       double2* x, const SolverState* st, double* partials) {
  if (!gate_open(st, G_ITER)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (s < g.V) {
    const double a = st->alpha;
    const PackedVec R{r}, X{x};
    const CVec tv = PackedVec{const_cast<double2*>(t)}.load(s);
    const CVec pv = PackedVec{const_cast<double2*>(p)}.load(s);
    CVec rv = R.load(s), xv = X.load(s);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      xv.v[i] = fma(a, pv.v[i], xv.v[i]);
      rv.v[i] = fma(-a, tv.v[i], rv.v[i]);
    }
    X.store(s, xv);
    R.store(s, rv);
    n2 = dot_re(rv, rv);
  }
  store_partial(n2, partials);
}

// p = r + beta p
__global__ __launch_bounds__(kBlock) void k_lap_p_update(Geom g, const double2* r, double2* p, const SolverState* st) {
  if (!gate_open(st, G_ITER)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const double beta = st->beta;
  const PackedVec P{p};
  const CVec rv = PackedVec{const_cast<double2*>(r)}.load(s);
  CVec pv = P.load(s);
#pragma unroll
  for (int i = 0; i < 6; ++i) pv.v[i] = fma(beta, pv.v[i], rv.v[i]);
  P.store(s, pv);
}

// |v|^2 per workgroup
__global__ __launch_bounds__(kBlock) void k_lap_norm2(Geom g, const double2* v, double* partials) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (s < g.V) {
    const CVec a = PackedVec{const_cast<double2*>(v)}.load(s);
    n2 = dot_re(a, a);
  }
  store_partial(n2, partials);
}

// dst = src (gated), or dst = 0 when src is null
__global__ __launch_bounds__(kBlock) void k_lap_copy(Geom g, const double2* src, double2* dst, int gate,
                                                     const SolverState* st) {
  if (!gate_open(st, gate)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t w = word_index(s, 3, c);
    dst[w] = src ? src[w] : make_double2(0.0, 0.0);
  }
}

// ============================================================= launchers

namespace {
template <typename... KArgs, typename... Args>
void launch_lap(void (*kernel)(KArgs...), const Geom& g, hipStream_t s, const EventPair* ev, Args... args) {
  if (ev)
    hipExtLaunchKernelGGL(kernel, dim3(g.nblocks), dim3(kBlock), 0, s, ev->begin, ev->end, 0,
                          static_cast<KArgs>(args)...);
  else
    kernel<<<dim3(g.nblocks), kBlock, 0, s>>>(static_cast<KArgs>(args)...);
}
}  // namespace

void launch_lap_canonical(const Geom& g, const void* U, const void* in, void* out, double m2, hipStream_t s) {
  k_lap_canonical<<<g.nblocks, kBlock, 0, s>>>(g, static_cast<const double2*>(U), static_cast<const double2*>(in),
                                               static_cast<double2*>(out), m2 + 8.0);
}

void launch_lap_pack(const Geom& g, const void* in, int c64, void* out, hipStream_t s) {
  k_lap_pack<<<g.nblocks, kBlock, 0, s>>>(g, in, c64, static_cast<double2*>(out));
}

void launch_lap_unpack(const Geom& g, const void* in, void* out, int c64, hipStream_t s) {
  k_lap_unpack<<<g.nblocks, kBlock, 0, s>>>(g, static_cast<const double2*>(in), out, c64);
}

void launch_lap_packed(const Geom& g, const void* U, const void* p, void* t, double m2, int gate, int fin,
                       SolverState* st, double* partials, hipStream_t s, const EventPair* ev) {
  if (g.tiled)
    launch_lap(k_lap_packed<true>, g, s, ev, g, U, static_cast<const double2*>(p), static_cast<double2*>(t), m2 + 8.0,
               gate, fin, st, partials);
  else
    launch_lap(k_lap_packed<false>, g, s, ev, g, U, static_cast<const double2*>(p), static_cast<double2*>(t), m2 + 8.0,
               gate, fin, st, partials);
  if (fin != F_NONE) launch_finalize_n(g.nblocks, partials, st, fin, gate, s);
}

void launch_lap_residual(const Geom& g, const void* U, const void* x, const void* b, void* r, double m2, int gate,
                         int fin, SolverState* st, double* partials, hipStream_t s) {
  if (g.tiled)
    k_lap_residual<true><<<g.nblocks, kBlock, 0, s>>>(g, U, static_cast<const double2*>(x),
                                                      static_cast<const double2*>(b), static_cast<double2*>(r),
                                                      m2 + 8.0, gate, st, partials);
  else
    k_lap_residual<false><<<g.nblocks, kBlock, 0, s>>>(g, U, static_cast<const double2*>(x),
                                                       static_cast<const double2*>(b), static_cast<double2*>(r),
                                                       m2 + 8.0, gate, st, partials);
  launch_finalize_n(g.nblocks, partials, st, fin, gate, s);
}

void launch_lap_update(const Geom& g, const void* t, void* r, const void* p, void* x, SolverState* st,
                       double* partials, hipStream_t s, const EventPair* ev) {
  const SolverState* cst = st;
  launch_lap(k_lap_update, g, s, ev, g, static_cast<const double2*>(t), static_cast<double2*>(r),
             static_cast<const double2*>(p), static_cast<double2*>(x), cst, partials);
  launch_finalize_n(g.nblocks, partials, st, F_BETA, G_ITER, s);
}

void launch_lap_p_update(const Geom& g, const void* r, void* p, SolverState* st, hipStream_t s, const EventPair* ev) {
  const SolverState* cst = st;
  launch_lap(k_lap_p_update, g, s, ev, g, static_cast<const double2*>(r), static_cast<double2*>(p), cst);
}

void launch_lap_norm2(const Geom& g, const void* v, int fin, SolverState* st, double* partials, hipStream_t s) {
  k_lap_norm2<<<g.nblocks, kBlock, 0, s>>>(g, static_cast<const double2*>(v), partials);
  launch_finalize_n(g.nblocks, partials, st, fin, G_ALWAYS, s);
}

void launch_lap_copy(const Geom& g, const void* src, void* dst, int gate, SolverState* st, hipStream_t s) {
  k_lap_copy<<<g.nblocks, kBlock, 0, s>>>(g, static_cast<const double2*>(src), static_cast<double2*>(dst), gate, st);
}

}  // namespace wd
