// HIP kernels of the Wilson-Dirac library for gfx950: packing, the Wilson
// stencil with fused solver epilogues, deterministic reductions, the CG
// vector updates and the gauge-link force.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "wd_dslash.hpp"
#include "wd_internal.hpp"
#include "wd_reduce.hpp"
#include "wd_tiled.hpp"

namespace wd {

// ------------------------------------------------------------ reductions

__device__ __forceinline__ bool finite_d(double x) { return x - x == 0.0; }

// Apply the end-of-reduction update to the solver state (one thread).
__device__ void finalize(SolverState* st, int fin, double sum) {
  switch (fin) {
    case F_BNORM:
      st->bnorm2 = sum;
      st->stop2 = st->stop2 * sum;   // host stored tol^2 in stop2
      break;
    case F_RHO_INIT:
      st->rho = sum;
      st->rho_true = sum;
      st->rho_update = sum;
      if (!finite_d(sum)) st->status = -4;
      else if (sum <= st->stop2) st->status = 1;
      break;
    case F_ALPHA:
    case F_ALPHA_RING:
      st->tnorm = sum;
      if (!finite_d(sum)) st->status = -4;
      else if (sum <= 0.0) st->status = -3;
      else st->alpha = st->rho / sum;
      if (fin == F_ALPHA_RING) {
        // the p just applied (ring slot npend) joins the pending x update.
        // The host folds the ring often enough that npend < ring_len here;
        // if not, D and the p update skipped their ring access: stop.
        if (st->npend >= st->ring_len) {
          st->status = -5;
        } else {
          st->alpha_hist[st->npend] = st->alpha;
          st->pcur = st->npend;
          st->npend += 1;
        }
      }
      break;
    case F_BETA: {
      st->rho_prev = st->rho;
      st->rho = sum;
      st->iter += 1;
      if (st->hist && st->iter <= st->hist_len) st->hist[st->iter - 1] = sqrt(sum / st->bnorm2);
      if (!finite_d(sum)) {
        st->status = -4;
      } else {
        st->beta = sum / st->rho_prev;
        if (sum <= st->stop2) {
          if (st->interval > 0) st->inner_done = 1;   // mixed: verify by a reliable update
          else st->status = 1;
        }
      }
      break;
    }
    case F_RELIABLE: {
      const double iterated = st->rho;
      st->rho_true = sum;
      st->rho_update = sum;
      st->rel_updates += 1;
      st->last_update = st->iter;
      st->inner_done = 0;
      st->npend = 0;   // the pending x update went into the accumulation before this
      if (!finite_d(sum)) st->status = -4;
      else if (sum <= st->stop2) st->status = 1;
      else {
        st->rho = sum;
        // keep the search direction (beta from the recomputed residual) unless
        // the low-precision recurrence has drifted far from the true residual,
        // or each recomputation starts a new inner solve (refinement)
        st->beta = (st->restart_on_update || sum > 4.0 * iterated) ? 0.0 : sum / st->rho_prev;
      }
      break;
    }
    case F_TRUE:
      st->rho_true = sum;
      break;
    case F_SU3MAX:
      st->su3_dev = sum;
      break;
    default:
      break;
  }
}

constexpr int kFinBlock = 1024;

// Sum of n partials in a fixed order, then the state update `fin`. Runs with
// the same gate as the kernel that wrote the partials (which did not change
// the state), so both are skipped or run together.
__global__ __launch_bounds__(kFinBlock) void k_finalize(const double* __restrict__ partials, int n, SolverState* st,
                                                        int fin, int gate, Rhs rb) {
  // one workgroup per system
  const long long off = (long long)blockIdx.x * rb.stride;
  partials = rhs_shift(partials, off);
  st = rhs_shift(st, off);
  if (!gate_open(st, gate)) return;
  __shared__ double wsum[kFinBlock / 64];
  const bool use_max = (fin == F_SU3MAX);
  // eight loads in flight per thread before any add (the partials were just
  // written by other XCDs, so each load is a full memory round trip)
  double v = 0.0;
  for (int base = 0; base < n; base += 8 * kFinBlock) {
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = base + k * kFinBlock + threadIdx.x;
      a[k] = i < n ? partials[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v = use_max ? fmax(v, a[k]) : v + a[k];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = use_max ? fmax(v, o) : v + o;
  }
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kFinBlock / 64; ++i) t = use_max ? fmax(t, wsum[i]) : t + wsum[i];
    finalize(st, fin, t);
  }
}

void launch_finalize_n(int n, double* partials, SolverState* st, int fin, int gate, hipStream_t s) {
  k_finalize<<<1, kFinBlock, 0, s>>>(partials, n, st, fin, gate, Rhs{});
}

static void launch_finalize(const Geom& g, double* partials, SolverState* st, int fin, int gate, hipStream_t s,
                            Rhs rb = {}) {
  k_finalize<<<rb.n, kFinBlock, 0, s>>>(partials, g.nblocks, st, fin, gate, rb);
}

// Where a tile kernel stores tile T's partial: the slot that the workgroup of
// tile T has in a single-system launch, so that a system's partials are
// summed in the same order whether it is solved alone or in a lockstep batch
// (identical iterates either way).
__device__ __forceinline__ int partial_slot(int T, const Rhs& rb) {
  return rb.n == 1 ? (int)blockIdx.x : xcd_tile_inv(T, (int)gridDim.x / rb.n);
}

// ------------------------------------------------------- spinor dispatch

template <int P> __device__ __forceinline__ PackedSpinor<P> spinor_of(const SpinorBuf& b) {
  PackedSpinor<P> s;
  s.data = reinterpret_cast<decltype(s.data)>(b.data);
  s.scale = b.scale;
  return s;
}
template <int P> __device__ __forceinline__ PackedGauge<P> gauge_of(const void* p) {
  PackedGauge<P> u;
  u.data = reinterpret_cast<decltype(u.data)>(p);
  return u;
}

// ---------------------------------------------------------------- packing

template <int P>
__global__ __launch_bounds__(kBlock) void k_pack_gauge(Geom g, const double2* __restrict__ U, void* out) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int c = canonical_index(g, s);
  for (int mu = 0; mu < 4; ++mu) {
    const double2* src = U + ((size_t)mu * g.V + c) * 9;
    for (int e = 0; e < 9; ++e) {
      const double2 d = src[e];
      const size_t w = word_index(s, 36, mu * 9 + e);
      if constexpr (P == P_F64) reinterpret_cast<double2*>(out)[w] = d;
      else if constexpr (P == P_F32) reinterpret_cast<float2*>(out)[w] = make_float2((float)d.x, (float)d.y);
      else if constexpr (P == P_BF16)
        reinterpret_cast<uint32_t*>(out)[w] = pack_bf16x2((float)d.x, (float)d.y);
      else   // FP16, and the FP16 links of the int8 storage
        reinterpret_cast<uint32_t*>(out)[w] = pack_f16x2((float)d.x, (float)d.y);
    }
  }
}

// Two-row (12-real) 16-bit copy of an SU(3) field: rows 0 and 1 of each link.
template <int P>
__global__ __launch_bounds__(kBlock) void k_pack_gauge_rows2(Geom g, const double2* __restrict__ U, uint32_t* out) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int c = canonical_index(g, s);
  for (int mu = 0; mu < 4; ++mu) {
    const double2* src = U + ((size_t)mu * g.V + c) * 9;
    for (int e = 0; e < 6; ++e) {
      const double2 d = src[e];
      out[word_index(s, 24, mu * 6 + e)] = (P == P_BF16) ? pack_bf16x2((float)d.x, (float)d.y)
                                                         : pack_f16x2((float)d.x, (float)d.y);
    }
  }
}

// Largest deviation of any link from SU(3): max over links of
// max_ij |(U U^+)_ij - delta_ij| and |det U - 1|, per workgroup.
__global__ __launch_bounds__(kBlock) void k_su3_check(Geom g, const double2* __restrict__ U, double* partials) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  double dev = 0.0;
  if (c < g.V) {
    for (int mu = 0; mu < 4; ++mu) {
      const double2* u = U + ((size_t)mu * g.V + c) * 9;
      double a[9][2];
      for (int e = 0; e < 9; ++e) {
        a[e][0] = u[e].x;
        a[e][1] = u[e].y;
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double re = 0.0, im = 0.0;
          for (int k = 0; k < 3; ++k) {   // sum_k U_ik conj(U_jk)
            re += a[i * 3 + k][0] * a[j * 3 + k][0] + a[i * 3 + k][1] * a[j * 3 + k][1];
            im += a[i * 3 + k][1] * a[j * 3 + k][0] - a[i * 3 + k][0] * a[j * 3 + k][1];
          }
          if (i == j) re -= 1.0;
          dev = fmax(dev, fmax(fabs(re), fabs(im)));
        }
      // det by the first row's cofactors
      double dr = 0.0, di = 0.0;
      for (int k = 0; k < 3; ++k) {
        const int p = (k + 1) % 3, q = (k + 2) % 3;
        const double cr = a[3 + p][0] * a[6 + q][0] - a[3 + p][1] * a[6 + q][1] - (a[3 + q][0] * a[6 + p][0] - a[3 + q][1] * a[6 + p][1]);
        const double ci = a[3 + p][0] * a[6 + q][1] + a[3 + p][1] * a[6 + q][0] - (a[3 + q][0] * a[6 + p][1] + a[3 + q][1] * a[6 + p][0]);
        dr += a[k][0] * cr - a[k][1] * ci;
        di += a[k][0] * ci + a[k][1] * cr;
      }
      dev = fmax(dev, fmax(fabs(dr - 1.0), fabs(di)));
      if (!(dev == dev)) dev = 1e300;   // NaN links are not SU(3)
    }
  }
  // workgroup max (fixed order)
  __shared__ double wmax[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) m = fmax(m, wmax[i]);
    partials[blockIdx.x] = m;
  }
}

template <int P, typename IO>
__global__ __launch_bounds__(kBlock) void k_pack_spinor(Geom g, const IO* __restrict__ in, SpinorBuf out) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  using R = typename PackedSpinor<P>::Real;
  R v[24];
  const IO* p = in + (size_t)canonical_index(g, s) * 12;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    v[2 * i] = (R)p[i].x;
    v[2 * i + 1] = (R)p[i].y;
  }
  spinor_of<P>(out).store(s, v);
}

template <int P, typename IO>
__global__ __launch_bounds__(kBlock) void k_unpack_spinor(Geom g, SpinorBuf in, IO* __restrict__ out) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  using R = typename PackedSpinor<P>::Real;
  R v[24];
  spinor_of<P>(in).load(s, v);
  IO* p = out + (size_t)canonical_index(g, s) * 12;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    IO d;
    d.x = v[2 * i];
    d.y = v[2 * i + 1];
    p[i] = d;
  }
}

template <int PA, int PB>
__global__ __launch_bounds__(kBlock) void k_convert(Geom g, SpinorBuf in, SpinorBuf out, int gate,
                                                    const SolverState* st) {
  if (!gate_open(st, gate)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  typename PackedSpinor<PA>::Real a[24];
  typename PackedSpinor<PB>::Real b[24];
  spinor_of<PA>(in).load(s, a);
#pragma unroll
  for (int i = 0; i < 24; ++i) b[i] = (typename PackedSpinor<PB>::Real)a[i];
  spinor_of<PB>(out).store(s, b);
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_zero(Geom g, SpinorBuf v, int gate, const SolverState* st) {
  if (!gate_open(st, gate)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  typename PackedSpinor<P>::Real z[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) z[i] = 0;
  spinor_of<P>(v).store(s, z);
}

// -------------------------------------------------------- Wilson operator

template <bool DAG>
__global__ __launch_bounds__(kBlock) void k_wilson_canonical(Geom g, CanonGauge U, CanonSpinor in, CanonSpinor out,
                                                             double diag) {
  const int s = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const Nbrs nb = neighbours(g, s);
  double o[24];
  wilson_site<DAG>(U, in, s, nb, diag, o);
  out.store(s, o);
}

// The stencil at site s of workgroup tile T: from the LDS-staged tile, each
// link read once, when TILE (FP64 / FP32 on the tiled order; every thread of
// the workgroup must get here), else straight from memory.
template <int P, bool DAG, bool TILE>
__device__ __forceinline__ void stencil_at(const Geom& g, const void* U, const SpinorBuf& in, int T, int s,
                                           typename PackedSpinor<P>::Real diag,
                                           typename PackedSpinor<P>::Real o[24]) {
  const Nbrs nb = neighbours(g, s);
  if constexpr (TILE) {
    __shared__ typename TileWord<P>::T lds[TileWord<P>::n * kTileSites];
    __shared__ UpBuf<typename PackedSpinor<P>::Real> up;
    const TileSrc<P> src = stage_own_tile<P>(in, T, lds);
    wilson_site_once<DAG>(gauge_of<P>(U), src, s, nb, diag, o, up);
  } else {
    wilson_site<DAG>(gauge_of<P>(U), spinor_of<P>(in), s, nb, diag, o);
  }
}

template <int P, bool DAG, bool TILE>
__global__ __launch_bounds__(kBlock) void k_wilson_packed(Geom g, const void* U, SpinorBuf in, SpinorBuf out,
                                                          double diag, int gate, int fin, SolverState* st,
                                                          double* partials, RingBuf ring, Rhs rb) {
  int k;
  const int T = rhs_split(xcd_tile(blockIdx.x, gridDim.x), rb, k);
  if (k) {
    const long long off = k * rb.stride;
    st = rhs_shift(st, off);
    partials = rhs_shift(partials, off);
    in = rhs_shift(in, off);
    out = rhs_shift(out, off);
    ring = rhs_shift(ring, off);
  }
  if (!gate_open(st, gate)) return;
  if (ring.data) {
    if (st->npend >= ring.len) return;   // never with the host's fold cadence
    in = ring.at(st->npend);
  }
  using R = typename PackedSpinor<P>::Real;
  const int s = T * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (TILE || s < g.V) {
    R o[24];
    stencil_at<P, DAG, TILE>(g, U, in, T, s, (R)diag, o);
    spinor_of<P>(out).store(s, o);
    if (fin != F_NONE) {
#pragma unroll
      for (int i = 0; i < 24; ++i) n2 += (double)o[i] * (double)o[i];
    }
  }
  if (fin != F_NONE) store_partial(n2, partials, partial_slot(T, rb));
}

// LDS-staged stencil (16-bit storage, tiled order): one workgroup per 4^4 tile.
// At most 128 VGPRs (4 waves per SIMD): without the bound the BF16
// instantiation hoists unpacking into 256+ registers and runs one wave per SIMD.
#define WD_TILED_OCCUPANCY __attribute__((amdgpu_waves_per_eu(4, 8)))

template <int P, bool C12, bool DAG>
__global__ __launch_bounds__(kBlock) WD_TILED_OCCUPANCY void k_wilson_tiled(Geom g, const void* U, SpinorBuf in, SpinorBuf out,
                                                         double diag, int gate, int fin, SolverState* st,
                                                         double* partials, RingBuf ring, Rhs rb) {
  int k;
  const int T = rhs_split(xcd_tile(blockIdx.x, gridDim.x), rb, k);
  if (k) {
    const long long off = k * rb.stride;
    st = rhs_shift(st, off);
    partials = rhs_shift(partials, off);
    in = rhs_shift(in, off);
    out = rhs_shift(out, off);
    ring = rhs_shift(ring, off);
  }
  if (!gate_open(st, gate)) return;
  if (ring.data) {
    if (st->npend >= ring.len) return;   // never with the host's fold cadence
    in = ring.at(st->npend);
  }
  __shared__ TileLds<P> lds;
  uint32_t lk[8][9];
  float o[24];
  if constexpr (P == P_I8 || P == P_F16) {
    tile_stage<P, C12>(g, T, U, in, lds, lk, -0.5f);
    __syncthreads();
    tile_links_late<C12>(g, T, U, lk);
    tile_wilson_h<C12, DAG>(lds, lk, -2.0f * (float)diag, o);
  } else {
    tile_stage<P, C12>(g, T, U, in, lds, lk);
    __syncthreads();
    tile_links_late<C12>(g, T, U, lk);
    tile_wilson<P, C12, DAG>(lds, lk, (float)diag, o);
  }
  spinor_of<P>(out).store(T * kTileSites + threadIdx.x, o);
  if (fin != F_NONE) {
    // the site's 24 squares summed in FP32 (relative 1e-7), the sites in FP64
    float s2 = 0.f;
#pragma unroll
    for (int i = 0; i < 24; ++i) s2 = fmaf(o[i], o[i], s2);
    store_partial((double)s2, partials, partial_slot(T, rb));
  }
}

// r update of the mixed solver with the LDS-staged D^+ (16- or 8-bit
// storage, tiled order): q = D^+ t (never stored), r -= alpha q, ||r||^2. The
// solution update is deferred (the search directions wait in a ring).
template <int P, bool C12>
__global__ __launch_bounds__(kBlock) WD_TILED_OCCUPANCY void k_cg_update_tiled(Geom g, const void* U, SpinorBuf t, SpinorBuf r,
                                                            double diag, SolverState* st, double* partials, Rhs rb) {
  int k;
  const int T = rhs_split(xcd_tile(blockIdx.x, gridDim.x), rb, k);
  if (k) {
    const long long off = k * rb.stride;
    st = rhs_shift(st, off);
    partials = rhs_shift(partials, off);
    t = rhs_shift(t, off);
    r = rhs_shift(r, off);
  }
  if (!gate_open(st, G_ITER)) return;
  __shared__ TileLds<P> lds;
  uint32_t lk[8][9];
  const int s = T * kTileSites + threadIdx.x;
  const float a = (float)st->alpha;
  float rv[24];
  const auto rs = spinor_of<P>(r);
  if constexpr (P == P_I8 || P == P_F16) {
    // y = -alpha D^+ t straight from the hops (kappa = alpha / 2), then
    // r = factor * (r's stored numbers) + y: no separate scaling of q or r
    tile_stage<P, C12>(g, T, U, t, lds, lk, 0.5f * a);
    __syncthreads();
    tile_links_late<C12>(g, T, U, lk);
    float y[24];
    tile_wilson_h<C12, true>(lds, lk, -2.0f * (float)diag, y);
    typename SpinorWord<P>::T dr[3];
#pragma unroll
    for (int w = 0; w < 3; ++w) dr[w] = rs.data[word_index(s, 3, w)];
    const float fr = PackedSpinor<P>::raw_factor(rs.load_scale(s));
    PackedSpinor<P>::unpack_raw(dr, rv);
#pragma unroll
    for (int i = 0; i < 24; ++i) rv[i] = fmaf(fr, rv[i], y[i]);
  } else {
    tile_stage<P, C12>(g, T, U, t, lds, lk);
    __syncthreads();
    tile_links_late<C12>(g, T, U, lk);
    float q[24];
    tile_wilson<P, C12, true>(lds, lk, (float)diag, q);
    rs.load(s, rv);
#pragma unroll
    for (int i = 0; i < 24; ++i) rv[i] = fmaf(-a, q[i], rv[i]);
  }
  typename SpinorWord<P>::T d[3];
  float sc;
  PackedSpinor<P>::pack(rv, d, sc);
  rs.store_raw(s, d, sc);
  // the norm of what the next iteration reads
  double n2 = 0.0;
  if constexpr (P == P_I8) {
    // factor^2 times the sum of the squared bytes, exact in int32 (<= 24 * 127^2)
    int q2 = 0;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      q2 = __builtin_amdgcn_sdot4((int)d[w].x, (int)d[w].x, q2, false);
      q2 = __builtin_amdgcn_sdot4((int)d[w].y, (int)d[w].y, q2, false);
    }
    const double f = (double)PackedSpinor<P>::raw_factor(sc);
    n2 = f * f * (double)q2;
  } else if constexpr (P == P_F16) {
    // scale^2 times the sum of the stored halves' squares (exact products, FP32 sums)
    float h2 = 0.f;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      h2 = dot2(d[w].x, d[w].x, h2);
      h2 = dot2(d[w].y, d[w].y, h2);
      h2 = dot2(d[w].z, d[w].z, h2);
      h2 = dot2(d[w].w, d[w].w, h2);
    }
    n2 = (double)sc * (double)sc * (double)h2;
  } else {
    PackedSpinor<P>::unpack(d, sc, rv);
#pragma unroll
    for (int i = 0; i < 24; ++i) n2 += (double)rv[i] * (double)rv[i];
  }
  store_partial(n2, partials, partial_slot(T, rb));
}

// q = D^+ t at site s; r -= alpha q; x += alpha p; reduce ||r||^2 (of the stored r).
template <int P, int PX, bool TILE, bool XP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_cg_update(Geom g, const void* U, SpinorBuf t, SpinorBuf r, SpinorBuf p,
                                                      SpinorBuf x, double diag, SolverState* st, double* partials) {
  if (!gate_open(st, G_ITER)) return;
  using R = typename PackedSpinor<P>::Real;
  using RX = typename PackedSpinor<PX>::Real;
  const int T = xcd_tile(blockIdx.x, gridDim.x);
  const int s = T * kBlock + threadIdx.x;
  const double alpha = st->alpha;
  double n2 = 0.0;
  if (TILE || s < g.V) {
    R q[24];
    stencil_at<P, true, TILE>(g, U, t, T, s, (R)diag, q);
    // the epilogue's loads are not hoisted into the stencil (register pressure)
    __builtin_amdgcn_sched_barrier(0);
    R rv[24];
    const auto rs = spinor_of<P>(r);
    rs.load(s, rv);
    if constexpr (XP) {
      R pv[24];
      RX xv[24];
      spinor_of<P>(p).load(s, pv);
      spinor_of<PX>(x).load(s, xv);
#pragma unroll
      for (int i = 0; i < 24; ++i) xv[i] = fma((RX)alpha, (RX)pv[i], xv[i]);
      spinor_of<PX>(x).store(s, xv);
    }
    const R a = (R)alpha;
#pragma unroll
    for (int i = 0; i < 24; ++i) rv[i] = fma(-a, q[i], rv[i]);
    rs.store(s, rv);
    if constexpr (P == P_F64 || P == P_F32) {
#pragma unroll
      for (int i = 0; i < 24; ++i) n2 += (double)rv[i] * (double)rv[i];
    } else {
      // the norm of what the next iteration will read
      rs.load(s, rv);
#pragma unroll
      for (int i = 0; i < 24; ++i) n2 += (double)rv[i] * (double)rv[i];
    }
  }
  store_partial(n2, partials);
}

// out = low(b - D^+ t) in FP64 arithmetic (t, b and links FP64); reduce the FP64 norm.
template <int PO, bool TILE>
__global__ __launch_bounds__(kBlock) void k_residual(Geom g, const void* U64, SpinorBuf t64, SpinorBuf b64,
                                                     SpinorBuf out, double diag, int gate, int fin, SolverState* st,
                                                     double* partials, Rhs rb) {
  int k;
  const int T = rhs_split(xcd_tile(blockIdx.x, gridDim.x), rb, k);
  if (k) {
    const long long off = k * rb.stride;
    st = rhs_shift(st, off);
    partials = rhs_shift(partials, off);
    t64 = rhs_shift(t64, off);
    b64 = rhs_shift(b64, off);
    out = rhs_shift(out, off);
  }
  if (!gate_open(st, gate)) return;
  const int s = T * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (TILE || s < g.V) {
    double q[24], b[24];
    stencil_at<P_F64, true, TILE>(g, U64, t64, T, s, diag, q);
    spinor_of<P_F64>(b64).load(s, b);
    typename PackedSpinor<PO>::Real o[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) {
      const double d = b[i] - q[i];
      n2 += d * d;
      o[i] = (typename PackedSpinor<PO>::Real)d;
    }
    spinor_of<PO>(out).store(s, o);
  }
  store_partial(n2, partials, partial_slot(T, rb));
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_p_update(Geom g, SpinorBuf r, SpinorBuf p, const SolverState* st) {
  if (!gate_open(st, G_ITER)) return;
  using R = typename PackedSpinor<P>::Real;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const R beta = (R)st->beta;
  R rv[24], pv[24];
  spinor_of<P>(r).load(s, rv);
  spinor_of<P>(p).load(s, pv);
#pragma unroll
  for (int i = 0; i < 24; ++i) pv[i] = fma(beta, pv[i], rv[i]);
  spinor_of<P>(p).store(s, pv);
}

template <int PX>
__global__ __launch_bounds__(kBlock) void k_accumulate(Geom g, SpinorBuf x64, SpinorBuf xhat, int gate,
                                                       const SolverState* st) {
  if (!gate_open(st, gate)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  double xv[24];
  typename PackedSpinor<PX>::Real hv[24];
  spinor_of<P_F64>(x64).load(s, xv);
  spinor_of<PX>(xhat).load(s, hv);
#pragma unroll
  for (int i = 0; i < 24; ++i) {
    xv[i] += (double)hv[i];
    hv[i] = 0;
  }
  spinor_of<P_F64>(x64).store(s, xv);
  spinor_of<PX>(xhat).store(s, hv);
}

// Mixed solver, deferred x update: ring[npend] = r + beta ring[pcur].
template <int P>
__global__ __launch_bounds__(kBlock) void k_p_update_ring(Geom g, SpinorBuf r, RingBuf ring, const SolverState* st,
                                                          Rhs rb) {
  int k;
  const int b = rhs_split(blockIdx.x, rb, k);
  if (k) {
    const long long off = k * rb.stride;
    st = rhs_shift(st, off);
    r = rhs_shift(r, off);
    ring = rhs_shift(ring, off);
  }
  if (!gate_open(st, G_ITER)) return;
  using R = typename PackedSpinor<P>::Real;
  const int s = b * kBlock + threadIdx.x;
  if (s >= g.V || st->npend >= ring.len) return;   // the latter never with the host's fold cadence
  const R beta = (R)st->beta;
  R rv[24], pv[24];
  spinor_of<P>(r).load(s, rv);
  spinor_of<P>(ring.at(st->pcur)).load(s, pv);
#pragma unroll
  for (int i = 0; i < 24; ++i) pv[i] = fma(beta, pv[i], rv[i]);
  spinor_of<P>(ring.at(st->npend)).store(s, pv);
}

// x(FP64) += sum_{j < npend} alpha_j p_j over the ring, in FP64 arithmetic.
template <int P>
__global__ __launch_bounds__(kBlock) void k_accumulate_ring(Geom g, SpinorBuf x64, RingBuf ring, int gate,
                                                            const SolverState* st, Rhs rb) {
  int k;
  const int b = rhs_split(blockIdx.x, rb, k);
  if (k) {
    const long long off = k * rb.stride;
    st = rhs_shift(st, off);
    x64 = rhs_shift(x64, off);
    ring = rhs_shift(ring, off);
  }
  if (!gate_open(st, gate)) return;
  const int s = b * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int n = st->npend;
  if (n == 0) return;
  double xv[24];
  spinor_of<P_F64>(x64).load(s, xv);
  for (int j = 0; j < n; ++j) {
    typename PackedSpinor<P>::Real pv[24];
    spinor_of<P>(ring.at(j)).load(s, pv);
    const double a = st->alpha_hist[j];
#pragma unroll
    for (int i = 0; i < 24; ++i) xv[i] = fma(a, (double)pv[i], xv[i]);
  }
  spinor_of<P_F64>(x64).store(s, xv);
}

__global__ void k_ring_reset(SolverState* st, Rhs rb) {
  if (threadIdx.x != 0) return;
  st = rhs_shift(st, (long long)blockIdx.x * rb.stride);   // one workgroup per system
  if (!gate_open(st, G_FLUSH)) return;
  st->npend = 0;
}

__global__ void k_gather_states(const SolverState* st, Rhs rb, SolverState* dst) {
  const int k = blockIdx.x;
  if (threadIdx.x != 0 || k >= rb.n) return;
  dst[k] = *rhs_shift(st, (long long)k * rb.stride);
}

__global__ void k_set_ring(SolverState* st, double* alpha_hist, int flush_at, int ring_len) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->alpha_hist = alpha_hist;
  st->flush_at = flush_at;
  st->ring_len = ring_len;
  st->npend = 0;
  st->pcur = 0;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_norm2(Geom g, SpinorBuf v, int gate, int fin, SolverState* st,
                                                  double* partials) {
  if (!gate_open(st, gate)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (s < g.V) {
    typename PackedSpinor<P>::Real a[24];
    spinor_of<P>(v).load(s, a);
#pragma unroll
    for (int i = 0; i < 24; ++i) n2 += (double)a[i] * (double)a[i];
  }
  store_partial(n2, partials);
}

// ------------------------------------------------------------------ force
// G(a, b)_mu(x) = 1/2 sum_spin [ ((1 - g_mu) a(x)) (x) b(x+mu)^* + b(x) (x) ((1 + g_mu) a(x+mu))^* ]
// In half-spinor form: (1 - g) a = [h; -A^+ h] with h = a_up - A a_dn, so
//   sum_spin ((1-g)a)_s (x) b_s^* = h (x) (b_up - A b_dn)^*  (two colour outer products),
// and likewise (1 + g): sum_spin b_s (x) ((1+g)a)_s^* = (b_up + A b_dn) (x) h'^*.

// f += sum_{k=0,1} u[k] (x) conj(v[k]) for half spinors u, v (index (k * 3 + c) * 2),
// each product added into f by its own FMA (four per complex term)
__device__ __forceinline__ void outer_acc(const double u[12], const double v[12], double f[18]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double ur = u[(k * 3 + i) * 2], ui = u[(k * 3 + i) * 2 + 1];
        const double vr = v[(k * 3 + j) * 2], vi = v[(k * 3 + j) * 2 + 1];
        f[(i * 3 + j) * 2] = fma(ur, vr, fma(ui, vi, f[(i * 3 + j) * 2]));
        f[(i * 3 + j) * 2 + 1] = fma(ui, vr, fma(-ur, vi, f[(i * 3 + j) * 2 + 1]));
      }
    }
  }
}

// ---- force kernel: one direction per wavefront. A workgroup owns 64
// consecutive sites (linear order) and stages their records of a and b in LDS
// once, coalesced; wavefront mu then computes G_mu for the 64 sites. Each
// wavefront has a single dependent load (its neighbours) between the staging
// and the store, where a workgroup that walks the four directions in turn has
// four, and the a and b records are read from memory once per workgroup.
constexpr int kForceSites = 64;
constexpr int kForcePad = kForceSites + 1;   // LDS row stride (bank spread)

__device__ __forceinline__ void staged_record(const double2* lds, int field, int site, double v[24]) {
#pragma unroll
  for (int w = 0; w < 12; ++w) {
    const double2 d = lds[(field * 12 + w) * kForcePad + site];
    v[2 * w] = d.x;
    v[2 * w + 1] = d.y;
  }
}

__device__ __forceinline__ int fwd_site(const Geom& g, int s, int mu) {
  int c[4];
  site_coords(g, s, c);
  const int st = g.stride[mu];
  return (c[mu] == g.L[mu] - 1) ? s - st * (g.L[mu] - 1) : s + st;
}

// 24 reals of a record from a generic pointer, word stride st (16-byte words)
__device__ __forceinline__ void load_record(const double2* p, int st, double v[24]) {
#pragma unroll
  for (int w = 0; w < 12; ++w) {
    const double2 d = p[w * st];
    v[2 * w] = d.x;
    v[2 * w + 1] = d.y;
  }
}

// The 64 records src[idx(lane)] of a wavefront into its LDS region buf
// ([word][lane], stride kForcePad), loaded 12 lanes to a record so that each
// load instruction covers about six whole records instead of one word of 64,
// then returned to each lane from LDS.
__device__ __forceinline__ void gather_wave(const double2* __restrict__ src, int idx, int l, double2* buf,
                                            double v[24]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const int e = k * 64 + l;            // element e of the 64 x 12 words
    const int r = e / 12;
    const int w = e - r * 12;
    const int sr = __shfl(idx, r, 64);
    buf[w * kForcePad + r] = src[(size_t)sr * 12 + w];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int w = 0; w < 12; ++w) {
    const double2 d = buf[w * kForcePad + l];
    v[2 * w] = d.x;
    v[2 * w + 1] = d.y;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// G_mu at the 64 sites of the block. x and y: the neighbour's record from the
// staged block when it lies there (one generic load path, LDS or memory); z
// and t: neighbours lie outside the block, gathered cooperatively.
template <int MU>
__device__ __forceinline__ void force_wave(const Geom& g, const double2* lds, double2* wbuf, const CanonSpinor& a,
                                           const CanonSpinor& b, int s0, int n, int l, double f[18]) {
  const int sf = fwd_site(g, s0 + min(l, n - 1), MU);
  const int j = sf - s0;
  const bool in_block = j >= 0 && j < n;
  const double2* nb_a = in_block ? lds + j : a.data + (size_t)sf * 12;
  const double2* nb_b = in_block ? lds + 12 * kForcePad + j : b.data + (size_t)sf * 12;
  const int st = in_block ? kForcePad : 1;
  double v[24], h[12], k[12];
  staged_record(lds, 0, l, v);
  project<MU, -1>(v, h);              // (1 - g) a(x), upper half
  if constexpr (MU >= 2) gather_wave(b.data, sf, l, wbuf, v);
  else load_record(nb_b, st, v);
  project<MU, -1>(v, k);              // matching combination of b(x + mu)
  outer_acc(h, k, f);
  // finish this half before the next record's loads are issued (the
  // compiler would otherwise hold all four records in registers at once)
#pragma unroll
  for (int i = 0; i < 18; ++i) asm volatile("" : "+v"(f[i]) : : "memory");
  staged_record(lds, 1, l, v);
  project<MU, +1>(v, h);              // (1 + g) b(x)
  if constexpr (MU >= 2) gather_wave(a.data, sf, l, wbuf, v);
  else load_record(nb_a, st, v);
  project<MU, +1>(v, k);              // (1 + g) a(x + mu)
  outer_acc(h, k, f);
}

// Workgroup -> block of 64 sites. Workgroups are dealt round-robin to the 8
// XCDs. When an xy-plane is a whole number of blocks and Lz a multiple of 8,
// XCD k takes the z-planes [k Lz/8, (k+1) Lz/8) of every t-plane and walks
// them xy-block fastest, then z, then t: a block's y neighbours are in the
// same XCD's next block, its z neighbours Lx Ly / 64 of its blocks later (on
// the next XCD for the last of its z-planes), its t neighbours Lx Ly Lz / 512
// of its blocks later. In linear order the y neighbours of a block's second
// x-row lay in the next block, on another XCD: each a and b record was fetched
// 1.78 times on 32^3 x 64, against 1.27 in this order. Otherwise blocks run in
// linear order.
__device__ __forceinline__ int force_block(const Geom& g, int b, int zsplit) {
  if (!zsplit) return b;
  const int cp = g.stride[2] / kForceSites;   // blocks per xy-plane
  const int zper = g.L[2] >> 3;
  const int p = b >> 3;
  const int q = p / cp;
  const int z = (b & 7) * zper + q % zper;
  return ((q / zper) * g.L[2] + z) * cp + (p - q * cp);
}

__global__ __launch_bounds__(kBlock) void k_force(Geom g, CanonSpinor a, CanonSpinor b, double coeff,
                                                  int accumulate, int zsplit, double2* __restrict__ F) {
  // rows of kForcePad words: [0, 24) the block's records of a and b
  // ([field][word][site]), [24, 48) the z and t wavefronts' gathers; after the
  // second barrier [0, 36) the link entries ([mu][entry][site])
  __shared__ double2 lds[48 * kForcePad];
  const int s0 = force_block(g, blockIdx.x, zsplit) * kForceSites;
  const int n = min(kForceSites, g.V - s0);
  const int nw = n * 12;
  for (int q = threadIdx.x; q < 2 * nw; q += kBlock) {
    const int fld = q >= nw;
    const int r = q - fld * nw;
    const int site = r / 12;
    lds[(fld * 12 + (r - site * 12)) * kForcePad + site] = (fld ? b.data : a.data)[(size_t)s0 * 12 + r];
  }
  __syncthreads();
  const int mu = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  double f[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) f[i] = 0.0;
  // every lane runs (the gathers need the whole wavefront); lanes past the
  // block's n sites compute a copy of the last site and store nothing
  if (mu == 0) force_wave<0>(g, lds, nullptr, a, b, s0, n, l, f);
  else if (mu == 1) force_wave<1>(g, lds, nullptr, a, b, s0, n, l, f);
  else if (mu == 2) force_wave<2>(g, lds, lds + 24 * kForcePad, a, b, s0, n, l, f);
  else force_wave<3>(g, lds, lds + 36 * kForcePad, a, b, s0, n, l, f);
  __syncthreads();   // every record read: the buffer now takes the link entries
  const double c = 0.5 * coeff;
#pragma unroll
  for (int e = 0; e < 9; ++e) lds[(mu * 9 + e) * kForcePad + l] = make_double2(c * f[2 * e], c * f[2 * e + 1]);
  __syncthreads();
  const int per = n * 9;
  for (int q = threadIdx.x; q < 4 * per; q += kBlock) {
    const int m = q / per;
    const int r = q - m * per;
    const int site = r / 9;
    double2 v = lds[(m * 9 + (r - site * 9)) * kForcePad + site];
    double2* dst = F + ((size_t)m * g.V + s0) * 9 + r;
    // G is written once and read by no later workgroup: streamed past the
    // caches, which keep the records that neighbouring blocks gather
    typedef double v2d __attribute__((ext_vector_type(2)));
    if (accumulate) {
      const v2d o = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(dst));
      v.x += o.x;
      v.y += o.y;
    }
    st_nt(dst, v);
  }
}

__global__ void k_init_state(SolverState* st, double tol, int interval, double delta, double* hist,
                             int hist_len) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  SolverState z{};
  z.stop2 = tol * tol;
  z.interval = interval;
  z.delta2 = delta * delta;
  z.hist = hist;
  z.hist_len = hist_len;
  z.alpha = 0.0;
  z.beta = 0.0;
  *st = z;
}

__global__ void k_set_restart(SolverState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->restart_on_update = 1;
}

__global__ void k_restart(SolverState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->status = 0;
  st->inner_done = 0;
  st->rho = st->rho_true;
}

// ============================================================= launchers

void launch_init_state(SolverState* st, double tol, int interval, double delta, double* hist, int hist_len,
                       hipStream_t s) {
  k_init_state<<<1, 64, 0, s>>>(st, tol, interval, delta, hist, hist_len);
}

void launch_restart(SolverState* st, hipStream_t s) { k_restart<<<1, 64, 0, s>>>(st); }

void launch_set_restart(SolverState* st, hipStream_t s) { k_set_restart<<<1, 64, 0, s>>>(st); }

static inline dim3 grid_of(const Geom& g) { return dim3(g.nblocks); }

void launch_pack_gauge(const Geom& g, const void* U, int prec, void* out, hipStream_t s) {
  const double2* u = static_cast<const double2*>(U);
  switch (prec) {
    case P_F64: k_pack_gauge<P_F64><<<grid_of(g), kBlock, 0, s>>>(g, u, out); break;
    case P_F32: k_pack_gauge<P_F32><<<grid_of(g), kBlock, 0, s>>>(g, u, out); break;
    case P_I8: k_pack_gauge<P_I8><<<grid_of(g), kBlock, 0, s>>>(g, u, out); break;
    case P_BF16: k_pack_gauge<P_BF16><<<grid_of(g), kBlock, 0, s>>>(g, u, out); break;
    default: k_pack_gauge<P_F16><<<grid_of(g), kBlock, 0, s>>>(g, u, out); break;
  }
}

template <typename IO>
static void pack_spinor_io(const Geom& g, const IO* in, SpinorBuf out, hipStream_t s) {
  switch (out.prec) {
    case P_F64: k_pack_spinor<P_F64, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
    case P_F32: k_pack_spinor<P_F32, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
    case P_I8: k_pack_spinor<P_I8, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
    case P_BF16: k_pack_spinor<P_BF16, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
    default: k_pack_spinor<P_F16, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
  }
}

void launch_pack_spinor(const Geom& g, const void* in, int io_c64, SpinorBuf out, hipStream_t s) {
  if (io_c64) pack_spinor_io(g, static_cast<const float2*>(in), out, s);
  else pack_spinor_io(g, static_cast<const double2*>(in), out, s);
}

template <typename IO>
static void unpack_spinor_io(const Geom& g, SpinorBuf in, IO* out, hipStream_t s) {
  switch (in.prec) {
    case P_F64: k_unpack_spinor<P_F64, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
    case P_F32: k_unpack_spinor<P_F32, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
    case P_I8: k_unpack_spinor<P_I8, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
    case P_BF16: k_unpack_spinor<P_BF16, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
    default: k_unpack_spinor<P_F16, IO><<<grid_of(g), kBlock, 0, s>>>(g, in, out); break;
  }
}

void launch_unpack_spinor(const Geom& g, SpinorBuf in, void* out, int io_c64, hipStream_t s) {
  if (io_c64) unpack_spinor_io(g, in, static_cast<float2*>(out), s);
  else unpack_spinor_io(g, in, static_cast<double2*>(out), s);
}

template <int PA>
static void convert_from(const Geom& g, SpinorBuf in, SpinorBuf out, int gate, SolverState* st, hipStream_t s) {
  switch (out.prec) {
    case P_F64: k_convert<PA, P_F64><<<grid_of(g), kBlock, 0, s>>>(g, in, out, gate, st); break;
    case P_F32: k_convert<PA, P_F32><<<grid_of(g), kBlock, 0, s>>>(g, in, out, gate, st); break;
    case P_I8: k_convert<PA, P_I8><<<grid_of(g), kBlock, 0, s>>>(g, in, out, gate, st); break;
    case P_BF16: k_convert<PA, P_BF16><<<grid_of(g), kBlock, 0, s>>>(g, in, out, gate, st); break;
    default: k_convert<PA, P_F16><<<grid_of(g), kBlock, 0, s>>>(g, in, out, gate, st); break;
  }
}

void launch_convert(const Geom& g, SpinorBuf in, SpinorBuf out, int gate, SolverState* st, hipStream_t s) {
  switch (in.prec) {
    case P_F64: convert_from<P_F64>(g, in, out, gate, st, s); break;
    case P_F32: convert_from<P_F32>(g, in, out, gate, st, s); break;
    case P_I8: convert_from<P_I8>(g, in, out, gate, st, s); break;
    case P_BF16: convert_from<P_BF16>(g, in, out, gate, st, s); break;
    default: convert_from<P_F16>(g, in, out, gate, st, s); break;
  }
}

void launch_zero(const Geom& g, SpinorBuf v, int gate, SolverState* st, hipStream_t s) {
  switch (v.prec) {
    case P_F64: k_zero<P_F64><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, st); break;
    case P_F32: k_zero<P_F32><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, st); break;
    case P_I8: k_zero<P_I8><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, st); break;
    case P_BF16: k_zero<P_BF16><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, st); break;
    default: k_zero<P_F16><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, st); break;
  }
}

void launch_wilson_canonical(const Geom& g, const void* U, const void* in, void* out, double mass, int dagger,
                             hipStream_t s) {
  CanonGauge u{static_cast<const double2*>(U), (size_t)g.V};
  CanonSpinor i{const_cast<double2*>(static_cast<const double2*>(in))};
  CanonSpinor o{static_cast<double2*>(out)};
  if (dagger) k_wilson_canonical<true><<<grid_of(g), kBlock, 0, s>>>(g, u, i, o, mass + 4.0);
  else k_wilson_canonical<false><<<grid_of(g), kBlock, 0, s>>>(g, u, i, o, mass + 4.0);
}

// Launch on the solver grid. With an event pair the events are attached to
// this dispatch (hipExtLaunchKernel), so they time the kernel alone, as the
// profiler's kernel trace does.
template <typename... KArgs, typename... Args>
static void launch_n(void (*kernel)(KArgs...), const Geom& g, int n, hipStream_t s, const EventPair* ev,
                     Args... args) {
  const dim3 grid(g.nblocks * n);
  if (ev)
    hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, s, ev->begin, ev->end, 0, static_cast<KArgs>(args)...);
  else
    kernel<<<grid, kBlock, 0, s>>>(static_cast<KArgs>(args)...);
}
template <typename... KArgs, typename... Args>
static void launch(void (*kernel)(KArgs...), const Geom& g, hipStream_t s, const EventPair* ev, Args... args) {
  launch_n(kernel, g, 1, s, ev, args...);
}

template <int P>
static void wilson_packed_p(const Geom& g, const void* U, SpinorBuf in, SpinorBuf out, double mass, int dagger,
                            int gate, int fin, SolverState* st, double* partials, hipStream_t s,
                            const EventPair* ev, int rows2, RingBuf ring, Rhs rb) {
  const double d = mass + 4.0;
  bool done = false;
  if constexpr (P == P_BF16 || P == P_F16 || P == P_I8) {
    if (g.tiled) {
      if (rows2 && dagger) launch_n(k_wilson_tiled<P, true, true>, g, rb.n, s, ev, g, U, in, out, d, gate, fin, st, partials, ring, rb);
      else if (rows2) launch_n(k_wilson_tiled<P, true, false>, g, rb.n, s, ev, g, U, in, out, d, gate, fin, st, partials, ring, rb);
      else if (dagger) launch_n(k_wilson_tiled<P, false, true>, g, rb.n, s, ev, g, U, in, out, d, gate, fin, st, partials, ring, rb);
      else launch_n(k_wilson_tiled<P, false, false>, g, rb.n, s, ev, g, U, in, out, d, gate, fin, st, partials, ring, rb);
      done = true;
    }
  }
  if constexpr (P == P_F64 || P == P_F32) {
    if (g.tiled) {
      if (dagger) launch_n(k_wilson_packed<P, true, true>, g, rb.n, s, ev, g, U, in, out, d, gate, fin, st, partials, ring, rb);
      else launch_n(k_wilson_packed<P, false, true>, g, rb.n, s, ev, g, U, in, out, d, gate, fin, st, partials, ring, rb);
      done = true;
    }
  }
  if (!done) {
    if (dagger) launch_n(k_wilson_packed<P, true, false>, g, rb.n, s, ev, g, U, in, out, d, gate, fin, st, partials, ring, rb);
    else launch_n(k_wilson_packed<P, false, false>, g, rb.n, s, ev, g, U, in, out, d, gate, fin, st, partials, ring, rb);
  }
  if (fin != F_NONE) launch_finalize(g, partials, st, fin, gate, s, rb);
}

void launch_wilson_packed(const Geom& g, int prec, const void* U, SpinorBuf in, SpinorBuf out, double mass,
                          int dagger, int gate, int fin, SolverState* st, double* partials, hipStream_t s,
                          const EventPair* ev, int rows2, const RingBuf* ring, Rhs rb) {
  RingBuf rg{};
  if (ring) rg = *ring;
  switch (prec) {
    case P_F64: wilson_packed_p<P_F64>(g, U, in, out, mass, dagger, gate, fin, st, partials, s, ev, 0, rg, rb); break;
    case P_F32: wilson_packed_p<P_F32>(g, U, in, out, mass, dagger, gate, fin, st, partials, s, ev, 0, rg, rb); break;
    case P_I8: wilson_packed_p<P_I8>(g, U, in, out, mass, dagger, gate, fin, st, partials, s, ev, rows2, rg, rb); break;
    case P_BF16: wilson_packed_p<P_BF16>(g, U, in, out, mass, dagger, gate, fin, st, partials, s, ev, rows2, rg, rb); break;
    default: wilson_packed_p<P_F16>(g, U, in, out, mass, dagger, gate, fin, st, partials, s, ev, rows2, rg, rb); break;
  }
}

void launch_pack_gauge_rows2(const Geom& g, const void* U, int prec, void* out, hipStream_t s) {
  const double2* u = static_cast<const double2*>(U);
  if (prec == P_BF16) k_pack_gauge_rows2<P_BF16><<<grid_of(g), kBlock, 0, s>>>(g, u, static_cast<uint32_t*>(out));
  else if (prec == P_I8) k_pack_gauge_rows2<P_I8><<<grid_of(g), kBlock, 0, s>>>(g, u, static_cast<uint32_t*>(out));
  else k_pack_gauge_rows2<P_F16><<<grid_of(g), kBlock, 0, s>>>(g, u, static_cast<uint32_t*>(out));
}

void launch_su3_check(const Geom& g, const void* U, SolverState* st, double* partials, hipStream_t s) {
  k_su3_check<<<grid_of(g), kBlock, 0, s>>>(g, static_cast<const double2*>(U), partials);
  launch_finalize(g, partials, st, F_SU3MAX, G_ALWAYS, s);
}

void launch_cg_update(const Geom& g, int prec, const void* U, SpinorBuf t, SpinorBuf r, SpinorBuf p, SpinorBuf x,
                      double mass, SolverState* st, double* partials, hipStream_t s, const EventPair* ev, int rows2) {
  const double diag = mass + 4.0;
  switch (prec) {
    case P_F64:
      if (g.tiled) launch(k_cg_update<P_F64, P_F64, true, true>, g, s, ev, g, U, t, r, p, x, diag, st, partials);
      else launch(k_cg_update<P_F64, P_F64, false, true>, g, s, ev, g, U, t, r, p, x, diag, st, partials);
      break;
    case P_F32:
      if (g.tiled) launch(k_cg_update<P_F32, P_F32, true, true>, g, s, ev, g, U, t, r, p, x, diag, st, partials);
      else launch(k_cg_update<P_F32, P_F32, false, true>, g, s, ev, g, U, t, r, p, x, diag, st, partials);
      break;
    default:   // the narrow storage formats use launch_r_update
      break;
  }
  launch_finalize(g, partials, st, F_BETA, G_ITER, s);
}

// r update without the x and p terms (the mixed solver's deferred x update).
template <int P>
static void r_update_p(const Geom& g, const void* U, SpinorBuf t, SpinorBuf r, double diag, SolverState* st,
                       double* partials, hipStream_t s, const EventPair* ev, int rows2, Rhs rb) {
  const SpinorBuf none{nullptr, nullptr, P};
  if constexpr (P == P_BF16 || P == P_F16 || P == P_I8) {
    if (g.tiled) {
      if (rows2) launch_n(k_cg_update_tiled<P, true>, g, rb.n, s, ev, g, U, t, r, diag, st, partials, rb);
      else launch_n(k_cg_update_tiled<P, false>, g, rb.n, s, ev, g, U, t, r, diag, st, partials, rb);
      return;
    }
    launch(k_cg_update<P, P_F32, false, false>, g, s, ev, g, U, t, r, none, none, diag, st, partials);
  } else {
    if (g.tiled) launch(k_cg_update<P, P, true, false>, g, s, ev, g, U, t, r, none, none, diag, st, partials);
    else launch(k_cg_update<P, P, false, false>, g, s, ev, g, U, t, r, none, none, diag, st, partials);
  }
}

void launch_r_update(const Geom& g, int prec, const void* U, SpinorBuf t, SpinorBuf r, double mass, SolverState* st,
                     double* partials, hipStream_t s, const EventPair* ev, int rows2, Rhs rb) {
  const double diag = mass + 4.0;
  switch (prec) {
    case P_F64: r_update_p<P_F64>(g, U, t, r, diag, st, partials, s, ev, 0, rb); break;
    case P_F32: r_update_p<P_F32>(g, U, t, r, diag, st, partials, s, ev, 0, rb); break;
    case P_I8: r_update_p<P_I8>(g, U, t, r, diag, st, partials, s, ev, rows2, rb); break;
    case P_BF16: r_update_p<P_BF16>(g, U, t, r, diag, st, partials, s, ev, rows2, rb); break;
    default: r_update_p<P_F16>(g, U, t, r, diag, st, partials, s, ev, rows2, rb); break;
  }
  launch_finalize(g, partials, st, F_BETA, G_ITER, s, rb);
}

void launch_p_update_ring(const Geom& g, SpinorBuf r, const RingBuf& ring, SolverState* st, hipStream_t s,
                          const EventPair* ev, Rhs rb) {
  const SolverState* cst = st;
  switch (ring.prec) {
    case P_F64: launch_n(k_p_update_ring<P_F64>, g, rb.n, s, ev, g, r, ring, cst, rb); break;
    case P_F32: launch_n(k_p_update_ring<P_F32>, g, rb.n, s, ev, g, r, ring, cst, rb); break;
    case P_I8: launch_n(k_p_update_ring<P_I8>, g, rb.n, s, ev, g, r, ring, cst, rb); break;
    case P_BF16: launch_n(k_p_update_ring<P_BF16>, g, rb.n, s, ev, g, r, ring, cst, rb); break;
    default: launch_n(k_p_update_ring<P_F16>, g, rb.n, s, ev, g, r, ring, cst, rb); break;
  }
}

void launch_accumulate_ring(const Geom& g, SpinorBuf x64, const RingBuf& ring, int gate, SolverState* st,
                            hipStream_t s, Rhs rb) {
  const SolverState* cst = st;
  switch (ring.prec) {
    case P_F64: launch_n(k_accumulate_ring<P_F64>, g, rb.n, s, nullptr, g, x64, ring, gate, cst, rb); break;
    case P_F32: launch_n(k_accumulate_ring<P_F32>, g, rb.n, s, nullptr, g, x64, ring, gate, cst, rb); break;
    case P_I8: launch_n(k_accumulate_ring<P_I8>, g, rb.n, s, nullptr, g, x64, ring, gate, cst, rb); break;
    case P_BF16: launch_n(k_accumulate_ring<P_BF16>, g, rb.n, s, nullptr, g, x64, ring, gate, cst, rb); break;
    default: launch_n(k_accumulate_ring<P_F16>, g, rb.n, s, nullptr, g, x64, ring, gate, cst, rb); break;
  }
}

void launch_ring_reset(SolverState* st, hipStream_t s, Rhs rb) { k_ring_reset<<<rb.n, 64, 0, s>>>(st, rb); }

void launch_gather_states(const SolverState* st, Rhs rb, SolverState* dst, hipStream_t s) {
  k_gather_states<<<rb.n, 64, 0, s>>>(st, rb, dst);
}

void launch_set_ring(SolverState* st, double* alpha_hist, int flush_at, int ring_len, hipStream_t s) {
  k_set_ring<<<1, 64, 0, s>>>(st, alpha_hist, flush_at, ring_len);
}

void launch_residual(const Geom& g, const void* U64, SpinorBuf t64, SpinorBuf b64, SpinorBuf out, double mass,
                     int gate, int fin, SolverState* st, double* partials, hipStream_t s, Rhs rb) {
  const double diag = mass + 4.0;
  if (g.tiled) {
    switch (out.prec) {
      case P_F64: launch_n(k_residual<P_F64, true>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
      case P_F32: launch_n(k_residual<P_F32, true>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
      case P_I8: launch_n(k_residual<P_I8, true>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
      case P_BF16: launch_n(k_residual<P_BF16, true>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
      default: launch_n(k_residual<P_F16, true>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
    }
  } else {
    switch (out.prec) {
      case P_F64: launch_n(k_residual<P_F64, false>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
      case P_F32: launch_n(k_residual<P_F32, false>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
      case P_I8: launch_n(k_residual<P_I8, false>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
      case P_BF16: launch_n(k_residual<P_BF16, false>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
      default: launch_n(k_residual<P_F16, false>, g, rb.n, s, nullptr, g, U64, t64, b64, out, diag, gate, fin, st, partials, rb); break;
    }
  }
  launch_finalize(g, partials, st, fin, gate, s, rb);
}

void launch_p_update(const Geom& g, SpinorBuf r, SpinorBuf p, SolverState* st, hipStream_t s, const EventPair* ev) {
  const SolverState* cst = st;
  switch (p.prec) {
    case P_F64: launch(k_p_update<P_F64>, g, s, ev, g, r, p, cst); break;
    case P_F32: launch(k_p_update<P_F32>, g, s, ev, g, r, p, cst); break;
    case P_I8: launch(k_p_update<P_I8>, g, s, ev, g, r, p, cst); break;
    case P_BF16: launch(k_p_update<P_BF16>, g, s, ev, g, r, p, cst); break;
    default: launch(k_p_update<P_F16>, g, s, ev, g, r, p, cst); break;
  }
}

void launch_accumulate(const Geom& g, SpinorBuf x64, SpinorBuf xhat, int gate, SolverState* st, hipStream_t s) {
  if (xhat.prec == P_F64) k_accumulate<P_F64><<<grid_of(g), kBlock, 0, s>>>(g, x64, xhat, gate, st);
  else k_accumulate<P_F32><<<grid_of(g), kBlock, 0, s>>>(g, x64, xhat, gate, st);
}

void launch_norm2(const Geom& g, SpinorBuf v, int gate, int fin, SolverState* st, double* partials, hipStream_t s) {
  switch (v.prec) {
    case P_F64: k_norm2<P_F64><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, fin, st, partials); break;
    case P_F32: k_norm2<P_F32><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, fin, st, partials); break;
    case P_I8: k_norm2<P_I8><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, fin, st, partials); break;
    case P_BF16: k_norm2<P_BF16><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, fin, st, partials); break;
    default: k_norm2<P_F16><<<grid_of(g), kBlock, 0, s>>>(g, v, gate, fin, st, partials); break;
  }
  launch_finalize(g, partials, st, fin, gate, s);
}

void launch_force(const Geom& g, const void* a, const void* b, double coeff, int accumulate, void* F, hipStream_t s) {
  CanonSpinor ca{const_cast<double2*>(static_cast<const double2*>(a))};
  CanonSpinor cb{const_cast<double2*>(static_cast<const double2*>(b))};
  const int zsplit = (g.stride[2] % kForceSites == 0) && (g.L[2] % 8 == 0);
  k_force<<<(unsigned)((g.V + kForceSites - 1) / kForceSites), kBlock, 0, s>>>(g, ca, cb, coeff, accumulate, zsplit,
                                                                               static_cast<double2*>(F));
}

}  // namespace wd
