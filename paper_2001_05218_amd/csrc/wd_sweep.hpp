// Wilson stencil for 16-bit fields as a sweep along t (2.5D blocking).
//
// The paper streams stencil inputs through on-chip cyclic buffers so that a
// datum crosses the memory interface once and is reused by the neighbouring
// stencils (Sec. 2). This kernel is that idea for gfx950:
//
// * A workgroup owns an 8x8x4 spatial block (2x2 tiles in x, y; wavefront w
//   owns one 4x4x4 cube) and sweeps it through a chunk of time slices.
// * The t-direction needs no halo: each thread keeps its own column's
//   spinors psi(x, t), psi(x, t+1) (and the incoming psi(x, t+2)) in
//   registers, and carries the backward-t hop U_t(x, t-1)^+ P psi(x, t-1)
//   computed one step earlier.
// * Spatial neighbours come from a two-plane ring in LDS: while step t reads
//   plane t (256 interior sites + the 256 sites of the six spatial faces), the
//   loads for plane t + 1 are in flight and land in the other plane.
// * The grid is sized so that every workgroup is resident at once and each
//   XCD holds one chunk of time slices over a compact spatial region; the
//   workgroups sweep in step, so a face one workgroup reads is an interior
//   another workgroup on the same XCD loads in the same step (an L2 hit).
//
// Requires the tiled order with an even number of tiles in x and y.
#pragma once

#include "wd_tiled.hpp"

namespace wd {

constexpr int kSweepSlots = 512;   // 256 interior + 256 face sites per plane

template <int P>
struct SweepPlane {
  uint4 w[3][kSweepSlots];
  float scale[kSweepSlots];
};

// Packed (tiled-order) index of lattice site (x, y, z, t), coordinates in range.
__device__ __forceinline__ int tiled_index(const Geom& g, int x, int y, int z, int t) {
  const int tile = (x >> 2) + g.tstride[1] * (y >> 2) + g.tstride[2] * (z >> 2) + g.tstride[3] * (t >> 2);
  return tile * kTileSites + (x & 3) + 4 * (y & 3) + 16 * (z & 3) + 64 * (t & 3);
}

__device__ __forceinline__ int wrap(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

// Sweep geometry of one workgroup: block origin (sites) and time chunk.
struct SweepPos {
  int x0, y0, z0;   // block origin
  int t0, nt;       // first time slice and number of slices
};

// Workgroup -> (time chunk, spatial block). Workgroups are dealt to the 8 XCDs
// round-robin; xcd_tile turns that into contiguous ranges per XCD, and within
// the range spatial blocks run x-fastest, so an XCD holds whole chunks of a
// compact spatial region.
__device__ __forceinline__ SweepPos sweep_pos(const Geom& g, int chunk_len) {
  const int nbx = g.nt[0] / 2, nby = g.nt[1] / 2, nbz = g.nt[2];
  const int nsb = nbx * nby * nbz;
  const int m = xcd_tile(blockIdx.x, gridDim.x);
  const int chunk = m / nsb;
  int sb = m - chunk * nsb;
  SweepPos p;
  const int bx = sb % nbx;
  sb /= nbx;
  const int by = sb % nby;
  const int bz = sb / nby;
  p.x0 = 8 * bx;
  p.y0 = 8 * by;
  p.z0 = 4 * bz;
  p.t0 = chunk * chunk_len;
  p.nt = chunk_len;
  return p;
}

// Block-local coordinates of this thread: wavefront w = (w & 1, w >> 1) tile in
// (x, y); lane = lx + 4 ly + 16 lz within the 4x4x4 cube.
struct SweepLocal {
  int i, j, k;      // 0..7, 0..7, 0..3
  int slot;         // interior slot i + 8 j + 64 k
};

__device__ __forceinline__ SweepLocal sweep_local() {
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  SweepLocal s;
  s.i = 4 * (w & 1) + (l & 3);
  s.j = 4 * (w >> 1) + ((l >> 2) & 3);
  s.k = l >> 4;
  s.slot = s.i + 8 * s.j + 64 * s.k;
  return s;
}

// Lattice coordinates of face site h (0..255) of a block: order x- x+ y- y+ (32
// each, index a + 8 b over the two other coordinates), then z- z+ (64 each).
__device__ __forceinline__ void face_site(const SweepPos& p, int h, const Geom& g, int& x, int& y, int& z) {
  if (h < 64) {            // x faces: a = j (0..7), b = k (0..3)
    const int side = h >> 5, r = h & 31;
    x = wrap(side ? p.x0 + 8 : p.x0 - 1, g.L[0]);
    y = p.y0 + (r & 7);
    z = p.z0 + (r >> 3);
  } else if (h < 128) {    // y faces: a = i, b = k
    const int side = (h - 64) >> 5, r = (h - 64) & 31;
    x = p.x0 + (r & 7);
    y = wrap(side ? p.y0 + 8 : p.y0 - 1, g.L[1]);
    z = p.z0 + (r >> 3);
  } else {                 // z faces: a = i, b = j
    const int side = (h - 128) >> 6, r = (h - 128) & 63;
    x = p.x0 + (r & 7);
    y = p.y0 + (r >> 3);
    z = wrap(side ? p.z0 + 4 : p.z0 - 1, g.L[2]);
  }
}

// LDS slot of the spatial neighbour of (i, j, k) in direction mu (0..2), step +-1.
template <int MU, int STEP>
__device__ __forceinline__ int nbr_slot(const SweepLocal& s) {
  if constexpr (MU == 0) {
    const bool in = STEP > 0 ? s.i < 7 : s.i > 0;
    return in ? s.slot + STEP : 256 + (STEP > 0 ? 32 : 0) + s.j + 8 * s.k;
  } else if constexpr (MU == 1) {
    const bool in = STEP > 0 ? s.j < 7 : s.j > 0;
    return in ? s.slot + 8 * STEP : 256 + 64 + (STEP > 0 ? 32 : 0) + s.i + 8 * s.k;
  } else {
    const bool in = STEP > 0 ? s.k < 3 : s.k > 0;
    return in ? s.slot + 64 * STEP : 256 + 128 + (STEP > 0 ? 64 : 0) + s.i + 8 * s.j;
  }
}

// Raw 16-bit spinor of one site (3 words + scale).
struct RawSpinor {
  uint4 d[3];
  float sc;
};

template <int P>
__device__ __forceinline__ RawSpinor load_raw(const SpinorBuf& in, int s) {
  const uint4* src = static_cast<const uint4*>(in.data);
  RawSpinor r;
#pragma unroll
  for (int w = 0; w < 3; ++w) r.d[w] = src[word_index(s, 3, w)];
  r.sc = (P == P_F16) ? in.scale[s] : 1.0f;
  return r;
}

template <int P>
__device__ __forceinline__ void put_plane(SweepPlane<P>& pl, int slot, const RawSpinor& r) {
#pragma unroll
  for (int w = 0; w < 3; ++w) pl.w[w][slot] = r.d[w];
  if constexpr (P == P_F16) pl.scale[slot] = r.sc;
}

template <int P>
__device__ __forceinline__ void plane_spinor(const SweepPlane<P>& pl, int slot, float v[24]) {
  uint4 d[3];
#pragma unroll
  for (int w = 0; w < 3; ++w) d[w] = pl.w[w][slot];
  PackedSpinor<P>::unpack(d, P == P_F16 ? pl.scale[slot] : 1.0f, v);
}

template <int P>
__device__ __forceinline__ void raw_spinor(const RawSpinor& r, float v[24]) {
  PackedSpinor<P>::unpack(r.d, r.sc, v);
}

template <int P, bool C12>
__device__ __forceinline__ void load_link_raw(const uint32_t* U, int s, int mu, uint32_t raw[9]) {
  constexpr int NE = LinkFormat<C12>::entries;
  constexpr int NW = LinkFormat<C12>::words;
#pragma unroll
  for (int e = 0; e < NE; ++e) raw[e] = U[word_index(s, NW, mu * NE + e)];
}

// One spatial hop pair (forward and backward in direction MU) from the plane.
template <int P, bool C12, int MU, bool DAG>
__device__ __forceinline__ void sweep_hop(const SweepPlane<P>& pl, const SweepLocal& sl, const uint32_t lf[9],
                                          const uint32_t lb[9], float acc[24]) {
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  float psi[24], h[12], w[12], u[18];
  plane_spinor<P>(pl, nbr_slot<MU, +1>(sl), psi);
  link_from<P, C12>(lf, u);
  project<MU, SF>(psi, h);
  su3_mul_half<false>(u, h, w);
  reconstruct_add<MU, SF>(acc, w);
  plane_spinor<P>(pl, nbr_slot<MU, -1>(sl), psi);
  link_from<P, C12>(lb, u);
  project<MU, SB>(psi, h);
  su3_mul_half<true>(u, h, w);
  reconstruct_add<MU, SB>(acc, w);
  __builtin_amdgcn_sched_barrier(0);
}

// Backward t-hop contribution of site (x, t) to (x, t + 1): U_t(x,t)^+ (1 + S g_t) psi(x,t)
// as the projected half spinor (the reconstruction happens at the next step).
template <int P, bool C12, bool DAG>
__device__ __forceinline__ void back_t_half(const uint32_t lt[9], const float psi[24], float hb[12]) {
  constexpr int SB = DAG ? -1 : +1;
  float h[12], u[18];
  link_from<P, C12>(lt, u);
  project<3, SB>(psi, h);
  su3_mul_half<true>(u, h, hb);
}

// The per-site result (D or D^+ psi at site s, time t) goes to `epi(s, t, o)`.
// `partial` accumulates whatever the epilogue returns (a norm), reduced per
// workgroup by the caller.
template <int P, bool C12, bool DAG, class Epi>
__device__ __forceinline__ double wilson_sweep(const Geom& g, const void* Uv, const SpinorBuf& in, float diag,
                                               int chunk_len, SweepPlane<P>* planes, Epi& epi) {
  const uint32_t* U = static_cast<const uint32_t*>(Uv);
  const SweepPos pos = sweep_pos(g, chunk_len);
  const SweepLocal sl = sweep_local();
  const int x = pos.x0 + sl.i, y = pos.y0 + sl.j, z = pos.z0 + sl.k;
  const int Lt = g.L[3];
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  double partial = 0.0;

  // ---- prime: plane t0, own psi(t0), psi(t0+1), carried hop from t0 - 1
  int t = pos.t0;
  const int tm = wrap(t - 1, Lt);
  float hb[12];
  {
    uint32_t lt_prev[9];
    load_link_raw<P, C12>(U, tiled_index(g, x, y, z, tm), 3, lt_prev);
    const RawSpinor prev = load_raw<P>(in, tiled_index(g, x, y, z, tm));
    float psi[24];
    raw_spinor<P>(prev, psi);
    back_t_half<P, C12, DAG>(lt_prev, psi, hb);
  }
  RawSpinor cur = load_raw<P>(in, tiled_index(g, x, y, z, t));
  RawSpinor nxt = load_raw<P>(in, tiled_index(g, x, y, z, wrap(t + 1, Lt)));
  {
    int fx, fy, fz;
    face_site(pos, threadIdx.x, g, fx, fy, fz);
    put_plane<P>(planes[0], 256 + threadIdx.x, load_raw<P>(in, tiled_index(g, fx, fy, fz, t)));
    put_plane<P>(planes[0], sl.slot, cur);
  }
  __syncthreads();

  for (int step = 0; step < pos.nt; ++step) {
    const int t1 = wrap(t + 1, Lt), t2 = wrap(t + 2, Lt);
    SweepPlane<P>& pl = planes[step & 1];
    SweepPlane<P>& pn = planes[(step + 1) & 1];
    const int s = tiled_index(g, x, y, z, t);
    // next plane's loads (used at the end of this step / the next step)
    const RawSpinor nn = load_raw<P>(in, tiled_index(g, x, y, z, t2));
    int fx, fy, fz;
    face_site(pos, threadIdx.x, g, fx, fy, fz);
    const RawSpinor face = load_raw<P>(in, tiled_index(g, fx, fy, fz, t1));
    // this step's links: own U_mu(x, t) and backward spatial U_mu(x - mu, t)
    uint32_t lf[4][9], lb[3][9];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) load_link_raw<P, C12>(U, s, mu, lf[mu]);
    load_link_raw<P, C12>(U, tiled_index(g, wrap(x - 1, g.L[0]), y, z, t), 0, lb[0]);
    load_link_raw<P, C12>(U, tiled_index(g, x, wrap(y - 1, g.L[1]), z, t), 1, lb[1]);
    load_link_raw<P, C12>(U, tiled_index(g, x, y, wrap(z - 1, g.L[2]), t), 2, lb[2]);

    float acc[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) acc[i] = 0.f;
    sweep_hop<P, C12, 0, DAG>(pl, sl, lf[0], lb[0], acc);
    sweep_hop<P, C12, 1, DAG>(pl, sl, lf[1], lb[1], acc);
    sweep_hop<P, C12, 2, DAG>(pl, sl, lf[2], lb[2], acc);
    {
      // forward t: U_t(x, t) (1 + SF g_t) psi(x, t + 1)
      float psi[24], h[12], w[12], u[18];
      raw_spinor<P>(nxt, psi);
      link_from<P, C12>(lf[3], u);
      project<3, SF>(psi, h);
      su3_mul_half<false>(u, h, w);
      reconstruct_add<3, SF>(acc, w);
      // backward t, carried from the previous step
      reconstruct_add<3, SB>(acc, hb);
    }
    float c[24];
    raw_spinor<P>(cur, c);
    back_t_half<P, C12, DAG>(lf[3], c, hb);   // for step t + 1
    float o[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) o[i] = fmaf(diag, c[i], -0.5f * acc[i]);
    partial += epi(s, o);

    // plane t + 1 into the other buffer (its last readers passed the previous barrier)
    put_plane<P>(pn, sl.slot, nxt);
    put_plane<P>(pn, 256 + threadIdx.x, face);
    __syncthreads();
    cur = nxt;
    nxt = nn;
    t = t1;
  }
  return partial;
}

// Time-chunk length for a lattice: about two workgroups per CU on 256 CUs,
// chunk lengths dividing Lt, at least 4 slices.
inline int sweep_chunk(const Geom& g) {
  const int nsb = (g.nt[0] / 2) * (g.nt[1] / 2) * g.nt[2];
  const int Lt = g.L[3];
  int best = Lt;
  for (int c = Lt; c >= 4; --c) {
    if (Lt % c) continue;
    best = c;
    if ((long long)nsb * (Lt / c) >= 512) break;
  }
  return best;
}

inline bool sweep_ok(const Geom& g) { return g.tiled && (g.nt[0] % 2 == 0) && (g.nt[1] % 2 == 0); }

}  // namespace wd
