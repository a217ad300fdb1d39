// LDS-staged Wilson stencil for 16-bit fields in the tiled site order.
//
// The paper keeps the inputs of neighbouring stencils on chip in cyclic
// buffers so that each datum crosses the memory interface once (Sec. 2).
// On gfx950 the caches cannot be trusted with that reuse: at full bandwidth
// an XCD's 4 MB L2 turns over in a few microseconds, less than the time a
// wavefront spends walking its eight hops, and measured L2 hit rates of the
// cache-only stencil are ~10 %. Here a workgroup owns one 4^4 tile and
//   1. issues, all at once, the loads of its 256 spinors plus the 8 halo
//      faces (64 sites each, read from the neighbouring tiles) into LDS, and
//      of its sites' 8 links (4 own, 4 backward) into registers;
//   2. after one barrier evaluates all 8 hops from LDS and registers.
// A workgroup's loads are thus in flight together; the faces it reads are the
// interiors of tiles that neighbouring workgroups of the same XCD stage at the
// same moment, so they are served by that XCD's L2.
//
// Slot map of the LDS staging area: 0..255 interior (slot = local index),
// 256 + (2 mu) * 64 + f: the +mu face, 256 + (2 mu + 1) * 64 + f: the -mu face,
// f = the local index with its 2 bits of coordinate mu removed.
#pragma once

#include "wd_dslash.hpp"

namespace wd {

constexpr int kTileSites = 256;
constexpr int kTileSlots = 768;

__device__ __forceinline__ int face_pos(int l, int mu) {
  const int lo = l & ((1 << (2 * mu)) - 1);
  const int hi = l >> (2 * mu + 2);
  return lo | (hi << (2 * mu));
}
__device__ __forceinline__ int face_insert(int f, int mu, int v) {
  const int lo = f & ((1 << (2 * mu)) - 1);
  const int hi = f >> (2 * mu);
  return lo | (v << (2 * mu)) | (hi << (2 * mu + 2));
}

template <int P>
struct TileLds {
  typename SpinorWord<P>::T w[3][kTileSlots];
  float scale[kTileSlots];
};

// Links are stored either as all 9 entries (18 reals) or, for SU(3) fields,
// as rows 0 and 1 only (12 reals; row 2 = conj(row0 x row1) is rebuilt on use).
template <bool C12> struct LinkFormat {
  static constexpr int entries = C12 ? 6 : 9;    // stored entries per link
  static constexpr int words = 4 * entries;      // per site, 4 directions
};

// Stage the tile's spinors and halo faces; prefetch the 8 links of site s.
template <int P, bool C12>
__device__ __forceinline__ void tile_stage(const Geom& g, int T, const void* Uv, const SpinorBuf& in, TileLds<P>& lds,
                                           uint32_t lk[8][9]) {
  constexpr int NE = LinkFormat<C12>::entries;
  constexpr int NW = LinkFormat<C12>::words;
  const int l = threadIdx.x;
  const int s = T * kTileSites + l;
  const uint32_t* U = static_cast<const uint32_t*>(Uv);
  const typename SpinorWord<P>::T* src = static_cast<const typename SpinorWord<P>::T*>(in.data);
  const Nbrs nb = neighbours(g, s);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
#pragma unroll
    for (int e = 0; e < NE; ++e) lk[mu][e] = U[word_index(s, NW, mu * NE + e)];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
#pragma unroll
    for (int e = 0; e < NE; ++e) lk[4 + mu][e] = U[word_index(nb.bwd[mu], NW, mu * NE + e)];
#pragma unroll
  for (int w = 0; w < 3; ++w) lds.w[w][l] = src[word_index(s, 3, w)];
  if constexpr (kScaled<P>) lds.scale[l] = in.scale[s];
  // halo: wavefront mu stages the two mu faces
  const int mu = l >> 6;
  const int f = l & 63;
  int b[4];
  tile_coords(g, (uint32_t)T, b);
  const int sp = tile_step(g, T, b, mu, +1) * kTileSites + face_insert(f, mu, 0);
  const int sm = tile_step(g, T, b, mu, -1) * kTileSites + face_insert(f, mu, 3);
  const int slot_p = kTileSites + (2 * mu) * 64 + f;
  const int slot_m = kTileSites + (2 * mu + 1) * 64 + f;
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    lds.w[w][slot_p] = src[word_index(sp, 3, w)];
    lds.w[w][slot_m] = src[word_index(sm, 3, w)];
  }
  if constexpr (kScaled<P>) {
    lds.scale[slot_p] = in.scale[sp];
    lds.scale[slot_m] = in.scale[sm];
  }
}

// ---- FP64 / FP32 stencils on the tiled order. A workgroup owns one 4^4
// tile; its 256 spinors are staged in LDS (48 KB in FP64) and the hops to
// sites inside the tile read them there. A hop across a tile face reads the
// neighbour from memory: each face site has a single consumer in this tile,
// so staging it would not save a load.
template <int P> struct TileWord;
template <> struct TileWord<P_F64> { using T = double2; static constexpr int n = 12; };
template <> struct TileWord<P_F32> { using T = float4; static constexpr int n = 6; };

template <int P>
struct TileSrc {
  using Word = typename TileWord<P>::T;
  using Real = typename PackedSpinor<P>::Real;
  static constexpr int NW = TileWord<P>::n;
  static constexpr bool kFence = true;
  const Word* lds;       // [NW][256]
  PackedSpinor<P> mem;
  int T;
  // One code path for both cases: a generic pointer into LDS (stride 256
  // words) or into memory (stride 64 words within the site's block).
  __device__ __forceinline__ void load(int s, Real v[24]) const {
    const bool in_tile = (s >> 8) == T;
    const Word* base = in_tile ? lds + (s & (kTileSites - 1)) : mem.data + word_index(s, NW, 0);
    const int stride = in_tile ? kTileSites : kSiteBlock;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const Word d = base[w * stride];
      if constexpr (P == P_F64) {
        v[2 * w] = d.x;
        v[2 * w + 1] = d.y;
      } else {
        v[4 * w] = d.x; v[4 * w + 1] = d.y; v[4 * w + 2] = d.z; v[4 * w + 3] = d.w;
      }
    }
  }
};

// Copy tile T of `in` to LDS (one site per thread) and return the source; ends
// with a barrier, so every thread of the workgroup must call it.
template <int P>
__device__ __forceinline__ TileSrc<P> stage_own_tile(const SpinorBuf& in, int T, typename TileWord<P>::T* lds) {
  using Word = typename TileWord<P>::T;
  constexpr int NW = TileWord<P>::n;
  const Word* src = static_cast<const Word*>(in.data);
  const int s = T * kTileSites + threadIdx.x;
#pragma unroll
  for (int w = 0; w < NW; ++w) lds[w * kTileSites + threadIdx.x] = src[word_index(s, NW, w)];
  __syncthreads();
  TileSrc<P> t;
  t.lds = lds;
  t.mem.data = static_cast<Word*>(in.data);
  t.mem.scale = in.scale;
  t.T = T;
  return t;
}

template <int P>
__device__ __forceinline__ void tile_spinor(const TileLds<P>& lds, int slot, float v[24]) {
  typename SpinorWord<P>::T d[3];
#pragma unroll
  for (int w = 0; w < 3; ++w) d[w] = lds.w[w][slot];
  PackedSpinor<P>::unpack(d, kScaled<P> ? lds.scale[slot] : 1.0f, v);
}

// The stored numbers of a staged spinor without its per-site factor, and the
// factor (value = f * raw): the hops apply f once, after the link multiply.
template <int P>
__device__ __forceinline__ float tile_spinor_raw(const TileLds<P>& lds, int slot, float v[24]) {
  typename SpinorWord<P>::T d[3];
#pragma unroll
  for (int w = 0; w < 3; ++w) d[w] = lds.w[w][slot];
  PackedSpinor<P>::unpack_raw(d, v);
  return PackedSpinor<P>::raw_factor(kScaled<P> ? lds.scale[slot] : 1.0f);
}

// Links as link_from returns them are the true links divided by kLinkUnit<P>
// (int16 fixed point is left unscaled until the hop factor).
template <int P> constexpr float kLinkUnit = (P == P_I8) ? 1.0f / kLinkFix : 1.0f;

// Unpack a prefetched link at its point of use. The empty asm makes each raw
// word opaque here, so the compiler cannot unpack all eight links right after
// their loads (which would keep 144 floats live instead of 72 raw words).
// For int16 fixed point the entries come back in units of 1 / kLinkFix (the
// hop multiplies by kLinkUnit<P> once); the rebuilt row 2 is brought to the
// same units.
template <int P, bool C12>
__device__ __forceinline__ void link_from(const uint32_t raw[9], float u[18]) {
  constexpr int NE = LinkFormat<C12>::entries;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    uint32_t r = raw[e];
    asm volatile("" : "+v"(r));
    if constexpr (P == P_I8) {
      u[2 * e] = i16_raw2f(r);
      u[2 * e + 1] = i16_raw2f(r >> 16);
    } else {
      unpack_link16<P>(r, u[2 * e], u[2 * e + 1]);
    }
  }
  if constexpr (C12) {
    su3_third_row(u);
    if constexpr (P == P_I8) {
#pragma unroll
      for (int i = 12; i < 18; ++i) u[i] *= 1.0f / kLinkFix;
    }
  }
}

template <int P, bool C12, int MU, bool DAG>
__device__ __forceinline__ void tile_hop(const TileLds<P>& lds, const uint32_t lk[8][9], int l, float acc[24]) {
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  constexpr int ls = 1 << (2 * MU);
  const int lm = (l >> (2 * MU)) & 3;
  const int fp = face_pos(l, MU);
  const int slot_f = (lm < 3) ? l + ls : kTileSites + (2 * MU) * 64 + fp;
  const int slot_b = (lm > 0) ? l - ls : kTileSites + (2 * MU + 1) * 64 + fp;
  float psi[24], h[12], w[12], u[18];
  float f = tile_spinor_raw<P>(lds, slot_f, psi) * kLinkUnit<P>;
  link_from<P, C12>(lk[MU], u);
  project<MU, SF>(psi, h);
  su3_mul_half<false>(u, h, w);
  reconstruct_fma<MU, SF>(acc, w, f);
  f = tile_spinor_raw<P>(lds, slot_b, psi) * kLinkUnit<P>;
  link_from<P, C12>(lk[4 + MU], u);
  project<MU, SB>(psi, h);
  su3_mul_half<true>(u, h, w);
  reconstruct_fma<MU, SB>(acc, w, f);
  // keep the scheduler from hoisting the next hop's LDS reads and unpacking
  // above this one (that multiplies the live registers for 16-bit data)
  __builtin_amdgcn_sched_barrier(0);
}

// out = D in (or D^+ in) at this thread's site of tile T, after tile_stage and a barrier.
template <int P, bool C12, bool DAG>
__device__ __forceinline__ void tile_wilson(const TileLds<P>& lds, const uint32_t lk[8][9], float diag,
                                            float out[24]) {
  const int l = threadIdx.x;
  float acc[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = 0.f;
  tile_hop<P, C12, 0, DAG>(lds, lk, l, acc);
  tile_hop<P, C12, 1, DAG>(lds, lk, l, acc);
  tile_hop<P, C12, 2, DAG>(lds, lk, l, acc);
  tile_hop<P, C12, 3, DAG>(lds, lk, l, acc);
  float c[24];
  const float dc = diag * tile_spinor_raw<P>(lds, l, c);
#pragma unroll
  for (int i = 0; i < 24; ++i) out[i] = fmaf(dc, c[i], -0.5f * acc[i]);
}

}  // namespace wd
