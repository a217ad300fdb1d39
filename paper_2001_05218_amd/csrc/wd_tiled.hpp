// LDS-staged Wilson stencils in the tiled site order: 16- and 8-bit fields
// (tile plus halo faces in LDS), FP64/FP32 fields (own tile in LDS, each link
// read once).
//
// The paper keeps the inputs of neighbouring stencils on chip in cyclic
// buffers so that each datum crosses the memory interface once (Sec. 2).
// On gfx950 the caches cannot be trusted with that reuse: at full bandwidth
// an XCD's 4 MB L2 turns over in a few microseconds, less than the time a
// wavefront spends walking its eight hops, and measured L2 hit rates of the
// cache-only stencil are ~10 %. Here a workgroup owns one 4^4 tile and
//   1. issues, all at once, the loads of its 256 spinors plus the 8 halo
//      faces (64 sites each, read from the neighbouring tiles) into LDS, and
//      of half of its sites' 8 links (4 own, 4 backward) into registers;
//   2. after one barrier loads the other half of the links and evaluates all
//      8 hops from LDS and registers.
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

// FP16 and int8 storage: 12 half2 words (one complex each, index
// spin * 3 + colour) per slot and the slot's value factor (FP16: the site's
// scale; int8: scale / 127, the bytes converted to half when staged), so that
// both run the same packed-half hops.
struct HalfTile {
  uint4 h[3][kTileSlots];
  float f[kTileSlots];
};
template <> struct TileLds<P_F16> : HalfTile {};
template <> struct TileLds<P_I8> : HalfTile {};

// Store one site's spinor words (and scale) into an LDS slot.
template <int P>
__device__ __forceinline__ void stage_slot(TileLds<P>& lds, int slot, const typename SpinorWord<P>::T* src,
                                           const float* scale, int s) {
#pragma unroll
  for (int w = 0; w < 3; ++w) lds.w[w][slot] = src[word_index(s, 3, w)];
  if constexpr (kScaled<P>) lds.scale[slot] = scale[s];
}
// FP16 and int8: the slot's factor is staged times kappa, a constant of the
// launch that the hops' sums then carry (see tile_wilson_h).
__device__ __forceinline__ void stage_slot(TileLds<P_F16>& lds, int slot, const uint4* src, const float* scale, int s,
                                           float kappa) {
#pragma unroll
  for (int w = 0; w < 3; ++w) lds.h[w][slot] = src[word_index(s, 3, w)];
  lds.f[slot] = scale[s] * kappa;
}
__device__ __forceinline__ void stage_slot(TileLds<P_I8>& lds, int slot, const uint2* src, const float* scale, int s,
                                           float kappa) {
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const uint2 d = src[word_index(s, 3, w)];
    lds.h[w][slot] = make_uint4(i8x2_to_h2(d.x, 0), i8x2_to_h2(d.x, 1), i8x2_to_h2(d.y, 0), i8x2_to_h2(d.y, 1));
  }
  lds.f[slot] = scale[s] * (kappa * (1.0f / 127.0f));
}
template <int P>
__device__ __forceinline__ void stage_slot(TileLds<P>& lds, int slot, const typename SpinorWord<P>::T* src,
                                           const float* scale, int s, float) {
  stage_slot(lds, slot, src, scale, s);
}

// Links are stored either as all 9 entries (18 reals) or, for SU(3) fields,
// as rows 0 and 1 only (12 reals; row 2 = conj(row0 x row1) is rebuilt on use).
template <bool C12> struct LinkFormat {
  static constexpr int entries = C12 ? 6 : 9;    // stored entries per link
  static constexpr int words = 4 * entries;      // per site, 4 directions
};

// Links of directions M0 <= mu < M1 of this thread's site into registers: the
// forward U_mu(s) in lk[mu], the backward U_mu(s - mu) in lk[4 + mu].
template <bool C12, int M0, int M1>
__device__ __forceinline__ void tile_links(const Geom& g, int T, const void* Uv, uint32_t lk[8][9]) {
  constexpr int NE = LinkFormat<C12>::entries;
  constexpr int NW = LinkFormat<C12>::words;
  const int s = T * kTileSites + threadIdx.x;
  const uint32_t* U = static_cast<const uint32_t*>(Uv);
  const Nbrs nb = neighbours(g, s);
#pragma unroll
  for (int mu = M0; mu < M1; ++mu)
#pragma unroll
    for (int e = 0; e < NE; ++e) lk[mu][e] = U[word_index(s, NW, mu * NE + e)];
#pragma unroll
  for (int mu = M0; mu < M1; ++mu)
#pragma unroll
    for (int e = 0; e < NE; ++e) lk[4 + mu][e] = U[word_index(nb.bwd[mu], NW, mu * NE + e)];
}

// Links of the first kEarlyDirs directions are loaded with the tile (before
// the barrier); the rest after it, so that their latency overlaps the first
// hops instead of the wait at the barrier.
constexpr int kEarlyDirs = 2;

// Stage the tile's spinors and halo faces; prefetch the early links of site s.
template <int P, bool C12>
__device__ __forceinline__ void tile_stage(const Geom& g, int T, const void* Uv, const SpinorBuf& in, TileLds<P>& lds,
                                           uint32_t lk[8][9], float kappa = 1.0f) {
  const int l = threadIdx.x;
  const int s = T * kTileSites + l;
  const typename SpinorWord<P>::T* src = static_cast<const typename SpinorWord<P>::T*>(in.data);
  stage_slot(lds, l, src, in.scale, s, kappa);
  // halo: wavefront mu stages the two mu faces
  const int mu = l >> 6;
  const int f = l & 63;
  int b[4];
  tile_coords(g, (uint32_t)T, b);
  const int sp = tile_step(g, T, b, mu, +1) * kTileSites + face_insert(f, mu, 0);
  const int sm = tile_step(g, T, b, mu, -1) * kTileSites + face_insert(f, mu, 3);
  const int slot_p = kTileSites + (2 * mu) * 64 + f;
  const int slot_m = kTileSites + (2 * mu + 1) * 64 + f;
  stage_slot(lds, slot_p, src, in.scale, sp, kappa);
  stage_slot(lds, slot_m, src, in.scale, sm, kappa);
  tile_links<C12, 0, kEarlyDirs>(g, T, Uv, lk);
}

// After tile_stage's barrier: the remaining links.
template <bool C12>
__device__ __forceinline__ void tile_links_late(const Geom& g, int T, const void* Uv, uint32_t lk[8][9]) {
  tile_links<C12, kEarlyDirs, 4>(g, T, Uv, lk);
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

// FP64 / FP32 tiles, each link read once. The thread at x loads U_mu(x),
// applies it to its forward neighbour and, as U_mu(x)^+ times the spin
// projection of its own spinor, hands the backward term of the site x + mu
// over through LDS (`up`, one direction at a time, two barriers per
// direction). Only a thread on the tile's lower mu face loads U_mu(x - mu)
// itself. Without this, every link is loaded twice (forward at x, backward at
// x + mu), and the second load mostly misses L2.
template <typename R> struct UpBuf { R v[12][kTileSites]; };

template <int MU, bool DAG, class Gauge, class Src, typename R>
__device__ __forceinline__ void hop_dir_once(const Gauge& U, const Src& in, int s, const Nbrs& nb, R acc[24],
                                             UpBuf<R>& up) {
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  constexpr int ls = 1 << (2 * MU);
  const int l = threadIdx.x;
  const int lm = (l >> (2 * MU)) & 3;
  R psi[24], h[12], w[12], u[18];
  U.load_fwd(s, MU, u);
  in.load(nb.fwd[MU], psi);
  project<MU, SF>(psi, h);
  su3_mul_half<false>(u, h, w);
  reconstruct_add<MU, SF>(acc, w);
  if (lm < 3) {
    in.load(s, psi);
    project<MU, SB>(psi, h);
    su3_mul_half<true>(u, h, w);
#pragma unroll
    for (int i = 0; i < 12; ++i) up.v[i][l + ls] = w[i];
  }
  __syncthreads();
  if (lm > 0) {
#pragma unroll
    for (int i = 0; i < 12; ++i) w[i] = up.v[i][l];
  } else {
    in.load(nb.bwd[MU], psi);
    U.load_bwd(nb.bwd[MU], MU, u);
    project<MU, SB>(psi, h);
    su3_mul_half<true>(u, h, w);
  }
  reconstruct_add<MU, SB>(acc, w);
  __syncthreads();   // `up` is rewritten by the next direction
#pragma unroll
  for (int i = 0; i < 24; ++i) asm volatile("" : "+v"(acc[i]));
  __builtin_amdgcn_sched_barrier(0);
}

// out = (m + 4) psi(x) - 1/2 sum_mu hops at site s of the staged tile; every
// thread of the workgroup must call it (barriers).
template <bool DAG, class Gauge, class Src, typename R>
__device__ __forceinline__ void wilson_site_once(const Gauge& U, const Src& in, int s, const Nbrs& nb, R diag,
                                                 R out[24], UpBuf<R>& up) {
  R acc[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = 0;
  hop_dir_once<0, DAG>(U, in, s, nb, acc, up);
  hop_dir_once<1, DAG>(U, in, s, nb, acc, up);
  hop_dir_once<2, DAG>(U, in, s, nb, acc, up);
  hop_dir_once<3, DAG>(U, in, s, nb, acc, up);
  R c[24];
  in.load(s, c);
#pragma unroll
  for (int i = 0; i < 24; ++i) out[i] = fma(diag, c[i], R(-0.5) * acc[i]);
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

// Unpack a prefetched link at its point of use. The empty asm makes each raw
// word opaque here, so the compiler cannot unpack all eight links right after
// their loads (which would keep 144 floats live instead of 72 raw words).
template <int P, bool C12>
__device__ __forceinline__ void link_from(const uint32_t raw[9], float u[18]) {
  constexpr int NE = LinkFormat<C12>::entries;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    uint32_t r = raw[e];
    asm volatile("" : "+v"(r));
    unpack_link16<P>(r, u[2 * e], u[2 * e + 1]);
  }
  if constexpr (C12) su3_third_row(u);
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
  float f = tile_spinor_raw<P>(lds, slot_f, psi);
  link_from<P, C12>(lk[MU], u);
  project<MU, SF>(psi, h);
  su3_mul_half<false>(u, h, w);
  reconstruct_fma<MU, SF>(acc, w, f);
  f = tile_spinor_raw<P>(lds, slot_b, psi);
  link_from<P, C12>(lk[4 + MU], u);
  project<MU, SB>(psi, h);
  su3_mul_half<true>(u, h, w);
  reconstruct_fma<MU, SB>(acc, w, f);
  // keep the scheduler from hoisting the next hop's LDS reads and unpacking
  // above this one (that multiplies the live registers for 16-bit data)
  __builtin_amdgcn_sched_barrier(0);
}

// ---- int8 storage: hops in packed half precision with FP32 dot products.
// gfx950's v_dot2_f32_f16 multiplies the two halves of two half2 words and
// adds both products to an FP32 accumulator, so a complex multiply-add takes
// two instructions instead of four FP32 FMAs, and a spin projection of two
// half2 complex numbers is one v_pk_add_f16. Nothing is lost to the format:
// the staged int8 values are exact in half, so are their projections
// (|q1 +- q2| <= 254), the products of two halves are exact in FP32, and the
// links are FP16 already; only the FP32 sums round, as in the FP32 path.

// a.x * b.x + a.y * b.y + c, FP32 sum of exact products.
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2(__builtin_bit_cast(wd_f16x2, a), __builtin_bit_cast(wd_f16x2, b), c, false);
}

// a.x * b.x + a.y * b.y, and its negative, as one VOP3P instruction with an
// inline zero addend (and negated second operand): given a zero accumulator the
// compiler otherwise picks the two-operand form and zeroes a register first,
// and negates results with a separate xor.
__device__ __forceinline__ float dot2z(uint32_t a, uint32_t b) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float ndot2z(uint32_t a, uint32_t b) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, 0 neg_lo:[0,1,0] neg_hi:[0,1,0]" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Written out: given the same sum as half2 vector code, the compiler builds
// the swapped or negated first operand with separate instructions (2-3 per
// form instead of none). v_pk_add_f16 is a plain VALU op: no wait states.
#define WD_PK_ADD_F16(r, a, b, MODS) asm("v_pk_add_f16 %0, %1, %2 " MODS : "=v"(r) : "v"(a), "v"(b))

// One form of h = a + i^N b (a, b, h complex as half2 (re, im)), in one
// v_pk_add_f16 whose source selects and negations build the form:
//   F = 0: (h.re, h.im)   F = 1: (h.re, -h.im)   F = 2: (h.im, h.re)   F = 3: (h.im, -h.re)
// U h needs forms 1 and 2 (re = sum dot2(u, form 1), im = sum dot2(u, form 2));
// U^+ h needs forms 0 and 3.
template <int N, int F>
__device__ __forceinline__ uint32_t proj_form(uint32_t a, uint32_t b) {
  uint32_t r;
  if constexpr (N == 0 && F == 0) WD_PK_ADD_F16(r, a, b, "op_sel:[0,0] op_sel_hi:[1,1] neg_lo:[0,0] neg_hi:[0,0]");
  if constexpr (N == 0 && F == 1) WD_PK_ADD_F16(r, a, b, "op_sel:[0,0] op_sel_hi:[1,1] neg_lo:[0,0] neg_hi:[1,1]");
  if constexpr (N == 0 && F == 2) WD_PK_ADD_F16(r, a, b, "op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,0] neg_hi:[0,0]");
  if constexpr (N == 0 && F == 3) WD_PK_ADD_F16(r, a, b, "op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,0] neg_hi:[1,1]");
  if constexpr (N == 1 && F == 0) WD_PK_ADD_F16(r, a, b, "op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1] neg_hi:[0,0]");
  if constexpr (N == 1 && F == 1) WD_PK_ADD_F16(r, a, b, "op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1] neg_hi:[1,1]");
  if constexpr (N == 1 && F == 2) WD_PK_ADD_F16(r, a, b, "op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,0] neg_hi:[0,1]");
  if constexpr (N == 1 && F == 3) WD_PK_ADD_F16(r, a, b, "op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,0] neg_hi:[1,0]");
  if constexpr (N == 2 && F == 0) WD_PK_ADD_F16(r, a, b, "op_sel:[0,0] op_sel_hi:[1,1] neg_lo:[0,1] neg_hi:[0,1]");
  if constexpr (N == 2 && F == 1) WD_PK_ADD_F16(r, a, b, "op_sel:[0,0] op_sel_hi:[1,1] neg_lo:[0,1] neg_hi:[1,0]");
  if constexpr (N == 2 && F == 2) WD_PK_ADD_F16(r, a, b, "op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[0,1]");
  if constexpr (N == 2 && F == 3) WD_PK_ADD_F16(r, a, b, "op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[1,0]");
  if constexpr (N == 3 && F == 0) WD_PK_ADD_F16(r, a, b, "op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,0] neg_hi:[0,1]");
  if constexpr (N == 3 && F == 1) WD_PK_ADD_F16(r, a, b, "op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,0] neg_hi:[1,0]");
  if constexpr (N == 3 && F == 2) WD_PK_ADD_F16(r, a, b, "op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1] neg_hi:[0,0]");
  if constexpr (N == 3 && F == 3) WD_PK_ADD_F16(r, a, b, "op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1] neg_hi:[1,1]");
  return r;
}

__device__ __forceinline__ uint32_t conj_h2(uint32_t u) { return u ^ 0x80000000u; }
__device__ __forceinline__ uint32_t swap_h2(uint32_t u) { return (u >> 16) | (u << 16); }

// Row 2 of an SU(3) link from FP16 rows 0 and 1 (words u[0..5]):
// u2_k = conj(u0_i u1_j - u0_j u1_i), (i, j, k) cyclic, summed in FP32.
__device__ __forceinline__ void su3_third_row_h(uint32_t u[9]) {
  uint32_t c1[3], s1[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    c1[j] = conj_h2(u[3 + j]);
    s1[j] = swap_h2(u[3 + j]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    const float re = dot2(u[i], c1[j], ndot2z(u[j], c1[i]));   // Re(u0_i u1_j - u0_j u1_i)
    const float im = dot2(u[j], s1[i], ndot2z(u[i], s1[j]));   // -Im(u0_i u1_j - u0_j u1_i)
    u[6 + k] = pack_f16x2(re, im);
  }
}

// acc += f * reconstruction of (U h) or (U^+ h), h the spin projection of the
// staged neighbour in `slot`, f its value factor.
// acc += f * reconstruction of (U h) or (U^+ h): h the spin projection of the
// half2 spinor words psi (index spin * 3 + colour), U the FP16 link words raw
// (rows 0 and 1 when C12), f the spinor's value factor.
template <int MU, int S, bool ADJ, bool C12>
__device__ __forceinline__ void hop_h_words(const uint32_t psi[12], float f, const uint32_t raw[9], float acc[24]) {
  using T = SpinTab<MU>;
  constexpr int sh = (S > 0) ? 0 : 2;
  constexpr int N0 = (T::n0 + sh) & 3, N1 = (T::n1 + sh) & 3;
  constexpr int FA = ADJ ? 0 : 1, FB = ADJ ? 3 : 2;
  uint32_t ha[6], hb[6];   // forms of the projection, index spin row * 3 + colour
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ha[c] = proj_form<N0, FA>(psi[c], psi[(2 + T::p0) * 3 + c]);
    hb[c] = proj_form<N0, FB>(psi[c], psi[(2 + T::p0) * 3 + c]);
    ha[3 + c] = proj_form<N1, FA>(psi[3 + c], psi[(2 + T::p1) * 3 + c]);
    hb[3 + c] = proj_form<N1, FB>(psi[3 + c], psi[(2 + T::p1) * 3 + c]);
  }
  constexpr int NE = LinkFormat<C12>::entries;
  uint32_t u[9];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    u[e] = raw[e];
    asm volatile("" : "+v"(u[e]));   // keep the link words opaque until their hop
  }
  if constexpr (C12) su3_third_row_h(u);
  float w[12];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int e0 = ADJ ? i : i * 3;
      float re = dot2z(u[e0], ha[k * 3]);
      float im = dot2z(u[e0], hb[k * 3]);
#pragma unroll
      for (int j = 1; j < 3; ++j) {
        const int e = ADJ ? (j * 3 + i) : (i * 3 + j);
        re = dot2(u[e], ha[k * 3 + j], re);
        im = dot2(u[e], hb[k * 3 + j], im);
      }
      w[(k * 3 + i) * 2] = re;
      w[(k * 3 + i) * 2 + 1] = im;
    }
  }
  reconstruct_fma<MU, S>(acc, w, f);
}

// The same for a staged FP16 or int8 slot.
template <int MU, int S, bool ADJ, bool C12>
__device__ __forceinline__ void hop_h(const HalfTile& lds, int slot, const uint32_t raw[9], float acc[24]) {
  uint32_t psi[12];
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const uint4 d = lds.h[w][slot];
    psi[4 * w] = d.x;
    psi[4 * w + 1] = d.y;
    psi[4 * w + 2] = d.z;
    psi[4 * w + 3] = d.w;
  }
  hop_h_words<MU, S, ADJ, C12>(psi, lds.f[slot], raw, acc);
}

template <bool C12, int MU, bool DAG>
__device__ __forceinline__ void tile_hop_h(const HalfTile& lds, const uint32_t lk[8][9], int l, float acc[24]) {
  constexpr int SF = DAG ? +1 : -1;
  constexpr int ls = 1 << (2 * MU);
  const int lm = (l >> (2 * MU)) & 3;
  const int fp = face_pos(l, MU);
  const int slot_f = (lm < 3) ? l + ls : kTileSites + (2 * MU) * 64 + fp;
  const int slot_b = (lm > 0) ? l - ls : kTileSites + (2 * MU + 1) * 64 + fp;
  hop_h<MU, SF, false, C12>(lds, slot_f, lk[MU], acc);
  hop_h<MU, -SF, true, C12>(lds, slot_b, lk[4 + MU], acc);
  __builtin_amdgcn_sched_barrier(0);
}

// out = D in (or D^+ in) at this thread's site of tile T, after tile_stage and a barrier.
template <int P, bool C12, bool DAG>
__device__ __forceinline__ void tile_wilson(const TileLds<P>& lds, const uint32_t lk[8][9], float diag,
                                            float out[24]) {
  static_assert(P != P_I8 && P != P_F16, "FP16 and int8 tiles use tile_wilson_h");
  const int l = threadIdx.x;
  float acc[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = 0.f;
  float c[24];
  tile_hop<P, C12, 0, DAG>(lds, lk, l, acc);
  tile_hop<P, C12, 1, DAG>(lds, lk, l, acc);
  tile_hop<P, C12, 2, DAG>(lds, lk, l, acc);
  tile_hop<P, C12, 3, DAG>(lds, lk, l, acc);
  const float dc = diag * tile_spinor_raw<P>(lds, l, c);
#pragma unroll
  for (int i = 0; i < 24; ++i) out[i] = fmaf(dc, c[i], -0.5f * acc[i]);
}

// FP16 and int8 tiles staged with factor kappa: out = dcoef * f_l * psi(x) +
// kappa * sum of hops, f_l the staged factor of the thread's own site. The
// launch chooses kappa so that no per-value scaling is left: D psi is
// kappa = -1/2, dcoef = -2 diag; -alpha D^+ t is kappa = alpha / 2, dcoef = -2 diag.
// The hops run in packed half precision with FP32 dot products: exact for
// int8 data; for FP16 data the spin projection rounds to half once (relative
// 2^-11, the resolution the values are stored with).
template <bool C12, bool DAG>
__device__ __forceinline__ void tile_wilson_h(const HalfTile& lds, const uint32_t lk[8][9], float dcoef,
                                              float out[24]) {
  const int l = threadIdx.x;
  float acc[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = 0.f;
  tile_hop_h<C12, 0, DAG>(lds, lk, l, acc);
  tile_hop_h<C12, 1, DAG>(lds, lk, l, acc);
  tile_hop_h<C12, 2, DAG>(lds, lk, l, acc);
  tile_hop_h<C12, 3, DAG>(lds, lk, l, acc);
  const float dc = dcoef * lds.f[l];
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const uint4 d = lds.h[w][l];
    const uint32_t q[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      out[8 * w + 2 * k] = fmaf(dc, h_bits2f(q[k]), acc[8 * w + 2 * k]);
      out[8 * w + 2 * k + 1] = fmaf(dc, h_bits2f(q[k] >> 16), acc[8 * w + 2 * k + 1]);
    }
  }
}

}  // namespace wd
