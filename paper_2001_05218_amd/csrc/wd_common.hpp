// Common device types for the Wilson-Dirac library (gfx950 / CDNA4).
//
// Storage precisions, lattice geometry with division-free neighbour lookup,
// and the packed (site-blocked, structure-of-arrays) field layouts used on the
// solver's hot loop.
//
// Packed layouts. Sites are grouped in blocks of 64 (one wavefront). Within a
// block every per-site record is split into fixed-width words and stored
// word-major, so that lane l of a wavefront reading word w of its own site
// touches address (block, w, l): each load instruction is one contiguous,
// fully coalesced 64 x word-width span.
//   spinor FP64 : 12 words x 16 B (one complex<double> per word)
//   spinor FP32 :  6 words x 16 B (two complex<float>)
//   spinor BF16 :  3 words x 16 B (four complex<bf16>)
//   spinor FP16 :  3 words x 16 B (four complex<fp16>) + one FP32 scale per site
//   spinor int8 :  3 words x  8 B (four complex<int8>) + one FP32 scale per site
//   links        : per site 4 directions x 9 words, one complex entry per
//                  word (16 B FP64, 8 B FP32, 4 B BF16/FP16; the int8
//                  storage keeps FP16 links), row-major colour
// The padded volume Vpad rounds V up to a multiple of 256 sites (one
// workgroup); padding sites are never read as neighbours and never written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wd {

enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_F16 = 3, P_I8 = 4 };

// Storage formats that carry one FP32 magnitude per site next to the spinor.
template <int P> constexpr bool kScaled = (P == P_F16 || P == P_I8);
// 16-byte-or-smaller word of a packed low-precision spinor (3 words per site).
template <int P> struct SpinorWord { using T = uint4; };   // BF16, FP16: 8 values per word
template <> struct SpinorWord<P_I8> { using T = uint2; };  // int8: 8 values per word

constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts)
constexpr int kSiteBlock = 64;   // sites per layout block (one wavefront)

// ---------------------------------------------------------------- geometry

// Division by a runtime constant d via one 64-bit multiply: exact for
// numerators below 2^31 (q = floor(n * m / 2^k), m = ceil(2^k / d),
// k = 31 + ceil(log2 d); then n * (m d - 2^k) < 2^k).
struct FastDiv {
  uint64_t m;
  uint32_t k;
  uint32_t d;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  FastDiv f;
  f.k = 31 + l;
  f.m = (((1ull << f.k) + d - 1) / d);
  f.d = d;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((uint64_t)n * f.m) >> f.k);
}

// Packed fields number their sites in one of two orders:
//  * linear: s = x + Lx (y + Ly (z + Lz t)), the canonical order;
//  * tiled (every extent a multiple of 4): the lattice is cut into 4^4 tiles of
//    256 sites; s = tile * 256 + local, local = lx + 4 ly + 16 lz + 64 lt, and
//    tiles are numbered x-fastest. One workgroup of 256 threads then owns one
//    compact tile, a wavefront one 4x4x4 cube of it, and a 64-site layout block
//    is exactly that cube.
// Kernels on the canonical boundary layout always use the linear order.
struct Geom {
  int L[4];        // Lx, Ly, Lz, Lt
  int V;           // sites
  int Vpad;        // V rounded up to kBlock
  int nblocks;     // Vpad / kBlock
  int stride[4];   // linear order: 1, Lx, Lx*Ly, Lx*Ly*Lz
  FastDiv dx, dy, dz;
  int tiled;       // 1: tiled order (see above)
  int nt[4];       // tiles per direction (L / 4)
  int tstride[4];  // tile-index strides: 1, nt0, nt0*nt1, nt0*nt1*nt2
  FastDiv tdx, tdy, tdz;
};

inline Geom make_geom(const int L[4], bool allow_tiled = false) {
  Geom g{};
  for (int i = 0; i < 4; ++i) g.L[i] = L[i];
  g.V = L[0] * L[1] * L[2] * L[3];
  g.Vpad = (g.V + kBlock - 1) / kBlock * kBlock;
  g.nblocks = g.Vpad / kBlock;
  g.stride[0] = 1;
  g.stride[1] = L[0];
  g.stride[2] = L[0] * L[1];
  g.stride[3] = L[0] * L[1] * L[2];
  g.dx = make_fastdiv(L[0]);
  g.dy = make_fastdiv(L[1]);
  g.dz = make_fastdiv(L[2]);
  g.tiled = allow_tiled && (L[0] % 4 == 0) && (L[1] % 4 == 0) && (L[2] % 4 == 0) && (L[3] % 4 == 0);
  for (int i = 0; i < 4; ++i) g.nt[i] = g.tiled ? L[i] / 4 : 0;
  if (g.tiled) {
    g.tstride[0] = 1;
    g.tstride[1] = g.nt[0];
    g.tstride[2] = g.nt[0] * g.nt[1];
    g.tstride[3] = g.nt[0] * g.nt[1] * g.nt[2];
    g.tdx = make_fastdiv(g.nt[0]);
    g.tdy = make_fastdiv(g.nt[1]);
    g.tdz = make_fastdiv(g.nt[2]);
  }
  return g;
}

// Tile coordinates of tile index T.
__device__ __forceinline__ void tile_coords(const Geom& g, uint32_t T, int b[4]) {
  uint32_t q = fdiv(T, g.tdx);
  b[0] = (int)(T - q * (uint32_t)g.nt[0]);
  T = q;
  q = fdiv(T, g.tdy);
  b[1] = (int)(T - q * (uint32_t)g.nt[1]);
  T = q;
  q = fdiv(T, g.tdz);
  b[2] = (int)(T - q * (uint32_t)g.nt[2]);
  b[3] = (int)q;
}

// Index of the tile next to tile T (coordinates b) in direction mu, step +-1.
__device__ __forceinline__ int tile_step(const Geom& g, int T, const int b[4], int mu, int step) {
  if (step > 0) return (b[mu] == g.nt[mu] - 1) ? T - (g.nt[mu] - 1) * g.tstride[mu] : T + g.tstride[mu];
  return (b[mu] == 0) ? T + (g.nt[mu] - 1) * g.tstride[mu] : T - g.tstride[mu];
}

// Lattice coordinates (x, y, z, t) of packed site s.
__device__ __forceinline__ void site_coords(const Geom& g, int s, int c[4]) {
  if (g.tiled) {
    int b[4];
    tile_coords(g, (uint32_t)(s >> 8), b);
    const int l = s & 255;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) c[mu] = 4 * b[mu] + ((l >> (2 * mu)) & 3);
  } else {
    uint32_t r = (uint32_t)s;
    uint32_t q = fdiv(r, g.dx);
    c[0] = (int)(r - q * (uint32_t)g.L[0]);
    r = q;
    q = fdiv(r, g.dy);
    c[1] = (int)(r - q * (uint32_t)g.L[1]);
    r = q;
    q = fdiv(r, g.dz);
    c[2] = (int)(r - q * (uint32_t)g.L[2]);
    c[3] = (int)q;
  }
}

// Canonical (linear) index of packed site s.
__device__ __forceinline__ int canonical_index(const Geom& g, int s) {
  if (!g.tiled) return s;
  int c[4];
  site_coords(g, s, c);
  return c[0] + g.stride[1] * c[1] + g.stride[2] * c[2] + g.stride[3] * c[3];
}

// Forward and backward neighbour indices of site s in all four directions.
struct Nbrs {
  int fwd[4];
  int bwd[4];
};

__device__ __forceinline__ Nbrs neighbours(const Geom& g, int s) {
  Nbrs n;
  if (g.tiled) {
    const int T = s >> 8;
    const int l = s & 255;
    int b[4];
    tile_coords(g, (uint32_t)T, b);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int lm = (l >> (2 * mu)) & 3;
      const int ls = 1 << (2 * mu);
      n.fwd[mu] = (lm < 3) ? s + ls : (tile_step(g, T, b, mu, +1) << 8) + (l - 3 * ls);
      n.bwd[mu] = (lm > 0) ? s - ls : (tile_step(g, T, b, mu, -1) << 8) + (l + 3 * ls);
    }
    return n;
  }
  int c[4];
  site_coords(g, s, c);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int st = g.stride[mu];
    const int span = st * (g.L[mu] - 1);
    n.fwd[mu] = (c[mu] == g.L[mu] - 1) ? s - span : s + st;
    n.bwd[mu] = (c[mu] == 0) ? s + span : s - st;
  }
  return n;
}

// Workgroup -> lattice tile. Workgroups are dealt round-robin to the 8 XCDs;
// remapping gives each XCD one contiguous range of tiles so that the
// neighbours a tile needs were recently fetched into the same XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int per = nb >> 3;
  if (b < (per << 3)) return (b & 7) * per + (b >> 3);
  return b;
}
// The workgroup index b with xcd_tile(b, nb) == T.
__device__ __forceinline__ int xcd_tile_inv(int T, int nb) {
  const int per = nb >> 3;
  if (T < (per << 3)) return (T % per) * 8 + T / per;
  return T;
}

// ----------------------------------------------------------- conversions

// Two floats -> two 16-bit values in one word (lo in bits 0..15), rounded to
// nearest even by gfx950's v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32.
typedef __bf16 wd_bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 wd_f16x2 __attribute__((ext_vector_type(2)));
typedef float wd_f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const wd_f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, wd_bf16x2));
}
__device__ __forceinline__ uint32_t pack_f16x2(float lo, float hi) {
  const wd_f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, wd_f16x2));
}
__device__ __forceinline__ float bf_bits2f(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ float h_bits2f(uint32_t b) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
}

// int8 values -> half2 words, exact (|q| <= 127 is an integer of FP16's range):
// flipping the sign bit makes each byte q + 128, and the half with high byte
// 0x64 and low byte q + 128 is 1024 + q + 128; one subtraction of 1152 leaves q.
// Returns the half2 (re, im) of the complex number in bytes 2j, 2j + 1 of d.
__device__ __forceinline__ uint32_t i8x2_to_h2(uint32_t d, int j) {
  const uint32_t x = d ^ 0x80808080u;
  const uint32_t biased = __builtin_amdgcn_perm(0x64646464u, x, j ? 0x04030402u : 0x04010400u);
  const wd_f16x2 bias = {(_Float16)1152.0f, (_Float16)1152.0f};
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(wd_f16x2, biased) - bias);
}

__device__ __forceinline__ size_t word_index(int s, int nwords, int w) {
  return ((size_t)(s >> 6) * nwords + w) * kSiteBlock + (s & 63);
}


// Non-temporal (streaming) store of a 4-, 8- or 16-byte value. Every packed
// field a kernel writes is read again only by a later launch, after the
// writing kernel's whole grid has streamed through the caches; marking the
// stores streaming keeps them from displacing the lines that the running
// stencil still reuses (neighbour faces, links), and measured 2-6 % faster
// stencils at 32^3 x 64 than plain stores.
template <class T> __device__ __forceinline__ void st_nt(T* p, const T& v) {
  if constexpr (sizeof(T) == 16) {
    typedef unsigned int v4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(__builtin_bit_cast(v4, v), reinterpret_cast<v4*>(p));
  } else if constexpr (sizeof(T) == 8) {
    typedef unsigned int v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(__builtin_bit_cast(v2, v), reinterpret_cast<v2*>(p));
  } else {
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned int, v), reinterpret_cast<unsigned int*>(p));
  }
}

// ------------------------------------------------- packed spinor access
// A site's spinor in registers: 24 reals, index (spin * 3 + colour) * 2 + {re, im}.

template <int P> struct PackedSpinor;

template <> struct PackedSpinor<P_F64> {
  using Real = double;
  static constexpr bool kFence = false;
  double2* data;
  float* scale;  // unused
  __device__ __forceinline__ void load(int s, Real v[24]) const {
#pragma unroll
    for (int w = 0; w < 12; ++w) {
      double2 d = data[word_index(s, 12, w)];
      v[2 * w] = d.x;
      v[2 * w + 1] = d.y;
    }
  }
  __device__ __forceinline__ void store(int s, const Real v[24]) const {
#pragma unroll
    for (int w = 0; w < 12; ++w) st_nt(&data[word_index(s, 12, w)], make_double2(v[2 * w], v[2 * w + 1]));
  }
};

template <> struct PackedSpinor<P_F32> {
  using Real = float;
  static constexpr bool kFence = false;
  float4* data;
  float* scale;
  __device__ __forceinline__ void load(int s, Real v[24]) const {
#pragma unroll
    for (int w = 0; w < 6; ++w) {
      float4 d = data[word_index(s, 6, w)];
      v[4 * w] = d.x; v[4 * w + 1] = d.y; v[4 * w + 2] = d.z; v[4 * w + 3] = d.w;
    }
  }
  __device__ __forceinline__ void store(int s, const Real v[24]) const {
#pragma unroll
    for (int w = 0; w < 6; ++w)
      st_nt(&data[word_index(s, 6, w)], make_float4(v[4 * w], v[4 * w + 1], v[4 * w + 2], v[4 * w + 3]));
  }
};

template <> struct PackedSpinor<P_BF16> {
  using Real = float;
  static constexpr bool kFence = false;
  uint4* data;
  float* scale;
  static __device__ __forceinline__ float raw_factor(float) { return 1.0f; }
  static __device__ __forceinline__ void unpack_raw(const uint4 d[3], Real v[24]) { unpack(d, 1.0f, v); }
  static __device__ __forceinline__ void unpack(const uint4 d[3], float, Real v[24]) {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const uint32_t u[4] = {d[w].x, d[w].y, d[w].z, d[w].w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[8 * w + 2 * k] = bf_bits2f(u[k] & 0xffffu);
        v[8 * w + 2 * k + 1] = bf_bits2f(u[k] >> 16);
      }
    }
  }
  __device__ __forceinline__ float load_scale(int) const { return 1.0f; }
  __device__ __forceinline__ void load(int s, Real v[24]) const {
    uint4 d[3];
#pragma unroll
    for (int w = 0; w < 3; ++w) d[w] = data[word_index(s, 3, w)];
    unpack(d, 1.0f, v);
  }
  // Rounded raw words of a spinor (the scale is always 1 for BF16).
  static __device__ __forceinline__ void pack(const Real v[24], uint4 d[3], float& sc) {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      uint32_t u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) u[k] = pack_bf16x2(v[8 * w + 2 * k], v[8 * w + 2 * k + 1]);
      d[w] = make_uint4(u[0], u[1], u[2], u[3]);
    }
    sc = 1.0f;
  }
  __device__ __forceinline__ void store_raw(int s, const uint4 d[3], float) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) st_nt(&data[word_index(s, 3, w)], d[w]);
  }
  __device__ __forceinline__ void store(int s, const Real v[24]) const {
    uint4 d[3];
    float sc;
    pack(v, d, sc);
    store_raw(s, d, sc);
  }
};

template <> struct PackedSpinor<P_F16> {
  using Real = float;
  static constexpr bool kFence = false;
  uint4* data;
  float* scale;   // per-site magnitude: stored value = v / scale, |stored| <= 1
  static __device__ __forceinline__ float raw_factor(float sc) { return sc; }
  static __device__ __forceinline__ void unpack_raw(const uint4 d[3], Real v[24]) {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const uint32_t u[4] = {d[w].x, d[w].y, d[w].z, d[w].w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[8 * w + 2 * k] = h_bits2f(u[k]);
        v[8 * w + 2 * k + 1] = h_bits2f(u[k] >> 16);
      }
    }
  }
  static __device__ __forceinline__ void unpack(const uint4 d[3], float sc, Real v[24]) {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const uint32_t u[4] = {d[w].x, d[w].y, d[w].z, d[w].w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[8 * w + 2 * k] = h_bits2f(u[k]) * sc;
        v[8 * w + 2 * k + 1] = h_bits2f(u[k] >> 16) * sc;
      }
    }
  }
  __device__ __forceinline__ float load_scale(int s) const { return scale[s]; }
  __device__ __forceinline__ void load(int s, Real v[24]) const {
    uint4 d[3];
#pragma unroll
    for (int w = 0; w < 3; ++w) d[w] = data[word_index(s, 3, w)];
    unpack(d, scale[s], v);
  }
  // Rounded raw words and scale of a spinor.
  static __device__ __forceinline__ void pack(const Real v[24], uint4 d[3], float& sc) {
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < 24; ++i) m = fmaxf(m, fabsf(v[i]));
    // 1 / m overflows for m below ~3e-39 (an FP32 denormal; such sites occur
    // far from a point source): capped, 0 stays 0 instead of 0 * inf = NaN and
    // the stored values come out too small by at most m, far below FP32
    // resolution of any field with a normal-range component.
    const float inv = (m > 0.f) ? fminf(1.0f / m, 3.4e38f) : 0.f;
    sc = m;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      uint32_t u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        u[k] = pack_f16x2(v[8 * w + 2 * k] * inv, v[8 * w + 2 * k + 1] * inv);
      d[w] = make_uint4(u[0], u[1], u[2], u[3]);
    }
  }
  __device__ __forceinline__ void store_raw(int s, const uint4 d[3], float sc) const {
    st_nt(&scale[s], sc);
#pragma unroll
    for (int w = 0; w < 3; ++w) st_nt(&data[word_index(s, 3, w)], d[w]);
  }
  __device__ __forceinline__ void store(int s, const Real v[24]) const {
    uint4 d[3];
    float sc;
    pack(v, d, sc);
    store_raw(s, d, sc);
  }
};

// int8 storage: value = q * scale / 127 for the stored signed byte q
// (-127..127), scale = the site's largest |component|. Converting a byte is one
// sign-extending convert; the factor scale / 127 can be applied after the
// linear algebra (raw_factor). A site with a NaN or Inf component gets a NaN
// scale (it stays NaN when read back).
template <> struct PackedSpinor<P_I8> {
  using Real = float;
  static constexpr bool kFence = false;
  uint2* data;
  float* scale;
  static __device__ __forceinline__ float raw_factor(float sc) { return sc * (1.0f / 127.0f); }
  static __device__ __forceinline__ void unpack_raw(const uint2 d[3], Real v[24]) {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const uint32_t u[2] = {d[w].x, d[w].y};
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          v[8 * w + 4 * k + b] = (float)(int)(int8_t)(uint8_t)((u[k] >> (8 * b)) & 0xffu);
    }
  }
  static __device__ __forceinline__ void unpack(const uint2 d[3], float sc, Real v[24]) {
    unpack_raw(d, v);
    const float f = raw_factor(sc);
#pragma unroll
    for (int i = 0; i < 24; ++i) v[i] *= f;
  }
  static __device__ __forceinline__ void pack(const Real v[24], uint2 d[3], float& sc) {
    float m = 0.f, chk = 0.f;
#pragma unroll
    for (int i = 0; i < 24; ++i) {
      m = fmaxf(m, fabsf(v[i]));
      chk = fmaf(v[i], 0.f, chk);   // NaN if any component is NaN or Inf
    }
    const float inv = (m > 0.f) ? fminf(127.0f / m, 3.4e38f) : 0.f;   // capped as for FP16
    sc = (chk == 0.f) ? m : __builtin_nanf("");
    // q = round(v * 127 / m) in [-127, 127] (|v| <= m), rounded to nearest even:
    // v_cvt_pk_u8_f32 rounds v * 127 / m + 128 (exact in FP32; 128 is even, so
    // the rounding is that of v * 127 / m) into a byte lane, and flipping each
    // byte's top bit turns the offset-binary q + 128 into two's complement q
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      uint32_t u[2] = {0u, 0u};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
#pragma unroll
        for (int b = 0; b < 4; ++b) u[k] = __builtin_amdgcn_cvt_pk_u8_f32(fmaf(v[8 * w + 4 * k + b], inv, 128.0f), b, u[k]);
        u[k] ^= 0x80808080u;
      }
      d[w] = make_uint2(u[0], u[1]);
    }
  }
  __device__ __forceinline__ float load_scale(int s) const { return scale[s]; }
  __device__ __forceinline__ void load(int s, Real v[24]) const {
    uint2 d[3];
#pragma unroll
    for (int w = 0; w < 3; ++w) d[w] = data[word_index(s, 3, w)];
    unpack(d, scale[s], v);
  }
  __device__ __forceinline__ void store_raw(int s, const uint2 d[3], float sc) const {
    st_nt(&scale[s], sc);
#pragma unroll
    for (int w = 0; w < 3; ++w) st_nt(&data[word_index(s, 3, w)], d[w]);
  }
  __device__ __forceinline__ void store(int s, const Real v[24]) const {
    uint2 d[3];
    float sc;
    pack(v, d, sc);
    store_raw(s, d, sc);
  }
};

// Canonical boundary layout: (Lt, Lz, Ly, Lx, 4, 3) complex128, AoS.
struct CanonSpinor {
  using Real = double;
  static constexpr bool kFence = false;
  double2* data;
  __device__ __forceinline__ void load(int s, Real v[24]) const {
    const double2* p = data + (size_t)s * 12;
#pragma unroll
    for (int w = 0; w < 12; ++w) {
      double2 d = p[w];
      v[2 * w] = d.x;
      v[2 * w + 1] = d.y;
    }
  }
  __device__ __forceinline__ void store(int s, const Real v[24]) const {
    double2* p = data + (size_t)s * 12;
#pragma unroll
    for (int w = 0; w < 12; ++w) p[w] = make_double2(v[2 * w], v[2 * w + 1]);
  }
};

// ---------------------------------------------------------- link access
// A link in registers: 18 reals, index (row * 3 + col) * 2 + {re, im}.
// The stencil asks for U_mu(x) through load_fwd(x, mu) and for U_mu(x - mu)
// through load_bwd(x - mu, mu); accessors that read memory directly forward
// both to load().
#define WD_GAUGE_FORWARDERS                                                              \
  template <typename R>                                                                  \
  __device__ __forceinline__ void load_fwd(int s, int mu, R u[18]) const { load(s, mu, u); } \
  template <typename R>                                                                  \
  __device__ __forceinline__ void load_bwd(int s, int mu, R u[18]) const { load(s, mu, u); }

template <int P> struct PackedGauge;

template <> struct PackedGauge<P_F64> {
  using Real = double;
  WD_GAUGE_FORWARDERS
  const double2* data;
  __device__ __forceinline__ void load(int s, int mu, Real u[18]) const {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      double2 d = data[word_index(s, 36, mu * 9 + e)];
      u[2 * e] = d.x;
      u[2 * e + 1] = d.y;
    }
  }
};

template <> struct PackedGauge<P_F32> {
  using Real = float;
  WD_GAUGE_FORWARDERS
  const float2* data;
  __device__ __forceinline__ void load(int s, int mu, Real u[18]) const {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      float2 d = data[word_index(s, 36, mu * 9 + e)];
      u[2 * e] = d.x;
      u[2 * e + 1] = d.y;
    }
  }
};

// One complex link entry from its 16-bit pair (re low, im high).
template <int P> __device__ __forceinline__ void unpack_link16(uint32_t d, float& re, float& im) {
  if constexpr (P == P_BF16) {
    re = bf_bits2f(d & 0xffffu);
    im = bf_bits2f(d >> 16);
  } else {   // FP16 pairs (also the links of the int8 storage)
    re = h_bits2f(d);
    im = h_bits2f(d >> 16);
  }
}

template <> struct PackedGauge<P_BF16> {
  using Real = float;
  WD_GAUGE_FORWARDERS
  const uint32_t* data;
  __device__ __forceinline__ void load(int s, int mu, Real u[18]) const {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      uint32_t d = data[word_index(s, 36, mu * 9 + e)];
      u[2 * e] = bf_bits2f(d & 0xffffu);
      u[2 * e + 1] = bf_bits2f(d >> 16);
    }
  }
};

template <> struct PackedGauge<P_F16> {
  using Real = float;
  WD_GAUGE_FORWARDERS
  const uint32_t* data;
  __device__ __forceinline__ void load(int s, int mu, Real u[18]) const {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      uint32_t d = data[word_index(s, 36, mu * 9 + e)];
      u[2 * e] = h_bits2f(d);
      u[2 * e + 1] = h_bits2f(d >> 16);
    }
  }
};

template <> struct PackedGauge<P_I8> : PackedGauge<P_F16> {};   // int8 storage keeps FP16 links

// Canonical boundary layout: (4, Lt, Lz, Ly, Lx, 3, 3) complex128.
struct CanonGauge {
  using Real = double;
  WD_GAUGE_FORWARDERS
  const double2* data;
  size_t V;
  __device__ __forceinline__ void load(int s, int mu, Real u[18]) const {
    const double2* p = data + ((size_t)mu * V + (size_t)s) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      double2 d = p[e];
      u[2 * e] = d.x;
      u[2 * e + 1] = d.y;
    }
  }
};

// Bytes of one packed field of V sites (padded volume).
inline size_t spinor_bytes(int P, int Vpad) {
  switch (P) {
    case P_F64: return (size_t)Vpad * 192;
    case P_F32: return (size_t)Vpad * 96;
    case P_I8: return (size_t)Vpad * 24;
    default: return (size_t)Vpad * 48;
  }
}
inline size_t spinor_scale_bytes(int P, int Vpad) { return (P == P_F16 || P == P_I8) ? (size_t)Vpad * 4 : 0; }
inline size_t gauge_bytes(int P, int Vpad) {
  switch (P) {
    case P_F64: return (size_t)Vpad * 4 * 9 * 16;
    case P_F32: return (size_t)Vpad * 4 * 9 * 8;
    default: return (size_t)Vpad * 4 * 9 * 4;
  }
}

}  // namespace wd
