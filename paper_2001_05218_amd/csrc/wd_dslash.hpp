// The Wilson hopping stencil at one lattice site.
//
// Operator (the Wilson-Dirac matrix of the lattice-QCD textbook the paper
// cites for it in Sec. 1; 3x3 links and 12-component spinors as in the
// Fig. 1 caption; lattice spacing 1, periodic):
//   (D psi)(x) = (m + 4) psi(x)
//              - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
// D^+ is the same stencil with g_mu -> -g_mu.
//
// The paper's stencil pipeline has four stages (Fig. 1): load, linear
// combinations, matrix-vector products, write-out. Here the same four stages
// run in registers per site: load a neighbour spinor, spin-project it to a
// half spinor (linear combinations with factors +-1, +-i), multiply its two
// colour vectors by the link, and rebuild the lower spin half while
// accumulating.
//
// Gamma basis: Euclidean chiral, g_mu = [[0, A_mu], [A_mu^+, 0]] with
//   A_x = -i sigma_1, A_y = -i sigma_2, A_z = -i sigma_3, A_t = 1.
// Each A_mu has one entry per row: (A v)_k = i^n_k v_perm(k).
// (1 + S g_mu) psi = [h ; S A_mu^+ h] with h = psi_up + S A_mu psi_dn.
#pragma once

#include "wd_common.hpp"

namespace wd {

template <int MU> struct SpinTab;
template <> struct SpinTab<0> { static constexpr int p0 = 1, p1 = 0, n0 = 3, n1 = 3; };  // -i, -i
template <> struct SpinTab<1> { static constexpr int p0 = 1, p1 = 0, n0 = 2, n1 = 0; };  // -1, +1
template <> struct SpinTab<2> { static constexpr int p0 = 0, p1 = 1, n0 = 3, n1 = 1; };  // -i, +i
template <> struct SpinTab<3> { static constexpr int p0 = 0, p1 = 1, n0 = 0, n1 = 0; };  // +1, +1

// (re, im) times i^N, N mod 4.
template <int N, typename R>
__device__ __forceinline__ void ipow(R re, R im, R& ore, R& oim) {
  constexpr int n = ((N % 4) + 4) % 4;
  if constexpr (n == 0) { ore = re; oim = im; }
  else if constexpr (n == 1) { ore = -im; oim = re; }
  else if constexpr (n == 2) { ore = -re; oim = -im; }
  else { ore = im; oim = -re; }
}

// h[k][c] = psi_up[k][c] + S * (A psi_dn)[k][c]; h indexed (k * 3 + c) * 2.
template <int MU, int S, typename R>
__device__ __forceinline__ void project(const R psi[24], R h[12]) {
  using T = SpinTab<MU>;
  constexpr int sh = (S > 0) ? 0 : 2;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R a, b;
    ipow<T::n0 + sh>(psi[((2 + T::p0) * 3 + c) * 2], psi[((2 + T::p0) * 3 + c) * 2 + 1], a, b);
    h[(0 * 3 + c) * 2] = psi[(0 * 3 + c) * 2] + a;
    h[(0 * 3 + c) * 2 + 1] = psi[(0 * 3 + c) * 2 + 1] + b;
    ipow<T::n1 + sh>(psi[((2 + T::p1) * 3 + c) * 2], psi[((2 + T::p1) * 3 + c) * 2 + 1], a, b);
    h[(1 * 3 + c) * 2] = psi[(1 * 3 + c) * 2] + a;
    h[(1 * 3 + c) * 2 + 1] = psi[(1 * 3 + c) * 2 + 1] + b;
  }
}

// acc_up[k] += w[k]; acc_dn[perm(k)] += S * conj(i^n_k) w[k]
template <int MU, int S, typename R>
__device__ __forceinline__ void reconstruct_add(R acc[24], const R w[12]) {
  using T = SpinTab<MU>;
  constexpr int sh = (S > 0) ? 0 : 2;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[(0 * 3 + c) * 2] += w[(0 * 3 + c) * 2];
    acc[(0 * 3 + c) * 2 + 1] += w[(0 * 3 + c) * 2 + 1];
    acc[(1 * 3 + c) * 2] += w[(1 * 3 + c) * 2];
    acc[(1 * 3 + c) * 2 + 1] += w[(1 * 3 + c) * 2 + 1];
    R a, b;
    ipow<4 - T::n0 + sh>(w[(0 * 3 + c) * 2], w[(0 * 3 + c) * 2 + 1], a, b);
    acc[((2 + T::p0) * 3 + c) * 2] += a;
    acc[((2 + T::p0) * 3 + c) * 2 + 1] += b;
    ipow<4 - T::n1 + sh>(w[(1 * 3 + c) * 2], w[(1 * 3 + c) * 2 + 1], a, b);
    acc[((2 + T::p1) * 3 + c) * 2] += a;
    acc[((2 + T::p1) * 3 + c) * 2 + 1] += b;
  }
}

// acc += f * (reconstruction of w): reconstruct_add with every term scaled by
// f, the FMA taking the place of the add (f carries the storage scales that
// the raw unpacking left out).
template <int MU, int S, typename R>
__device__ __forceinline__ void reconstruct_fma(R acc[24], const R w[12], R f) {
  using T = SpinTab<MU>;
  constexpr int sh = (S > 0) ? 0 : 2;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[(0 * 3 + c) * 2] = fma(f, w[(0 * 3 + c) * 2], acc[(0 * 3 + c) * 2]);
    acc[(0 * 3 + c) * 2 + 1] = fma(f, w[(0 * 3 + c) * 2 + 1], acc[(0 * 3 + c) * 2 + 1]);
    acc[(1 * 3 + c) * 2] = fma(f, w[(1 * 3 + c) * 2], acc[(1 * 3 + c) * 2]);
    acc[(1 * 3 + c) * 2 + 1] = fma(f, w[(1 * 3 + c) * 2 + 1], acc[(1 * 3 + c) * 2 + 1]);
    R a, b;
    ipow<4 - T::n0 + sh>(w[(0 * 3 + c) * 2], w[(0 * 3 + c) * 2 + 1], a, b);
    acc[((2 + T::p0) * 3 + c) * 2] = fma(f, a, acc[((2 + T::p0) * 3 + c) * 2]);
    acc[((2 + T::p0) * 3 + c) * 2 + 1] = fma(f, b, acc[((2 + T::p0) * 3 + c) * 2 + 1]);
    ipow<4 - T::n1 + sh>(w[(1 * 3 + c) * 2], w[(1 * 3 + c) * 2 + 1], a, b);
    acc[((2 + T::p1) * 3 + c) * 2] = fma(f, a, acc[((2 + T::p1) * 3 + c) * 2]);
    acc[((2 + T::p1) * 3 + c) * 2 + 1] = fma(f, b, acc[((2 + T::p1) * 3 + c) * 2 + 1]);
  }
}

// Row 2 of an SU(3) matrix from rows 0 and 1: u2_k = conj(u0_i u1_j - u0_j u1_i),
// (i, j, k) cyclic (unitarity with unit determinant).
template <typename R>
__device__ __forceinline__ void su3_third_row(R u[18]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    const R ar = u[2 * i] * u[2 * (3 + j)] - u[2 * i + 1] * u[2 * (3 + j) + 1];
    const R ai = u[2 * i] * u[2 * (3 + j) + 1] + u[2 * i + 1] * u[2 * (3 + j)];
    const R br = u[2 * j] * u[2 * (3 + i)] - u[2 * j + 1] * u[2 * (3 + i) + 1];
    const R bi = u[2 * j] * u[2 * (3 + i) + 1] + u[2 * j + 1] * u[2 * (3 + i)];
    u[2 * (6 + k)] = ar - br;
    u[2 * (6 + k) + 1] = -(ai - bi);
  }
}

// w = U h (ADJ = false) or U^+ h (ADJ = true), for both spin rows of h.
template <bool ADJ, typename R>
__device__ __forceinline__ void su3_mul_half(const R u[18], const R h[12], R w[12]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      R re = 0, im = 0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int e = ADJ ? (j * 3 + i) : (i * 3 + j);
        const R ur = u[2 * e];
        const R ui = ADJ ? -u[2 * e + 1] : u[2 * e + 1];
        const R hr = h[(k * 3 + j) * 2];
        const R hi = h[(k * 3 + j) * 2 + 1];
        re = fma(ur, hr, re);
        re = fma(-ui, hi, re);
        im = fma(ur, hi, im);
        im = fma(ui, hr, im);
      }
      w[(k * 3 + i) * 2] = re;
      w[(k * 3 + i) * 2 + 1] = im;
    }
  }
}

// One direction's forward and backward hop, accumulated into acc.
// DAG = false: forward (1 - g), backward (1 + g); DAG = true: signs swapped.
template <int MU, bool DAG, class Gauge, class Src, typename R>
__device__ __forceinline__ void hop_dir(const Gauge& U, const Src& in, int s, const Nbrs& nb, R acc[24]) {
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  R psi[24], h[12], w[12], u[18];
  // forward: U_mu(x) psi(x + mu)
  in.load(nb.fwd[MU], psi);
  U.load_fwd(s, MU, u);
  project<MU, SF>(psi, h);
  su3_mul_half<false>(u, h, w);
  reconstruct_add<MU, SF>(acc, w);
  // backward: U_mu(x - mu)^+ psi(x - mu)
  in.load(nb.bwd[MU], psi);
  U.load_bwd(nb.bwd[MU], MU, u);
  project<MU, SB>(psi, h);
  su3_mul_half<true>(u, h, w);
  reconstruct_add<MU, SB>(acc, w);
  // Sources that read LDS: finish this direction's arithmetic here. Without
  // the empty asm the optimiser sinks every hop's arithmetic to the final
  // sum, which keeps all eight neighbours' loaded values live at once.
  if constexpr (Src::kFence) {
#pragma unroll
    for (int i = 0; i < 24; ++i) asm volatile("" : "+v"(acc[i]));
    __builtin_amdgcn_sched_barrier(0);
  }
}

// out = (m + 4) psi(x) - 1/2 sum_mu hops, arithmetic in R.
template <bool DAG, class Gauge, class Src, typename R>
__device__ __forceinline__ void wilson_site(const Gauge& U, const Src& in, int s, const Nbrs& nb, R diag,
                                            R out[24]) {
  R acc[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = 0;
  hop_dir<0, DAG>(U, in, s, nb, acc);
  hop_dir<1, DAG>(U, in, s, nb, acc);
  hop_dir<2, DAG>(U, in, s, nb, acc);
  hop_dir<3, DAG>(U, in, s, nb, acc);
  R c[24];
  in.load(s, c);
#pragma unroll
  for (int i = 0; i < 24; ++i) out[i] = fma(diag, c[i], R(-0.5) * acc[i]);
}

}  // namespace wd
