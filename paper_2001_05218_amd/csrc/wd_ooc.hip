// Out-of-core FP64 CG: the gauge field and every CG vector stay in pinned host
// memory and stream through the GPU in slabs of time planes.
//
// The paper's accelerator starts on the first complete set of inputs while the
// rest of the data is still arriving over the host link, which frees the
// computation from the size of the accelerator's local memory (Sec. 2;
// Sec. 3.1; Sec. 4 and Fig. 2, three input streams and one output stream).
// Here the same holds per t-slab: a sweep walks the lattice slab by slab with
// three HIP streams (host-to-device copies, kernels, device-to-host copies)
// and two device buffer sets, so that while slab k is computed, slab k + 1 is
// copied in and slab k - 1 copied out. The stencil needs the planes on both
// sides of a slab; the window copied in holds them (a lower and an upper halo
// plane, periodic in t), and the links of the plane below.
//
// One CGNR iteration k is two sweeps (b' = D^+ b or b, M = D^+ D):
//   S1  p_k = r_k + beta_{k-1} p_{k-1} (on the whole window), t = D p_k,
//       x += alpha_{k-1} p_{k-1}       in: U, r and p windows, x
//                                      out: p_k, t, x     ||t||^2 -> alpha_k
//   S2  r_{k+1} = r_k - alpha_k D^+ t  in: U, t window, r  out: r  ||r||^2 -> beta_k
// The solution update lags one iteration behind (x is not needed by the
// recurrences): S1 applies the previous step's alpha p while it holds that p,
// and a last short sweep applies the final one. The scalars never leave the
// device (finalize kernels on the kernel stream); the host reads the state
// once per iteration.
// Each sweep may start copying in as soon as the slabs it reads have been
// written back by the sweep before: a sweep whose input is a window starts one
// slab later than the sweep before it (its first slab then needs only slabs
// that were written back first), so consecutive sweeps overlap instead of
// draining the pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <utility>
#include <vector>

#include "wd_dslash.hpp"
#include "wd_internal.hpp"
#include "wd_reduce.hpp"

namespace wd {

// ---------------------------------------------------------------- geometry

// A window: `ts` slab planes plus one halo plane below (window plane 0) and
// one above; sites numbered canonically within it (x fastest, plane-major).
struct SlabGeom {
  int L[3];      // Lx, Ly, Lz
  int plane;     // Lx * Ly * Lz
  int ts;        // planes of this slab
  FastDiv dx, dy, dz;
};

__device__ __forceinline__ Nbrs slab_neighbours(const SlabGeom& g, int w) {
  uint32_t q = fdiv((uint32_t)w, g.dx);
  const int x = w - (int)q * g.L[0];
  const uint32_t q2 = fdiv(q, g.dy);
  const int y = (int)q - (int)q2 * g.L[1];
  const uint32_t q3 = fdiv(q2, g.dz);
  const int z = (int)q2 - (int)q3 * g.L[2];
  const int c[3] = {x, y, z};
  const int st[3] = {1, g.L[0], g.L[0] * g.L[1]};
  Nbrs n;
#pragma unroll
  for (int mu = 0; mu < 3; ++mu) {
    const int span = st[mu] * (g.L[mu] - 1);
    n.fwd[mu] = (c[mu] == g.L[mu] - 1) ? w - span : w + st[mu];
    n.bwd[mu] = (c[mu] == 0) ? w + span : w - st[mu];
  }
  n.fwd[3] = w + g.plane;   // the halo planes make t local
  n.bwd[3] = w - g.plane;
  return n;
}

// ------------------------------------------------------------------ kernels
// Thread i works on slab site i (window site plane + i). Partial sums go to
// partials[blockIdx.x] (the host offsets the pointer per slab).

template <bool DAG>
__global__ __launch_bounds__(kBlock) void k_ooc_apply(SlabGeom g, CanonGauge U, CanonSpinor in,
                                                      double2* __restrict__ out, double diag,
                                                      double* __restrict__ partials) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (i < g.ts * g.plane) {
    const int w = g.plane + i;
    double o[24];
    wilson_site<DAG>(U, in, w, slab_neighbours(g, w), diag, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      out[(size_t)i * 12 + k] = make_double2(o[2 * k], o[2 * k + 1]);
      n2 += o[2 * k] * o[2 * k] + o[2 * k + 1] * o[2 * k + 1];
    }
  }
  store_partial(n2, partials);
}

// r = b' - D^+ t (and p = r when p is given); ||r||^2.
__global__ __launch_bounds__(kBlock) void k_ooc_residual(SlabGeom g, CanonGauge U, CanonSpinor t,
                                                         const double2* __restrict__ bp, double2* __restrict__ r,
                                                         double2* __restrict__ p, double diag,
                                                         double* __restrict__ partials) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (i < g.ts * g.plane) {
    const int w = g.plane + i;
    double q[24];
    wilson_site<true>(U, t, w, slab_neighbours(g, w), diag, q);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const size_t e = (size_t)i * 12 + k;
      const double2 b = bp[e];
      const double2 v = make_double2(b.x - q[2 * k], b.y - q[2 * k + 1]);
      r[e] = v;
      if (p) p[e] = v;
      n2 += v.x * v.x + v.y * v.y;
    }
  }
  store_partial(n2, partials);
}

// The search direction over a whole window (ts + 2 planes): p = r + beta p.
// On the slab's own planes (window planes 1 .. ts) also x += alpha p_old, the
// deferred solution update of the previous iteration.
__global__ __launch_bounds__(kBlock) void k_ooc_pwin(size_t n_win, size_t lo, size_t hi, const double2* __restrict__ r,
                                                     double2* __restrict__ p, double2* __restrict__ x,
                                                     const SolverState* __restrict__ st) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n_win) return;
  const double beta = st->beta;
  const double2 rv = r[e];
  const double2 po = p[e];
  if (e >= lo && e < hi) {
    const double alpha = st->alpha;
    double2 xv = x[e - lo];
    xv.x = fma(alpha, po.x, xv.x);
    xv.y = fma(alpha, po.y, xv.y);
    x[e - lo] = xv;
  }
  p[e] = make_double2(fma(beta, po.x, rv.x), fma(beta, po.y, rv.y));
}

// x += alpha p over n complex numbers (the last deferred solution update).
__global__ __launch_bounds__(kBlock) void k_ooc_axpy(size_t n, double2* __restrict__ x, const double2* __restrict__ p,
                                                     const SolverState* __restrict__ st) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const double alpha = st->alpha;
  const double2 pv = p[e];
  double2 xv = x[e];
  xv.x = fma(alpha, pv.x, xv.x);
  xv.y = fma(alpha, pv.y, xv.y);
  x[e] = xv;
}

// alpha = beta = 0: the next S1 starts a new Krylov space (p = r) and adds
// nothing to x.
__global__ void k_ooc_reset_ab(SolverState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->alpha = 0.0;
  st->beta = 0.0;
}

// r -= alpha D^+ t; ||r||^2.
__global__ __launch_bounds__(kBlock) void k_ooc_rupdate(SlabGeom g, CanonGauge U, CanonSpinor t,
                                                        double2* __restrict__ r, double diag,
                                                        const SolverState* __restrict__ st,
                                                        double* __restrict__ partials) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (i < g.ts * g.plane) {
    const int w = g.plane + i;
    double q[24];
    wilson_site<true>(U, t, w, slab_neighbours(g, w), diag, q);
    const double a = st->alpha;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const size_t e = (size_t)i * 12 + k;
      double2 rv = r[e];
      rv.x = fma(-a, q[2 * k], rv.x);
      rv.y = fma(-a, q[2 * k + 1], rv.y);
      r[e] = rv;
      n2 += rv.x * rv.x + rv.y * rv.y;
    }
  }
  store_partial(n2, partials);
}

// ||v||^2 of n sites.
__global__ __launch_bounds__(kBlock) void k_ooc_norm2(int n, const double2* __restrict__ v,
                                                      double* __restrict__ partials) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double n2 = 0.0;
  if (i < n) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double2 a = v[(size_t)i * 12 + k];
      n2 += a.x * a.x + a.y * a.y;
    }
  }
  store_partial(n2, partials);
}

// Copies between pinned host memory and device memory as one kernel: up to
// kMaxSeg segments of 16-byte words, each word one lane's coalesced load and
// store (consecutive lanes, consecutive addresses), eight words in flight per
// thread. Host memory is read and written in place over the host link; one
// launch per slab replaces the slab's separate runtime copies, each of which
// cost tens of microseconds of set-up between transfers.
constexpr int kMaxSeg = 16;   // a slab's largest list: 8 link pieces, 3 window pieces, 3 slabs
struct SegList {
  const uint4* src[kMaxSeg];
  uint4* dst[kMaxSeg];
  size_t start[kMaxSeg + 1];   // prefix sums of the segments' words
  int n;
};

constexpr size_t kMoveBlocks = 128;

__global__ __launch_bounds__(kBlock) void k_ooc_move(SegList L) {
  const size_t total = L.start[L.n];
  const size_t stride = (size_t)gridDim.x * kBlock * 8;
  for (size_t base = (size_t)blockIdx.x * kBlock * 8 + threadIdx.x; base < total; base += stride) {
    uint4 v[8];
    int seg[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const size_t w = base + (size_t)u * kBlock;
      int k = 0;
      while (k + 1 < L.n && w >= L.start[k + 1]) ++k;
      seg[u] = k;
      if (w < total) v[u] = L.src[k][w - L.start[k]];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const size_t w = base + (size_t)u * kBlock;
      if (w < total) L.dst[seg[u]][w - L.start[seg[u]]] = v[u];
    }
  }
}

// ------------------------------------------------------------------ layout

namespace {

constexpr size_t kSpinorSite = 12 * sizeof(double2);   // 192 B
constexpr size_t kLinkSite = 9 * sizeof(double2);      // 144 B per direction

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

struct OocSet {
  double2* U;      // 4 x (ts + 1) planes of links (window planes 0 .. ts)
  double2* win;    // ts + 2 planes of a spinor (window)
  double2* win2;   // a second window
  double2* s[3];   // ts planes each
};

struct OocLayout {
  SolverState* st;
  double* hist;
  double* partials;   // nslab x bps
  OocSet set[2];
  size_t bytes;
};

int blocks_per_slab(int ts, int plane) { return (ts * plane + kBlock - 1) / kBlock; }

OocLayout ooc_layout(void* base, int plane, int T, int ts, int hist_len) {
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t n) -> void* {
    void* p = b ? b + off : nullptr;
    off += align256(n);
    return p;
  };
  OocLayout L{};
  const int nslab = (T + ts - 1) / ts;
  L.st = static_cast<SolverState*>(take(sizeof(SolverState)));
  L.hist = static_cast<double*>(take(sizeof(double) * (size_t)std::max(hist_len, 1)));
  L.partials = static_cast<double*>(take(sizeof(double) * (size_t)nslab * blocks_per_slab(ts, plane)));
  for (int j = 0; j < 2; ++j) {
    L.set[j].U = static_cast<double2*>(take(4 * (size_t)(ts + 1) * plane * kLinkSite));
    L.set[j].win = static_cast<double2*>(take((size_t)(ts + 2) * plane * kSpinorSite));
    L.set[j].win2 = static_cast<double2*>(take((size_t)(ts + 2) * plane * kSpinorSite));
    for (int k = 0; k < 3; ++k) L.set[j].s[k] = static_cast<double2*>(take((size_t)ts * plane * kSpinorSite));
  }
  L.bytes = off;
  return L;
}

// Per-device streams and state mirror, created on first use (default
// priority, non-blocking).
struct OocDevice {
  hipStream_t h2d = nullptr, comp = nullptr, d2h = nullptr;
  SolverState* mirror = nullptr;   // pinned, two slots (one iteration runs ahead)
  hipEvent_t mirror_ev[2] = {nullptr, nullptr};
  bool ready = false;
};
std::mutex g_ooc_mu;
OocDevice g_ooc[64];

#define OOC_TRY(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      snprintf(err, errlen, "%s: %s", #call, hipGetErrorString(e_));                          \
      return WD_ERR_HIP;                                                                      \
    }                                                                                         \
  } while (0)

int ooc_device(OocDevice** out, char* err, size_t errlen) {
  int dev = 0;
  OOC_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    snprintf(err, errlen, "device index %d out of range", dev);
    return WD_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(g_ooc_mu);
  OocDevice& d = g_ooc[dev];
  if (!d.ready) {
    OOC_TRY(hipStreamCreateWithFlags(&d.h2d, hipStreamNonBlocking));
    OOC_TRY(hipStreamCreateWithFlags(&d.comp, hipStreamNonBlocking));
    OOC_TRY(hipStreamCreateWithFlags(&d.d2h, hipStreamNonBlocking));
    OOC_TRY(hipHostMalloc(reinterpret_cast<void**>(&d.mirror), 2 * sizeof(SolverState), hipHostMallocDefault));
    OOC_TRY(hipEventCreateWithFlags(&d.mirror_ev[0], hipEventDisableTiming));
    OOC_TRY(hipEventCreateWithFlags(&d.mirror_ev[1], hipEventDisableTiming));
    d.ready = true;
  }
  *out = &d;
  return WD_OK;
}

// The sweep machinery of one solve.
struct Ooc {
  // lattice
  int T = 0, plane = 0, ts = 0, nslab = 0;
  SlabGeom sg{};
  double diag = 0.0;
  // host fields (canonical complex128)
  const double2* U = nullptr;   // (4, T, plane, 9)
  const double2* b = nullptr;
  double2* x = nullptr;
  // host vectors; the search direction is double-buffered: S1 reads p (its
  // window's halo planes belong to neighbouring slabs) and writes p_next, so
  // that no slab's new p can overwrite a plane another slab has yet to read
  double2 *bp = nullptr, *r = nullptr, *p = nullptr, *p_next = nullptr, *t = nullptr;
  // device
  OocLayout L{};
  OocDevice* dev = nullptr;
  // Per slab, the write-back of the previous sweep and of the current one
  // (out_ev[par] and out_ev[par ^ 1]). No sweep reads host data that it
  // writes itself (the search direction is double-buffered for that), so a
  // slab's copy-in waits only for the previous sweep's write-backs of the
  // slabs it reads: in stream order those finish after every earlier one.
  std::vector<hipEvent_t> out_ev[2];
  int par = 0;
  hipEvent_t in_ready[2]{}, comp_done[2]{}, set_free[2]{};
  int start = 0;                        // first slab of the current sweep order
  char* err = nullptr;
  size_t errlen = 0;

  int t0_of(int k) const { return k * ts; }
  int ts_of(int k) const { return std::min(ts, T - k * ts); }
  size_t sp_plane() const { return (size_t)plane * 12; }   // double2 per spinor plane
  size_t u_plane() const { return (size_t)plane * 9; }     // double2 per link plane (one mu)
  double* partials_of(int k) const { return L.partials + (size_t)k * blocks_per_slab(ts, plane); }
  int total_partials() const { return nslab * blocks_per_slab(ts, plane); }

  // A pending list of copies for one k_ooc_move launch.
  struct Moves {
    SegList L{};
    size_t words = 0;
  };
  bool overflow = false;
  void add(Moves& m, void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    SegList& L = m.L;
    if (L.n == kMaxSeg) {   // cannot happen with the sweeps below (at most 14 pieces)
      overflow = true;
      return;
    }
    L.src[L.n] = static_cast<const uint4*>(src);
    L.dst[L.n] = static_cast<uint4*>(dst);
    L.start[L.n] = m.words;
    m.words += bytes / 16;
    L.n += 1;
    L.start[L.n] = m.words;
  }
  int launch_moves(Moves& m, hipStream_t s) {
    if (overflow) {
      snprintf(err, errlen, "internal: more than %d copy segments for one slab", kMaxSeg);
      return WD_ERR_HIP;
    }
    if (m.L.n == 0) return WD_OK;
    // 128 workgroups (8 x 16 B in flight per thread, 4 MiB in all) keep the
    // host link busy; more of them only crowd the slab kernels that run
    // beside the copies (their host reads hold CU slots for microseconds).
    // Measured on 16^3x32 under 64 MiB: 1024 -> 2.02 s, 128 -> 1.74 s, 32 -> 2.22 s.
    const size_t per = (size_t)kBlock * 8;
    const size_t blocks = std::min<size_t>((m.words + per - 1) / per, kMoveBlocks);
    k_ooc_move<<<(unsigned)blocks, kBlock, 0, s>>>(m.L);
    OOC_TRY(hipGetLastError());
    return WD_OK;
  }
  // planes [first, first + n) of a host spinor field (first may be -1 or T:
  // periodic) into consecutive device planes
  void planes_in(Moves& m, double2* dst, const double2* src, int first, int n) {
    int done = 0;
    while (done < n) {
      const int tp = ((first + done) % T + T) % T;
      const int run = std::min(n - done, T - tp);
      add(m, dst + (size_t)done * sp_plane(), src + (size_t)tp * sp_plane(), (size_t)run * sp_plane() * sizeof(double2));
      done += run;
    }
  }
  void window_in(Moves& m, double2* dst, const double2* src, int k) { planes_in(m, dst, src, t0_of(k) - 1, ts_of(k) + 2); }
  void slab_in(Moves& m, double2* dst, const double2* src, int k) {
    add(m, dst, src + (size_t)t0_of(k) * sp_plane(), (size_t)ts_of(k) * sp_plane() * sizeof(double2));
  }
  void slab_out(Moves& m, double2* dst, const double2* src, int k) {
    add(m, dst + (size_t)t0_of(k) * sp_plane(), src, (size_t)ts_of(k) * sp_plane() * sizeof(double2));
  }
  // links of window planes 0 .. ts (lattice planes t0 - 1 .. t0 + ts - 1) for each mu;
  // in the device window the directions are ts_max + 1 planes apart
  void links_in(Moves& m, double2* dst, int k) {
    const int n = ts_of(k) + 1;
    for (int mu = 0; mu < 4; ++mu) {
      double2* d = dst + (size_t)mu * (ts + 1) * u_plane();
      const double2* src = U + (size_t)mu * T * u_plane();
      int done = 0;
      const int first = t0_of(k) - 1;
      while (done < n) {
        const int tp = ((first + done) % T + T) % T;
        const int run = std::min(n - done, T - tp);
        add(m, d + (size_t)done * u_plane(), src + (size_t)tp * u_plane(), (size_t)run * u_plane() * sizeof(double2));
        done += run;
      }
    }
  }
  SlabGeom geom_of(int k) const {
    SlabGeom g = sg;
    g.ts = ts_of(k);
    return g;
  }
  CanonGauge gauge_of(const OocSet& S) const {
    CanonGauge G;
    G.data = S.U;
    G.V = (size_t)(ts + 1) * plane;
    return G;
  }
  CanonSpinor win_of(const OocSet& S) const {
    CanonSpinor c;
    c.data = S.win;
    return c;
  }
  // every slab launches the full slab's workgroups (a thinner last slab's
  // extra ones store zero partials), so that no stale partial is summed
  unsigned grid_of(int) const { return (unsigned)blocks_per_slab(ts, plane); }

  // One pass over the slabs. `in` queues slab k's copies into buffer set S on
  // the copy-in stream, `kern` its kernel on the kernel stream, `out` its
  // write-back on the copy-out stream. `window`: slab k reads host data of
  // slabs k - 1 and k + 1 too.
  template <class In, class Kern, class Out>
  int sweep(bool window, In in, Kern kern, Out out) {
    if (window) start = (start + 1) % nslab;
    OocDevice& D = *dev;
    for (int i = 0; i < nslab; ++i) {
      const int k = (start + i) % nslab;
      const int j = i & 1;
      OocSet& S = L.set[j];
      const std::vector<hipEvent_t>& prev = out_ev[par];
      OOC_TRY(hipStreamWaitEvent(D.h2d, set_free[j], 0));
      OOC_TRY(hipStreamWaitEvent(D.h2d, prev[k], 0));
      if (window) {
        OOC_TRY(hipStreamWaitEvent(D.h2d, prev[(k + nslab - 1) % nslab], 0));
        OOC_TRY(hipStreamWaitEvent(D.h2d, prev[(k + 1) % nslab], 0));
      }
      Moves mi;
      in(k, S, mi);
      int rc = launch_moves(mi, D.h2d);
      if (rc) return rc;
      OOC_TRY(hipEventRecord(in_ready[j], D.h2d));
      OOC_TRY(hipStreamWaitEvent(D.comp, in_ready[j], 0));
      kern(k, S, D.comp);
      OOC_TRY(hipGetLastError());
      OOC_TRY(hipEventRecord(comp_done[j], D.comp));
      OOC_TRY(hipStreamWaitEvent(D.d2h, comp_done[j], 0));
      Moves mo;
      out(k, S, mo);
      if ((rc = launch_moves(mo, D.d2h))) return rc;
      OOC_TRY(hipEventRecord(out_ev[par ^ 1][k], D.d2h));
      OOC_TRY(hipEventRecord(set_free[j], D.d2h));
    }
    par ^= 1;
    return WD_OK;
  }
  void finalize(int fin, int gate = G_ALWAYS) {
    launch_finalize_n(total_partials(), L.partials, L.st, fin, gate, dev->comp);
  }

  // ---- the sweeps of the solver
  // b' = D^+ b (source) or b (normal); r = p = b'; ||b'||^2 -> bnorm, rho; x = 0 if asked
  int sweep_setup(bool source, bool zero_x) {
    auto in = [&](int k, OocSet& S, Moves& m) {
      if (source) {
        links_in(m, S.U, k);
        window_in(m, S.win, b, k);
      } else {
        slab_in(m, S.s[0], b, k);
      }
    };
    auto kern = [&](int k, OocSet& S, hipStream_t s) {
      if (source)
        k_ooc_apply<true><<<grid_of(k), kBlock, 0, s>>>(geom_of(k), gauge_of(S), win_of(S), S.s[0], diag,
                                                        partials_of(k));
      else
        k_ooc_norm2<<<grid_of(k), kBlock, 0, s>>>(ts_of(k) * plane, S.s[0], partials_of(k));
      if (zero_x) (void)hipMemsetAsync(S.s[1], 0, (size_t)ts_of(k) * sp_plane() * sizeof(double2), s);
    };
    auto out = [&](int k, OocSet& S, Moves& m) {
      slab_out(m, bp, S.s[0], k);
      slab_out(m, r, S.s[0], k);
      slab_out(m, p, S.s[0], k);
      if (zero_x) slab_out(m, x, S.s[1], k);
    };
    int rc = sweep(source, in, kern, out);
    if (rc) return rc;
    finalize(F_BNORM);
    finalize(F_RHO_INIT);
    return WD_OK;
  }
  // t = D v (v = p in the iteration, x for a residual); ||t||^2 -> fin
  int sweep_D(const double2* v, int fin) {
    auto in = [&](int k, OocSet& S, Moves& m) {
      links_in(m, S.U, k);
      window_in(m, S.win, v, k);
    };
    auto kern = [&](int k, OocSet& S, hipStream_t s) {
      k_ooc_apply<false><<<grid_of(k), kBlock, 0, s>>>(geom_of(k), gauge_of(S), win_of(S), S.s[0], diag,
                                                       partials_of(k));
    };
    auto out = [&](int k, OocSet& S, Moves& m) { slab_out(m, t, S.s[0], k); };
    int rc = sweep(true, in, kern, out);
    if (rc) return rc;
    if (fin != F_NONE) finalize(fin);
    return WD_OK;
  }
  // S1: p = r + beta p on the window, t = D p, x += alpha p_old; ||t||^2 -> alpha
  int sweep_s1() {
    auto in = [&](int k, OocSet& S, Moves& m) {
      links_in(m, S.U, k);
      window_in(m, S.win2, r, k);
      window_in(m, S.win, p, k);
      slab_in(m, S.s[0], x, k);
    };
    auto kern = [&](int k, OocSet& S, hipStream_t s) {
      const size_t n_win = (size_t)(ts_of(k) + 2) * sp_plane();
      k_ooc_pwin<<<(unsigned)((n_win + kBlock - 1) / kBlock), kBlock, 0, s>>>(
          n_win, sp_plane(), (size_t)(ts_of(k) + 1) * sp_plane(), S.win2, S.win, S.s[0], L.st);
      k_ooc_apply<false><<<grid_of(k), kBlock, 0, s>>>(geom_of(k), gauge_of(S), win_of(S), S.s[1], diag,
                                                       partials_of(k));
    };
    auto out = [&](int k, OocSet& S, Moves& m) {
      slab_out(m, p_next, S.win + sp_plane(), k);   // the window's own planes
      slab_out(m, t, S.s[1], k);
      slab_out(m, x, S.s[0], k);
    };
    int rc = sweep(true, in, kern, out);
    if (rc) return rc;
    std::swap(p, p_next);
    finalize(F_ALPHA, G_ITER);   // frozen once the solve has stopped (see the loop)
    return WD_OK;
  }
  // S2: r -= alpha D^+ t; ||r||^2 -> beta
  int sweep_s2() {
    auto in = [&](int k, OocSet& S, Moves& m) {
      links_in(m, S.U, k);
      window_in(m, S.win, t, k);
      slab_in(m, S.s[0], r, k);
    };
    auto kern = [&](int k, OocSet& S, hipStream_t s) {
      k_ooc_rupdate<<<grid_of(k), kBlock, 0, s>>>(geom_of(k), gauge_of(S), win_of(S), S.s[0], diag, L.st,
                                                  partials_of(k));
    };
    auto out = [&](int k, OocSet& S, Moves& m) { slab_out(m, r, S.s[0], k); };
    int rc = sweep(true, in, kern, out);
    if (rc) return rc;
    finalize(F_BETA, G_ITER);
    return WD_OK;
  }
  // the deferred x += alpha p of the last iteration
  int sweep_x_update() {
    auto in = [&](int k, OocSet& S, Moves& m) {
      slab_in(m, S.s[0], x, k);
      slab_in(m, S.s[1], p, k);
    };
    auto kern = [&](int k, OocSet& S, hipStream_t s) {
      const size_t n = (size_t)ts_of(k) * sp_plane();
      k_ooc_axpy<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, S.s[0], S.s[1], L.st);
    };
    auto out = [&](int k, OocSet& S, Moves& m) { slab_out(m, x, S.s[0], k); };
    return sweep(false, in, kern, out);
  }
  // r = b' - D^+ t (p = r too when restart); ||r||^2 -> fin
  int sweep_residual(int fin, bool set_p) {
    auto in = [&](int k, OocSet& S, Moves& m) {
      links_in(m, S.U, k);
      window_in(m, S.win, t, k);
      slab_in(m, S.s[0], bp, k);
    };
    auto kern = [&](int k, OocSet& S, hipStream_t s) {
      k_ooc_residual<<<grid_of(k), kBlock, 0, s>>>(geom_of(k), gauge_of(S), win_of(S), S.s[0], S.s[1],
                                                   set_p ? S.s[2] : nullptr, diag, partials_of(k));
    };
    auto out = [&](int k, OocSet& S, Moves& m) {
      slab_out(m, r, S.s[1], k);
      if (set_p) slab_out(m, p, S.s[2], k);
    };
    int rc = sweep(true, in, kern, out);
    if (rc) return rc;
    finalize(fin);
    return WD_OK;
  }
  // the device state, after everything queued so far on the kernel stream,
  // into mirror slot k
  int post_state(int k) {
    OOC_TRY(hipMemcpyAsync(dev->mirror + k, L.st, sizeof(SolverState), hipMemcpyDeviceToHost, dev->comp));
    OOC_TRY(hipEventRecord(dev->mirror_ev[k], dev->comp));
    return WD_OK;
  }
  int wait_state(int k, SolverState* out) {
    OOC_TRY(hipEventSynchronize(dev->mirror_ev[k]));
    *out = dev->mirror[k];
    return WD_OK;
  }
};

}  // namespace

size_t ooc_device_bytes(const int L[4], int slab_planes, int hist_len) {
  const int plane = L[0] * L[1] * L[2];
  return ooc_layout(nullptr, plane, L[3], slab_planes, hist_len).bytes;
}

size_t ooc_host_bytes(const int L[4]) {
  return 5 * (size_t)L[0] * L[1] * L[2] * L[3] * kSpinorSite;   // b', r, p, p_next, t
}

int ooc_slab_planes(const int L[4], size_t device_bytes, int hist_len) {
  const int T = L[3];
  const int cap = std::max(1, (T + 3) / 4);   // at least about four slabs, so that copies overlap
  int best = 0;
  for (int ts = 1; ts <= cap; ++ts)
    if (ooc_device_bytes(L, ts, hist_len) <= device_bytes) best = ts;
  return best;
}

int ooc_solve(const int Ldims[4], double mass, const void* U, const void* b, void* x, const ::wd_cg_params* p,
              ::wd_cg_result* res, void* host_ws, void* dev_ws, size_t dev_ws_bytes, hipStream_t caller,
              char* err, size_t errlen) {
  const auto t0 = std::chrono::steady_clock::now();
  Ooc o;
  o.err = err;
  o.errlen = errlen;
  o.T = Ldims[3];
  o.plane = Ldims[0] * Ldims[1] * Ldims[2];
  o.ts = ooc_slab_planes(Ldims, dev_ws_bytes, p->history_len);
  if (o.ts < 1) {
    snprintf(err, errlen, "device workspace of %zu bytes is below the minimum of %zu (one-plane slabs)", dev_ws_bytes,
             ooc_device_bytes(Ldims, 1, p->history_len));
    return WD_ERR_WORKSPACE;
  }
  o.nslab = (o.T + o.ts - 1) / o.ts;
  for (int i = 0; i < 3; ++i) o.sg.L[i] = Ldims[i];
  o.sg.plane = o.plane;
  o.sg.dx = make_fastdiv(Ldims[0]);
  o.sg.dy = make_fastdiv(Ldims[1]);
  o.sg.dz = make_fastdiv(Ldims[2]);
  o.diag = mass + 4.0;
  o.U = static_cast<const double2*>(U);
  o.b = static_cast<const double2*>(b);
  o.x = static_cast<double2*>(x);
  const size_t V = (size_t)o.plane * o.T;
  double2* hw = static_cast<double2*>(host_ws);
  o.bp = hw;
  o.r = hw + V * 12;
  o.p = hw + 2 * V * 12;
  o.p_next = hw + 3 * V * 12;
  o.t = hw + 4 * V * 12;
  o.L = ooc_layout(dev_ws, o.plane, o.T, o.ts, p->history_len);
  int rc = ooc_device(&o.dev, err, errlen);
  if (rc) return rc;
  OocDevice& D = *o.dev;

  // events of this solve (recorded once so that the first waits pass)
  std::vector<hipEvent_t> evs;
  auto make_ev = [&](hipEvent_t* e) -> int {
    OOC_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    evs.push_back(*e);
    return WD_OK;
  };
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(D.h2d);
    (void)hipStreamSynchronize(D.comp);
    (void)hipStreamSynchronize(D.d2h);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  };
  for (int h = 0; h < 2; ++h) {
    o.out_ev[h].assign(o.nslab, nullptr);
    for (int k = 0; k < o.nslab && !rc; ++k) rc = make_ev(&o.out_ev[h][k]);
  }
  for (int j = 0; j < 2 && !rc; ++j)
    rc = make_ev(&o.in_ready[j]) || make_ev(&o.comp_done[j]) || make_ev(&o.set_free[j]) ? WD_ERR_HIP : WD_OK;
  hipEvent_t caller_ev = nullptr;
  if (!rc) rc = make_ev(&caller_ev);
  if (rc) {
    cleanup();
    return rc;
  }
  // everything after the caller's queued work
  auto run = [&]() -> int {
    OOC_TRY(hipEventRecord(caller_ev, caller));
    OOC_TRY(hipStreamWaitEvent(D.h2d, caller_ev, 0));
    OOC_TRY(hipStreamWaitEvent(D.comp, caller_ev, 0));
    OOC_TRY(hipStreamWaitEvent(D.d2h, caller_ev, 0));
    for (int h = 0; h < 2; ++h)
      for (hipEvent_t e : o.out_ev[h]) OOC_TRY(hipEventRecord(e, D.d2h));
    for (int j = 0; j < 2; ++j) OOC_TRY(hipEventRecord(o.set_free[j], D.d2h));

    launch_init_state(o.L.st, p->tol, 0, 0.0, o.L.hist, p->history_len, D.comp);
    const bool source = p->rhs_mode == WD_RHS_SOURCE;
    int r2 = o.sweep_setup(source, p->zero_guess != 0);
    if (r2) return r2;
    if (!p->zero_guess) {
      // r = b' - D^+ D x0, p = r
      if ((r2 = o.sweep_D(o.x, F_NONE)) || (r2 = o.sweep_residual(F_RHO_INIT, true))) return r2;
    }
    // The host reads the state of one iteration while the next is already
    // queued, so that the copies of consecutive iterations overlap. The
    // alpha and beta updates are gated on the state: an iteration queued past
    // the one that stopped the solve changes no scalar, and its first sweep
    // applies the stopping iteration's deferred x += alpha p (its second
    // sweep leaves a residual that the confirmation below recomputes).
    int slot = 0, wait_slot = 0, queued = 0;
    auto sync_state = [&](SolverState* out) -> int {   // everything queued so far
      int rc = o.post_state(slot);
      if (!rc) rc = o.wait_state(slot, out);
      return rc;
    };
    SolverState st{};
    if ((r2 = sync_state(&st))) return r2;
    int restarts = 0;
    // alpha = beta = 0 (from the state's initialisation): the first S1 sets
    // p = r and adds nothing to x
    bool pending_x = false;   // x lacks the last alpha p
    for (;;) {
      while (st.status == 0 && queued < 2 && st.iter + queued < p->max_iter) {
        if ((r2 = o.sweep_s1()) || (r2 = o.sweep_s2()) || (r2 = o.post_state(slot))) return r2;
        slot ^= 1;
        ++queued;
      }
      if (queued == 0) break;   // max_iter reached
      if ((r2 = o.wait_state(wait_slot, &st))) return r2;
      wait_slot ^= 1;
      --queued;
      pending_x = true;
      if (st.status == 0) continue;
      while (queued > 0) {      // the iteration queued beyond the stop: x is complete after it
        if ((r2 = o.wait_state(wait_slot, &st))) return r2;
        wait_slot ^= 1;
        --queued;
        pending_x = false;
      }
      if (st.status != 1) break;   // breakdown or NaN
      // complete x, then confirm with the residual recomputed from it
      if (pending_x && (r2 = o.sweep_x_update())) return r2;
      pending_x = false;
      if ((r2 = o.sweep_D(o.x, F_NONE)) || (r2 = o.sweep_residual(F_TRUE, true))) return r2;
      if ((r2 = sync_state(&st))) return r2;
      if (st.rho_true <= st.stop2 || st.iter >= p->max_iter || restarts >= 5) break;
      ++restarts;   // the recurrence drifted: continue from the recomputed residual (r = p = it)
      launch_restart(o.L.st, D.comp);
      k_ooc_reset_ab<<<1, 64, 0, D.comp>>>(o.L.st);
      if ((r2 = sync_state(&st))) return r2;
    }
    if (pending_x && st.status >= 0 && (r2 = o.sweep_x_update())) return r2;
    if (st.status == 0 || (st.status == 1 && st.rho_true > st.stop2)) {
      // stopped by max_iter: the true residual of the last iterate
      if ((r2 = o.sweep_D(o.x, F_NONE)) || (r2 = o.sweep_residual(F_TRUE, false))) return r2;
      if ((r2 = sync_state(&st))) return r2;
    }
    if (p->history && p->history_len > 0) {
      const int n = std::min(st.iter, p->history_len);
      if (n > 0) {
        OOC_TRY(hipMemcpyAsync(p->history, o.L.hist, sizeof(double) * n, hipMemcpyDeviceToHost, D.comp));
        OOC_TRY(hipStreamSynchronize(D.comp));
      }
      for (int i = n; i < p->history_len; ++i) p->history[i] = 0.0;
    }
    OOC_TRY(hipStreamSynchronize(D.h2d));
    OOC_TRY(hipStreamSynchronize(D.comp));
    OOC_TRY(hipStreamSynchronize(D.d2h));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    const double bn = st.bnorm2 > 0 ? st.bnorm2 : 1.0;
    int code;
    if (st.status == -3) code = WD_ERR_BREAKDOWN;
    else if (st.status == -4) code = WD_ERR_NAN;
    else if (st.rho_true <= st.stop2 && st.status == 1) code = WD_OK;
    else code = WD_NOT_CONVERGED;
    if (code == WD_ERR_BREAKDOWN) snprintf(err, errlen, "CG breakdown: <p, A p> <= 0");
    if (code == WD_ERR_NAN) snprintf(err, errlen, "NaN or Inf encountered in a CG reduction");
    if (code == WD_NOT_CONVERGED)
      snprintf(err, errlen, "not converged in %d iterations (true rel. residual %.3e)", st.iter,
               std::sqrt(st.rho_true / bn));
    if (res) {
      res->iterations = st.iter;
      res->reliable_updates = 0;
      res->status = code;
      res->two_row_links = 0;
      res->true_rel_res = std::sqrt(st.rho_true / bn);
      res->iter_rel_res = std::sqrt(st.rho / bn);
      res->seconds = secs;
      for (int j = 0; j < 3; ++j) res->kernel_seconds[j] = 0.0;
      res->ooc_slab_planes = o.ts;
      res->ooc_slabs = o.nslab;
    }
    return code;
  };
  rc = run();
  cleanup();
  return rc;
}

}  // namespace wd
