// Internal interface between the host driver (wd_api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/wilson.h"
#include "wd_common.hpp"

namespace wd {

// Device-resident solver state. All scalars of the CG recurrences live here,
// are produced by the one-workgroup finalize kernel of a reduction, and are read by
// the following kernels; the host reads a copy only when it polls.
struct SolverState {
  double rho;        // <r, r> of the current (inner) residual
  double rho_prev;   // value before the last update (beta = rho / rho_prev)
  double alpha;
  double beta;
  double tnorm;      // <t, t> = <p, D^+ D p>
  double bnorm2;     // ||b'||^2
  double stop2;      // (tol ||b'||)^2
  double rho_true;   // ||b' - D^+ D x||^2 from the last FP64 recomputation
  double rho_update; // rho right after the last reliable update (or at the start)
  double su3_dev;    // largest deviation of a link from SU(3) (F_SU3MAX)
  double delta2;     // mixed: also update once rho <= delta2 * rho_update
  int iter;          // inner iterations completed
  int status;        // 0 running, 1 converged, -3 breakdown, -4 NaN/Inf, -5 ring overflow
  int inner_done;    // mixed: inner residual reached the target; update pending
  int last_update;   // iteration of the last reliable update
  int interval;      // reliable-update interval (mixed)
  int rel_updates;   // reliable updates performed
  int restart_on_update;  // refinement: every FP64 recomputation restarts the Krylov space (beta = 0)
  int hist_len;      // capacity of hist
  int npend;         // mixed: p vectors in the ring whose x update is still pending
  int pcur;          // mixed: ring slot of the current search direction p
  int flush_at;      // mixed: fold the ring into x once npend reaches this (0: never)
  int ring_len;      // mixed: slots in the ring (npend never exceeds it; -5 status if it would)
  double* hist;      // per-iteration relative residual (device, in the workspace)
  double* alpha_hist;  // mixed: alpha of the p in each ring slot (device, in the workspace)
};

// When a kernel runs. Decided identically by every workgroup from the state,
// which only finalize kernels change; a reducing kernel and its finalize
// kernel carry the same gate and so run or skip together.
enum Gate : int {
  G_ALWAYS = 0,   // unconditional
  G_ITER = 1,     // a CG iteration: status == 0 and no reliable update pending
  G_RELIABLE = 2, // reliable-update slot: status == 0 and (pending, interval reached, or
                  //   residual reduced by delta since the last update)
  G_FINAL = 3,    // final FP64 recomputation: unconditional
  G_FLUSH = 4,    // mixed: status == 0 and the ring of pending p vectors is nearly full
};

// What the last workgroup does with the reduced sum.
enum Fin : int {
  F_NONE = 0,
  F_BNORM = 1,     // bnorm2 = sum; stop2 = tol^2 sum
  F_RHO_INIT = 2,  // rho = sum (start of the solve)
  F_ALPHA = 3,     // tnorm = sum; alpha = rho / tnorm
  F_BETA = 4,      // rho_prev = rho; rho = sum; beta = rho / rho_prev; iter++; convergence test
  F_RELIABLE = 5,  // rho_true = sum; converged? else rho = sum, beta = rho / rho_prev
                   //   (beta = 0, a restart, if the true residual exceeds twice the iterated one)
  F_TRUE = 6,      // rho_true = sum (final recomputation)
  F_SU3MAX = 7,    // su3_dev = max of the partials (the finalize takes a maximum, not a sum)
  F_ALPHA_RING = 8,  // F_ALPHA, then alpha_hist[npend] = alpha, pcur = npend, npend += 1
};

// Optional pair of events recorded on the launch stream right before and
// right after a kernel (not around its finalize kernel).
struct EventPair {
  hipEvent_t begin;
  hipEvent_t end;
};

struct SpinorBuf {
  void* data;
  float* scale;   // FP16 storage only
  int prec;
};

// Ring of search directions for the deferred solution update of the mixed
// solver: slot j holds a packed spinor at data + j * stride (FP16 scales at
// scale + j * scale_stride). A null `data` means "no ring".
struct RingBuf {
  char* data;
  char* scale;
  long long stride;
  long long scale_stride;
  int prec;
  int len;
  __host__ __device__ SpinorBuf at(int j) const {
    SpinorBuf b;
    b.data = data + j * stride;
    b.scale = scale ? reinterpret_cast<float*>(scale + j * scale_stride) : nullptr;
    b.prec = prec;
    return b;
  }
};

// Several systems in one launch (the lockstep batched solver): the state,
// partials, vectors and ring of system k lie `stride` bytes after those of
// system k - 1; the gauge fields are shared and not offset. The default is a
// single system.
struct Rhs {
  int n = 1;
  long long stride = 0;
};

// ---- launchers (wd_kernels.hip). All asynchronous on `stream`.
// Reset the state: stop2 = tol^2 (scaled by ||b'||^2 at F_BNORM), interval 0 = plain CG.
void launch_init_state(SolverState* st, double tol, int interval, double delta, double* hist, int hist_len,
                       hipStream_t s);
// Continue after a failed final check: status = 0, rho = rho_true.
void launch_restart(SolverState* st, hipStream_t s);
// Make every reliable update a restart (iterative refinement).
void launch_set_restart(SolverState* st, hipStream_t s);
void launch_pack_gauge(const Geom& g, const void* U_c128, int prec, void* out, hipStream_t s);
void launch_pack_spinor(const Geom& g, const void* in, int io_c64, SpinorBuf out, hipStream_t s);
void launch_unpack_spinor(const Geom& g, SpinorBuf in, void* out, int io_c64, hipStream_t s);
void launch_convert(const Geom& g, SpinorBuf in, SpinorBuf out, int gate, SolverState* st, hipStream_t s);
void launch_zero(const Geom& g, SpinorBuf v, int gate, SolverState* st, hipStream_t s);

// out = D in (dagger = 0) or D^+ in on canonical complex128 fields.
void launch_wilson_canonical(const Geom& g, const void* U, const void* in, void* out, double mass, int dagger,
                             hipStream_t s);
// out = D in / D^+ in on packed fields of one precision; optional reduction of ||out||^2.
// With `ring`, the input is ring slot st->npend instead of `in` (mixed solver).
void launch_wilson_packed(const Geom& g, int prec, const void* U, SpinorBuf in, SpinorBuf out, double mass,
                          int dagger, int gate, int fin, SolverState* st, double* partials, hipStream_t s,
                          const EventPair* ev = nullptr, int rows2 = 0, const RingBuf* ring = nullptr,
                          Rhs rb = {});
// Two-row (12-real) 16-bit gauge copy (BF16 or FP16), tiled lattices; the
// tiled 16-bit kernels rebuild row 2 from unitarity (rows2 = 1).
void launch_pack_gauge_rows2(const Geom& g, const void* U_c128, int prec, void* out, hipStream_t s);
// su3_dev = largest deviation of a canonical complex128 gauge field from SU(3).
void launch_su3_check(const Geom& g, const void* U_c128, SolverState* st, double* partials, hipStream_t s);
// Plain CG (FP64 or FP32 storage): q = D^+ t (never stored); r -= alpha q;
// x += alpha p; ||r||^2 -> F_BETA.
void launch_cg_update(const Geom& g, int prec, const void* U, SpinorBuf t, SpinorBuf r, SpinorBuf p, SpinorBuf x,
                      double mass, SolverState* st, double* partials, hipStream_t s, const EventPair* ev = nullptr,
                      int rows2 = 0);
// out = low(b - D^+ t) with FP64 arithmetic on FP64 fields; ||b - D^+ t||^2 -> fin.
void launch_residual(const Geom& g, const void* U64, SpinorBuf t64, SpinorBuf b64, SpinorBuf out, double mass,
                     int gate, int fin, SolverState* st, double* partials, hipStream_t s, Rhs rb = {});
// p = r + beta p
void launch_p_update(const Geom& g, SpinorBuf r, SpinorBuf p, SolverState* st, hipStream_t s,
                     const EventPair* ev = nullptr);
// Mixed solver with a ring of search directions (the deferred x update):
//   t = D ring[npend] (+ ||t||^2 -> F_ALPHA_RING) is launch_wilson_packed with `ring`;
//   q = D^+ t (never stored); r -= alpha q; ||r||^2 -> F_BETA.
void launch_r_update(const Geom& g, int prec, const void* U, SpinorBuf t, SpinorBuf r, double mass, SolverState* st,
                     double* partials, hipStream_t s, const EventPair* ev = nullptr, int rows2 = 0,
                     Rhs rb = {});
//   ring[npend] = r + beta ring[pcur] (in place when the two slots coincide).
void launch_p_update_ring(const Geom& g, SpinorBuf r, const RingBuf& ring, SolverState* st, hipStream_t s,
                          const EventPair* ev = nullptr, Rhs rb = {});
//   x(FP64) += sum_{j < npend} alpha_hist[j] ring[j], accumulated in FP64.
void launch_accumulate_ring(const Geom& g, SpinorBuf x64, const RingBuf& ring, int gate, SolverState* st,
                            hipStream_t s, Rhs rb = {});
//   npend = 0 when G_FLUSH is open (after launch_accumulate_ring with G_FLUSH).
void launch_ring_reset(SolverState* st, hipStream_t s, Rhs rb = {});
// dst[k] = the state of system k (a contiguous copy for the host to read).
void launch_gather_states(const SolverState* st, Rhs rb, SolverState* dst, hipStream_t s);
//   alpha_hist, flush_at and ring_len of the state.
void launch_set_ring(SolverState* st, double* alpha_hist, int flush_at, int ring_len, hipStream_t s);
// x(FP64) += xhat; xhat = 0
void launch_accumulate(const Geom& g, SpinorBuf x64, SpinorBuf xhat, int gate, SolverState* st, hipStream_t s);
// Sum of the first n per-workgroup partials, then the state update fin (gated).
void launch_finalize_n(int n, double* partials, SolverState* st, int fin, int gate, hipStream_t s);
// ||v||^2 -> fin
void launch_norm2(const Geom& g, SpinorBuf v, int gate, int fin, SolverState* st, double* partials, hipStream_t s);
// Workspace of the batched persistent solver (wd_batched.hip).
size_t batched_workspace_bytes(const Geom& g, int nrhs, int hist_len, int inner_prec);
// Batched solve after argument validation; writes a message to err on failure.
int batched_solve(const Geom& g, double mass, const void* U, int nrhs, const void* B, void* X,
                  const ::wd_cg_params* p, ::wd_cg_result* res, void* ws, hipStream_t s, char* err, size_t errlen);

// ---- gauge-covariant Laplacian on colour vectors (wd_laplace.hip); packed
// colour fields are FP64, 3 words per site; links are the FP64 packed gauge field.
// out = L in on canonical (V, 3) complex128 fields
void launch_lap_canonical(const Geom& g, const void* U, const void* in, void* out, double m2, hipStream_t s);
// canonical (V, 3) colour field (complex128, or complex64 if c64) <-> packed FP64
void launch_lap_pack(const Geom& g, const void* in, int c64, void* out, hipStream_t s);
void launch_lap_unpack(const Geom& g, const void* in, void* out, int c64, hipStream_t s);
// t = L p; Re <p, t> -> fin (F_ALPHA in the solver, F_NONE for a plain application)
void launch_lap_packed(const Geom& g, const void* U, const void* p, void* t, double m2, int gate, int fin,
                       SolverState* st, double* partials, hipStream_t s, const EventPair* ev = nullptr);
// r = b - L x; ||r||^2 -> fin
void launch_lap_residual(const Geom& g, const void* U, const void* x, const void* b, void* r, double m2, int gate,
                         int fin, SolverState* st, double* partials, hipStream_t s);
// x += alpha p; r -= alpha t; ||r||^2 -> F_BETA (gate G_ITER)
void launch_lap_update(const Geom& g, const void* t, void* r, const void* p, void* x, SolverState* st,
                       double* partials, hipStream_t s, const EventPair* ev = nullptr);
// p = r + beta p (gate G_ITER)
void launch_lap_p_update(const Geom& g, const void* r, void* p, SolverState* st, hipStream_t s,
                         const EventPair* ev = nullptr);
// ||v||^2 -> fin
void launch_lap_norm2(const Geom& g, const void* v, int fin, SolverState* st, double* partials, hipStream_t s);
// dst = src, or dst = 0 when src is null (gated)
void launch_lap_copy(const Geom& g, const void* src, void* dst, int gate, SolverState* st, hipStream_t s);

// ---- out-of-core FP64 CG (wd_ooc.hip): host-resident fields streamed in t-slabs.
// Device bytes for slabs of `slab_planes` time planes; host bytes of the CG vectors.
size_t ooc_device_bytes(const int L[4], int slab_planes, int hist_len);
size_t ooc_host_bytes(const int L[4]);
// Thickest slab (planes) that fits `device_bytes`, at most about a quarter of Lt; 0 if none.
int ooc_slab_planes(const int L[4], size_t device_bytes, int hist_len);
// The solve after argument validation; writes a message to err on a non-zero return.
int ooc_solve(const int L[4], double mass, const void* U, const void* b, void* x, const ::wd_cg_params* p,
              ::wd_cg_result* res, void* host_ws, void* dev_ws, size_t dev_ws_bytes, hipStream_t caller, char* err,
              size_t errlen);

// ---- streaming kernels (wd_stream.hip): kind 0 copy, 1 read (XOR per workgroup
// into dst), 2 write zeros; bytes a multiple of 16.
void launch_stream(int kind, const void* src, void* dst, size_t bytes, hipStream_t s);
unsigned stream_read_partials(size_t bytes);

// G(a, b) force on canonical complex128 spinors -> canonical complex128 links.
void launch_force(const Geom& g, const void* a, const void* b, double coeff, int accumulate, void* F, hipStream_t s);

}  // namespace wd
