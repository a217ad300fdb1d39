// C ABI of the Wilson-Dirac library: argument validation, workspace layout,
// and the host side of the conjugate-gradient drivers.
//
// The paper's host part owns the CG vectors and evaluates the stopping test
// on the host, invoking the accelerator once per operator application
// (Sec. 3.1, Sec. 3.1.1). Here every vector and every CG scalar stays in HBM:
// the reductions finish on the device (a one-workgroup finalize kernel), alpha and beta
// never leave it, and the host only enqueues chunks of iterations and polls a
// copy of the device state between chunks. A device-side status flag turns
// the kernels of iterations enqueued past convergence into no-ops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/wilson.h"
#include "wd_internal.hpp"

using namespace wd;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail(WD_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_));     \
  } while (0)

int check_lattice(const wd_lattice* lat) {
  if (!lat) return fail(WD_ERR_INVALID, "lattice is NULL");
  long long v = 1;
  for (int i = 0; i < 4; ++i) {
    if (lat->L[i] < 2) return fail(WD_ERR_INVALID, "lattice extent L[%d] = %d (must be >= 2)", i, lat->L[i]);
    if (lat->L[i] > (1 << 20)) return fail(WD_ERR_INVALID, "lattice extent L[%d] = %d too large", i, lat->L[i]);
    v *= lat->L[i];
  }
  if (v > (1ll << 28)) return fail(WD_ERR_INVALID, "lattice volume %lld exceeds 2^28 sites", v);
  return WD_OK;
}

// Geometry of the packed (solver-internal) fields: tiled site order when every
// extent is a multiple of 4.
Geom packed_geom(const wd_lattice* lat) { return make_geom(lat->L, true); }

bool valid_prec(int p) { return p == WD_F64 || p == WD_F32 || p == WD_BF16 || p == WD_F16 || p == WD_I8; }

// Low-precision storage whose links may be kept as two rows (and whose tiled
// kernels stage 16-bit or 8-bit words).
bool narrow_prec(int p) { return p == WD_BF16 || p == WD_F16 || p == WD_I8; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

// Carves a caller-owned workspace into 256-byte aligned pieces.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t n) {
    void* p = base ? base + off : nullptr;
    off += align_up(n);
    return p;
  }
};

SpinorBuf take_spinor(Carver& c, int prec, const Geom& g) {
  SpinorBuf b;
  b.prec = prec;
  b.data = c.take(spinor_bytes(prec, g.Vpad));
  b.scale = spinor_scale_bytes(prec, g.Vpad) ? static_cast<float*>(c.take(spinor_scale_bytes(prec, g.Vpad))) : nullptr;
  return b;
}

// Layout of the single-RHS solver workspace. With base == nullptr it only
// measures.
struct CgWorkspace {
  SolverState* st;
  double* partials;
  double* hist;
  void* U64;
  void* Ulow;
  SpinorBuf b64, x64, r64, p64, t64;   // plain FP64 CG (r64/p64 unused by mixed)
  SpinorBuf rh, th;                     // mixed: low-precision r, t
  RingBuf ring;                         // mixed: search directions since the last x update
  double* alpha_hist;                   // mixed: their alphas
  size_t bytes;
};

constexpr int kSlotEvery = 5;   // mixed: a reliable-update slot after every 5th enqueued iteration
constexpr size_t kRingBudget = size_t(8) << 30;   // default ring: at most 8 GiB

int reliable_interval_of(const wd_cg_params* p) {
  if (p->scheme == WD_ITERATIVE_REFINEMENT) return 1 << 30;   // no periodic recomputation
  return p->reliable_interval > 0 ? p->reliable_interval : 50;
}

// Besides every `interval` iterations, a mixed solve recomputes the residual
// whenever the iterated residual has fallen by this factor since the last
// update, so that the low-precision drift (~ unit roundoff x the residual at
// the last update) stays well below the residual being iterated.
double reliable_delta(const wd_cg_params* p) {
  if (p->inner_tol > 0.0) return p->inner_tol;
  if (p->scheme == WD_ITERATIVE_REFINEMENT) return 0.1;
  const int P = p->inner_prec;
  return (P == WD_BF16 || P == WD_I8) ? 0.1 : (P == WD_F16) ? 1e-2 : 1e-4;
}

// Ring slots: the caller's ring_len, else enough that the ring is folded only
// at reliable updates (interval + kSlotEvery), within kRingBudget bytes.
int ring_length(const wd_cg_params* p, const Geom& g) {
  if (p->ring_len > 0) return p->ring_len;
  const size_t per = align_up(spinor_bytes(p->inner_prec, g.Vpad)) + align_up(spinor_scale_bytes(p->inner_prec, g.Vpad));
  const long long by_mem = (long long)(kRingBudget / per);
  const long long want = std::min<long long>((long long)reliable_interval_of(p) + kSlotEvery, by_mem);
  return (int)std::max<long long>(8, std::min<long long>(256, want));
}

CgWorkspace layout_cg(void* base, const Geom& g, int inner, int hist_len, int ring_len) {
  Carver c(base);
  CgWorkspace w{};
  w.st = static_cast<SolverState*>(c.take(sizeof(SolverState)));
  w.partials = static_cast<double*>(c.take(sizeof(double) * (size_t)g.nblocks));
  w.hist = static_cast<double*>(c.take(sizeof(double) * (size_t)(hist_len > 0 ? hist_len : 1)));
  w.U64 = c.take(gauge_bytes(P_F64, g.Vpad));
  w.b64 = take_spinor(c, P_F64, g);
  w.x64 = take_spinor(c, P_F64, g);
  w.t64 = take_spinor(c, P_F64, g);
  if (inner == WD_F64) {
    w.r64 = take_spinor(c, P_F64, g);
    w.p64 = take_spinor(c, P_F64, g);
  } else {
    w.Ulow = c.take(gauge_bytes(inner, g.Vpad));
    w.rh = take_spinor(c, inner, g);
    w.th = take_spinor(c, inner, g);
    w.alpha_hist = static_cast<double*>(c.take(sizeof(double) * (size_t)ring_len));
    w.ring.prec = inner;
    w.ring.len = ring_len;
    w.ring.stride = (long long)align_up(spinor_bytes(inner, g.Vpad));
    w.ring.data = static_cast<char*>(c.take((size_t)w.ring.stride * ring_len));
    if (spinor_scale_bytes(inner, g.Vpad)) {
      w.ring.scale_stride = (long long)align_up(spinor_scale_bytes(inner, g.Vpad));
      w.ring.scale = static_cast<char*>(c.take((size_t)w.ring.scale_stride * ring_len));
    }
  }
  w.bytes = c.off;
  return w;
}

// ---- lockstep batched solver (WD_BATCH_LOCKSTEP): the shared gauge copies,
// a contiguous copy of the systems' states for the host, then one region per
// system (the single-system layout without the gauge fields) at a fixed stride.
constexpr int kMaxBatch = 16;

struct LockstepWorkspace {
  void* U64;
  void* Ulow;
  SolverState* states;
  CgWorkspace sys0;    // system 0; its U64 / Ulow are the shared copies
  long long stride;    // bytes from one system's region to the next
  size_t bytes;
};

// Ring slots per system: the single-system rule, with a budget of 16 GiB
// shared by the systems (16 systems on 32^3 x 64: 16 slots each, a fold every
// ~12 iterations; on 24^3 x 48: 31 slots, more than the reliable updates leave
// pending).
constexpr size_t kBatchRingBudget = size_t(16) << 30;
int ring_length_batch(const wd_cg_params* p, const Geom& g, int nrhs) {
  if (p->ring_len > 0) return p->ring_len;
  const size_t per = align_up(spinor_bytes(p->inner_prec, g.Vpad)) + align_up(spinor_scale_bytes(p->inner_prec, g.Vpad));
  const long long by_mem = (long long)(kBatchRingBudget / ((size_t)nrhs * per));
  const long long want = std::min<long long>((long long)reliable_interval_of(p) + kSlotEvery, by_mem);
  return (int)std::max<long long>(8, std::min<long long>(256, want));
}

LockstepWorkspace layout_lockstep(void* base, const Geom& g, int inner, int ring_len, int nrhs) {
  Carver c(base);
  LockstepWorkspace L{};
  L.U64 = c.take(gauge_bytes(P_F64, g.Vpad));
  L.Ulow = c.take(gauge_bytes(inner, g.Vpad));
  L.states = static_cast<SolverState*>(c.take(sizeof(SolverState) * kMaxBatch));
  const size_t start = c.off;
  CgWorkspace& w = L.sys0;
  w.st = static_cast<SolverState*>(c.take(sizeof(SolverState)));
  w.partials = static_cast<double*>(c.take(sizeof(double) * (size_t)g.nblocks));
  w.hist = static_cast<double*>(c.take(sizeof(double)));
  w.b64 = take_spinor(c, P_F64, g);
  w.x64 = take_spinor(c, P_F64, g);
  w.t64 = take_spinor(c, P_F64, g);
  w.rh = take_spinor(c, inner, g);
  w.th = take_spinor(c, inner, g);
  w.alpha_hist = static_cast<double*>(c.take(sizeof(double) * (size_t)ring_len));
  w.ring.prec = inner;
  w.ring.len = ring_len;
  w.ring.stride = (long long)align_up(spinor_bytes(inner, g.Vpad));
  w.ring.data = static_cast<char*>(c.take((size_t)w.ring.stride * ring_len));
  if (spinor_scale_bytes(inner, g.Vpad)) {
    w.ring.scale_stride = (long long)align_up(spinor_scale_bytes(inner, g.Vpad));
    w.ring.scale = static_cast<char*>(c.take((size_t)w.ring.scale_stride * ring_len));
  }
  w.U64 = L.U64;
  w.Ulow = L.Ulow;
  L.stride = (long long)(c.off - start);
  c.off = start + (size_t)L.stride * (size_t)nrhs;
  L.bytes = c.off;
  return L;
}

template <class T>
T* shift_ptr(T* p, long long off) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<char*>(p) + off) : p;
}
SpinorBuf shift_buf(SpinorBuf b, long long off) {
  b.data = shift_ptr(static_cast<char*>(b.data), off);
  b.scale = shift_ptr(b.scale, off);
  return b;
}

// System k's region seen as a single-system workspace.
CgWorkspace system_view(const LockstepWorkspace& L, int k) {
  const long long off = (long long)k * L.stride;
  CgWorkspace w = L.sys0;
  w.st = shift_ptr(w.st, off);
  w.partials = shift_ptr(w.partials, off);
  w.hist = shift_ptr(w.hist, off);
  w.b64 = shift_buf(w.b64, off);
  w.x64 = shift_buf(w.x64, off);
  w.t64 = shift_buf(w.t64, off);
  w.rh = shift_buf(w.rh, off);
  w.th = shift_buf(w.th, off);
  w.alpha_hist = shift_ptr(w.alpha_hist, off);
  w.ring.data = shift_ptr(w.ring.data, off);
  w.ring.scale = shift_ptr(w.ring.scale, off);
  return w;
}

// The lockstep kernels exist for 16- and 8-bit storage with reliable updates
// on the tiled site order.
bool lockstep_possible(const Geom& g, const wd_cg_params* p) {
  return g.tiled && narrow_prec(p->inner_prec) && p->scheme == WD_RELIABLE_UPDATE;
}
bool use_lockstep(const Geom& g, const wd_cg_params* p) {
  return p->batch_schedule == WD_BATCH_LOCKSTEP || (p->batch_schedule == WD_BATCH_AUTO && lockstep_possible(g, p));
}

// The blocking solvers share per-device pinned state mirrors and event sets,
// so solves on one device are serialised: a call from a second host thread
// waits until the first has returned.
std::mutex g_solve_mu[64];

int lock_device(std::unique_lock<std::mutex>& lk) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(WD_ERR_HIP, "device index %d out of range", dev);
  lk = std::unique_lock<std::mutex>(g_solve_mu[dev]);
  return WD_OK;
}

// Host mirrors of the device state, pinned, one pair per device.
struct HostMirror {
  SolverState* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
};
std::mutex g_mirror_mu;
HostMirror g_mirror[64];

int get_mirror(HostMirror** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(WD_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mirror_mu);
  HostMirror& m = g_mirror[dev];
  if (!m.buf[0]) {
    for (int i = 0; i < 2; ++i) {
      HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&m.buf[i]), sizeof(SolverState), hipHostMallocDefault));
      HIP_TRY(hipEventCreateWithFlags(&m.ev[i], hipEventDisableTiming));
    }
  }
  *out = &m;
  return WD_OK;
}

// Events for params->profile: per device, 3 kernel kinds x kClockSamples
// iterations x (begin, end), created on first use.
constexpr int kClockSamples = 64;
struct KernelClock {
  EventPair ev[3][kClockSamples];
  bool ready = false;
};
KernelClock g_clock[64];

int get_clock(KernelClock** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(WD_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mirror_mu);
  KernelClock& c = g_clock[dev];
  if (!c.ready) {
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < kClockSamples; ++i) {
        HIP_TRY(hipEventCreate(&c.ev[k][i].begin));
        HIP_TRY(hipEventCreate(&c.ev[k][i].end));
      }
    c.ready = true;
  }
  *out = &c;
  return WD_OK;
}

// Event pair of kernel kind k at enqueued iteration i, or null when not sampled.
const EventPair* clock_at(KernelClock* c, int k, int i) {
  return (c && i < kClockSamples) ? &c->ev[k][i] : nullptr;
}

// Average device time per kernel kind over the sampled iterations (stream
// synchronised); kinds beyond `kinds` were not launched and read 0.
void clock_read(KernelClock* c, int n, int kinds, double out[3]) {
  for (int k = 0; k < 3; ++k) out[k] = 0.0;
  if (!c) return;
  n = std::min(n, kClockSamples);
  for (int k = 0; k < kinds; ++k) {
    double sum = 0.0;
    int cnt = 0;
    for (int i = 0; i < n; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[k][i].begin, c->ev[k][i].end) == hipSuccess) {
        sum += ms * 1e-3;
        ++cnt;
      }
    }
    out[k] = cnt ? sum / cnt : 0.0;
  }
}

int fill_result(wd_cg_result* res, const SolverState& st, int code, double secs, double iter_rel) {
  if (!res) return code;
  res->iterations = st.iter;
  res->reliable_updates = st.rel_updates;
  res->status = code;
  const double bn = st.bnorm2 > 0 ? st.bnorm2 : 1.0;
  res->true_rel_res = std::sqrt(st.rho_true / bn);
  res->iter_rel_res = iter_rel;
  res->seconds = secs;
  return code;
}
// (kernel_seconds is filled by the drivers before fill_result)

int status_to_code(int status) {
  if (status == 1) return WD_OK;
  if (status == -3) return fail(WD_ERR_BREAKDOWN, "CG breakdown: <p, A p> <= 0 (A not positive definite)");
  if (status == -4) return fail(WD_ERR_NAN, "NaN or Inf encountered in a CG reduction");
  if (status == -5) return fail(WD_ERR_HIP, "internal: search-direction ring overflow");
  return WD_OK;
}

int validate_params(const wd_cg_params* p) {
  if (!p) return fail(WD_ERR_INVALID, "params is NULL");
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return fail(WD_ERR_INVALID, "tol = %g must be positive", p->tol);
  if (p->max_iter < 1) return fail(WD_ERR_INVALID, "max_iter = %d must be >= 1", p->max_iter);
  if (!valid_prec(p->inner_prec)) return fail(WD_ERR_INVALID, "inner_prec = %d unknown", p->inner_prec);
  if (p->reliable_interval < 0) return fail(WD_ERR_INVALID, "reliable_interval = %d", p->reliable_interval);
  if (p->rhs_mode != WD_RHS_SOURCE && p->rhs_mode != WD_RHS_NORMAL)
    return fail(WD_ERR_INVALID, "rhs_mode = %d unknown", p->rhs_mode);
  if (p->io_dtype != WD_C128 && p->io_dtype != WD_C64) return fail(WD_ERR_INVALID, "io_dtype = %d unknown", p->io_dtype);
  if (p->history_len < 0) return fail(WD_ERR_INVALID, "history_len = %d", p->history_len);
  if (p->history_len > 0 && !p->history) return fail(WD_ERR_INVALID, "history is NULL but history_len > 0");
  if (p->scheme != WD_RELIABLE_UPDATE && p->scheme != WD_ITERATIVE_REFINEMENT)
    return fail(WD_ERR_INVALID, "scheme = %d unknown", p->scheme);
  if (!(p->inner_tol >= 0.0 && p->inner_tol < 1.0)) return fail(WD_ERR_INVALID, "inner_tol = %g not in [0, 1)", p->inner_tol);
  if (p->ring_len != 0 && (p->ring_len < 8 || p->ring_len > 256))
    return fail(WD_ERR_INVALID, "ring_len = %d must be 0 or in [8, 256]", p->ring_len);
  if (p->batch_schedule != WD_BATCH_AUTO && p->batch_schedule != WD_BATCH_PERSISTENT &&
      p->batch_schedule != WD_BATCH_LOCKSTEP)
    return fail(WD_ERR_INVALID, "batch_schedule = %d unknown", p->batch_schedule);
  return WD_OK;
}

// The documented workspace size: for nrhs = 1 it covers both cg_solve and a
// single-system cg_solve_batched.
size_t required_bytes(const Geom& g, const wd_cg_params* p, int nrhs) {
  size_t batched = batched_workspace_bytes(g, nrhs, p->history_len, p->inner_prec);
  if (use_lockstep(g, p) && lockstep_possible(g, p))
    batched = std::max(batched, layout_lockstep(nullptr, g, p->inner_prec, ring_length_batch(p, g, nrhs), nrhs).bytes);
  if (nrhs == 1)
    return std::max(layout_cg(nullptr, g, p->inner_prec, p->history_len, ring_length(p, g)).bytes, batched);
  return batched;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

const char* wd_last_error(void) { return g_err.c_str(); }

int wd_device_count(void) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return fail(WD_ERR_HIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
  return n;
}

static int apply_common(const wd_lattice* lat, double mass, const void* U, const void* psi, void* out, void* stream,
                        int dagger) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (!U || !psi || !out) return fail(WD_ERR_INVALID, "NULL field pointer");
  if (psi == out) return fail(WD_ERR_INVALID, "in and out must not alias");
  if (!std::isfinite(mass)) return fail(WD_ERR_INVALID, "mass is not finite");
  const Geom g = make_geom(lat->L, false);
  launch_wilson_canonical(g, U, psi, out, mass, dagger, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

int wilson_apply(const wd_lattice* lat, double mass, const void* U, const void* psi, void* out, void* stream) {
  return apply_common(lat, mass, U, psi, out, stream, 0);
}

int wilson_apply_dagger(const wd_lattice* lat, double mass, const void* U, const void* psi, void* out,
                        void* stream) {
  return apply_common(lat, mass, U, psi, out, stream, 1);
}

// prec of a packed gauge field, possibly with WD_TWO_ROW_LINKS: returns the
// precision, sets *rows2; fails unless two rows are asked for a 16-bit field on
// a tiled lattice.
static int gauge_format(const wd_lattice* lat, int32_t prec, int* rows2) {
  *rows2 = (prec & WD_TWO_ROW_LINKS) ? 1 : 0;
  const int p = prec & ~WD_TWO_ROW_LINKS;
  if (!valid_prec(p)) return fail(WD_ERR_INVALID, "prec = %d unknown", prec);
  if (*rows2 && !narrow_prec(p))
    return fail(WD_ERR_INVALID, "two-row links exist for WD_BF16, WD_F16 and WD_I8 only");
  if (*rows2 && !packed_geom(lat).tiled)
    return fail(WD_ERR_INVALID, "two-row links need every lattice extent to be a multiple of 4");
  return WD_OK;
}

size_t wd_gauge_bytes(const wd_lattice* lat, int32_t prec) {
  if (check_lattice(lat)) return 0;
  int rows2 = 0;
  if (gauge_format(lat, prec, &rows2)) return 0;
  const int p = prec & ~WD_TWO_ROW_LINKS;
  const Geom g = packed_geom(lat);
  return rows2 ? (size_t)g.Vpad * 4 * 6 * 4 : gauge_bytes(p, g.Vpad);
}

size_t wd_spinor_bytes(const wd_lattice* lat, int32_t prec) {
  if (check_lattice(lat)) return 0;
  if (!valid_prec(prec)) { fail(WD_ERR_INVALID, "prec = %d unknown", prec); return 0; }
  const Geom g = packed_geom(lat);
  return spinor_bytes(prec, g.Vpad) + spinor_scale_bytes(prec, g.Vpad);
}

static SpinorBuf packed_view(const Geom& g, int prec, const void* p) {
  SpinorBuf b;
  b.prec = prec;
  b.data = const_cast<void*>(p);
  b.scale = spinor_scale_bytes(prec, g.Vpad)
                ? reinterpret_cast<float*>(static_cast<char*>(b.data) + spinor_bytes(prec, g.Vpad))
                : nullptr;
  return b;
}

int wd_pack_gauge(const wd_lattice* lat, const void* U, int32_t prec, void* out, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  int rows2 = 0;
  if ((rc = gauge_format(lat, prec, &rows2))) return rc;
  if (!U || !out) return fail(WD_ERR_INVALID, "NULL field pointer");
  const int p = prec & ~WD_TWO_ROW_LINKS;
  if (rows2) launch_pack_gauge_rows2(packed_geom(lat), U, p, out, as_stream(stream));
  else launch_pack_gauge(packed_geom(lat), U, p, out, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

int wd_pack_spinor(const wd_lattice* lat, const void* in, int32_t io_dtype, int32_t prec, void* out, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (!valid_prec(prec)) return fail(WD_ERR_INVALID, "prec = %d unknown", prec);
  if (io_dtype != WD_C128 && io_dtype != WD_C64) return fail(WD_ERR_INVALID, "io_dtype = %d unknown", io_dtype);
  if (!in || !out) return fail(WD_ERR_INVALID, "NULL field pointer");
  const Geom g = packed_geom(lat);
  launch_pack_spinor(g, in, io_dtype == WD_C64, packed_view(g, prec, out), as_stream(stream));
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

int wd_unpack_spinor(const wd_lattice* lat, const void* in, int32_t prec, void* out, int32_t io_dtype,
                     void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (!valid_prec(prec)) return fail(WD_ERR_INVALID, "prec = %d unknown", prec);
  if (io_dtype != WD_C128 && io_dtype != WD_C64) return fail(WD_ERR_INVALID, "io_dtype = %d unknown", io_dtype);
  if (!in || !out) return fail(WD_ERR_INVALID, "NULL field pointer");
  const Geom g = packed_geom(lat);
  launch_unpack_spinor(g, packed_view(g, prec, in), out, io_dtype == WD_C64, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

int wilson_apply_packed(const wd_lattice* lat, double mass, int32_t prec, const void* U_packed,
                        const void* in_packed, void* out_packed, int32_t dagger, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  int rows2 = 0;
  if ((rc = gauge_format(lat, prec, &rows2))) return rc;
  if (!U_packed || !in_packed || !out_packed) return fail(WD_ERR_INVALID, "NULL field pointer");
  if (in_packed == out_packed) return fail(WD_ERR_INVALID, "in and out must not alias");
  const int p = prec & ~WD_TWO_ROW_LINKS;
  const Geom g = packed_geom(lat);
  launch_wilson_packed(g, p, U_packed, packed_view(g, p, in_packed), packed_view(g, p, out_packed), mass,
                       dagger ? 1 : 0, G_ALWAYS, F_NONE, nullptr, nullptr, as_stream(stream), nullptr, rows2);
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

int wilson_force(const wd_lattice* lat, const void* a, const void* b, double coeff, int32_t accumulate, void* F,
                 void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (!a || !b || !F) return fail(WD_ERR_INVALID, "NULL field pointer");
  if (!std::isfinite(coeff)) return fail(WD_ERR_INVALID, "coeff is not finite");
  launch_force(make_geom(lat->L, false), a, b, coeff, accumulate ? 1 : 0, F, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

size_t wd_workspace_bytes(const wd_lattice* lat, const wd_cg_params* params, int32_t nrhs) {
  if (check_lattice(lat)) return 0;
  if (validate_params(params)) return 0;
  if (nrhs < 1) { fail(WD_ERR_INVALID, "nrhs = %d must be >= 1", nrhs); return 0; }
  if (nrhs > 16) { fail(WD_ERR_INVALID, "nrhs = %d exceeds 16", nrhs); return 0; }
  return required_bytes(packed_geom(lat), params, nrhs);
}

}  // extern "C"

// ============================================================ CG drivers

namespace {

// Polls device state between chunks of enqueued iterations. Two chunks are
// in flight: while the host waits for chunk k, chunk k + 1 is already queued.
// Without a pinned mirror (m == nullptr: the allocation-free solve) a wait
// synchronises the stream and copies the state into host memory directly, so
// it sees the state after every chunk posted so far.
struct Poller {
  HostMirror* m;
  SolverState* dst;
  hipStream_t s;
  int slot = 0;
  int pending = 0;
  SolverState* src = nullptr;
  int post(SolverState* st) {
    if (!m) {
      src = st;
      ++pending;
      return WD_OK;
    }
    HIP_TRY(hipMemcpyAsync(m->buf[slot], st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(m->ev[slot], s));
    slot ^= 1;
    ++pending;
    return WD_OK;
  }
  // Wait for the oldest posted copy.
  int wait(SolverState* out) {
    if (!m) {
      HIP_TRY(hipMemcpyAsync(out, src, sizeof(SolverState), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      --pending;
      return WD_OK;
    }
    const int k = pending == 2 ? slot : slot ^ 1;
    HIP_TRY(hipEventSynchronize(m->ev[k]));
    *out = *m->buf[k];
    --pending;
    return WD_OK;
  }
  int drain(SolverState* out) {
    while (pending > 0) {
      int rc = wait(out);
      if (rc) return rc;
    }
    return WD_OK;
  }
};

// The device state, now (stream synchronised), through the pinned mirror or,
// without one, straight into host memory.
int read_state(HostMirror* m, const SolverState* st, hipStream_t s, SolverState* out) {
  if (!m) {
    HIP_TRY(hipMemcpyAsync(out, st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return WD_OK;
  }
  HIP_TRY(hipMemcpyAsync(m->buf[0], st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = *m->buf[0];
  return WD_OK;
}

// Iterations to enqueue next, from the observed convergence rate.
int next_chunk(const SolverState& s, int enqueued, int max_iter) {
  int left = max_iter - enqueued;
  if (left <= 0) return 0;
  int n = 16;
  if (s.iter >= 4 && s.rho > 0 && s.bnorm2 > 0 && s.stop2 > 0) {
    const double rate = std::log(s.rho / s.bnorm2) / s.iter;  // < 0 when converging
    if (rate < 0) {
      const double need = std::log(s.stop2 / s.bnorm2) - std::log(s.rho / s.bnorm2);
      const int est = (int)std::ceil(need / rate);
      n = std::max(2, std::min(32, est / 2 + 1));
    }
  }
  return std::min(n, left);
}

int copy_history(const double* hist, const wd_cg_params* p, hipStream_t s, int iters) {
  if (!p->history || p->history_len <= 0) return WD_OK;
  const int n = std::min(iters, p->history_len);
  if (n > 0) HIP_TRY(hipMemcpyAsync(p->history, hist, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = n; i < p->history_len; ++i) p->history[i] = 0.0;
  return WD_OK;
}

// Shared set-up: pack U and b, form b', zero or pack x, and the initial
// residual r = b' - D^+ D x written to `rout` in its precision.
int cg_setup(const Geom& g, double mass, const void* U, const void* b, void* x, const wd_cg_params* p,
             const CgWorkspace& w, int interval, double delta, SpinorBuf rout, hipStream_t s, bool pack_u = true) {
  launch_init_state(w.st, p->tol, interval, delta, w.hist, p->history_len, s);
  if (pack_u) launch_pack_gauge(g, U, P_F64, w.U64, s);
  const int c64 = p->io_dtype == WD_C64;
  if (p->rhs_mode == WD_RHS_SOURCE) {
    launch_pack_spinor(g, b, c64, w.t64, s);
    launch_wilson_packed(g, P_F64, w.U64, w.t64, w.b64, mass, 1, G_ALWAYS, F_NONE, w.st, w.partials, s);
  } else {
    launch_pack_spinor(g, b, c64, w.b64, s);
  }
  launch_norm2(g, w.b64, G_ALWAYS, F_BNORM, w.st, w.partials, s);
  if (p->zero_guess) {
    // x = 0: the initial residual is b' itself (D 0 = 0 exactly), no stencils
    launch_zero(g, w.x64, G_ALWAYS, w.st, s);
    launch_norm2(g, w.b64, G_ALWAYS, F_RHO_INIT, w.st, w.partials, s);
    launch_convert(g, w.b64, rout, G_ALWAYS, w.st, s);
  } else {
    launch_pack_spinor(g, x, c64, w.x64, s);
    launch_wilson_packed(g, P_F64, w.U64, w.x64, w.t64, mass, 0, G_ALWAYS, F_NONE, w.st, w.partials, s);
    launch_residual(g, w.U64, w.t64, w.b64, rout, mass, G_ALWAYS, F_RHO_INIT, w.st, w.partials, s);
  }
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

// noalloc: no pinned mirror and no timing events (cg_solve_noalloc).
int cg_plain(const Geom& g, double mass, const void* U, const void* b, void* x, const wd_cg_params* p,
             wd_cg_result* res, void* ws, hipStream_t s, std::chrono::steady_clock::time_point t0,
             bool noalloc = false) {
  const CgWorkspace w = layout_cg(ws, g, WD_F64, p->history_len, ring_length(p, g));
  int rc = cg_setup(g, mass, U, b, x, p, w, 0, 0.0, w.r64, s);
  if (rc) return rc;
  launch_convert(g, w.r64, w.p64, G_ALWAYS, w.st, s);

  HostMirror* m = nullptr;
  if (!noalloc && (rc = get_mirror(&m))) return rc;
  KernelClock* clk = nullptr;
  if (p->profile && (rc = get_clock(&clk))) return rc;
  Poller poll{m, nullptr, s};
  SolverState st{};
  st.stop2 = 1;
  int enqueued = 0;
  int restarts = 0;
  for (;;) {
    // keep two chunks in flight
    while (poll.pending < 2) {
      const int n = next_chunk(st, enqueued, p->max_iter);
      if (n <= 0) break;
      for (int k = 0; k < n; ++k) {
        const int i = enqueued + k;
        launch_wilson_packed(g, P_F64, w.U64, w.p64, w.t64, mass, 0, G_ITER, F_ALPHA, w.st, w.partials, s,
                             clock_at(clk, 0, i));
        launch_cg_update(g, P_F64, w.U64, w.t64, w.r64, w.p64, w.x64, mass, w.st, w.partials, s,
                         clock_at(clk, 1, i));
        launch_p_update(g, w.r64, w.p64, w.st, s, clock_at(clk, 2, i));
      }
      enqueued += n;
      HIP_TRY(hipGetLastError());
      if ((rc = poll.post(w.st))) return rc;
    }
    if (poll.pending == 0) break;
    if ((rc = poll.wait(&st))) return rc;
    if (st.status != 0) {
      if ((rc = poll.drain(&st))) return rc;
      if (st.status != 1) break;
      // verify with the FP64 residual recomputed from x
      launch_wilson_packed(g, P_F64, w.U64, w.x64, w.t64, mass, 0, G_FINAL, F_NONE, w.st, w.partials, s);
      launch_residual(g, w.U64, w.t64, w.b64, w.r64, mass, G_FINAL, F_TRUE, w.st, w.partials, s);
      if ((rc = poll.post(w.st))) return rc;
      if ((rc = poll.drain(&st))) return rc;
      if (st.rho_true <= st.stop2 || enqueued >= p->max_iter || restarts >= 5) break;
      // the recurrence drifted from the true residual: restart from it
      ++restarts;
      launch_restart(w.st, s);
      launch_convert(g, w.r64, w.p64, G_ALWAYS, w.st, s);
      HIP_TRY(hipGetLastError());
      continue;
    }
  }
  if ((rc = poll.drain(&st))) return rc;
  double iter_rel = std::sqrt(st.rho / (st.bnorm2 > 0 ? st.bnorm2 : 1.0));
  if (st.status != 1 || st.rho_true > st.stop2) {
    if (st.status == 0 || st.status == 1) {
      // not converged within max_iter: report the true residual of the last iterate
      launch_wilson_packed(g, P_F64, w.U64, w.x64, w.t64, mass, 0, G_FINAL, F_NONE, w.st, w.partials, s);
      launch_residual(g, w.U64, w.t64, w.b64, w.r64, mass, G_FINAL, F_TRUE, w.st, w.partials, s);
      if ((rc = poll.post(w.st))) return rc;
      if ((rc = poll.drain(&st))) return rc;
    }
  }
  launch_unpack_spinor(g, w.x64, x, p->io_dtype == WD_C64, s);
  HIP_TRY(hipGetLastError());
  if ((rc = copy_history(w.hist, p, s, st.iter))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (res) clock_read(clk, enqueued, 3, res->kernel_seconds);
  int code;
  if (st.status < 0) code = status_to_code(st.status);
  else if (st.rho_true <= st.stop2) code = WD_OK;
  else code = fail(WD_NOT_CONVERGED, "not converged in %d iterations (true rel. residual %.3e)", st.iter,
                   std::sqrt(st.rho_true / (st.bnorm2 > 0 ? st.bnorm2 : 1.0)));
  return fill_result(res, st, code, secs, iter_rel);
}

// Reliable-update mixed precision: inner CG in FP32 arithmetic on
// low-precision fields; the solution accumulates in FP32 between updates and
// is flushed into FP64 x, where the residual is recomputed exactly.
int cg_mixed(const Geom& g, double mass, const void* U, const void* b, void* x, const wd_cg_params* p,
             wd_cg_result* res, void* ws, hipStream_t s, std::chrono::steady_clock::time_point t0,
             bool noalloc = false) {
  const int P = p->inner_prec;
  const bool refine = p->scheme == WD_ITERATIVE_REFINEMENT;
  // refinement: no periodic recomputation, only after each inner solve
  const int interval = reliable_interval_of(p);
  const CgWorkspace w = layout_cg(ws, g, P, p->history_len, ring_length(p, g));
  const double delta = reliable_delta(p);
  int rc = cg_setup(g, mass, U, b, x, p, w, interval, delta, w.rh, s);
  if (refine) launch_set_restart(w.st, s);
  if (rc) return rc;
  HostMirror* m = nullptr;
  if (!noalloc && (rc = get_mirror(&m))) return rc;
  // 16-bit inner links: two rows per link (row 2 rebuilt from unitarity) when
  // every link is SU(3) to 1e-9; the full 9 entries otherwise.
  int rows2 = 0;
  if (narrow_prec(P) && g.tiled) {
    launch_su3_check(g, U, w.st, w.partials, s);
    SolverState chk;
    if ((rc = read_state(m, w.st, s, &chk))) return rc;
    rows2 = chk.su3_dev <= 1e-9;
  }
  if (rows2) launch_pack_gauge_rows2(g, U, P, w.Ulow, s);
  else launch_pack_gauge(g, U, P, w.Ulow, s);
  // p_0 = r_0 in ring slot 0; fold the ring into x before it overflows: at
  // most kSlotEvery iterations pass between two checks
  launch_convert(g, w.rh, w.ring.at(0), G_ALWAYS, w.st, s);
  launch_set_ring(w.st, w.alpha_hist, w.ring.len - (kSlotEvery - 1), w.ring.len, s);
  HIP_TRY(hipGetLastError());

  KernelClock* clk = nullptr;
  if (p->profile && (rc = get_clock(&clk))) return rc;
  Poller poll{m, nullptr, s};
  SolverState st{};
  st.stop2 = 1;
  int enqueued = 0;
  for (;;) {
    while (poll.pending < 2) {
      int n = next_chunk(st, enqueued, p->max_iter);
      if (n <= 0) break;
      for (int k = 0; k < n; ++k) {
        const int i = enqueued + k;
        // t = D p (p = ring slot npend), alpha; r -= alpha D^+ t, beta
        launch_wilson_packed(g, P, w.Ulow, w.rh, w.th, mass, 0, G_ITER, F_ALPHA_RING, w.st, w.partials, s,
                             clock_at(clk, 0, i), rows2, &w.ring);
        launch_r_update(g, P, w.Ulow, w.th, w.rh, mass, w.st, w.partials, s, clock_at(clk, 1, i), rows2);
        if ((enqueued + k + 1) % kSlotEvery == 0) {
          // ring nearly full: x += sum alpha_j p_j without a residual recomputation
          launch_accumulate_ring(g, w.x64, w.ring, G_FLUSH, w.st, s);
          launch_ring_reset(w.st, s);
          // reliable update: x += sum alpha_j p_j, r = b' - D^+ D x in FP64
          launch_accumulate_ring(g, w.x64, w.ring, G_RELIABLE, w.st, s);
          launch_wilson_packed(g, P_F64, w.U64, w.x64, w.t64, mass, 0, G_RELIABLE, F_NONE, w.st, w.partials, s);
          launch_residual(g, w.U64, w.t64, w.b64, w.rh, mass, G_RELIABLE, F_RELIABLE, w.st, w.partials, s);
        }
        // next p into ring slot npend
        launch_p_update_ring(g, w.rh, w.ring, w.st, s, clock_at(clk, 2, i));
      }
      enqueued += n;
      HIP_TRY(hipGetLastError());
      if ((rc = poll.post(w.st))) return rc;
    }
    if (poll.pending == 0) break;
    if ((rc = poll.wait(&st))) return rc;
    if (st.status != 0) break;
    if (st.inner_done && enqueued >= p->max_iter) break;
  }
  if ((rc = poll.drain(&st))) return rc;
  const double iter_rel = std::sqrt(st.rho / (st.bnorm2 > 0 ? st.bnorm2 : 1.0));
  if (st.status != 1) {
    // max_iter reached (or an error): fold the pending p vectors into x and
    // measure the true residual
    launch_accumulate_ring(g, w.x64, w.ring, G_FINAL, w.st, s);
    launch_wilson_packed(g, P_F64, w.U64, w.x64, w.t64, mass, 0, G_FINAL, F_NONE, w.st, w.partials, s);
    launch_residual(g, w.U64, w.t64, w.b64, w.rh, mass, G_FINAL, F_TRUE, w.st, w.partials, s);
    if ((rc = poll.post(w.st))) return rc;
    if ((rc = poll.drain(&st))) return rc;
  }
  launch_unpack_spinor(g, w.x64, x, p->io_dtype == WD_C64, s);
  HIP_TRY(hipGetLastError());
  if ((rc = copy_history(w.hist, p, s, st.iter))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (res) {
    clock_read(clk, enqueued, 3, res->kernel_seconds);
    res->two_row_links = rows2;
  }
  int code;
  if (st.status < 0) code = status_to_code(st.status);
  else if (st.rho_true <= st.stop2) code = WD_OK;
  else code = fail(WD_NOT_CONVERGED, "not converged in %d iterations (true rel. residual %.3e)", st.iter,
                   std::sqrt(st.rho_true / (st.bnorm2 > 0 ? st.bnorm2 : 1.0)));
  return fill_result(res, st, code, secs, iter_rel);
}

// ---- lockstep batched solve: cg_mixed's schedule with every launch of the
// inner loop and of the reliable-update slots covering all systems (Rhs).
// Each system keeps its own state, so a converged system's workgroups exit
// at its closed gates while the others continue.

struct BatchMirror {
  SolverState* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
};
BatchMirror g_batch_mirror[64];

int get_batch_mirror(BatchMirror** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(WD_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mirror_mu);
  BatchMirror& m = g_batch_mirror[dev];
  if (!m.buf[0]) {
    for (int i = 0; i < 2; ++i) {
      HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&m.buf[i]), sizeof(SolverState) * kMaxBatch,
                            hipHostMallocDefault));
      HIP_TRY(hipEventCreateWithFlags(&m.ev[i], hipEventDisableTiming));
    }
  }
  *out = &m;
  return WD_OK;
}

int cg_mixed_lockstep(const Geom& g, double mass, const void* U, int nrhs, const void* B, void* X,
                      const wd_cg_params* p, wd_cg_result* res, void* ws, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int P = p->inner_prec;
  const int interval = reliable_interval_of(p);
  const LockstepWorkspace L = layout_lockstep(ws, g, P, ring_length_batch(p, g, nrhs), nrhs);
  const CgWorkspace& w = L.sys0;
  const Rhs rb{nrhs, L.stride};
  const double delta = reliable_delta(p);
  const int c64 = p->io_dtype == WD_C64;
  const size_t io_stride = (size_t)g.V * 12 * (c64 ? 8 : 16);
  wd_cg_params q = *p;   // per-system set-up, without a residual history
  q.history = nullptr;
  q.history_len = 0;
  int rc;
  BatchMirror* m;
  if ((rc = get_batch_mirror(&m))) return rc;

  // shared links: FP64 for the reliable updates; low precision, two rows when SU(3)
  launch_pack_gauge(g, U, P_F64, L.U64, s);
  launch_init_state(w.st, p->tol, interval, delta, w.hist, 0, s);
  launch_su3_check(g, U, w.st, w.partials, s);
  HIP_TRY(hipMemcpyAsync(m->buf[0], w.st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int rows2 = m->buf[0]->su3_dev <= 1e-9;
  if (rows2) launch_pack_gauge_rows2(g, U, P, L.Ulow, s);
  else launch_pack_gauge(g, U, P, L.Ulow, s);
  for (int k = 0; k < nrhs; ++k) {
    const CgWorkspace wk = system_view(L, k);
    const void* bk = static_cast<const char*>(B) + k * io_stride;
    void* xk = static_cast<char*>(X) + k * io_stride;
    if ((rc = cg_setup(g, mass, U, bk, xk, &q, wk, interval, delta, wk.rh, s, false))) return rc;
    launch_convert(g, wk.rh, wk.ring.at(0), G_ALWAYS, wk.st, s);
    launch_set_ring(wk.st, wk.alpha_hist, wk.ring.len - (kSlotEvery - 1), wk.ring.len, s);
  }
  HIP_TRY(hipGetLastError());

  SolverState st[kMaxBatch];
  for (int k = 0; k < nrhs; ++k) {
    st[k] = SolverState{};
    st[k].stop2 = 1;
  }
  int slot = 0, pending = 0, enqueued = 0;
  auto post = [&]() -> int {
    launch_gather_states(w.st, rb, L.states, s);
    HIP_TRY(hipMemcpyAsync(m->buf[slot], L.states, sizeof(SolverState) * nrhs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(m->ev[slot], s));
    slot ^= 1;
    ++pending;
    return WD_OK;
  };
  auto wait = [&]() -> int {   // the oldest posted copy
    const int j = pending == 2 ? slot : slot ^ 1;
    HIP_TRY(hipEventSynchronize(m->ev[j]));
    for (int k = 0; k < nrhs; ++k) st[k] = m->buf[j][k];
    --pending;
    return WD_OK;
  };
  for (;;) {
    while (pending < 2) {
      // enough iterations for the slowest system still running
      int n = 0;
      for (int k = 0; k < nrhs; ++k)
        if (st[k].status == 0) n = std::max(n, next_chunk(st[k], enqueued, p->max_iter));
      if (n <= 0) break;
      for (int i = 0; i < n; ++i) {
        launch_wilson_packed(g, P, w.Ulow, w.rh, w.th, mass, 0, G_ITER, F_ALPHA_RING, w.st, w.partials, s, nullptr,
                             rows2, &w.ring, rb);
        launch_r_update(g, P, w.Ulow, w.th, w.rh, mass, w.st, w.partials, s, nullptr, rows2, rb);
        if ((enqueued + i + 1) % kSlotEvery == 0) {
          launch_accumulate_ring(g, w.x64, w.ring, G_FLUSH, w.st, s, rb);
          launch_ring_reset(w.st, s, rb);
          launch_accumulate_ring(g, w.x64, w.ring, G_RELIABLE, w.st, s, rb);
          launch_wilson_packed(g, P_F64, w.U64, w.x64, w.t64, mass, 0, G_RELIABLE, F_NONE, w.st, w.partials, s,
                               nullptr, 0, nullptr, rb);
          launch_residual(g, w.U64, w.t64, w.b64, w.rh, mass, G_RELIABLE, F_RELIABLE, w.st, w.partials, s, rb);
        }
        launch_p_update_ring(g, w.rh, w.ring, w.st, s, nullptr, rb);
      }
      enqueued += n;
      HIP_TRY(hipGetLastError());
      if ((rc = post())) return rc;
    }
    if (pending == 0) break;
    if ((rc = wait())) return rc;
    bool more = false;   // a system still running that more iterations can serve
    for (int k = 0; k < nrhs; ++k)
      if (st[k].status == 0 && !(st[k].inner_done && enqueued >= p->max_iter)) more = true;
    if (!more) break;
  }
  while (pending > 0)
    if ((rc = wait())) return rc;
  double iter_rel[kMaxBatch];
  for (int k = 0; k < nrhs; ++k) {
    iter_rel[k] = std::sqrt(st[k].rho / (st[k].bnorm2 > 0 ? st[k].bnorm2 : 1.0));
    if (st[k].status == 1) continue;
    // max_iter reached (or an error): fold the pending directions, measure the true residual
    const CgWorkspace wk = system_view(L, k);
    launch_accumulate_ring(g, wk.x64, wk.ring, G_FINAL, wk.st, s);
    launch_wilson_packed(g, P_F64, wk.U64, wk.x64, wk.t64, mass, 0, G_FINAL, F_NONE, wk.st, wk.partials, s);
    launch_residual(g, wk.U64, wk.t64, wk.b64, wk.rh, mass, G_FINAL, F_TRUE, wk.st, wk.partials, s);
  }
  for (int k = 0; k < nrhs; ++k)
    launch_unpack_spinor(g, system_view(L, k).x64, static_cast<char*>(X) + k * io_stride, c64, s);
  HIP_TRY(hipGetLastError());
  if ((rc = post())) return rc;
  if ((rc = wait())) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int code = WD_OK;
  for (int k = 0; k < nrhs; ++k) {
    const SolverState& sk = st[k];
    int ck;
    if (sk.status == -4) ck = WD_ERR_NAN;
    else if (sk.status == -3) ck = WD_ERR_BREAKDOWN;
    else if (sk.status < 0) ck = WD_ERR_HIP;
    else if (sk.rho_true <= sk.stop2) ck = WD_OK;
    else ck = WD_NOT_CONVERGED;
    if (ck < 0 && (code >= 0 || ck < code)) code = ck;
    else if (ck == WD_NOT_CONVERGED && code == WD_OK) code = WD_NOT_CONVERGED;
    if (res) {
      fill_result(&res[k], sk, ck, secs, iter_rel[k]);
      res[k].two_row_links = rows2;
      for (int j = 0; j < 3; ++j) res[k].kernel_seconds[j] = 0.0;
    }
  }
  if (code == WD_NOT_CONVERGED)
    return fail(code, "at least one system did not converge in %d iterations", p->max_iter);
  if (code == WD_ERR_HIP) return fail(code, "internal: search-direction ring overflow");
  if (code < 0) return fail(code, "a system ended with status %d (NaN/Inf or breakdown)", code);
  return WD_OK;
}

// ---- the gauge-covariant Laplacian: the same state, gates, reductions and
// host loop as cg_plain, with the colour-vector stencil and updates.

struct LapWorkspace {
  SolverState* st;
  double* partials;
  double* hist;
  void* U64;
  void *b, *x, *r, *p, *t;   // packed FP64 colour fields
  size_t bytes;
};

LapWorkspace layout_lap(void* base, const Geom& g, int hist_len) {
  Carver c(base);
  LapWorkspace w{};
  w.st = static_cast<SolverState*>(c.take(sizeof(SolverState)));
  w.partials = static_cast<double*>(c.take(sizeof(double) * (size_t)g.nblocks));
  w.hist = static_cast<double*>(c.take(sizeof(double) * (size_t)(hist_len > 0 ? hist_len : 1)));
  w.U64 = c.take(gauge_bytes(P_F64, g.Vpad));
  const size_t vb = (size_t)g.Vpad * 3 * sizeof(double2);
  w.b = c.take(vb);
  w.x = c.take(vb);
  w.r = c.take(vb);
  w.p = c.take(vb);
  w.t = c.take(vb);
  w.bytes = c.off;
  return w;
}

int validate_lap_params(const wd_cg_params* p) {
  int rc = validate_params(p);
  if (rc) return rc;
  if (p->inner_prec != WD_F64) return fail(WD_ERR_INVALID, "laplace_cg_solve runs FP64 CG: inner_prec must be WD_F64");
  return WD_OK;
}

int lap_cg(const Geom& g, double m2, const void* U, const void* b, void* x, const wd_cg_params* p,
           wd_cg_result* res, void* ws, hipStream_t s, std::chrono::steady_clock::time_point t0) {
  const LapWorkspace w = layout_lap(ws, g, p->history_len);
  const int c64 = p->io_dtype == WD_C64;
  launch_init_state(w.st, p->tol, 0, 0.0, w.hist, p->history_len, s);
  launch_pack_gauge(g, U, P_F64, w.U64, s);
  launch_lap_pack(g, b, c64, w.b, s);
  launch_lap_norm2(g, w.b, F_BNORM, w.st, w.partials, s);
  if (p->zero_guess) launch_lap_copy(g, nullptr, w.x, G_ALWAYS, w.st, s);
  else launch_lap_pack(g, x, c64, w.x, s);
  launch_lap_residual(g, w.U64, w.x, w.b, w.r, m2, G_ALWAYS, F_RHO_INIT, w.st, w.partials, s);
  launch_lap_copy(g, w.r, w.p, G_ALWAYS, w.st, s);
  HIP_TRY(hipGetLastError());

  int rc;
  HostMirror* m;
  if ((rc = get_mirror(&m))) return rc;
  KernelClock* clk = nullptr;
  if (p->profile && (rc = get_clock(&clk))) return rc;
  Poller poll{m, nullptr, s};
  SolverState st{};
  st.stop2 = 1;
  int enqueued = 0;
  int restarts = 0;
  for (;;) {
    while (poll.pending < 2) {
      const int n = next_chunk(st, enqueued, p->max_iter);
      if (n <= 0) break;
      for (int k = 0; k < n; ++k) {
        const int i = enqueued + k;
        // t = L p, alpha = rho / <p, t>; x += alpha p, r -= alpha t, beta; p = r + beta p
        launch_lap_packed(g, w.U64, w.p, w.t, m2, G_ITER, F_ALPHA, w.st, w.partials, s, clock_at(clk, 0, i));
        launch_lap_update(g, w.t, w.r, w.p, w.x, w.st, w.partials, s, clock_at(clk, 1, i));
        launch_lap_p_update(g, w.r, w.p, w.st, s, clock_at(clk, 2, i));
      }
      enqueued += n;
      HIP_TRY(hipGetLastError());
      if ((rc = poll.post(w.st))) return rc;
    }
    if (poll.pending == 0) break;
    if ((rc = poll.wait(&st))) return rc;
    if (st.status != 0) {
      if ((rc = poll.drain(&st))) return rc;
      if (st.status != 1) break;
      // verify with the residual recomputed from x
      launch_lap_residual(g, w.U64, w.x, w.b, w.r, m2, G_FINAL, F_TRUE, w.st, w.partials, s);
      if ((rc = poll.post(w.st))) return rc;
      if ((rc = poll.drain(&st))) return rc;
      if (st.rho_true <= st.stop2 || enqueued >= p->max_iter || restarts >= 5) break;
      ++restarts;
      launch_restart(w.st, s);
      launch_lap_copy(g, w.r, w.p, G_ALWAYS, w.st, s);
      HIP_TRY(hipGetLastError());
      continue;
    }
  }
  if ((rc = poll.drain(&st))) return rc;
  const double iter_rel = std::sqrt(st.rho / (st.bnorm2 > 0 ? st.bnorm2 : 1.0));
  if ((st.status != 1 || st.rho_true > st.stop2) && (st.status == 0 || st.status == 1)) {
    // not converged within max_iter: report the true residual of the last iterate
    launch_lap_residual(g, w.U64, w.x, w.b, w.r, m2, G_FINAL, F_TRUE, w.st, w.partials, s);
    if ((rc = poll.post(w.st))) return rc;
    if ((rc = poll.drain(&st))) return rc;
  }
  launch_lap_unpack(g, w.x, x, c64, s);
  HIP_TRY(hipGetLastError());
  if ((rc = copy_history(w.hist, p, s, st.iter))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (res) clock_read(clk, enqueued, 3, res->kernel_seconds);
  int code;
  if (st.status < 0) code = status_to_code(st.status);
  else if (st.rho_true <= st.stop2) code = WD_OK;
  else code = fail(WD_NOT_CONVERGED, "not converged in %d iterations (true rel. residual %.3e)", st.iter,
                   std::sqrt(st.rho_true / (st.bnorm2 > 0 ? st.bnorm2 : 1.0)));
  return fill_result(res, st, code, secs, iter_rel);
}

}  // namespace

extern "C" int laplace_apply(const wd_lattice* lat, double m2, const void* U, const void* psi, void* out,
                             void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (!U || !psi || !out) return fail(WD_ERR_INVALID, "NULL field pointer");
  if (psi == out) return fail(WD_ERR_INVALID, "in and out must not alias");
  if (!std::isfinite(m2)) return fail(WD_ERR_INVALID, "m2 is not finite");
  launch_lap_canonical(make_geom(lat->L, false), U, psi, out, m2, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

extern "C" size_t laplace_workspace_bytes(const wd_lattice* lat, const wd_cg_params* params) {
  if (check_lattice(lat)) return 0;
  if (validate_lap_params(params)) return 0;
  return layout_lap(nullptr, packed_geom(lat), params->history_len).bytes;
}

extern "C" int laplace_cg_solve(const wd_lattice* lat, double m2, const void* U, const void* b, void* x,
                                const wd_cg_params* params, wd_cg_result* result, void* workspace, size_t ws_bytes,
                                void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (result) std::memset(result, 0, sizeof(*result));
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = validate_lap_params(params))) return rc;
  if (!U || !b || !x) return fail(WD_ERR_INVALID, "NULL field pointer");
  if (b == x) return fail(WD_ERR_INVALID, "b and x must not alias");
  if (!std::isfinite(m2)) return fail(WD_ERR_INVALID, "m2 is not finite");
  const Geom g = packed_geom(lat);
  const size_t need = layout_lap(nullptr, g, params->history_len).bytes;
  if (!workspace || ws_bytes < need)
    return fail(WD_ERR_WORKSPACE, "workspace of %zu bytes given, %zu needed", workspace ? ws_bytes : 0, need);
  std::unique_lock<std::mutex> lk;
  if ((rc = lock_device(lk))) return rc;
  return lap_cg(g, m2, U, b, x, params, result, workspace, as_stream(stream), t0);
}

extern "C" int cg_solve(const wd_lattice* lat, double mass, const void* U, const void* b, void* x,
                        const wd_cg_params* params, wd_cg_result* result, void* workspace, size_t ws_bytes,
                        void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (result) std::memset(result, 0, sizeof(*result));
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = validate_params(params))) return rc;
  if (!U || !b || !x) return fail(WD_ERR_INVALID, "NULL field pointer");
  if (b == x) return fail(WD_ERR_INVALID, "b and x must not alias");
  if (!std::isfinite(mass)) return fail(WD_ERR_INVALID, "mass is not finite");
  const Geom g = packed_geom(lat);
  const size_t need = required_bytes(g, params, 1);
  if (!workspace || ws_bytes < need)
    return fail(WD_ERR_WORKSPACE, "workspace of %zu bytes given, %zu needed", workspace ? ws_bytes : 0, need);
  const hipStream_t s = as_stream(stream);
  std::unique_lock<std::mutex> lk;
  if ((rc = lock_device(lk))) return rc;
  if (params->inner_prec == WD_F64) return cg_plain(g, mass, U, b, x, params, result, workspace, s, t0);
  return cg_mixed(g, mass, U, b, x, params, result, workspace, s, t0);
}

extern "C" int cg_solve_batched(const wd_lattice* lat, double mass, const void* U, int32_t nrhs, const void* B,
                                void* X, const wd_cg_params* params, wd_cg_result* results, void* workspace,
                                size_t ws_bytes, void* stream) {
  if (results && nrhs > 0 && nrhs <= 16) std::memset(results, 0, sizeof(wd_cg_result) * nrhs);
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = validate_params(params))) return rc;
  if (nrhs < 1 || nrhs > 16) return fail(WD_ERR_INVALID, "nrhs = %d must be in 1..16", nrhs);
  if (params->inner_prec == WD_F64)
    return fail(WD_ERR_INVALID, "batched solves run FP32 inner iterations: inner_prec must be WD_F32, WD_BF16, "
                                "WD_F16 or WD_I8");
  if (!U || !B || !X) return fail(WD_ERR_INVALID, "NULL field pointer");
  if (B == X) return fail(WD_ERR_INVALID, "B and X must not alias");
  if (!std::isfinite(mass)) return fail(WD_ERR_INVALID, "mass is not finite");
  const Geom g = packed_geom(lat);
  const size_t need = required_bytes(g, params, nrhs);
  if (!workspace || ws_bytes < need)
    return fail(WD_ERR_WORKSPACE, "workspace of %zu bytes given, %zu needed", workspace ? ws_bytes : 0, need);
  if (params->batch_schedule == WD_BATCH_LOCKSTEP && !lockstep_possible(g, params))
    return fail(WD_ERR_INVALID, "lockstep batching needs BF16, FP16 or int8 inner storage, reliable updates "
                                "and lattice extents that are multiples of 4");
  if (use_lockstep(g, params)) {
    std::unique_lock<std::mutex> lk;
    if ((rc = lock_device(lk))) return rc;
    return cg_mixed_lockstep(g, mass, U, nrhs, B, X, params, results, workspace, as_stream(stream));
  }
  char err[512] = {0};
  rc = batched_solve(g, mass, U, nrhs, B, X, params, results, workspace, as_stream(stream), err, sizeof(err));
  if (rc != WD_OK) return fail(rc, "%s", err);
  return WD_OK;
}

// ---- allocation-free solve: cg_solve with the workspace in a static device
// array instead of a caller-owned buffer, for callers that cannot allocate
// (HIP graph capture, serving loops). Each device the library runs on holds
// its own copy of the array, from the library's load to the process's end.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` per device (the name itself is a host-side
// stand-in), looked up once per device with that device current.
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

int scratch_ptr(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(WD_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(WD_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return WD_OK;
}

}  // namespace

extern "C" int cg_solve_noalloc(const wd_lattice* lat, double mass, const void* U, const void* b, void* x,
                                const wd_cg_params* params, wd_cg_result* result, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (result) std::memset(result, 0, sizeof(*result));
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = validate_params(params))) return rc;
  if (params->profile) return fail(WD_ERR_INVALID, "cg_solve_noalloc: profile needs timing events (use cg_solve)");
  if (!U || !b || !x) return fail(WD_ERR_INVALID, "NULL field pointer");
  if (b == x) return fail(WD_ERR_INVALID, "b and x must not alias");
  if (!std::isfinite(mass)) return fail(WD_ERR_INVALID, "mass is not finite");
  const Geom g = packed_geom(lat);
  const size_t need = layout_cg(nullptr, g, params->inner_prec, params->history_len, ring_length(params, g)).bytes;
  if (need > kScratchBytes)
    return fail(WD_ERR_WORKSPACE,
                "cg_solve_noalloc: this solve needs %zu bytes of workspace, the static scratch holds %zu "
                "(use cg_solve with a caller-owned workspace, or a smaller ring_len)",
                need, kScratchBytes);
  void* ws = nullptr;
  if ((rc = scratch_ptr(&ws))) return rc;
  const hipStream_t s = as_stream(stream);
  std::unique_lock<std::mutex> lk;
  if ((rc = lock_device(lk))) return rc;
  if (params->inner_prec == WD_F64) return cg_plain(g, mass, U, b, x, params, result, ws, s, t0, true);
  return cg_mixed(g, mass, U, b, x, params, result, ws, s, t0, true);
}

// ---- out-of-core solve (wd_ooc.hip) and the streaming measurement kernels

namespace {

// Host memory the GPU can read and write in place: pinned (page-locked) and
// known to the HIP runtime. *dev receives the address kernels use for it.
bool pinned_host(const void* p, const void** dev) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // pageable memory: clear the error the query left
    return false;
  }
  if (a.type != hipMemoryTypeHost) return false;
  *dev = p;
  if (a.devicePointer && a.hostPointer)
    *dev = static_cast<const char*>(a.devicePointer) + (static_cast<const char*>(p) - static_cast<const char*>(a.hostPointer));
  return true;
}

}  // namespace

extern "C" int wd_ooc_workspace_bytes(const wd_lattice* lat, int32_t slab_planes, int32_t history_len,
                                      size_t* device_bytes, size_t* host_bytes) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (slab_planes < 1 || slab_planes > lat->L[3])
    return fail(WD_ERR_INVALID, "slab_planes = %d must be in [1, Lt = %d]", slab_planes, lat->L[3]);
  if (history_len < 0) return fail(WD_ERR_INVALID, "history_len = %d", history_len);
  if (device_bytes) *device_bytes = ooc_device_bytes(lat->L, slab_planes, history_len);
  if (host_bytes) *host_bytes = ooc_host_bytes(lat->L);
  return WD_OK;
}

extern "C" int cg_solve_ooc(const wd_lattice* lat, double mass, const void* U, const void* b, void* x,
                            const wd_cg_params* params, wd_cg_result* result, void* host_workspace,
                            size_t host_ws_bytes, void* device_workspace, size_t device_ws_bytes, void* stream) {
  if (result) std::memset(result, 0, sizeof(*result));
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = validate_params(params))) return rc;
  if (params->inner_prec != WD_F64) return fail(WD_ERR_INVALID, "cg_solve_ooc runs FP64 CG: inner_prec must be WD_F64");
  if (params->io_dtype != WD_C128) return fail(WD_ERR_INVALID, "cg_solve_ooc takes complex128 fields (io_dtype WD_C128)");
  if (params->profile) return fail(WD_ERR_INVALID, "cg_solve_ooc does not profile kernels (profile must be 0)");
  if (!U || !b || !x || !host_workspace) return fail(WD_ERR_INVALID, "NULL field or host workspace pointer");
  if (b == x) return fail(WD_ERR_INVALID, "b and x must not alias");
  if (!std::isfinite(mass)) return fail(WD_ERR_INVALID, "mass is not finite");
  const void* host_ptrs[4] = {U, b, x, host_workspace};
  const void* dev_ptrs[4] = {nullptr, nullptr, nullptr, nullptr};
  const char* names[4] = {"U", "b", "x", "host_workspace"};
  for (int i = 0; i < 4; ++i)
    if (!pinned_host(host_ptrs[i], &dev_ptrs[i]))
      return fail(WD_ERR_INVALID, "cg_solve_ooc: %s is not pinned host memory (hipHostMalloc or a pinned tensor)",
                  names[i]);
  const size_t host_need = ooc_host_bytes(lat->L);
  if (host_ws_bytes < host_need)
    return fail(WD_ERR_WORKSPACE, "host workspace of %zu bytes given, %zu needed", host_ws_bytes, host_need);
  if (!device_workspace || ooc_slab_planes(lat->L, device_ws_bytes, params->history_len) < 1)
    return fail(WD_ERR_WORKSPACE, "device workspace of %zu bytes is below the %zu of one-plane slabs",
                device_workspace ? device_ws_bytes : 0, ooc_device_bytes(lat->L, 1, params->history_len));
  std::unique_lock<std::mutex> lk;
  if ((rc = lock_device(lk))) return rc;
  char err[512] = {0};
  // the kernels read and write the host fields in place, through their device addresses
  rc = ooc_solve(lat->L, mass, dev_ptrs[0], dev_ptrs[1], const_cast<void*>(dev_ptrs[2]),
                 params, result, const_cast<void*>(dev_ptrs[3]), device_workspace, device_ws_bytes,
                 as_stream(stream), err, sizeof(err));
  if (rc != WD_OK) return fail(rc, "%s", err);
  return WD_OK;
}

extern "C" int wd_stream(int32_t kind, const void* src, void* dst, size_t bytes, void* stream) {
  if (kind < 0 || kind > 2) return fail(WD_ERR_INVALID, "kind = %d unknown", kind);
  if (bytes % 16) return fail(WD_ERR_INVALID, "bytes = %zu is not a multiple of 16", bytes);
  if ((kind != 2 && !src) || !dst) return fail(WD_ERR_INVALID, "NULL pointer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
    return fail(WD_ERR_INVALID, "pointers must be 16-byte aligned");
  if (bytes == 0) return WD_OK;
  launch_stream(kind, src, dst, bytes, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return WD_OK;
}

extern "C" size_t wd_stream_partials(size_t bytes) { return stream_read_partials(bytes); }
