/*
 * wilson.h -- C ABI of the MI355X (gfx950) Wilson-Dirac conjugate-gradient library.
 *
 * What is computed. The Wilson-Dirac operator on a periodic 4D lattice with
 * 3x3 complex (SU(3)) link matrices acting on 12-component complex spinors
 * (paper Sec. 1 and the Fig. 1 caption name the operator and its data; the
 * definition is the one of the lattice-QCD textbook the paper cites there),
 * in mass form with lattice spacing 1:
 *
 *   (D psi)(x) = (m + 4) psi(x)
 *              - 1/2 sum_{mu=0..3} [ (1 - g_mu) U_mu(x) psi(x + mu)
 *                                  + (1 + g_mu) U_mu(x - mu)^+ psi(x - mu) ]
 *
 * (equivalently (1 / 2 kappa)(1 - kappa H) with kappa = 1 / (2 m + 8)),
 * g_mu the Euclidean chiral gamma matrices, mu = 0, 1, 2, 3 = x, y, z, t.
 * D^+ is the same stencil with g_mu -> -g_mu. The solver is the
 * conjugate-gradient method (Sec. 1, Sec. 3.1) on the normal equations
 * D^+ D x = D^+ b, optionally in the two-precision form of Sec. 2 / Sec. 3.2
 * (low-precision iterations corrected by occasional FP64 recomputation of
 * the residual).
 *
 * Layouts at the boundary (row-major, x fastest):
 *   lattice dims   L[0] = Lx, L[1] = Ly, L[2] = Lz, L[3] = Lt, each >= 2
 *   gauge field U  complex128 (4, Lt, Lz, Ly, Lx, 3, 3); U[mu][site] is the
 *                  colour matrix on the link site -> site + mu, row-major
 *   spinor psi     (Lt, Lz, Ly, Lx, 4, 3) complex128 (or complex64 where an
 *                  io_dtype says so): spin index then colour index
 *   force F        same shape and type as U
 *
 * Pointers: every field pointer is DEVICE memory owned by the caller (for
 * example a PyTorch tensor's data_ptr()); the library keeps no pointer after
 * a call returns and never frees caller memory. `stream` is a hipStream_t
 * (NULL = the default stream). Input and output fields must not overlap.
 *
 * Errors: every int-returning call returns WD_OK (0), WD_NOT_CONVERGED (1)
 * or a negative WD_ERR_* code; wd_last_error() returns a message for the
 * calling thread's last non-zero return. Argument errors are detected before
 * any device work is issued. Nothing aborts or throws across the ABI.
 *
 * Threads: the blocking solvers (cg_solve, cg_solve_batched, laplace_cg_solve)
 * share pinned host buffers per device, so their calls on one device are
 * serialised (a second thread's call waits for the first to return). The
 * current device (hipSetDevice) selects the GPU.
 */
#ifndef WILSON_MI355X_H
#define WILSON_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t L[4]; /* Lx, Ly, Lz, Lt; each >= 2; Lx*Ly*Lz*Lt <= 2^28 */
} wd_lattice;

/* storage / arithmetic precision of the solver's inner iterations.
 * WD_F16 spinors carry one FP32 magnitude per site (values stored divided by it).
 * WD_I8 is fixed point: spinors as 24 signed bytes per site, q = round(127 v / m)
 * with m the site's largest |component| (kept as FP32 per site); links as FP16,
 * as for WD_F16 (the stencil then runs its products in half precision with
 * FP32 sums, exact for these inputs). */
enum { WD_F64 = 0, WD_F32 = 1, WD_BF16 = 2, WD_F16 = 3, WD_I8 = 4 };
/* OR-ed into the precision of a packed GAUGE field (wd_gauge_bytes, wd_pack_gauge,
 * wilson_apply_packed): store rows 0 and 1 of each link only and rebuild row 2
 * as conj(row0 x row1). Valid for SU(3) links (the caller guarantees it),
 * WD_BF16 / WD_F16 / WD_I8, and lattices whose extents are all multiples of 4. */
enum { WD_TWO_ROW_LINKS = 0x100 };
/* which system cg_solve solves */
enum { WD_RHS_SOURCE = 0, /* D^+ D x = D^+ b  (x = D^-1 b) */
       WD_RHS_NORMAL = 1  /* D^+ D x = b                   */ };
/* element type of b and x at the boundary */
enum { WD_C128 = 0, WD_C64 = 1 };
/* two-precision scheme of a mixed solve (inner_prec != WD_F64) */
enum { WD_RELIABLE_UPDATE = 0,      /* one Krylov space; the FP64 residual replaces the
                                       low-precision one every reliable_interval iterations
                                       and after each inner_tol reduction (default) */
       WD_ITERATIVE_REFINEMENT = 1  /* defect correction: x += e with D^+D e = r solved in low
                                       precision to inner_tol from e = 0 (a new Krylov space
                                       per cycle), r recomputed in FP64 after each cycle */ };

enum {
  WD_OK = 0,
  WD_NOT_CONVERGED = 1,   /* max_iter reached; x holds the last iterate */
  WD_ERR_INVALID = -1,    /* bad argument; nothing was launched */
  WD_ERR_HIP = -2,        /* a HIP runtime call failed */
  WD_ERR_BREAKDOWN = -3,  /* <p, D^+ D p> <= 0 */
  WD_ERR_NAN = -4,        /* NaN or Inf in a reduction (for example a NaN in b) */
  WD_ERR_WORKSPACE = -5   /* workspace NULL or smaller than wd_workspace_bytes() */
};

typedef struct {
  double tol;                /* stop when ||b' - D^+ D x|| / ||b'|| <= tol (b' = D^+ b or b) */
  int32_t max_iter;          /* CG iterations (inner iterations for mixed precision) */
  int32_t inner_prec;        /* WD_F64: plain FP64 CG. WD_F32 / WD_BF16 / WD_F16 / WD_I8: FP32
                                arithmetic on that storage, FP64 reliable updates */
  int32_t reliable_interval; /* mixed only: FP64 residual recomputation every this many
                                iterations (0 -> 50) */
  int32_t rhs_mode;          /* WD_RHS_SOURCE or WD_RHS_NORMAL */
  int32_t io_dtype;          /* WD_C128 or WD_C64: element type of b and x */
  int32_t zero_guess;        /* nonzero: start from x = 0 and ignore x's input contents */
  double* history;           /* HOST array, may be NULL: iterated relative residual per iteration */
  int32_t history_len;       /* capacity of history (entries beyond are dropped) */
  int32_t profile;           /* nonzero (cg_solve only): time the inner loop's kernels with HIP
                                events on `stream` over the first 64 iterations (see wd_cg_result) */
  int32_t scheme;            /* WD_RELIABLE_UPDATE or WD_ITERATIVE_REFINEMENT (cg_solve, mixed) */
  int32_t ring_len;          /* mixed (cg_solve): search directions kept in the workspace before
                                they are folded into x (x += sum alpha_j p_j, in FP64); 8..256, or
                                0 -> reliable_interval + 5 (so that folds coincide with the FP64
                                recomputations) limited to what fits in 8 GiB, at least 8. The
                                fold runs at each FP64 recomputation and whenever ring_len - 4
                                directions are pending. Workspace grows by ring_len
                                low-precision spinors. */
  double inner_tol;          /* residual reduction between FP64 recomputations; 0 -> the default
                                (reliable updates: 0.1 BF16 and I8, 1e-2 FP16, 1e-4 FP32;
                                refinement: 0.1) */
  int32_t batch_schedule;    /* cg_solve_batched only: WD_BATCH_AUTO, WD_BATCH_PERSISTENT or
                                WD_BATCH_LOCKSTEP (see below) */
} wd_cg_params;

/* How cg_solve_batched runs its systems.
   WD_BATCH_PERSISTENT: one cooperative persistent launch for the whole solve, with
     per-system convergence masks; every storage precision and lattice.
   WD_BATCH_LOCKSTEP: the single-system mixed solver's kernels, each CG step one launch
     over all systems (workgroups of one tile and all systems run back to back, so each
     link is read from HBM once per step for all of them); BF16, FP16 or int8 storage,
     reliable updates, every lattice extent a multiple of 4.
   WD_BATCH_AUTO (0): lockstep where it applies, persistent otherwise. */
enum { WD_BATCH_AUTO = 0, WD_BATCH_PERSISTENT = 1, WD_BATCH_LOCKSTEP = 2 };

typedef struct {
  int32_t iterations;        /* iterations performed (inner iterations for mixed) */
  int32_t reliable_updates;  /* FP64 residual recomputations (mixed) */
  int32_t status;            /* same value as the call's return code */
  int32_t two_row_links;     /* 1 if the inner iterations used two-row (12-real) links: cg_solve does
                                so for WD_BF16 / WD_F16 / WD_I8 on tileable lattices whose links are SU(3)
                                to 1e-9 (checked on the device); 0 otherwise */
  double true_rel_res;       /* ||b' - D^+ D x|| / ||b'|| recomputed in FP64 at the end */
  double iter_rel_res;       /* the recurrence's own residual at the end */
  double seconds;            /* host wall time of the call */
  double kernel_seconds[3];  /* with params->profile: average device time of one launch of the inner
                                loop's (0) t = D p kernel, (1) fused D^+ t / r update kernel (plain
                                FP64 CG: also x += alpha p), (2) p = r + beta p kernel; 0 otherwise */
  int32_t ooc_slab_planes;   /* cg_solve_ooc: time planes per slab of its schedule; 0 otherwise */
  int32_t ooc_slabs;         /* cg_solve_ooc: slabs per sweep; 0 otherwise */
} wd_cg_result;

/* Thread-local text of the last non-zero return on the calling thread. */
const char* wd_last_error(void);

/* Number of HIP devices visible, or a negative WD_ERR_HIP. */
int wd_device_count(void);

/*
 * out = D psi. U, psi, out: device, canonical complex128 layouts above.
 * Asynchronous on `stream`; no host synchronisation, no workspace.
 */
int wilson_apply(const wd_lattice* lat, double mass, const void* U, const void* psi, void* out, void* stream);

/* out = D^+ psi (the same stencil with g_mu -> -g_mu). As wilson_apply. */
int wilson_apply_dagger(const wd_lattice* lat, double mass, const void* U, const void* psi, void* out,
                        void* stream);

/*
 * Device workspace needed by cg_solve (nrhs = 1) or cg_solve_batched
 * (nrhs = number of right-hand sides) for these parameters, in bytes
 * (for batched solves it depends on params->batch_schedule: the lockstep
 * schedule keeps a ring of search directions per system).
 * Returns 0 on an invalid argument (see wd_last_error()).
 */
size_t wd_workspace_bytes(const wd_lattice* lat, const wd_cg_params* params, int32_t nrhs);

/*
 * Solve D^+ D x = D^+ b (rhs_mode WD_RHS_SOURCE) or D^+ D x = b
 * (WD_RHS_NORMAL) by conjugate gradient.
 *   U          device, canonical complex128 gauge field
 *   b          device, canonical spinor of element type params->io_dtype
 *   x          device, same type: initial guess on entry (unless
 *              params->zero_guess), solution on return
 *   workspace  device, at least wd_workspace_bytes(lat, params, 1) bytes,
 *              owned by the caller, contents need not be initialised
 *   result     host, filled on return (may be NULL)
 * Runs on `stream` and BLOCKS until the solve ends (the host polls the
 * device-side residual to stop). Returns WD_OK, WD_NOT_CONVERGED (x holds the
 * last iterate, usable as a restart guess) or a WD_ERR_* code.
 */
int cg_solve(const wd_lattice* lat, double mass, const void* U, const void* b, void* x,
             const wd_cg_params* params, wd_cg_result* result, void* workspace, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cg_solve
 * with its workspace taken from a static device array of 256 MiB that the
 * library holds on every device it runs on, from its load to the end of the
 * process, instead of a caller-owned buffer. Arguments, results, return codes
 * and blocking behaviour as cg_solve; the caller still owns U, b and x. The
 * call itself allocates nothing: no hipMalloc / hipFree, no pinned host
 * buffers and no events (the device state is polled by synchronous copies
 * into host memory), so params->profile must be 0 (else WD_ERR_INVALID).
 * A solve whose single-system workspace (the layout cg_solve would carve; at
 * most wd_workspace_bytes(lat, params, 1)) exceeds 256 MiB is rejected with
 * WD_ERR_WORKSPACE before anything is launched: e.g. FP64 CG fits lattices
 * up to about 16^3 x 32; a mixed solve's ring of search directions may need
 * a smaller params->ring_len. Every call on a device shares that device's
 * array and leaves its contents behind; nothing in it needs to start at zero
 * (each solve initialises its state). Calls on one device are serialised
 * with cg_solve's (one device mutex) and each returns after its device work
 * has finished, so calls from several host threads do not overlap; work
 * that a caller enqueues on the array by other means would race with them.
 */
int cg_solve_noalloc(const wd_lattice* lat, double mass, const void* U, const void* b, void* x,
                     const wd_cg_params* params, wd_cg_result* result, void* stream);

/*
 * Solve nrhs systems sharing one gauge field (the batched multi-RHS form of
 * the mixed-precision CG, Sec. 2 and Sec. 3.2 applied per system).
 * B, X: device, (nrhs, Lt, Lz, Ly, Lx, 4, 3) of element type params->io_dtype.
 * Inner iterations run in FP32 arithmetic; p, r and t are stored in
 * params->inner_prec (WD_F32, WD_BF16, WD_F16 or WD_I8; WD_F64 is rejected).
 * Each system carries its own alpha, beta and convergence mask; FP64 reliable
 * updates (every params->reliable_interval iterations, and whenever a
 * system's residual has fallen by params->inner_tol, default as for cg_solve)
 * recompute each residual from an FP64 solution.
 * params->batch_schedule selects how (see WD_BATCH_*):
 *   persistent  ONE cooperative launch for the whole solve; FP32 links staged
 *               in LDS per 64-site block and reused by every system; the
 *               solution increment in FP32.
 *   lockstep    cg_solve's mixed-precision kernels, each CG step one launch over
 *               all systems (tile-major, so a tile's links are fetched from HBM
 *               once per step for all systems); each system's iterates equal
 *               those of cg_solve on it alone. BF16 / FP16 / int8 storage,
 *               reliable updates, lattice extents multiples of 4 (else
 *               WD_ERR_INVALID); more workspace (a ring of search directions
 *               per system).
 * results: host array of nrhs entries (may be NULL). 1 <= nrhs <= 16. Blocks
 * until all systems end. Returns WD_OK if every system converged,
 * WD_NOT_CONVERGED if any did not, or a WD_ERR_* code.
 */
int cg_solve_batched(const wd_lattice* lat, double mass, const void* U, int32_t nrhs, const void* B, void* X,
                     const wd_cg_params* params, wd_cg_result* results, void* workspace, size_t ws_bytes,
                     void* stream);

/*
 * Gauge-link gradient kernel (the derivative of 1/2 Re<a, H b> with respect to
 * the links, in the convention grad = d/dRe U + i d/dIm U):
 *   G(a, b)_mu(x) = 1/2 sum_spin [ ((1 - g_mu) a(x)) (x) b(x + mu)^*
 *                                + b(x) (x) ((1 + g_mu) a(x + mu))^* ]
 * with (u (x) v^*)_ij = u_i conj(v_j). F = coeff * G(a, b), or F += coeff * G(a, b)
 * when accumulate is nonzero. a, b: device canonical complex128 spinors;
 * F: device canonical complex128 gauge-shaped field. Asynchronous on `stream`.
 * For chi = (D^+D)^-1 phi and an upstream gradient g, lambda = (D^+D)^-1 g:
 *   dL/dU = G(D chi, lambda) + G(D lambda, chi).
 */
int wilson_force(const wd_lattice* lat, const void* a, const void* b, double coeff, int32_t accumulate, void* F,
                 void* stream);

/* ---- out-of-core solve: fields larger than (or kept out of) device memory ----
 *
 * The paper's accelerator computes on the first complete inputs while later
 * data is still streaming in over the host link, which removes the limit that
 * local memory would put on the problem size (Sec. 2, Sec. 3.1, Sec. 4 and
 * Fig. 2). cg_solve_ooc runs the plain FP64 CG of cg_solve with the gauge
 * field, b, x and the CG vectors in HOST memory: each operator application
 * streams the lattice through the GPU in slabs of whole time planes (each slab
 * with one halo plane on either side, periodic in t), on three HIP streams
 * (copies in, kernels, copies out) and two device buffer sets, so that copies
 * of neighbouring slabs overlap the kernels. The copies are kernels that read
 * and write the pinned host memory in place (one launch per slab and
 * direction). One iteration is two sweeps (t = D p with the search-direction
 * and deferred solution updates; r -= alpha D^+ t) and moves about 2.1 KB per
 * site to the device and 0.8 KB back (more for slabs of few planes, whose
 * halo planes are a larger share). */

/* Workspace of cg_solve_ooc for slabs of slab_planes time planes
 * (1 <= slab_planes <= Lt) and a residual history of history_len entries:
 * *device_bytes (device memory) and *host_bytes (pinned host memory: five
 * FP64 spinor fields, b', r, two search directions, t). Either pointer may be NULL. Returns WD_OK or
 * WD_ERR_INVALID. */
int wd_ooc_workspace_bytes(const wd_lattice* lat, int32_t slab_planes, int32_t history_len, size_t* device_bytes,
                           size_t* host_bytes);

/*
 * Out-of-core D^+ D x = D^+ b (or b) by plain FP64 CG.
 *   U, b, x          PINNED HOST memory (hipHostMalloc, or a pinned torch tensor),
 *                    canonical complex128 layouts; x: initial guess unless
 *                    params->zero_guess, solution on return
 *   host_workspace   pinned host memory, >= host_bytes of wd_ooc_workspace_bytes
 *   device_workspace device memory of device_ws_bytes: the device budget. The
 *                    solve uses the thickest slabs (at most about Lt / 4 planes,
 *                    so that there are slabs to overlap) whose buffers fit;
 *                    WD_ERR_WORKSPACE if not even one-plane slabs fit.
 * params: tol, max_iter, rhs_mode, zero_guess, history / history_len as for
 * cg_solve; inner_prec must be WD_F64, io_dtype WD_C128, profile 0 (else
 * WD_ERR_INVALID). result->ooc_slab_planes / ooc_slabs report the schedule.
 * The solve starts after the work already queued on `stream` and BLOCKS until
 * it ends (it runs on the library's own streams). Returns WD_OK,
 * WD_NOT_CONVERGED (x holds the last iterate), or a WD_ERR_* code (pageable
 * host memory: WD_ERR_INVALID).
 */
int cg_solve_ooc(const wd_lattice* lat, double mass, const void* U, const void* b, void* x,
                 const wd_cg_params* params, wd_cg_result* result, void* host_workspace, size_t host_ws_bytes,
                 void* device_workspace, size_t device_ws_bytes, void* stream);

/* ---- measurement: plain streaming kernels, the practical HBM ceiling ----
 * The paper states that its stencil is limited only by memory bandwidth
 * (Sec. 3.1.2); these kernels measure what a perfectly coalesced stream gets
 * from HBM on this device, for comparison with the stencils. kind 0: dst = src
 * (bytes read and bytes written); 1: read src, an XOR of all words per
 * workgroup goes to dst (wd_stream_partials(bytes) 16-byte words); 2: dst = 0
 * (bytes written). Device pointers, 16-byte aligned; bytes a multiple of 16.
 * Asynchronous on `stream`. */
int wd_stream(int32_t kind, const void* src, void* dst, size_t bytes, void* stream);
size_t wd_stream_partials(size_t bytes);

/* ---- packed fields: the solver's internal site-blocked layout, for callers that
 *      apply D repeatedly without repacking (and for timing the hot kernel). ---- */

/* Bytes of a packed gauge field / spinor field in precision `prec` (0 on bad args). */
size_t wd_gauge_bytes(const wd_lattice* lat, int32_t prec);
size_t wd_spinor_bytes(const wd_lattice* lat, int32_t prec);

/* Pack canonical complex128 U into `out` (device, wd_gauge_bytes bytes). Asynchronous. */
int wd_pack_gauge(const wd_lattice* lat, const void* U, int32_t prec, void* out, void* stream);
/* Canonical spinor (element type io_dtype) <-> packed spinor of precision prec. Asynchronous. */
int wd_pack_spinor(const wd_lattice* lat, const void* in, int32_t io_dtype, int32_t prec, void* out, void* stream);
int wd_unpack_spinor(const wd_lattice* lat, const void* in, int32_t prec, void* out, int32_t io_dtype,
                     void* stream);

/* out = D in (dagger = 0) or D^+ in on packed fields of precision prec (FP32
 * arithmetic for WD_F32/WD_BF16/WD_F16/WD_I8, FP64 for WD_F64). The kernel of the
 * solver's inner iterations. Asynchronous. */
int wilson_apply_packed(const wd_lattice* lat, double mass, int32_t prec, const void* U_packed,
                        const void* in_packed, void* out_packed, int32_t dagger, void* stream);

/* ---- a second operator through the same solver: the gauge-covariant Laplacian ----
 *
 * The paper presents its CG design as a backbone on which other linear
 * operators can be solved with the data movement unchanged (abstract,
 * Sec. 3.2, Sec. 7). This operator acts on colour vectors (3 complex numbers
 * per site) with the same links and the same nearest-neighbour stencil shape,
 * without spin:
 *
 *   (L psi)(x) = (m2 + 8) psi(x) - sum_{mu=0..3} [ U_mu(x) psi(x + mu) + U_mu(x - mu)^+ psi(x - mu) ]
 *
 * Hermitian; for unitary links the hopping sum has norm <= 8, so L is positive
 * definite for m2 > 0 (spectrum in [m2, m2 + 16]) and CG solves L x = b
 * directly. Colour field layout: (Lt, Lz, Ly, Lx, 3), complex128 (complex64
 * for solver I/O where params->io_dtype says so). U as above. */

/* out = L psi on canonical complex128 fields (device). Asynchronous on
 * `stream`; no workspace. Any finite m2 is accepted. */
int laplace_apply(const wd_lattice* lat, double m2, const void* U, const void* psi, void* out, void* stream);

/* Device workspace of laplace_cg_solve for these parameters, in bytes; 0 on an
 * invalid argument. */
size_t laplace_workspace_bytes(const wd_lattice* lat, const wd_cg_params* params);

/*
 * Solve L x = b by plain FP64 conjugate gradient, on the Wilson solver's
 * machinery (device-resident state, deterministic reductions, host polling).
 * Uses params->tol (||b - L x|| / ||b||, confirmed by an FP64 recomputation),
 * max_iter, io_dtype, zero_guess, history / history_len and profile
 * (kernel_seconds: (0) t = L p with <p, t>, (1) x += alpha p and r -= alpha t
 * with ||r||^2, (2) p = r + beta p). inner_prec must be WD_F64; rhs_mode,
 * scheme, reliable_interval, inner_tol and ring_len are ignored.
 *   U, b, x, workspace: device, owned by the caller (x: initial guess unless
 *   zero_guess, solution on return); result: host, may be NULL.
 * BLOCKS until the solve ends. Returns WD_OK, WD_NOT_CONVERGED (x holds the
 * last iterate), WD_ERR_BREAKDOWN if <p, L p> <= 0 (L not positive definite),
 * or another WD_ERR_* code.
 */
int laplace_cg_solve(const wd_lattice* lat, double m2, const void* U, const void* b, void* x,
                     const wd_cg_params* params, wd_cg_result* result, void* workspace, size_t ws_bytes,
                     void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WILSON_MI355X_H */
