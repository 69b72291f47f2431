/*
 * wilson.h -- C ABI of the MI355X (gfx950) Wilson-Dirac operator and solver library.
 *
 * The operator is the Wilson fermion matrix of Kanamori & Matsufuru, Sec. 2.1, Eq. (1):
 *
 *   D(x,y) = delta_{x,y} - kappa * sum_{mu=1..4} [ (1 - gamma_mu) U_mu(x) delta_{x+mu,y}
 *                                                + (1 + gamma_mu) U_mu(x-mu)^dag delta_{x-mu,y} ]
 *          = 1 - kappa * H,
 *
 * acting on complex fields with 4 spin x 3 colour components per site and SU(3) links
 * U_mu(x) on the 4 directions (Sec. 2).  The linear system D x = b is solved with
 * BiCGStab, the Krylov method of Sec. 2, here on the even-odd preconditioned Schur
 * system, with CG on the normal equations as a second method, and in a mixed-precision
 * variant (FP32 / FP16 inner solve, FP64 outer correction); Sec. 2 motivates the latter:
 * in practice the single-precision inner solve dominates the cost of the whole solve.
 *
 * CONVENTIONS (all entry points)
 *   dims  = {Lx, Ly, Lz, Lt}; every extent even and >= 2.  V = Lx*Ly*Lz*Lt.
 *   site  s = x + Lx*(y + Ly*(z + Lz*t)), 0-based; parity of a site = (x+y+z+t) mod 2.
 *   mu    = 0..3 <-> x, y, z, t.
 *   Complex numbers are interleaved (re, im) doubles (double _Complex layout).
 *   Spinor element (s, spin, colour) is complex number (s*4 + spin)*3 + colour
 *     (12*V complex = 24*V doubles per field; nrhs fields are stored back to back).
 *   Link U_mu(s)[a][b] is complex number ((s*4 + mu)*3 + a)*3 + b (36*V complex).
 *   gamma_mu in the Dirac basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = x,y,z),
 *     gamma_t = diag(1, 1, -1, -1); gamma_5 = gamma_x gamma_y gamma_z gamma_t.
 *   Boundaries: periodic in x, y, z; antiperiodic in t.  The caller passes periodic
 *     links; the library applies the sign -1 to the hops that cross t = Lt-1 <-> 0.
 *
 * POINTERS AND OWNERSHIP
 *   Every buffer is owned by the caller.  Array arguments may be host or device memory
 *   (detected per pointer).  With device pointers the call is enqueued on the context's
 *   stream and returns without waiting, except where stated; with host pointers the
 *   call copies through device memory and returns when the result is on the host.
 *   The library keeps no caller pointer after a call returns.  Handles (contexts,
 *   gauge fields, batches) are owned by the library and released by their _free /
 *   _destroy call.  A context and everything created from it is used by one host thread
 *   at a time; distinct contexts may be used concurrently.
 *
 * ERRORS
 *   Every int-returning call returns a wilson_status code; no C++ exception crosses
 *   the ABI.  wilson_strerror() gives text, wilson_last_error() the detail of the last
 *   failure on the calling thread.
 *
 * ENVIRONMENT (read by the library; none is needed)
 *   WILSON_TUNE=0          no launch-shape tuning: built-in default shapes.
 *   WILSON_TUNE_CACHE=path tuned shapes read from this JSON-lines file at start and new
 *                          ones appended (tuning costs a few hundred ms per new shape).
 *   WILSON_TUNE_VERBOSE=1  print every timed candidate shape to stderr.
 *   WILSON_HOP_CFG=block,rpt,xcd,zblk[,lds_kb[,wsplit[,shx[,dsplit[,ldsl[,tm]]]]]]
 *                          pin the parity-hop launch shape of contexts created after it
 *                          is set (testing).
 *   WILSON_RECON=18        keep all 18 reals of every link (default: the first two rows
 *                          when every link is SU(3) to 1e-13, the third rebuilt in the
 *                          kernels).
 *   WILSON_GRAPHS=1        on lattices up to 2^16 sites per parity, replay solver
 *                          iterations in chunks of four from captured HIP graphs (same
 *                          results bit for bit; measured slower than direct launches on
 *                          ROCm 7.2, so off by default).
 */
#ifndef WILSON_H
#define WILSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WILSON_OK = 0,
    WILSON_NOT_CONVERGED = 1,  /* x holds the last iterate; info is filled */
    WILSON_INVALID_ARG = -1,   /* null, odd or < 2 extent, bad kappa/tol/maxiter/parity, ... */
    WILSON_OUT_OF_MEMORY = -2,
    WILSON_DEVICE_ERROR = -3,  /* a HIP call failed; see wilson_last_error() */
    WILSON_BREAKDOWN = -4,     /* Krylov breakdown persisted through restarts */
    WILSON_NONFINITE = -5,     /* NaN or Inf in the input or an iterate */
    WILSON_REJECTED = -6,      /* admission refused (memory budget) */
    WILSON_BUSY = -7           /* batch slot occupied / not ready */
} wilson_status;

/* Arithmetic/storage precision of spinors and links inside the library. */
typedef enum {
    WILSON_FP64 = 0,      /* FP64 spinors and links */
    WILSON_FP32 = 1,      /* FP32 spinors and links, FP64 reduction accumulators */
    WILSON_FP16 = 2,      /* FP16 spinors with one FP32 scale per site, FP16 links */
    WILSON_FP16_L32 = 3   /* FP16 spinors with one FP32 scale per site, FP32 links */
} wilson_precision;

/* Bits of wilson_gauge_load's `precisions`: which link copies to keep resident. */
#define WILSON_GAUGE_FP64 1u
#define WILSON_GAUGE_FP32 2u
#define WILSON_GAUGE_FP16 4u

typedef enum {
    WILSON_SOLVER_BICGSTAB_EO = 0, /* BiCGStab on M_ee = 1 - kappa^2 H_eo H_oe */
    WILSON_SOLVER_CGNR_EO = 1,     /* CG on M_ee^dag M_ee (CGLS form), M_ee^dag = g5 M_ee g5 */
    WILSON_SOLVER_BLOCK_BICGSTAB_EO = 2
    /* Block BiCGStab on M_ee (Guennouni, Jbilou and Sadok 2003; the paper's BiCGStab of
       Sec. 2 with the s right-hand sides of one call sharing one Krylov space: alpha and
       beta become s x s matrices solved against the shadow block R~ = R_0, omega is one
       Frobenius ratio).  wilson_solve_ex only, FP64 only (precision WILSON_FP64,
       mixed_update 0), every kappa[k] equal (one matrix).  The right-hand sides are taken
       in blocks of up to 16 consecutive non-zero ones (a zero b_k gets x_k = 0 and is left
       out); each block stops when every column meets its tol[k] on the iterated residual,
       and is then checked in FP64 like the other solvers.  A block whose s x s matrix
       R~^H V is singular to working precision (pivot below 1e-13 of its largest entry:
       e.g. linearly dependent right-hand sides) restarts from its current solution with
       one BiCGStab recurrence per right-hand side (counted in `restarts`).  info[k]
       .iterations counts block iterations (plus those of such a restart). */
} wilson_solver;

typedef struct wilson_ctx wilson_ctx;
typedef struct wilson_gauge wilson_gauge;
typedef struct wilson_batch wilson_batch;

typedef struct {
    int32_t solver;        /* wilson_solver */
    int32_t precision;     /* WILSON_FP64: plain FP64 solve; FP32 / FP16 / FP16_L32: mixed
                              precision, inner solve in that precision, FP64 outer defect
                              correction (residual, solution and reductions in FP64) */
    int32_t maxiter;       /* cap on inner iterations summed over all cycles (> 0) */
    int32_t max_restarts;  /* FP64 path: restarts when the true residual misses tol (<0: 5) */
    double inner_tol;      /* mixed: relative tolerance of each inner solve (<=0: default
                              1e-5 for FP32, 1e-2 for FP16) */
    int32_t use_x0;        /* nonzero: x holds the initial guess on entry */
    int32_t poll_every;    /* iterations between host convergence polls (<=0: default) */
    int32_t mixed_update;  /* mixed precision with BiCGStab: 0 defect correction (each cycle
                              restarts the inner solve on the normalised FP64 residual),
                              1 reliable updates (Sleijpen and van der Vorst 1996: one inner
                              recurrence through all cycles; at each cycle the FP64 residual
                              replaces the iterated one; inner_tol is the drop per cycle
                              with the same defaults).  Batches take 0. */
    void *workspace;       /* optional caller-owned device memory (e.g. a torch tensor's
                              storage), 256-byte aligned, for every device buffer of the call:
                              wilson_solve_ex uses it for that call only (nothing is kept in it
                              afterwards), wilson_batch_create for the batch's lifetime (the
                              caller keeps it alive until wilson_batch_destroy).  NULL: the
                              library allocates and caches its own (the default). */
    size_t workspace_bytes;/* size of workspace; at least wilson_footprint_bytes(dims, nrhs or
                              nslots, opts), else the call fails with WILSON_INVALID_ARG */
} wilson_solve_opts;

typedef struct {
    int32_t iterations;    /* inner iterations (BiCGStab / CG steps) */
    int32_t outer_cycles;  /* defect-correction cycles (0 for the FP64 path) */
    int32_t restarts;
    int32_t converged;     /* 1 if |b - D x| / |b| < tol in FP64 */
    double true_residual;  /* |b - D x| / |b| recomputed in FP64 after the solve */
    double ms;             /* wall time of the call on the host */
    double hop_launches;   /* parity-hop launches issued (this and the next two: for the
                              whole call, the same in every record) */
    double bytes;          /* algorithmic bytes of the call's parity hops and solver vector
                              kernels: each operand field read or written once per launch,
                              a link counted as 18 reals (conversions at the boundary and
                              the scalar steps not included) */
    double flops;          /* operator flops of those hops: 1320 per output site and
                              right-hand side (Table 1's convention), 1896 with a clover
                              site term; vector-kernel flops not included */
} wilson_solve_info;

/* ---------------------------------------------------------------------------------- */
/* Plain entry points (the library's two-call form).                                  */
/* ---------------------------------------------------------------------------------- */

/*
 * Apply the Wilson operator (Eq. (1)) in FP64.
 *   parity 0 or 1: out = -kappa * H * in on the sites of that parity only (the
 *                  parity-hop block D_{p,1-p}); sites of the other parity in `out` are
 *                  not written, and `in` is read only on parity 1-p, so out == in is
 *                  allowed.
 *   parity 2:      out = D * in = in - kappa * H * in on every site; out == in is rejected.
 * out, in: 12*V complex each.  U: 36*V complex (periodic links).  kappa finite.
 * Uses an internal context on the default stream; synchronous.
 */
int wilson_dslash(double *out, const double *in, const double *U, double kappa, const int32_t dims[4],
                  int32_t parity);

/*
 * Solve D x = b (Eq. (1)) with FP64 even-odd BiCGStab from x = 0.  Converged when the
 * FP64 true residual |b - D x| / |b| < tol (recomputed after the iteration stops; the
 * solve restarts from x if the iterated residual was optimistic).  b = 0 gives x = 0.
 * Returns WILSON_OK, WILSON_NOT_CONVERGED (x = last iterate) or an error.  Synchronous.
 */
int wilson_solve(double *x, const double *b, const double *U, double kappa, const int32_t dims[4], double tol,
                 int32_t maxiter);

/* ---------------------------------------------------------------------------------- */
/* Context, resident gauge fields, extended calls.                                    */
/* ---------------------------------------------------------------------------------- */

/* Create a context bound to the current HIP device and to `hip_stream` (a hipStream_t;
 * NULL = the null stream).  All work of calls on this context goes to that stream. */
int wilson_context_create(wilson_ctx **ctx, void *hip_stream);
int wilson_context_destroy(wilson_ctx *ctx);

/* Upload links (canonical layout, periodic, host or device) and keep them resident in
 * the library's layout with the antiperiodic sign applied, in each precision requested
 * by `precisions` (WILSON_GAUGE_* bits; FP64 is always kept).  Links must be SU(3)
 * (|U_ab| <= 1 is what the FP16 copy relies on). */
int wilson_gauge_load(wilson_ctx *ctx, wilson_gauge **g, const double *U, const int32_t dims[4],
                      uint32_t precisions);
int wilson_gauge_free(wilson_ctx *ctx, wilson_gauge *g);
/* Device bytes held by a resident gauge field (links and any clover term). */
size_t wilson_gauge_bytes(const wilson_gauge *g);
/* Device bytes wilson_gauge_load would keep for this lattice and `precisions` (WILSON_GAUGE_*
 * bits; FP64 always), with links stored as link_reals = 18 (full) or 12 (the first two rows,
 * which wilson_gauge_load uses when every link is SU(3) to 1e-13): for admission before a
 * field is loaded (18 gives an upper bound).  0 for invalid arguments. */
size_t wilson_gauge_footprint_bytes(const int32_t dims[4], uint32_t precisions, int32_t link_reals);

/*
 * Clover term (Sec. 2.1.2 of the paper): the clover fermion matrix adds a site term,
 * D_clov(x,y) = D(x,y) + F(x) delta_{x,y}, with F(x) a Hermitian 12x12 matrix that is
 * block diagonal, two Hermitian 6x6 blocks, in the chiral basis (equivalently: F
 * commutes with gamma5).  The paper stores F like the links and does not build it; the
 * caller supplies it.
 *
 * wilson_gauge_attach_clover attaches F to a resident gauge field.  From then on every
 * call on g uses D_clov: wilson_dslash_ex with parity 2 applies D_clov (parity 0/1 is the
 * off-diagonal block -kappa*H, common to both matrices); wilson_solve_ex and the batch
 * API solve D_clov x = b (even-odd: M_ee = T_ee - kappa^2 H_eo T_oo^-1 H_oe with
 * T = 1 + F, x_o = T_oo^-1 (b_o + kappa H_oe x_e)), in every precision and solver.
 *   F: V x 12 x 12 complex doubles (interleaved re, im), F[s][a][b] at complex offset
 *      (s*12 + a)*12 + b, site s in canonical order, a, b = 3*spin + colour in the
 *      library's Dirac basis (gamma5 = -[[0,1],[1,0]] on the spin pairs (0,2), (1,3));
 *      host or device; read during the call only.
 * The library keeps T and T^-1 per site as packed chiral blocks in FP64 and FP32
 * (1728 bytes per site).  Attaching again replaces the term.  The term must not change
 * (attach or detach) while a batch on g has busy slots or a call on g is in progress.
 * Errors: INVALID_ARG (NULL; F not Hermitian or not commuting with gamma5 beyond a
 * relative 1e-12; T singular at some site), OUT_OF_MEMORY, DEVICE_ERROR; on error the
 * field keeps its previous state.
 */
int wilson_gauge_attach_clover(wilson_ctx *ctx, wilson_gauge *g, const double *F);
/* Remove the clover term: g is a plain Wilson field again. */
int wilson_gauge_detach_clover(wilson_ctx *ctx, wilson_gauge *g);

/*
 * Dslash on a resident gauge field, for nrhs fields stored back to back (canonical
 * layout, complex128, host or device).  Semantics of `parity` as wilson_dslash.
 * `precision` selects the arithmetic: inputs are rounded to it (FP16: per-site scale),
 * the result is returned as complex128.  nrhs in 1..64.
 */
int wilson_dslash_ex(wilson_ctx *ctx, const wilson_gauge *g, double *out, const double *in, double kappa,
                     int32_t parity, int32_t precision, int32_t nrhs);

/*
 * Solve D x_k = b_k for k = 0..nrhs-1 on a resident gauge field with per-RHS kappa[k]
 * and tol[k] (arrays of nrhs doubles, host memory).  opts may be NULL (plain FP64
 * even-odd BiCGStab).  info, if not NULL, is an array of nrhs records.  The RHS are
 * solved together: every kernel processes all of them in one launch and each link is
 * read once per site for all RHS.  Returns the worst status over the RHS.  Synchronous.
 */
int wilson_solve_ex(wilson_ctx *ctx, const wilson_gauge *g, double *x, const double *b, int32_t nrhs,
                    const double *kappa, const double *tol, const wilson_solve_opts *opts,
                    wilson_solve_info *info);

/* Host check of the site indexing the kernels use on lattice dims (no device work; the
 * library's own index functions, compiled for the host, replayed over every site of
 * both parities): coordinates decoded from every checkerboard index, the eight
 * neighbour indices of the hop (in range, at the right coordinates, on the other
 * parity, each direction a permutation), every plane-blocked visiting order and the
 * XCD-contiguous block order of the launch grids.  Returns WILSON_OK, a negative
 * error code for invalid dims, or the number of violations (> 0; the first is
 * described by wilson_last_error()).  Diagnostic: cost O(V) time and 64 bytes per
 * site of host memory. */
int wilson_index_check(const int32_t dims[4]);

/* Device bytes wilson_solve_ex would allocate for this lattice, nrhs and options
 * (workspace only; the resident gauge field is wilson_gauge_bytes); also the smallest
 * opts->workspace_bytes a caller-owned workspace may have. */
size_t wilson_footprint_bytes(const int32_t dims[4], int32_t nrhs, const wilson_solve_opts *opts);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): wilson_solve_ex without any
 * allocation.  Same arguments, semantics and results as wilson_solve_ex, with these
 * differences:
 *   - x and b must be device memory (host pointers: WILSON_INVALID_ARG);
 *   - every device buffer of the solve lives in one static array of the library
 *     (256 MiB per GPU, part of the library's code object: each GPU the library runs on
 *     holds it from the library's first use on that device until the process ends); a
 *     solve needing more, wilson_footprint_bytes(dims, nrhs, opts) > 256 MiB (for
 *     example FP64 1 RHS up to 16^3x32, 12 RHS at 8^4), fails with WILSON_INVALID_ARG
 *     and a message naming both sizes; opts->workspace must be NULL;
 *   - host resources come from the context (created with it);
 *   - launch shapes come from the tuning table filled by earlier calls of this process,
 *     else the built-in defaults; no tuning runs; event timing is suspended for the call.
 * The call allocates no device, pinned or managed memory (no hipMalloc, hipFree or
 * allocating library routine).  All calls on one GPU share that GPU's array, which keeps
 * the last call's contents (the solve clears what must start at zero): calls that overlap
 * on one GPU (other threads, other contexts) race and must be serialised by the caller.
 * Synchronous, like wilson_solve_ex.
 */
int wilson_solve_noalloc(wilson_ctx *ctx, const wilson_gauge *g, double *x, const double *b, int32_t nrhs,
                         const double *kappa, const double *tol, const wilson_solve_opts *opts,
                         wilson_solve_info *info);

/* ---------------------------------------------------------------------------------- */
/* Batched step API for continuous batching (a serving loop keeps one batch per        */
/* resident gauge field and refills slots as right-hand sides converge).              */
/* ---------------------------------------------------------------------------------- */

/* A batch of `nslots` independent solves on one resident gauge field; all slots use
 * opts (solver, precision, inner_tol; workspace, if given, holds the batch's device
 * buffers until wilson_batch_destroy); kappa and tol are per slot. */
int wilson_batch_create(wilson_ctx *ctx, const wilson_gauge *g, int32_t nslots, const wilson_solve_opts *opts,
                        wilson_batch **batch);
int wilson_batch_destroy(wilson_batch *batch);
/* Copy b (12*V complex, host or device) into a free slot and start its solve.
 * WILSON_BUSY if the slot is in use. */
int wilson_batch_attach(wilson_batch *batch, int32_t slot, const double *b, double kappa, double tol,
                        int32_t maxiter);
/* Enqueue up to `iters` iterations for every active slot; returns without waiting. */
int wilson_batch_step(wilson_batch *batch, int32_t iters);
/* Per-slot state after the work enqueued so far has completed on the device:
 * state[k] = 0 free, 1 running, 2 finished (status[k] holds its wilson_status).
 * Blocks until the device has finished the enqueued steps. */
int wilson_batch_poll(wilson_batch *batch, int32_t *state, int32_t *status);
/* Copy a finished slot's solution (12*V complex) to x (host or device) and free the slot.
 * info may be NULL. */
int wilson_batch_detach(wilson_batch *batch, int32_t slot, double *x, wilson_solve_info *info);

/* ---------------------------------------------------------------------------------- */
/* Measurement helpers.                                                                */
/* ---------------------------------------------------------------------------------- */

/* Kernel classes timed with HIP events when timing is enabled on a context. */
typedef enum { WILSON_KERNEL_HOP = 0, WILSON_KERNEL_BLAS = 1, WILSON_KERNEL_COUNT = 2 } wilson_kernel_class;

/* Enable (1) / disable (0) event timing of every launch of the timed kernel classes
 * on the context's stream; enabling clears the accumulators. */
int wilson_timing_enable(wilson_ctx *ctx, int32_t enable);
/* Sum of launch durations (ms), launch count and algorithmic bytes of a kernel class
 * since timing was enabled.  Waits for outstanding timed work. */
int wilson_timing_read(wilson_ctx *ctx, int32_t kernel_class, double *total_ms, int64_t *launches,
                       double *bytes);

/* Device-to-device copy of `bytes` bytes with a plain streaming kernel on the context
 * stream (reference for bandwidth and hardware-counter calibration). */
int wilson_stream_copy(wilson_ctx *ctx, void *dst, const void *src, size_t bytes);
/* Read `bytes` bytes of device memory with a plain streaming kernel on the context stream
 * (read-only bandwidth reference; the data is not modified). */
int wilson_stream_read(wilson_ctx *ctx, const void *src, size_t bytes);

/* ---------------------------------------------------------------------------------- */
/* Layout ablation.                                                                    */
/* ---------------------------------------------------------------------------------- */

/* Storage layouts of wilson_layout_hop (Sec. 4.1 compares folding consecutive x-sites
 * into one SIMD vector, its layout 1, with folding one site of each of several
 * sub-lattices into it, its layout 2; Sec. 5 also compares both with the
 * array-of-structures base code).  A GPU wavefront plays the vector. */
typedef enum {
    WILSON_LAYOUT_SOA = 0,    /* component planes over checkerboard sites: 64 consecutive
                                 x-sites per wavefront (layout 1; the library's own) */
    WILSON_LAYOUT_AOS = 1,    /* the 12 complex of a site contiguous, the 4 links of a site
                                 contiguous (the base code's array of structures) */
    WILSON_LAYOUT_AOSOA = 2,  /* tiles of 64 sites, component planes inside a tile */
    WILSON_LAYOUT_VNODE = 3   /* 1 x 4 x 4 x 4 sub-lattices; lane l of a wavefront holds
                                 sub-lattice l (layout 2); needs Ly, Lz, Lt multiples of 8 */
} wilson_layout;

/* The parity hop out = -kappa H_{p,1-p} in (Eq. (1); the same operation as
 * wilson_dslash_ex with parity p), computed by one kernel whose spinor and link fields
 * are stored in `layout`; everything but the addressing is shared by the layouts.
 *   out, in   canonical complex128 fields of the whole lattice (12*V complex, layout of
 *             wilson_dslash), device memory.  in is read on the sites of parity 1-parity;
 *             out receives the hop on the sites of `parity` and zero on the others.
 *   U         canonical complex128 links (4*V*9 complex), device memory.
 *   parity    0 or 1.
 *   precision WILSON_FP64 or WILSON_FP32: storage and arithmetic of fields and links.
 *   link_reals 18 (full links) or 12 (first two rows; U must then be SU(3) to 1e-13).
 *   reps      >= 0 further launches after the one whose result is returned, timed with
 *             HIP events on the context stream; *us_per_launch (may be NULL) receives
 *             their mean duration in microseconds (0 when reps == 0).
 * The call packs the fields into the layout in device buffers of its own (freed before
 * it returns; not part of the timing) and synchronizes the context stream.
 * Errors: WILSON_INVALID_ARG (NULL or host pointer, extents not allowed for the layout,
 * bad parity/precision/layout/link_reals/reps, U not SU(3) with link_reals 12),
 * WILSON_OUT_OF_MEMORY, WILSON_DEVICE_ERROR. */
int wilson_layout_hop(wilson_ctx *ctx, double *out, const double *in, const double *U, const int32_t dims[4],
                      double kappa, int32_t parity, int32_t precision, int32_t layout, int32_t link_reals,
                      int32_t reps, double *us_per_launch);

const char *wilson_strerror(int code);
const char *wilson_last_error(void);
/* Library version string. */
const char *wilson_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WILSON_H */
