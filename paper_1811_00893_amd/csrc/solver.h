// Krylov solvers on the even-odd preconditioned Wilson system.
//
// With D = [[1, -k H_eo], [-k H_oe, 1]] in (even, odd) blocks (Eq. (1) couples only
// nearest neighbours, which have opposite parity), D x = b is equivalent to
//     M_ee x_e = b'_e,   M_ee = 1 - k^2 H_eo H_oe,   b'_e = b_e + k H_eo b_o,
//     x_o = b_o + k H_oe x_e,
// and the residual of the full system equals the even residual (r_o = 0).
//
// Methods: BiCGStab (the paper's Krylov method, Sec. 2) and CG on the normal equations
// M^dag M x = M^dag b' in its CGLS form, with M^dag = g5 M g5.  Every scalar of the
// iteration lives on the device; the host enqueues iterations ahead and polls a
// host-mapped copy of the per-RHS state a few iterations behind, so the GPU never waits
// for the host.  Mixed precision: an FP64 outer defect correction on the even system
// (r_e = b'_e - M x_e in FP64, x_e accumulated in FP64) around inner solves in FP32 or
// FP16-with-per-site-scale.  All right-hand sides of a call run in lockstep in the
// same launches with their own scalars; finished ones are masked out.
#pragma once
#include "runtime.h"

namespace wl {

// Bump allocator over one device region: buffers at increasing 256-byte aligned offsets.
// With no base it only measures (the pointers it hands out are then null).
struct Arena {
    char *base = nullptr;
    size_t used = 0;
    void *take(size_t bytes) {
        used = (used + 255) & ~size_t(255);
        void *p = base ? base + used : nullptr;
        used += bytes;
        return p;
    }
};

struct FieldBuf {
    DevBuf buf;   // owning storage (make); empty when the field is placed in an arena
    Spinor f;
    void make(int prec, const Geom &g, int nrhs);
    void place(int prec, const Geom &g, int nrhs, Arena &A);
};

// Device memory of one even-odd problem with nrhs right-hand sides: every field, the
// reduction partials and the per-RHS states, carved in a fixed order out of one region
// (the library's own allocation, a caller's workspace, or the static scratch array).
struct EoMem {
    FieldBuf b_e, b_o, x_e, x_o, bp;          // FP64 problem
    FieldBuf r64, tmp64;                      // FP64 outer residual (mixed only)
    FieldBuf r, rh, p, v, s, t, tmp, rf, xin; // inner Krylov fields
    double *partials = nullptr;
    double *partials2 = nullptr;              // partials of the hops whose finalize a vector kernel runs
    RhsState *st_in = nullptr, *st_out = nullptr;
    RhsState *st_alt = nullptr;               // states between such a kernel and the iteration's end
    BlockState *bstate = nullptr;             // block BiCGStab only
    size_t bytes = 0;                         // size of the region
    // places every buffer from base (nullptr: sizes only); returns the region's size
    size_t carve(char *base, const Geom &g, int nrhs, int precision, int method);
};

struct SolveParams {
    int method = WILSON_SOLVER_BICGSTAB_EO;
    int precision = WILSON_FP64;
    int maxiter = 10000;
    int max_restarts = 5;
    double inner_tol = 0.0;
    bool use_x0 = false;
    int poll_every = 1;
    bool reliable = false;  // mixed precision: reliable updates instead of defect correction
    void *workspace = nullptr;    // device region for every buffer of the solve (null: the library's)
    size_t workspace_bytes = 0;
    bool no_tune = false;         // launch shapes from the tuning table or the defaults, no tuning runs
    bool graphs = true;           // small lattices may replay iteration chunks as HIP graphs (WILSON_GRAPHS=1)
};

// Solves for nrhs right-hand sides given in canonical layout on the device.
// x_canon (in/out) and b_canon are device pointers.
int solve_device(wilson_ctx *ctx, const wilson_gauge *G, double *x_canon, const double *b_canon, int nrhs,
                 const double *kappa, const double *tol, const SolveParams &p, wilson_solve_info *info);

size_t solve_footprint(const Geom &g, int nrhs, const SolveParams &p);

// Dslash on device canonical fields (see wilson_dslash_ex).
void dslash_device(wilson_ctx *ctx, const wilson_gauge *G, double *out, const double *in, double kappa, int parity,
                   int prec, int nrhs);

// ---- continuous-batching engine (one resident gauge field, nslots RHS slots) ----
class BatchEngine;
BatchEngine *batch_create(wilson_ctx *ctx, const wilson_gauge *G, int nslots, const SolveParams &p);
void batch_destroy(BatchEngine *b);
int batch_attach(BatchEngine *b, int slot, const double *b_canon_dev, double kappa, double tol, int maxiter);
void batch_step(BatchEngine *b, int iters);
void batch_poll(BatchEngine *b, int32_t *state, int32_t *status);
int batch_detach(BatchEngine *b, int slot, double *x_canon_dev, wilson_solve_info *info);
wilson_ctx *batch_ctx(BatchEngine *b);
size_t batch_spinor_bytes(BatchEngine *b);  // bytes of one canonical complex128 field

}  // namespace wl
