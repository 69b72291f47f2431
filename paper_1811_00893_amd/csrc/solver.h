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

struct FieldBuf {
    DevBuf buf;
    Spinor f;
    void make(int prec, const Geom &g, int nrhs);
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
