// Finalize of a reduction (Sec. 2: the scalar steps of the Krylov solvers run on the
// device): the per-block partial sums of each right-hand side are added in a fixed
// order, then the scalar step of the iteration (FinOp) updates that right-hand side's
// state.  The finalize kernel (blas.hip) and the vector kernels that run a finalize
// before their own work (PreFin) share these functions, so both give the same bits.
#pragma once
#include "common.h"
#include "device.h"

namespace wl {

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

template <int OP>
__device__ __forceinline__ void fin_op(RhsState *st, const double a0, const double a1, const double a2) {
    auto fail = [&](int code) {
        st->phase = PH_FAIL;
        st->fail = code;
    };
    if constexpr (OP == FIN_STORE_AUX) {
        st->aux = a0;
    } else if constexpr (OP == FIN_ADD_AUX) {
        st->aux += a0;
    } else if constexpr (OP == FIN_BICG_INIT) {
        st->r2 = a0;
        st->rhat2 = a0;
        st->rho_re = a0; st->rho_im = 0.0;
        st->alpha_re = 1.0; st->alpha_im = 0.0;
        st->omega_re = 1.0; st->omega_im = 0.0;
        st->beta_re = 0.0; st->beta_im = 0.0;
        st->fail = FAIL_NONE;
        if (!finite(a0)) fail(FAIL_NONFINITE);
        else if (a0 <= st->stop2) st->phase = PH_DONE;
        else st->phase = PH_RUN;
    } else if constexpr (OP == FIN_BICG_ALPHA) {
        // alpha = rho / <rhat, v>
        const double den = a0 * a0 + a1 * a1;
        if (!finite(den)) { fail(FAIL_NONFINITE); return; }
        if (den == 0.0) { fail(FAIL_BREAKDOWN); return; }
        st->alpha_re = (st->rho_re * a0 + st->rho_im * a1) / den;
        st->alpha_im = (st->rho_im * a0 - st->rho_re * a1) / den;
    } else if constexpr (OP == FIN_BICG_S) {
        st->s2 = a0;
        if (!finite(a0)) { fail(FAIL_NONFINITE); return; }
        if (a0 <= st->stop2) {
            st->phase = PH_SCONV;  // x += alpha p and stop: omega = 0 makes the last update exactly that
            st->omega_re = 0.0;
            st->omega_im = 0.0;
        }
    } else if constexpr (OP == FIN_BICG_OMEGA) {
        if (st->phase != PH_RUN) return;
        if (!finite(a2) || !finite(a0) || !finite(a1)) { fail(FAIL_NONFINITE); return; }
        if (a2 == 0.0) { fail(FAIL_BREAKDOWN); return; }
        st->omega_re = a0 / a2;
        st->omega_im = a1 / a2;
        if (st->omega_re == 0.0 && st->omega_im == 0.0) fail(FAIL_BREAKDOWN);
    } else if constexpr (OP == FIN_BICG_RHO) {
        st->r2 = a0;
        st->iter += 1;
        if (!finite(a0)) { fail(FAIL_NONFINITE); return; }
        const bool stop = st->phase == PH_SCONV || a0 <= st->stop2;
        const double rn = sqrt(a1 * a1 + a2 * a2);
        if (st->phase != PH_SCONV && rn > 1e-30 * sqrt(st->rhat2 * a0)) {
            // beta = (rho'/rho) (alpha/omega); also on the last iteration of a cycle, so that
            // a recurrence resumed after its residual was replaced continues from here
            const double d1 = st->rho_re * st->rho_re + st->rho_im * st->rho_im;
            const double q1r = (a1 * st->rho_re + a2 * st->rho_im) / d1, q1i = (a2 * st->rho_re - a1 * st->rho_im) / d1;
            const double d2 = st->omega_re * st->omega_re + st->omega_im * st->omega_im;
            const double q2r = (st->alpha_re * st->omega_re + st->alpha_im * st->omega_im) / d2;
            const double q2i = (st->alpha_im * st->omega_re - st->alpha_re * st->omega_im) / d2;
            st->beta_re = q1r * q2r - q1i * q2i;
            st->beta_im = q1r * q2i + q1i * q2r;
            st->rho_re = a1;
            st->rho_im = a2;
        } else if (!stop) {
            fail(FAIL_BREAKDOWN);
            return;
        }
        if (stop) st->phase = PH_DONE;
    } else if constexpr (OP == FIN_CG_R2) {
        st->r2 = a0;
        st->fail = FAIL_NONE;
        if (!finite(a0)) fail(FAIL_NONFINITE);
        else if (a0 <= st->stop2) st->phase = PH_DONE;
        else st->phase = PH_RUN;
    } else if constexpr (OP == FIN_CG_ZZ) {
        st->zz = a0;
        if (!finite(a0)) fail(FAIL_NONFINITE);
        else if (a0 == 0.0) fail(FAIL_BREAKDOWN);
    } else if constexpr (OP == FIN_CG_ALPHA) {
        if (!finite(a0)) { fail(FAIL_NONFINITE); return; }
        if (a0 == 0.0) { fail(FAIL_BREAKDOWN); return; }
        st->alpha_re = st->zz / a0;
        st->alpha_im = 0.0;
    } else if constexpr (OP == FIN_CG_R) {
        st->r2 = a0;
        st->iter += 1;
        if (!finite(a0)) fail(FAIL_NONFINITE);
        else if (a0 <= st->stop2) st->phase = PH_DONE;
    } else if constexpr (OP == FIN_BLOCK_TS) {
        st->omega_re = a0;
        st->omega_im = a1;
        st->aux = a2;
    } else if constexpr (OP == FIN_CG_BETA) {
        if (!finite(a0)) { fail(FAIL_NONFINITE); return; }
        if (st->zz == 0.0) { fail(FAIL_BREAKDOWN); return; }
        st->beta_re = a0 / st->zz;
        st->beta_im = 0.0;
        st->zz = a0;
    }
}

// One compiled copy (not inlined) serves the finalize kernel and the vector kernels that
// run a finalize: inlined into different kernels, the compiler may contract the scalar
// arithmetic into fused multiply-adds differently, and the two paths would differ in the
// last bits.
static __device__ __noinline__ void fin_op_rt(int op, RhsState *st, double a0, double a1, double a2) {
#define FIN_RT(X) \
    case X: fin_op<X>(st, a0, a1, a2); break;
    switch (op) {
        FIN_RT(FIN_STORE_AUX)
        FIN_RT(FIN_BICG_INIT)
        FIN_RT(FIN_BICG_ALPHA)
        FIN_RT(FIN_BICG_S)
        FIN_RT(FIN_BICG_OMEGA)
        FIN_RT(FIN_BICG_RHO)
        FIN_RT(FIN_CG_R2)
        FIN_RT(FIN_CG_ZZ)
        FIN_RT(FIN_CG_ALPHA)
        FIN_RT(FIN_CG_R)
        FIN_RT(FIN_CG_BETA)
        FIN_RT(FIN_ADD_AUX)
        FIN_RT(FIN_BLOCK_TS)
        default: break;
    }
#undef FIN_RT
}

// Sum of n partials by one wave: lane l adds elements l + 64 (8 m + u) into its
// accumulator u (eight loads in flight), adds its accumulators pairwise, then the lanes
// are added by a butterfly.  Every lane returns the same value; the grouping depends on
// n alone.
__device__ __forceinline__ double wave_sum_fixed(const double *p, int n) {
    const int lane = (int)threadIdx.x & 63;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int j0 = lane;
    for (; j0 + 7 * 64 < n; j0 += 512) {
#pragma unroll
        for (int u = 0; u < 8; u++) acc[u] += p[j0 + u * 64];
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const int j = j0 + u * 64;
        if (j < n) acc[u] += p[j];
    }
    double v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return 0.0 + v;
}

// Finalize of right-hand side `rhs` by one whole wave.  mirror (optional, host-mapped):
// the state is copied there after the step, so the host can poll convergence without a
// device-to-host copy on the stream.
__device__ __forceinline__ void fin_rhs_wave(int op, const double *partials, int nv, int nblocks, int rhs,
                                             RhsState *state, int run_mask, RhsState *mirror) {
    RhsState *st = &state[rhs];
    const bool lane0 = (threadIdx.x & 63) == 0;
    if (st->phase & run_mask) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < nv; k++) v[k] = wave_sum_fixed(partials + ((size_t)rhs * nv + k) * nblocks, nblocks);
        if (lane0) fin_op_rt(op, st, v[0], v[1], v[2]);
    }
    if (mirror && lane0) mirror[rhs] = *st;
}

// Finalize run at the start of the vector kernel that consumes it (PreFin; short partial
// rows only): wave 0 of every block sums the partials of its right-hand side in the
// finalize kernel's order and applies the scalar step to a copy of the state `src`
// held in LDS, which the block then uses; the blocks of grid column 0 store that copy
// to `dst` (a second state buffer, so that no block reads a state another block is
// writing).  The copy is complete (every field) and written for every right-hand side.
// Called by all threads of the block (it holds a barrier).
__device__ __forceinline__ const RhsState *pre_finalize(const PreFin &f, int rhs, RhsState *loc) {
    const double *partials = f.partials;
    if (threadIdx.x < 64) {
        if (threadIdx.x == 0) *loc = f.src[rhs];
        double v[3] = {0.0, 0.0, 0.0};
        const bool run = (f.src[rhs].phase & f.run_mask) != 0;
        if (run)
            for (int k = 0; k < f.nv; k++) v[k] = wave_sum_fixed(partials + ((size_t)rhs * f.nv + k) * f.nblocks, f.nblocks);
        if (threadIdx.x == 0) {
            if (run) fin_op_rt(f.op, loc, v[0], v[1], v[2]);
            if (blockIdx.x == 0) f.dst[rhs] = *loc;
        }
    }
    __syncthreads();
    return loc;
}

}  // namespace wl
