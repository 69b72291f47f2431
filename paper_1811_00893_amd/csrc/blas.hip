// Fused vector kernels of the Krylov solvers and their deterministic reductions.
//
// BiCGStab (van der Vorst's form; the paper names the method in Sec. 2 and notes in
// Sec. 5 that its separate BLAS-like routines each reload their operands) is fused
// into three vector kernels per iteration:
//   p = r + beta (p - omega v)
//   s = r - alpha v                                  with |s|^2
//   x += alpha p + omega s;  r = s - omega t         with |r|^2 and <rhat, r>
// and the CG-on-normal-equations (CGLS) path into two:
//   x += alpha p;  r -= alpha w                      with |r|^2
//   p = z + beta p
// The remaining dot products are fused into the operator's epilogue (dslash.hip).
//
// Reductions accumulate in FP64 whatever the storage precision.  Each block writes
// one partial per value; a one-block-per-RHS finalize kernel sums the partials in a
// fixed order (so results are bitwise reproducible run to run and independent of
// which other right-hand sides share the launch) and runs the scalar step of the
// iteration on the device.
#include "common.h"
#include "device.h"

namespace wl {

constexpr int kBlasBlock = 256;

int blas_nblocks(const Geom &g) { return (g.Vh + kBlasBlock - 1) / kBlasBlock; }

template <int PK, int PX, int OP>
__global__ void __launch_bounds__(kBlasBlock) blas_kernel(const BlasArgs a) {
    using R = real_t<PK>;
    using RX = real_t<PX>;
    const int rhs = blockIdx.y;
    const RhsState *st = a.state ? &a.state[rhs] : nullptr;
    if (st && !(st->phase & a.run_mask)) return;
    const int stride = a.g.stride;
    const int i_raw = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i_raw < a.g.Vh;
    const int i = valid ? i_raw : a.g.Vh - 1;
    double *dst = a.partials;
    const int ps = a.pstride ? a.pstride : (int)gridDim.x;

    if constexpr (OP == BL_P_UPDATE) {
        const Cx<R> beta = {(R)st->beta_re, (R)st->beta_im};
        const Cx<R> omega = {(R)st->omega_re, (R)st->omega_im};
        Cx<R> p[12], r[12], v[12];
        load_site<PK, R>(p, a.a, stride, rhs, i);
        load_site<PK, R>(r, a.b, stride, rhs, i);
        load_site<PK, R>(v, a.c, stride, rhs, i);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            Cx<R> q = csub(p[k], cmul(omega, v[k]));
            p[k] = cadd(r[k], cmul(beta, q));
        }
        if (valid) store_site<PK, R>(a.a, stride, rhs, i, p);
    } else if constexpr (OP == BL_S_UPDATE) {
        const Cx<R> alpha = {(R)st->alpha_re, (R)st->alpha_im};
        Cx<R> r[12], v[12], s[12];
        load_site<PK, R>(r, a.b, stride, rhs, i);
        load_site<PK, R>(v, a.c, stride, rhs, i);
        double n2[1] = {0.0};
#pragma unroll
        for (int k = 0; k < 12; k++) {
            s[k] = csub(r[k], cmul(alpha, v[k]));
            n2[0] += (double)s[k].re * s[k].re + (double)s[k].im * s[k].im;
        }
        if (valid) store_site<PK, R>(a.a, stride, rhs, i, s);
        else n2[0] = 0.0;
        block_reduce_to<1>(n2, dst + (size_t)rhs * ps + blockIdx.x, ps);
    } else if constexpr (OP == BL_XR_UPDATE) {
        const Cx<RX> alpha = {(RX)st->alpha_re, (RX)st->alpha_im};
        const Cx<RX> omega_x = {(RX)st->omega_re, (RX)st->omega_im};
        const Cx<R> omega = {(R)st->omega_re, (R)st->omega_im};
        Cx<R> p[12], s[12], t[12], rh[12];
        Cx<RX> x[12];
        load_site<PK, R>(p, a.a, stride, rhs, i);
        load_site<PK, R>(s, a.b, stride, rhs, i);
        load_site<PK, R>(t, a.d, stride, rhs, i);
        load_site<PK, R>(rh, a.e, stride, rhs, i);
        load_site<PX, RX>(x, a.x, stride, rhs, i);
        double red[3] = {0.0, 0.0, 0.0};
        Cx<R> r[12];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const Cx<RX> pk = {(RX)p[k].re, (RX)p[k].im}, sk = {(RX)s[k].re, (RX)s[k].im};
            x[k] = cadd(x[k], cadd(cmul(alpha, pk), cmul(omega_x, sk)));
            r[k] = csub(s[k], cmul(omega, t[k]));
            red[0] += (double)r[k].re * r[k].re + (double)r[k].im * r[k].im;
            red[1] += (double)rh[k].re * r[k].re + (double)rh[k].im * r[k].im;  // <rhat, r>
            red[2] += (double)rh[k].re * r[k].im - (double)rh[k].im * r[k].re;
        }
        if (valid) {
            store_site<PX, RX>(a.x, stride, rhs, i, x);
            store_site<PK, R>(a.c, stride, rhs, i, r);
        } else {
            red[0] = red[1] = red[2] = 0.0;
        }
        block_reduce_to<3>(red, dst + (size_t)rhs * 3 * ps + blockIdx.x, ps);
    } else if constexpr (OP == BL_COPY_NORM) {
        Cx<R> v[12];
        load_site<PK, R>(v, a.b, stride, rhs, i);
        double n2[1] = {0.0};
#pragma unroll
        for (int k = 0; k < 12; k++) n2[0] += (double)v[k].re * v[k].re + (double)v[k].im * v[k].im;
        if (valid) store_site<PK, R>(a.a, stride, rhs, i, v);
        else n2[0] = 0.0;
        block_reduce_to<1>(n2, dst + (size_t)rhs * ps + blockIdx.x, ps);
    } else if constexpr (OP == BL_CG_XR) {
        const RX alpha_x = (RX)st->alpha_re;
        const R alpha = (R)st->alpha_re;
        Cx<R> p[12], r[12], w[12];
        Cx<RX> x[12];
        load_site<PK, R>(p, a.a, stride, rhs, i);
        load_site<PK, R>(r, a.b, stride, rhs, i);
        load_site<PK, R>(w, a.c, stride, rhs, i);
        load_site<PX, RX>(x, a.x, stride, rhs, i);
        double n2[1] = {0.0};
#pragma unroll
        for (int k = 0; k < 12; k++) {
            x[k] = cadd(x[k], cscale(Cx<RX>{(RX)p[k].re, (RX)p[k].im}, alpha_x));
            r[k] = csub(r[k], cscale(w[k], alpha));
            n2[0] += (double)r[k].re * r[k].re + (double)r[k].im * r[k].im;
        }
        if (valid) {
            store_site<PX, RX>(a.x, stride, rhs, i, x);
            store_site<PK, R>(a.b, stride, rhs, i, r);
        } else {
            n2[0] = 0.0;
        }
        block_reduce_to<1>(n2, dst + (size_t)rhs * ps + blockIdx.x, ps);
    } else if constexpr (OP == BL_CG_P) {
        const R beta = (R)st->beta_re;
        Cx<R> p[12], z[12];
        load_site<PK, R>(p, a.a, stride, rhs, i);
        load_site<PK, R>(z, a.b, stride, rhs, i);
#pragma unroll
        for (int k = 0; k < 12; k++) p[k] = cadd(z[k], cscale(p[k], beta));
        if (valid) store_site<PK, R>(a.a, stride, rhs, i, p);
    } else if constexpr (OP == BL_NORM2) {
        Cx<R> v[12];
        load_site<PK, R>(v, a.a, stride, rhs, i);
        double n2[1] = {0.0};
        if (valid)
#pragma unroll
            for (int k = 0; k < 12; k++) n2[0] += (double)v[k].re * v[k].re + (double)v[k].im * v[k].im;
        block_reduce_to<1>(n2, dst + (size_t)rhs * ps + blockIdx.x, ps);
    }
}

template <int PK, int PX>
static hipError_t launch_blas_t(int op, const BlasArgs &a, hipStream_t s) {
    dim3 grid(blas_nblocks(a.g), a.nrhs), block(kBlasBlock);
    switch (op) {
        case BL_P_UPDATE: hipLaunchKernelGGL((blas_kernel<PK, PX, BL_P_UPDATE>), grid, block, 0, s, a); break;
        case BL_S_UPDATE: hipLaunchKernelGGL((blas_kernel<PK, PX, BL_S_UPDATE>), grid, block, 0, s, a); break;
        case BL_XR_UPDATE: hipLaunchKernelGGL((blas_kernel<PK, PX, BL_XR_UPDATE>), grid, block, 0, s, a); break;
        case BL_COPY_NORM: hipLaunchKernelGGL((blas_kernel<PK, PX, BL_COPY_NORM>), grid, block, 0, s, a); break;
        case BL_CG_XR: hipLaunchKernelGGL((blas_kernel<PK, PX, BL_CG_XR>), grid, block, 0, s, a); break;
        case BL_CG_P: hipLaunchKernelGGL((blas_kernel<PK, PX, BL_CG_P>), grid, block, 0, s, a); break;
        case BL_NORM2: hipLaunchKernelGGL((blas_kernel<PK, PX, BL_NORM2>), grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_blas(int op, const BlasArgs &a, hipStream_t s) {
    const int pk = a.a.prec, px = a.x.data ? a.x.prec : pk;
    if (pk == P64 && px == P64) return launch_blas_t<P64, P64>(op, a, s);
    if (pk == P32 && px == P32) return launch_blas_t<P32, P32>(op, a, s);
    if (pk == P16 && px == P32) return launch_blas_t<P16, P32>(op, a, s);
    if (pk == P16 && px == P16) return launch_blas_t<P16, P16>(op, a, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------
// Finalize: sum the per-block partials of one RHS in a fixed order, then the scalar
// step.  One block per RHS.
__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

template <int OP>
__device__ void fin_op(RhsState *st, double a0, double a1, double a2);

// mirror (optional, host-mapped): every RHS's state is copied there after the step, so
// the host can poll convergence without a device-to-host copy on the stream.
template <int OP>
__global__ void __launch_bounds__(256) finalize_kernel(const double *partials, int nv, int nblocks,
                                                       RhsState *state, int run_mask, RhsState *mirror) {
    const int rhs = blockIdx.x;
    RhsState *st = &state[rhs];
    if (st->phase & run_mask) {
        __shared__ double tot[3];
        double v[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < nv; k++) {
            // 8 independent accumulators keep 8 loads in flight per thread; the grouping
            // is fixed, so the sum is the same on every run
            const double *p = partials + ((size_t)rhs * nv + k) * nblocks;
            double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            const int step = blockDim.x * 8;
            int j0 = threadIdx.x;
            for (; j0 + 7 * (int)blockDim.x < nblocks; j0 += step) {
#pragma unroll
                for (int u = 0; u < 8; u++) acc[u] += p[j0 + u * blockDim.x];
            }
            for (int u = 0; u < 8; u++) {
                const int j = j0 + u * blockDim.x;
                if (j < nblocks) acc[u] += p[j];
            }
            v[k] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        }
        block_reduce_to<3>(v, tot, 1);
        if (threadIdx.x == 0) fin_op<OP>(st, tot[0], tot[1], tot[2]);
    }
    if (mirror && threadIdx.x == 0) mirror[rhs] = *st;
}

template <int OP>
__device__ void fin_op(RhsState *st, const double a0, const double a1, const double a2) {
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
        if (st->phase == PH_SCONV || a0 <= st->stop2) { st->phase = PH_DONE; return; }
        const double rn = sqrt(a1 * a1 + a2 * a2);
        if (!(rn > 1e-30 * sqrt(st->rhat2 * a0))) { fail(FAIL_BREAKDOWN); return; }
        // beta = (rho'/rho) (alpha/omega)
        const double d1 = st->rho_re * st->rho_re + st->rho_im * st->rho_im;
        const double q1r = (a1 * st->rho_re + a2 * st->rho_im) / d1, q1i = (a2 * st->rho_re - a1 * st->rho_im) / d1;
        const double d2 = st->omega_re * st->omega_re + st->omega_im * st->omega_im;
        const double q2r = (st->alpha_re * st->omega_re + st->alpha_im * st->omega_im) / d2;
        const double q2i = (st->alpha_im * st->omega_re - st->alpha_re * st->omega_im) / d2;
        st->beta_re = q1r * q2r - q1i * q2i;
        st->beta_im = q1r * q2i + q1i * q2r;
        st->rho_re = a1;
        st->rho_im = a2;
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
    } else if constexpr (OP == FIN_CG_BETA) {
        if (!finite(a0)) { fail(FAIL_NONFINITE); return; }
        if (st->zz == 0.0) { fail(FAIL_BREAKDOWN); return; }
        st->beta_re = a0 / st->zz;
        st->beta_im = 0.0;
        st->zz = a0;
    }
}

hipError_t launch_finalize(int op, const double *partials, int nvals, int nblocks, int nrhs, RhsState *state,
                           int run_mask, hipStream_t s, RhsState *mirror) {
    dim3 grid(nrhs), block(256);
#define FIN_CASE(X) \
    case X: hipLaunchKernelGGL((finalize_kernel<X>), grid, block, 0, s, partials, nvals, nblocks, state, run_mask, mirror); break;
    switch (op) {
        FIN_CASE(FIN_STORE_AUX)
        FIN_CASE(FIN_BICG_INIT)
        FIN_CASE(FIN_BICG_ALPHA)
        FIN_CASE(FIN_BICG_S)
        FIN_CASE(FIN_BICG_OMEGA)
        FIN_CASE(FIN_BICG_RHO)
        FIN_CASE(FIN_CG_R2)
        FIN_CASE(FIN_CG_ZZ)
        FIN_CASE(FIN_CG_ALPHA)
        FIN_CASE(FIN_CG_R)
        FIN_CASE(FIN_CG_BETA)
        FIN_CASE(FIN_ADD_AUX)
        default: return hipErrorInvalidValue;
    }
#undef FIN_CASE
    return hipGetLastError();
}

// Fill kernel (used instead of a memset so that the sequence stays capturable).
__global__ void zero_kernel(uint4 *p, size_t n16) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n16; k += (size_t)gridDim.x * blockDim.x)
        p[k] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_zero(const Spinor &f, const Geom &g, int nrhs, hipStream_t s) {
    const size_t bytes = (size_t)nrhs * 12 * spinor_plane_bytes(f.prec, g);
    // plane strides are multiples of 64 elements, so every size here is a multiple of 16 bytes
    hipLaunchKernelGGL(zero_kernel, dim3(1024), dim3(256), 0, s, (uint4 *)f.data, bytes / 16);
    if (f.prec == P16 && f.scale)
        hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(256), 0, s, (uint4 *)f.scale, (size_t)nrhs * g.stride * 4 / 16);
    return hipGetLastError();
}

}  // namespace wl
