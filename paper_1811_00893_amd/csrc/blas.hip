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
// This file is compiled without multiply-add contraction (build.py): which product of a
// complex multiply the compiler would fuse depends on where the scalars come from (scalar
// registers, or LDS when a kernel runs the finalize of its input), and both forms of a
// kernel must give the same bits.
//
// Reductions accumulate in FP64 whatever the storage precision.  Each block writes
// one partial per value; a one-block-per-RHS finalize kernel sums the partials in a
// fixed order (so results are bitwise reproducible run to run and independent of
// which other right-hand sides share the launch) and runs the scalar step of the
// iteration on the device.
#include "common.h"
#include "device.h"
#include "finalize.h"

namespace wl {

// Operands of the ops (BlasOp in common.h), by slot: which are read and which written.
enum : int { SA = 1, SB = 2, SC = 4, SD = 8, SE = 16, SX = 32 };
template <int OP>
struct OpShape;
template <> struct OpShape<BL_P_UPDATE> { static constexpr int LD = SA | SB | SC, ST = SA, NV = 0; };
template <> struct OpShape<BL_S_UPDATE> { static constexpr int LD = SB | SC, ST = SA, NV = 1; };
template <> struct OpShape<BL_XR_UPDATE> { static constexpr int LD = SA | SB | SD | SE | SX, ST = SC | SX, NV = 3; };
template <> struct OpShape<BL_COPY_NORM> { static constexpr int LD = SB, ST = SA, NV = 1; };
template <> struct OpShape<BL_CG_XR> { static constexpr int LD = SA | SB | SC | SX, ST = SB | SX, NV = 1; };
template <> struct OpShape<BL_CG_P> { static constexpr int LD = SA | SB, ST = SA, NV = 0; };
template <> struct OpShape<BL_NORM2> { static constexpr int LD = SA, ST = 0, NV = 1; };

// N complex numbers of every operand slot (a whole site, or one 16-byte element).
template <int N, typename R, typename RX>
struct Opnds {
    Cx<R> a[N], b[N], c[N], d[N], e[N];
    Cx<RX> x[N];
};

template <typename R>
__device__ __forceinline__ double norm2_of(Cx<R> v) {
    return (double)v.re * v.re + (double)v.im * v.im;
}

// The arithmetic of one op on N complex numbers; reductions accumulate into red (FP64).
template <int OP, int N, typename R, typename RX>
__device__ __forceinline__ void blas_math(const RhsState *st, Opnds<N, R, RX> &o, double (&red)[3]) {
    if constexpr (OP == BL_P_UPDATE) {
        const Cx<R> beta = {(R)st->beta_re, (R)st->beta_im};
        const Cx<R> omega = {(R)st->omega_re, (R)st->omega_im};
#pragma unroll
        for (int k = 0; k < N; k++) o.a[k] = cadd(o.b[k], cmul(beta, csub(o.a[k], cmul(omega, o.c[k]))));
    } else if constexpr (OP == BL_S_UPDATE) {
        const Cx<R> alpha = {(R)st->alpha_re, (R)st->alpha_im};
#pragma unroll
        for (int k = 0; k < N; k++) {
            o.a[k] = csub(o.b[k], cmul(alpha, o.c[k]));
            red[0] += norm2_of(o.a[k]);
        }
    } else if constexpr (OP == BL_XR_UPDATE) {
        const Cx<RX> alpha = {(RX)st->alpha_re, (RX)st->alpha_im};
        const Cx<RX> omega_x = {(RX)st->omega_re, (RX)st->omega_im};
        const Cx<R> omega = {(R)st->omega_re, (R)st->omega_im};
#pragma unroll
        for (int k = 0; k < N; k++) {
            const Cx<RX> pk = {(RX)o.a[k].re, (RX)o.a[k].im}, sk = {(RX)o.b[k].re, (RX)o.b[k].im};
            o.x[k] = cadd(o.x[k], cadd(cmul(alpha, pk), cmul(omega_x, sk)));
            const Cx<R> r = csub(o.b[k], cmul(omega, o.d[k]));
            o.c[k] = r;
            red[0] += norm2_of(r);
            red[1] += (double)o.e[k].re * r.re + (double)o.e[k].im * r.im;  // <rhat, r>
            red[2] += (double)o.e[k].re * r.im - (double)o.e[k].im * r.re;
        }
    } else if constexpr (OP == BL_COPY_NORM) {
#pragma unroll
        for (int k = 0; k < N; k++) {
            o.a[k] = o.b[k];
            red[0] += norm2_of(o.b[k]);
        }
    } else if constexpr (OP == BL_CG_XR) {
        const RX alpha_x = (RX)st->alpha_re;
        const R alpha = (R)st->alpha_re;
#pragma unroll
        for (int k = 0; k < N; k++) {
            o.x[k] = cadd(o.x[k], cscale(Cx<RX>{(RX)o.a[k].re, (RX)o.a[k].im}, alpha_x));
            o.b[k] = csub(o.b[k], cscale(o.c[k], alpha));
            red[0] += norm2_of(o.b[k]);
        }
    } else if constexpr (OP == BL_CG_P) {
        const R beta = (R)st->beta_re;
#pragma unroll
        for (int k = 0; k < N; k++) o.a[k] = cadd(o.b[k], cscale(o.a[k], beta));
    } else if constexpr (OP == BL_NORM2) {
#pragma unroll
        for (int k = 0; k < N; k++) red[0] += norm2_of(o.a[k]);
    }
}

// FP64 and FP32 storage: one 16-byte element (1 or 2 complex numbers) of one site per
// thread.  Every op is elementwise over the spinor components, so a thread holds one
// element of each operand: few registers, many waves in flight, and each wave reads and
// writes whole contiguous runs of one plane.  A block covers kElemBlock consecutive sites
// of one element plane (blockIdx.x = plane * nbs + site block) and leaves one partial per
// reduced value.
constexpr int kElemBlock = 1024;

template <int P, int OP, bool PRE = false, bool NT = false>
__global__ void __launch_bounds__(kElemBlock) blas_elem_kernel(const BlasArgs a, int nbs) {
    using R = real_t<P>;
    using S = OpShape<OP>;
    constexpr int CPE = SpinorPack<P>::CPE, NEL = SpinorPack<P>::NEL;
    const int rhs = blockIdx.y;
    const RhsState *st = a.state ? &a.state[rhs] : nullptr;
    if constexpr (PRE) {  // the finalize of this op's input, then its state (in LDS) is the one used
        __shared__ RhsState pre_st;
        st = pre_finalize(a.pre, rhs, &pre_st);
    }
    if (st && !(st->phase & a.run_mask)) return;
    const int e = blockIdx.x / nbs;
    const int i_raw = (blockIdx.x - e * nbs) * kElemBlock + threadIdx.x;
    const bool valid = i_raw < a.g.Vh;
    const unsigned off = (unsigned)(valid ? i_raw : a.g.Vh - 1) * 16u;
    const int plane = rhs * NEL + e, stride = a.g.stride;
    Opnds<CPE, R, R> o;
    if constexpr (S::LD & SA) ld_elem<P, R, NT>(o.a, splane(a.a.data, plane, stride), off);
    if constexpr (S::LD & SB) ld_elem<P, R, NT>(o.b, splane(a.b.data, plane, stride), off);
    if constexpr (S::LD & SC) ld_elem<P, R, NT>(o.c, splane(a.c.data, plane, stride), off);
    if constexpr (S::LD & SD) ld_elem<P, R, NT>(o.d, splane(a.d.data, plane, stride), off);
    if constexpr (S::LD & SE) ld_elem<P, R, NT>(o.e, splane(a.e.data, plane, stride), off);
    if constexpr (S::LD & SX) ld_elem<P, R, NT>(o.x, splane(a.x.data, plane, stride), off);
    double red[3] = {0.0, 0.0, 0.0};
    blas_math<OP, CPE, R, R>(st, o, red);
    if (valid) {
        if constexpr (S::ST & SA) st_elem<P, R, NT>(const_cast<gchar *>(splane(a.a.data, plane, stride)), off, o.a);
        if constexpr (S::ST & SB) st_elem<P, R, NT>(const_cast<gchar *>(splane(a.b.data, plane, stride)), off, o.b);
        if constexpr (S::ST & SC) st_elem<P, R, NT>(const_cast<gchar *>(splane(a.c.data, plane, stride)), off, o.c);
        if constexpr (S::ST & SX) st_elem<P, R, NT>(const_cast<gchar *>(splane(a.x.data, plane, stride)), off, o.x);
    } else {
        red[0] = red[1] = red[2] = 0.0;
    }
    if constexpr (S::NV > 0) {
        const int ps = a.pstride ? a.pstride : (int)gridDim.x;
        double v[S::NV];
#pragma unroll
        for (int k = 0; k < S::NV; k++) v[k] = red[k];
        block_reduce_to<S::NV>(v, a.partials + (size_t)rhs * S::NV * ps + blockIdx.x, ps);
    }
}

// FP16 storage: the per-site scale couples all 24 reals of a site, so one thread takes a
// whole site (x may be FP32 or FP16).
constexpr int kSiteBlock = 256;

template <int PK, int PX, int OP, bool PRE = false, bool NT = false>
__global__ void __launch_bounds__(kSiteBlock) blas_site_kernel(const BlasArgs a) {
    using R = real_t<PK>;
    using RX = real_t<PX>;
    using S = OpShape<OP>;
    const int rhs = blockIdx.y;
    const RhsState *st = a.state ? &a.state[rhs] : nullptr;
    if constexpr (PRE) {  // the finalize of this op's input, then its state (in LDS) is the one used
        __shared__ RhsState pre_st;
        st = pre_finalize(a.pre, rhs, &pre_st);
    }
    if (st && !(st->phase & a.run_mask)) return;
    const int stride = a.g.stride;
    const int i_raw = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i_raw < a.g.Vh;
    const int i = valid ? i_raw : a.g.Vh - 1;
    Opnds<12, R, RX> o;
    if constexpr (S::LD & SA) load_site<PK, R, NT>(o.a, a.a, stride, rhs, i);
    if constexpr (S::LD & SB) load_site<PK, R, NT>(o.b, a.b, stride, rhs, i);
    if constexpr (S::LD & SC) load_site<PK, R, NT>(o.c, a.c, stride, rhs, i);
    if constexpr (S::LD & SD) load_site<PK, R, NT>(o.d, a.d, stride, rhs, i);
    if constexpr (S::LD & SE) load_site<PK, R, NT>(o.e, a.e, stride, rhs, i);
    if constexpr (S::LD & SX) load_site<PX, RX, NT>(o.x, a.x, stride, rhs, i);
    double red[3] = {0.0, 0.0, 0.0};
    blas_math<OP, 12, R, RX>(st, o, red);
    if (valid) {
        if constexpr (S::ST & SA) store_site<PK, R, NT>(a.a, stride, rhs, i, o.a);
        if constexpr (S::ST & SB) store_site<PK, R, NT>(a.b, stride, rhs, i, o.b);
        if constexpr (S::ST & SC) store_site<PK, R, NT>(a.c, stride, rhs, i, o.c);
        if constexpr (S::ST & SX) store_site<PX, RX, NT>(a.x, stride, rhs, i, o.x);
    } else {
        red[0] = red[1] = red[2] = 0.0;
    }
    if constexpr (S::NV > 0) {
        const int ps = a.pstride ? a.pstride : (int)gridDim.x;
        double v[S::NV];
#pragma unroll
        for (int k = 0; k < S::NV; k++) v[k] = red[k];
        block_reduce_to<S::NV>(v, a.partials + (size_t)rhs * S::NV * ps + blockIdx.x, ps);
    }
}

int blas_nblocks(const Geom &g, int prec) {
    if (prec == P16) return (g.Vh + kSiteBlock - 1) / kSiteBlock;
    return (prec == P64 ? 12 : 6) * ((g.Vh + kElemBlock - 1) / kElemBlock);
}

// Vectors above this size are loaded and stored non-temporally (NT): about eight of them
// stream through each BiCGStab iteration, more than the 256 MB Infinity Cache holds, so no
// kernel finds the previous one's output there, and streaming hints let a copy-shaped
// kernel move 6.5 instead of 6.1 TB/s.  Smaller vectors keep ordinary loads and stores,
// so the next kernel of the iteration can find them in the caches.
constexpr size_t kStreamBytes = (size_t)32 << 20;
static bool streaming(const BlasArgs &a, int pk) {
    return (size_t)a.nrhs * spinor_field_bytes(pk, a.g) > kStreamBytes;
}
template <int OP, bool PRE>
static void launch_op_elem(int pk, const BlasArgs &a, hipStream_t s) {
    const int nbs = (a.g.Vh + kElemBlock - 1) / kElemBlock;
    const dim3 grid(blas_nblocks(a.g, pk), a.nrhs), block(kElemBlock);
    if constexpr (!PRE) {  // (the finalizing variants run on small lattices only)
        if (streaming(a, pk)) {
            if (pk == P64) hipLaunchKernelGGL((blas_elem_kernel<P64, OP, false, true>), grid, block, 0, s, a, nbs);
            else hipLaunchKernelGGL((blas_elem_kernel<P32, OP, false, true>), grid, block, 0, s, a, nbs);
            return;
        }
    }
    if (pk == P64) hipLaunchKernelGGL((blas_elem_kernel<P64, OP, PRE>), grid, block, 0, s, a, nbs);
    else hipLaunchKernelGGL((blas_elem_kernel<P32, OP, PRE>), grid, block, 0, s, a, nbs);
}
template <int PX, int OP, bool PRE>
static void launch_op_site(const BlasArgs &a, hipStream_t s) {
    const dim3 grid(blas_nblocks(a.g, P16), a.nrhs), block(kSiteBlock);
    if constexpr (!PRE) {
        if (streaming(a, P16)) {
            hipLaunchKernelGGL((blas_site_kernel<P16, PX, OP, false, true>), grid, block, 0, s, a);
            return;
        }
    }
    hipLaunchKernelGGL((blas_site_kernel<P16, PX, OP, PRE>), grid, block, 0, s, a);
}
template <int OP, bool PRE>
static hipError_t launch_op_t(int pk, int px, const BlasArgs &a, hipStream_t s) {
    if ((pk == P64 || pk == P32) && px == pk) launch_op_elem<OP, PRE>(pk, a, s);
    else if (pk == P16 && px == P32) launch_op_site<P32, OP, PRE>(a, s);
    else if (pk == P16 && px == P16) launch_op_site<P16, OP, PRE>(a, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}
// the vector kernels of the BiCGStab iteration may run the finalize of their input first
template <int OP>
static hipError_t launch_op(int pk, int px, const BlasArgs &a, hipStream_t s) {
    if constexpr (OP == BL_S_UPDATE || OP == BL_XR_UPDATE) {
        if (a.pre.on) {
            if (a.pre.nblocks > kPreFinMax || a.pre.nv > 3 || !a.pre.partials || a.pre.partials == a.partials ||
                !a.pre.src || !a.pre.dst || a.pre.src == a.pre.dst)
                return hipErrorInvalidValue;
            return launch_op_t<OP, true>(pk, px, a, s);
        }
    } else {
        if (a.pre.on) return hipErrorInvalidValue;
    }
    return launch_op_t<OP, false>(pk, px, a, s);
}

hipError_t launch_blas(int op, const BlasArgs &a, hipStream_t s) {
    const int pk = a.a.prec, px = a.x.data ? a.x.prec : pk;
    if (a.nrhs < 1 || a.nrhs > 65535) return hipErrorInvalidValue;
    switch (op) {
        case BL_P_UPDATE: return launch_op<BL_P_UPDATE>(pk, px, a, s);
        case BL_S_UPDATE: return launch_op<BL_S_UPDATE>(pk, px, a, s);
        case BL_XR_UPDATE: return launch_op<BL_XR_UPDATE>(pk, px, a, s);
        case BL_COPY_NORM: return launch_op<BL_COPY_NORM>(pk, px, a, s);
        case BL_CG_XR: return launch_op<BL_CG_XR>(pk, px, a, s);
        case BL_CG_P: return launch_op<BL_CG_P>(pk, px, a, s);
        case BL_NORM2: return launch_op<BL_NORM2>(pk, px, a, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------------
// Finalize kernel: one block per RHS sums that RHS's partials in a fixed order and runs
// the scalar step (finalize.h).  Rows a vector kernel could finalize (up to kPreFinMax
// partials) take one wave, exactly as that kernel does (PreFin); longer rows 256 threads,
// beyond 4096 partials 1024 (each thread with the same grouping, then the waves in order).
template <int OP>
__global__ void __launch_bounds__(1024) finalize_kernel(const double *partials, int nv, int nblocks,
                                                       RhsState *state, int run_mask, RhsState *mirror) {
    const int rhs = blockIdx.x;
    if (blockDim.x == 64) {
        fin_rhs_wave(OP, partials, nv, nblocks, rhs, state, run_mask, mirror);
        return;
    }
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

hipError_t launch_finalize(int op, const double *partials, int nvals, int nblocks, int nrhs, RhsState *state,
                           int run_mask, hipStream_t s, RhsState *mirror) {
    // a wider block keeps more loads in flight over long partial rows; the block size is a
    // function of the row length alone, so the summation order stays fixed
    dim3 grid(nrhs), block(nblocks <= kPreFinMax ? 64 : (nblocks > 4096 ? 1024 : 256));
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
        FIN_CASE(FIN_BLOCK_TS)
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
