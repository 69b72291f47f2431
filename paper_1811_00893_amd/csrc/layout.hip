// Layout and precision conversion kernels (boundary of the library, not the hot loop).
//
//   * canonical complex128 spinors [rhs][site][spin][colour]  <->  parity-split planes;
//   * FP64 -> FP32 / FP16-with-per-site-scale encodings (FP16: scale s = max |component|
//     over the 24 reals of the site in FP32, h = fp16_rne(fp32(v / s)));
//   * gauge packing: canonical links -> parity-split planes.  Full (18-real) links carry
//     the antiperiodic sign of the time boundary folded into U_t(x) on the slice
//     t = Lt - 1 (that link serves both the forward hop out of t = Lt-1 and the backward
//     hop out of t = 0).  SU(3) links may instead be stored as their first two rows
//     (12 reals): the third row of a special unitary matrix is the complex conjugate of
//     the cross product of the first two, and the hop kernel rebuilds it and applies the
//     boundary sign itself (a folded sign would flip det U and break that identity);
//   * the defect-correction glue (scaled conversion of the residual, FP64 accumulation
//     of the correction), and a plain streaming copy used as a bandwidth reference.
#include "common.h"
#include "device.h"

namespace wl {

__device__ __forceinline__ int full_site(const Geom &g, int i, int par, int *t_out) {
    const SiteXY c = cb_coords(g, i, par);
    const int x = 2 * c.xh + c.b;
    if (t_out) *t_out = c.t;
    return x + g.L[0] * (c.y + g.L[1] * (c.z + g.L[2] * c.t));
}

template <int P>
__global__ void __launch_bounds__(256) to_parity_kernel(Spinor f, const double2 *canon, Geom g, int par,
                                                        double scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.Vh) return;
    const int rhs = blockIdx.y;
    const size_t V = (size_t)g.Vh * 2;
    const int s = full_site(g, i, par, nullptr);
    const double2 *src = canon + ((size_t)rhs * V + s) * 12;
    using R = real_t<P>;
    Cx<R> v[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const double2 d = src[k];
        v[k] = {(R)(d.x * scale), (R)(d.y * scale)};
    }
    store_site<P, R>(f, g.stride, rhs, i, v);
}

template <int P>
__global__ void __launch_bounds__(256) from_parity_kernel(double2 *canon, Spinor f, Geom g, int par) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.Vh) return;
    const int rhs = blockIdx.y;
    const size_t V = (size_t)g.Vh * 2;
    const int s = full_site(g, i, par, nullptr);
    using R = real_t<P>;
    Cx<R> v[12];
    load_site<P, R>(v, f, g.stride, rhs, i);
    double2 *dst = canon + ((size_t)rhs * V + s) * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) dst[k] = make_double2((double)v[k].re, (double)v[k].im);
}

template <int PD>
__global__ void __launch_bounds__(256) convert_kernel(Spinor dst, Spinor src, Geom g, const RhsState *state,
                                                      int inv_sqrt_aux) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.Vh) return;
    const int rhs = blockIdx.y;
    double c = 1.0;
    if (state && inv_sqrt_aux) {
        const double a = state[rhs].aux;
        c = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
    }
    Cx<double> v[12];
    load_site<P64, double>(v, src, g.stride, rhs, i);
    using R = real_t<PD>;
    Cx<R> o[12];
#pragma unroll
    for (int k = 0; k < 12; k++) o[k] = {(R)(v[k].re * c), (R)(v[k].im * c)};
    store_site<PD, R>(dst, g.stride, rhs, i, o);
}

template <int PE>
__global__ void __launch_bounds__(256) axpy_f64_kernel(Spinor x, Spinor e, Geom g, const RhsState *state,
                                                       int sqrt_aux) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.Vh) return;
    const int rhs = blockIdx.y;
    double c = 1.0;
    if (sqrt_aux) {
        const double a = state[rhs].aux;
        c = a > 0.0 ? sqrt(a) : 0.0;
    }
    using R = real_t<PE>;
    Cx<R> ev[12];
    load_site<PE, R>(ev, e, g.stride, rhs, i);
    Cx<double> xv[12];
    load_site<P64, double>(xv, x, g.stride, rhs, i);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        xv[k].re = fma(c, (double)ev[k].re, xv[k].re);
        xv[k].im = fma(c, (double)ev[k].im, xv[k].im);
    }
    store_site<P64, double>(x, g.stride, rhs, i, xv);
}

template <int P>
__global__ void __launch_bounds__(256) gauge_pack_kernel(void *dst, const double2 *canon, Geom g, int recon) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.Vh) return;
    const int par = blockIdx.y >> 2, mu = blockIdx.y & 3;
    int t;
    const int s = full_site(g, i, par, &t);
    const int ne = recon == 12 ? 6 : 9;
    const int nl = link_elems(P, ne);
    constexpr int CPL = LinkPack<P>::CPL;
    const double sgn = (recon == 18 && mu == 3 && t == g.L[3] - 1) ? -1.0 : 1.0;
    const double2 *src = canon + ((size_t)s * 4 + mu) * 9;
    using R = real_t<P>;
    const unsigned off = (unsigned)i * LinkPack<P>::EB;
    for (int e = 0; e < nl; e++) {
        Cx<R> x[CPL];
        for (int k = 0; k < CPL; k++) {
            const int idx = e * CPL + k;  // entries past the last are padding
            const double2 d = idx < ne ? src[idx] : make_double2(0.0, 0.0);
            x[k] = {(R)(sgn * d.x), (R)(sgn * d.y)};
        }
        st_link_elem<P, R>(const_cast<gchar *>(lplane<P>(dst, (par * 4 + mu) * nl + e, g.stride)), off, x);
    }
}

// max over entries of |U U^dag - 1| and |det U - 1| for each link; flag if above tol
__global__ void su3_check_kernel(const double2 *canon, size_t nlinks, double tol, int *flag) {
    bool bad = false;
    for (size_t l = blockIdx.x * (size_t)blockDim.x + threadIdx.x; l < nlinks; l += (size_t)gridDim.x * blockDim.x) {
        Cx<double> u[3][3];
        for (int e = 0; e < 9; e++) u[e / 3][e % 3] = {canon[l * 9 + e].x, canon[l * 9 + e].y};
        double dev = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                Cx<double> acc = {a == b ? -1.0 : 0.0, 0.0};
                for (int k = 0; k < 3; k++) acc = cfma_conj(acc, u[b][k], u[a][k]);  // (U U^dag)_ab - d_ab
                dev = fmax(dev, fabs(acc.re) + fabs(acc.im));
            }
        // det via the first row and the cofactors of rows 1, 2
        const Cx<double> c0 = csub(cmul(u[1][1], u[2][2]), cmul(u[1][2], u[2][1]));
        const Cx<double> c1 = csub(cmul(u[1][2], u[2][0]), cmul(u[1][0], u[2][2]));
        const Cx<double> c2 = csub(cmul(u[1][0], u[2][1]), cmul(u[1][1], u[2][0]));
        const Cx<double> det = cadd(cadd(cmul(u[0][0], c0), cmul(u[0][1], c1)), cmul(u[0][2], c2));
        dev = fmax(dev, fabs(det.re - 1.0) + fabs(det.im));
        bad |= !(dev <= tol);
    }
    if (bad) atomicOr(flag, 1);
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Bandwidth probes.  One 16-byte element per thread and no loop: a wave moves one
// contiguous 1 KiB run and ends, which keeps the most requests in flight on gfx950 (a
// thread that loops waits for its own earlier stores before its next loads return).
// Loads and stores are non-temporal, the fastest one-pass pattern measured (a 2 GiB copy
// 6.5-6.6 TB/s against 6.1 with ordinary loads and stores; two or more elements per
// thread were slower still).
__global__ void __launch_bounds__(256) stream_copy_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                          size_t n16) {
    const size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (k < n16)
        __builtin_nontemporal_store(__builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(src) + k),
                                    reinterpret_cast<u32x4 *>(dst) + k);
}

// Read-only stream: each lane folds its 16 bytes into one word and, only when that word
// equals an arbitrary constant, XORs it into one of kStreamSink words.  The branch depends
// on the data, so no load can be elided, and almost no lane ever writes.
constexpr unsigned kStreamSink = 8192;
__global__ void __launch_bounds__(256) stream_read_kernel(const uint4 *__restrict__ src, size_t n16,
                                                          unsigned *sink) {
    const size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (k < n16) {
        const u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(src) + k);
        const unsigned w = a.x ^ a.y ^ a.z ^ a.w;
        if (w == 0x9E3779B9u) atomicXor(&sink[k % kStreamSink], w);
    }
}

__global__ void copy_tail_kernel(unsigned char *dst, const unsigned char *src, size_t n) {
    const size_t k = threadIdx.x;
    if (k < n) dst[k] = src[k];
}

__global__ void check_finite_kernel(const double *p, size_t n, int *flag) {
    bool bad = false;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(p[k]);
    if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------------
static inline dim3 site_grid(const Geom &g, int ny) { return dim3((g.Vh + 255) / 256, ny); }

hipError_t launch_to_parity(Spinor f, const double *canon, const Geom &g, int par, int nrhs, double scale,
                            hipStream_t s) {
    const dim3 grid = site_grid(g, nrhs), block(256);
    const double2 *c = reinterpret_cast<const double2 *>(canon);
    switch (f.prec) {
        case P64: hipLaunchKernelGGL(to_parity_kernel<P64>, grid, block, 0, s, f, c, g, par, scale); break;
        case P32: hipLaunchKernelGGL(to_parity_kernel<P32>, grid, block, 0, s, f, c, g, par, scale); break;
        case P16: hipLaunchKernelGGL(to_parity_kernel<P16>, grid, block, 0, s, f, c, g, par, scale); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_from_parity(double *canon, Spinor f, const Geom &g, int par, int nrhs, hipStream_t s) {
    const dim3 grid = site_grid(g, nrhs), block(256);
    double2 *c = reinterpret_cast<double2 *>(canon);
    switch (f.prec) {
        case P64: hipLaunchKernelGGL(from_parity_kernel<P64>, grid, block, 0, s, c, f, g, par); break;
        case P32: hipLaunchKernelGGL(from_parity_kernel<P32>, grid, block, 0, s, c, f, g, par); break;
        case P16: hipLaunchKernelGGL(from_parity_kernel<P16>, grid, block, 0, s, c, f, g, par); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(Spinor dst, Spinor src, const Geom &g, int nrhs, const RhsState *state, int inv_sqrt_aux,
                          hipStream_t s) {
    if (src.prec != P64) return hipErrorInvalidValue;
    const dim3 grid = site_grid(g, nrhs), block(256);
    switch (dst.prec) {
        case P64: hipLaunchKernelGGL(convert_kernel<P64>, grid, block, 0, s, dst, src, g, state, inv_sqrt_aux); break;
        case P32: hipLaunchKernelGGL(convert_kernel<P32>, grid, block, 0, s, dst, src, g, state, inv_sqrt_aux); break;
        case P16: hipLaunchKernelGGL(convert_kernel<P16>, grid, block, 0, s, dst, src, g, state, inv_sqrt_aux); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_axpy_f64(Spinor x64, Spinor e, const Geom &g, int nrhs, const RhsState *state, int sqrt_aux,
                           hipStream_t s) {
    if (x64.prec != P64 || (sqrt_aux && !state)) return hipErrorInvalidValue;
    const dim3 grid = site_grid(g, nrhs), block(256);
    switch (e.prec) {
        case P64: hipLaunchKernelGGL(axpy_f64_kernel<P64>, grid, block, 0, s, x64, e, g, state, sqrt_aux); break;
        case P32: hipLaunchKernelGGL(axpy_f64_kernel<P32>, grid, block, 0, s, x64, e, g, state, sqrt_aux); break;
        case P16: hipLaunchKernelGGL(axpy_f64_kernel<P16>, grid, block, 0, s, x64, e, g, state, sqrt_aux); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gauge_pack(void *dst, int prec, const double *canon, const Geom &g, int recon, hipStream_t s) {
    if (recon != 12 && recon != 18) return hipErrorInvalidValue;
    const dim3 grid = site_grid(g, 8), block(256);
    const double2 *c = reinterpret_cast<const double2 *>(canon);
    switch (prec) {
        case P64: hipLaunchKernelGGL(gauge_pack_kernel<P64>, grid, block, 0, s, dst, c, g, recon); break;
        case P32: hipLaunchKernelGGL(gauge_pack_kernel<P32>, grid, block, 0, s, dst, c, g, recon); break;
        case P16: hipLaunchKernelGGL(gauge_pack_kernel<P16>, grid, block, 0, s, dst, c, g, recon); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_su3_check(const double *canon, size_t nlinks, double tol, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(su3_check_kernel, dim3(2048), dim3(256), 0, s, reinterpret_cast<const double2 *>(canon),
                       nlinks, tol, flag);
    return hipGetLastError();
}

hipError_t launch_stream_read(const void *src, size_t bytes, unsigned *sink, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16) hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s,
                                (const uint4 *)src, n16, sink);
    return hipGetLastError();
}

hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16)
        hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s, (uint4 *)dst,
                           (const uint4 *)src, n16);
    const size_t tail = bytes - n16 * 16;
    if (tail)
        hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(64), 0, s, (unsigned char *)dst + n16 * 16,
                           (const unsigned char *)src + n16 * 16, tail);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double *p, size_t n, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(check_finite_kernel, dim3(1024), dim3(256), 0, s, p, n, flag);
    return hipGetLastError();
}

}  // namespace wl
