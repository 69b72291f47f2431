// Device-side helpers: complex arithmetic, per-precision storage access, block reductions.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"

namespace wl {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

template <typename R>
struct Cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> csub(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
// a + i b, a - i b
template <typename R>
__device__ __forceinline__ Cx<R> cadd_i(Cx<R> a, Cx<R> b) { return {a.re - b.im, a.im + b.re}; }
template <typename R>
__device__ __forceinline__ Cx<R> csub_i(Cx<R> a, Cx<R> b) { return {a.re + b.im, a.im - b.re}; }
template <typename R>
__device__ __forceinline__ Cx<R> cscale(Cx<R> a, R s) { return {a.re * s, a.im * s}; }
// a * b
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// acc + a * b
template <typename R>
__device__ __forceinline__ Cx<R> cfma(Cx<R> acc, Cx<R> a, Cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
    return acc;
}
// acc + conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cfma_conj(Cx<R> acc, Cx<R> a, Cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
    return acc;
}

template <int P>
using real_t = typename std::conditional<P == P64, double, float>::type;

// ---- storage access: one complex number at element index idx of a plane array ----
template <int P, typename R>
__device__ __forceinline__ Cx<R> ld_c(const void *base, size_t idx) {
    if constexpr (P == P64) {
        double2 v = reinterpret_cast<const double2 *>(base)[idx];
        return {(R)v.x, (R)v.y};
    } else if constexpr (P == P32) {
        float2 v = reinterpret_cast<const float2 *>(base)[idx];
        return {(R)v.x, (R)v.y};
    } else {
        half2_t v = reinterpret_cast<const half2_t *>(base)[idx];
        return {(R)(float)v.x, (R)(float)v.y};
    }
}

// Streaming (read-once) variant for links: non-temporal so they do not evict spinors.
template <int P, typename R>
__device__ __forceinline__ Cx<R> ld_c_nt(const void *base, size_t idx) {
    if constexpr (P == P64) {
        const dvec2 *p = reinterpret_cast<const dvec2 *>(base) + idx;
        dvec2 v = __builtin_nontemporal_load(p);
        return {(R)v.x, (R)v.y};
    } else if constexpr (P == P32) {
        const fvec2 *p = reinterpret_cast<const fvec2 *>(base) + idx;
        fvec2 v = __builtin_nontemporal_load(p);
        return {(R)v.x, (R)v.y};
    } else {
        const half2_t *p = reinterpret_cast<const half2_t *>(base) + idx;
        half2_t v = __builtin_nontemporal_load(p);
        return {(R)(float)v.x, (R)(float)v.y};
    }
}

template <int P, typename R>
__device__ __forceinline__ void st_c(void *base, size_t idx, Cx<R> v) {
    if constexpr (P == P64) {
        reinterpret_cast<double2 *>(base)[idx] = make_double2((double)v.re, (double)v.im);
    } else if constexpr (P == P32) {
        reinterpret_cast<float2 *>(base)[idx] = make_float2((float)v.re, (float)v.im);
    } else {
        half2_t h;
        h.x = (_Float16)(float)v.re;
        h.y = (_Float16)(float)v.im;
        reinterpret_cast<half2_t *>(base)[idx] = h;
    }
}

// ---- plane addressing: a wave-uniform plane base plus one 32-bit per-lane byte offset,
// so that every plane load of a site shares the same offset register and the base
// stays in scalar registers ----
template <int P>
struct Elem {
    static constexpr unsigned bytes = P == P64 ? 16u : (P == P32 ? 8u : 4u);
};
template <int P>
__device__ __forceinline__ const char *plane_ptr(const void *base, int plane, int stride) {
    return static_cast<const char *>(base) + (size_t)plane * stride * Elem<P>::bytes;
}
template <int P, typename R>
__device__ __forceinline__ Cx<R> ld_p(const char *plane, unsigned off) {
    if constexpr (P == P64) {
        double2 v = *reinterpret_cast<const double2 *>(plane + off);
        return {(R)v.x, (R)v.y};
    } else if constexpr (P == P32) {
        float2 v = *reinterpret_cast<const float2 *>(plane + off);
        return {(R)v.x, (R)v.y};
    } else {
        half2_t v = *reinterpret_cast<const half2_t *>(plane + off);
        return {(R)(float)v.x, (R)(float)v.y};
    }
}
template <int P, typename R>
__device__ __forceinline__ Cx<R> ld_p_nt(const char *plane, unsigned off) {
    if constexpr (P == P64) {
        dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(plane + off));
        return {(R)v.x, (R)v.y};
    } else if constexpr (P == P32) {
        fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const fvec2 *>(plane + off));
        return {(R)v.x, (R)v.y};
    } else {
        half2_t v = __builtin_nontemporal_load(reinterpret_cast<const half2_t *>(plane + off));
        return {(R)(float)v.x, (R)(float)v.y};
    }
}
template <int P, typename R>
__device__ __forceinline__ void st_p(char *plane, unsigned off, Cx<R> v) {
    if constexpr (P == P64) {
        *reinterpret_cast<double2 *>(plane + off) = make_double2((double)v.re, (double)v.im);
    } else if constexpr (P == P32) {
        *reinterpret_cast<float2 *>(plane + off) = make_float2((float)v.re, (float)v.im);
    } else {
        half2_t h;
        h.x = (_Float16)(float)v.re;
        h.y = (_Float16)(float)v.im;
        *reinterpret_cast<half2_t *>(plane + off) = h;
    }
}

// Full site (12 complex) of rhs `r` of a parity field; FP16 values are rescaled.
template <int P, typename R>
__device__ __forceinline__ void load_site(Cx<R> (&v)[12], const Spinor &f, int stride, int r, int i) {
    const unsigned off = (unsigned)i * Elem<P>::bytes;
#pragma unroll
    for (int c = 0; c < 12; c++) v[c] = ld_p<P, R>(plane_ptr<P>(f.data, r * 12 + c, stride), off);
    if constexpr (P == P16) {
        const R s = (R)f.scale[(size_t)r * stride + i];
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] = cscale(v[c], s);
    }
}

// FP16 encoding of a site: s = max |component| (FP32), h = fp16_rne(fp32(v / s)), s = 0 -> zeros.
template <int P, typename R>
__device__ __forceinline__ void store_site(const Spinor &f, int stride, int r, int i, const Cx<R> (&v)[12]) {
    const unsigned off = (unsigned)i * Elem<P>::bytes;
    if constexpr (P == P16) {
        float vf[24];
#pragma unroll
        for (int c = 0; c < 12; c++) {
            vf[2 * c] = (float)v[c].re;
            vf[2 * c + 1] = (float)v[c].im;
        }
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < 24; k++) s = fmaxf(s, fabsf(vf[k]));
        const float sd = s > 0.f ? s : 1.f;
#pragma unroll
        for (int c = 0; c < 12; c++) {
            half2_t h;
            h.x = (_Float16)(s > 0.f ? vf[2 * c] / sd : 0.f);
            h.y = (_Float16)(s > 0.f ? vf[2 * c + 1] / sd : 0.f);
            *reinterpret_cast<half2_t *>(const_cast<char *>(plane_ptr<P>(f.data, r * 12 + c, stride)) + off) = h;
        }
        f.scale[(size_t)r * stride + i] = s;
    } else {
#pragma unroll
        for (int c = 0; c < 12; c++) st_p<P, R>(const_cast<char *>(plane_ptr<P>(f.data, r * 12 + c, stride)), off, v[c]);
    }
}

// ---- deterministic block reduction of NV doubles; result written by thread 0 ----
template <int NV>
__device__ __forceinline__ void block_reduce_to(double (&v)[NV], double *dst, size_t dst_stride) {
    __shared__ double lds[NV][16];
#pragma unroll
    for (int k = 0; k < NV; k++) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) lds[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) {
            double s = 0.0;
            for (int w = 0; w < nw; w++) s += lds[k][w];
            dst[(size_t)k * dst_stride] = s;
        }
    }
    __syncthreads();
}

// Site coordinates of checkerboard index i on output parity par.
struct SiteXY {
    int xh, b, y, z, t;
};
__device__ __forceinline__ SiteXY cb_coords(const Geom &g, int i, int par) {
    SiteXY c;
    c.xh = i % g.Lxh;
    int rest = i / g.Lxh;
    c.y = rest % g.L[1];
    rest /= g.L[1];
    c.z = rest % g.L[2];
    c.t = rest / g.L[2];
    c.b = (c.y + c.z + c.t + par) & 1;  // x = 2*xh + b
    return c;
}

// Processing order of sites.  zblk = 0: memory order (x, y, z, t).  zblk > 0: the
// (z, t) planes of Lxh*Ly sites are visited z-block by z-block, and within a block
// t-major then z, so that the spinor read by the +t and -t hops of neighbouring planes is
// still in L2 when the second hop needs it (in memory order the two uses lie 2*Lz planes
// apart).  Requires zblk | Lz; with Lxh*Ly a multiple of the block size every block stays
// inside one plane, so loads stay coalesced.
__device__ __forceinline__ int visit_order(int l, const Geom &g, int zblk) {
    if (zblk <= 0) return l;
    const int S = g.Lxh * g.L[1];
    const int pl = l / S, within = l - pl * S;
    const int per_zb = zblk * g.L[3];
    const int zb = pl / per_zb, rem = pl - zb * per_zb;
    const int t = rem / zblk, zi = rem - t * zblk;
    return ((zb * zblk + zi) + g.L[2] * t) * S + within;
}

// Block index remapped so that each XCD (blocks are dealt round-robin to 8 XCDs)
// processes one contiguous range of tiles: neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n >> 3, rem = n & 7;
    const int k = b & 7, j = b >> 3;
    return (k < rem) ? k * (q + 1) + j : rem * (q + 1) + (k - rem) * q + j;
}

}  // namespace wl
