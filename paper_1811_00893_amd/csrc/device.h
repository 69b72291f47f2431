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

// ---- storage: packed 16-byte plane elements ------------------------------------------
// Spinor planes hold 16-byte elements: 1 complex (FP64), 2 (FP32) or 4 (FP16) consecutive
// components, so every lane moves 16 bytes per load in every precision (narrower loads
// would make the per-CU load units, not HBM, the limit).  Component c of a site lives in
// element plane c / CPE, slot c % CPE; a field of one parity has NEL = 12 / CPE planes
// per right-hand side.  Links use 16-byte elements of 1 (FP64) or 2 (FP32) complex and
// 8-byte elements of 2 complex (FP16).
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef _Float16 hvec4 __attribute__((ext_vector_type(4)));
typedef _Float16 hvec8 __attribute__((ext_vector_type(8)));

// Fields in device memory are addressed through pointers of the global address space, so
// their loads and stores are global_load / global_store.  Through a generic pointer they
// would be flat accesses, which also count against the counter of LDS and scalar loads:
// every wait for an LDS read or a kernel argument would then also wait for all memory
// loads in flight.  (A generic pointer loses its address space in the integer round trip
// of uniform_ptr below, and a field pointer read from a kernel's argument struct has none.)
#define WL_GLOBAL __attribute__((address_space(1)))
typedef WL_GLOBAL char gchar;
template <typename T>
__device__ __forceinline__ const WL_GLOBAL T *gptr(const T *p) {
    return (const WL_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ WL_GLOBAL T *gptr_w(T *p) {
    return (WL_GLOBAL T *)p;
}

template <int P>
struct SpinorPack {
    static constexpr int CPE = P == P64 ? 1 : (P == P32 ? 2 : 4);  // complex per element
    static constexpr int NEL = 12 / CPE;                            // elements per site
};
template <int P>
struct LinkPack {
    static constexpr int CPL = P == P64 ? 1 : 2;          // complex per element
    static constexpr unsigned EB = P == P16 ? 8u : 16u;  // element bytes
};
template <int P, int NE>
struct LinkElems {
    static constexpr int N = (NE + LinkPack<P>::CPL - 1) / LinkPack<P>::CPL;
};
__host__ __device__ constexpr int link_elems(int prec, int ne) { return prec == P64 ? ne : (ne + 1) / 2; }
__host__ __device__ constexpr unsigned link_elem_bytes(int prec) { return prec == P16 ? 8u : 16u; }

// plane addressing: a wave-uniform plane base plus one 32-bit per-lane byte offset, so the
// loads of a site share one offset register and the bases stay in scalar registers
// The plane base is passed through readfirstlane, so every caller must pass a base and a
// plane index that are the same on all lanes of the wavefront (a kernel whose lanes may
// belong to different fields or parities takes them from blockIdx, not from the lane).
// Without it the compiler folds the lane offset into the base first and then adds each
// plane's offset with a 64-bit per-lane multiply-add, instead of one scalar base per plane.
__device__ __forceinline__ const gchar *uniform_ptr(const char *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const gchar *>(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ const gchar *splane(const void *base, int plane, int stride) {
    return uniform_ptr(static_cast<const char *>(base) + (size_t)plane * stride * 16u);
}
template <int P>
__device__ __forceinline__ const gchar *lplane(const void *base, int plane, int stride) {
    return uniform_ptr(static_cast<const char *>(base) + (size_t)plane * stride * LinkPack<P>::EB);
}

// Loads and stores of data that a launch touches once (the hop's y, z and w operands and
// its output, links when one launch group covers every right-hand side) are non-temporal
// (NT), so they do not evict from L2 the neighbour spinors that are still to be re-read.
template <typename T, bool NT>
__device__ __forceinline__ T ld_maybe_nt(const gchar *p) {
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const WL_GLOBAL T *>(p));
    else return *reinterpret_cast<const WL_GLOBAL T *>(p);
}
template <int P, typename R, bool NT = false>
__device__ __forceinline__ void ld_elem(Cx<R> *o, const gchar *plane, unsigned off) {
    if constexpr (P == P64) {
        const dvec2 v = ld_maybe_nt<dvec2, NT>(plane + off);
        o[0] = {(R)v.x, (R)v.y};
    } else if constexpr (P == P32) {
        const fvec4 v = ld_maybe_nt<fvec4, NT>(plane + off);
        o[0] = {(R)v.x, (R)v.y};
        o[1] = {(R)v.z, (R)v.w};
    } else {
        const hvec8 v = ld_maybe_nt<hvec8, NT>(plane + off);
#pragma unroll
        for (int k = 0; k < 4; k++) o[k] = {(R)(float)v[2 * k], (R)(float)v[2 * k + 1]};
    }
}
template <typename T, bool NT>
__device__ __forceinline__ void st_maybe_nt(gchar *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<WL_GLOBAL T *>(p));
    else *reinterpret_cast<WL_GLOBAL T *>(p) = v;
}
template <int P, typename R, bool NT = false>
__device__ __forceinline__ void st_elem(gchar *plane, unsigned off, const Cx<R> *x) {
    if constexpr (P == P64) {
        dvec2 v;
        v.x = (double)x[0].re;
        v.y = (double)x[0].im;
        st_maybe_nt<dvec2, NT>(plane + off, v);
    } else if constexpr (P == P32) {
        fvec4 v;
        v.x = (float)x[0].re;
        v.y = (float)x[0].im;
        v.z = (float)x[1].re;
        v.w = (float)x[1].im;
        st_maybe_nt<fvec4, NT>(plane + off, v);
    } else {
        hvec8 v;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            v[2 * k] = (_Float16)(float)x[k].re;
            v[2 * k + 1] = (_Float16)(float)x[k].im;
        }
        st_maybe_nt<hvec8, NT>(plane + off, v);
    }
}
// link element: NT when a launch reads each link once; ordinary loads when several
// right-hand-side groups read the same links one after another and must find them in L2.
template <int P, typename R, bool NT>
__device__ __forceinline__ void ld_link_elem(Cx<R> *o, const gchar *plane, unsigned off) {
    if constexpr (P == P64) {
        const dvec2 v = ld_maybe_nt<dvec2, NT>(plane + off);
        o[0] = {(R)v.x, (R)v.y};
    } else if constexpr (P == P32) {
        const fvec4 v = ld_maybe_nt<fvec4, NT>(plane + off);
        o[0] = {(R)v.x, (R)v.y};
        o[1] = {(R)v.z, (R)v.w};
    } else {
        const hvec4 v = ld_maybe_nt<hvec4, NT>(plane + off);
        o[0] = {(R)(float)v[0], (R)(float)v[1]};
        o[1] = {(R)(float)v[2], (R)(float)v[3]};
    }
}
// the same element from a block's LDS copy of the links (a __shared__ buffer)
template <int P, typename R>
__device__ __forceinline__ void ld_link_elem_lds(Cx<R> *o, const char *lds, unsigned off) {
    if constexpr (P == P64) {
        const dvec2 v = *reinterpret_cast<const dvec2 *>(lds + off);
        o[0] = {(R)v.x, (R)v.y};
    } else if constexpr (P == P32) {
        const fvec4 v = *reinterpret_cast<const fvec4 *>(lds + off);
        o[0] = {(R)v.x, (R)v.y};
        o[1] = {(R)v.z, (R)v.w};
    } else {
        const hvec4 v = *reinterpret_cast<const hvec4 *>(lds + off);
        o[0] = {(R)(float)v[0], (R)(float)v[1]};
        o[1] = {(R)(float)v[2], (R)(float)v[3]};
    }
}
template <int P, typename R>
__device__ __forceinline__ void st_link_elem(gchar *plane, unsigned off, const Cx<R> *x) {
    if constexpr (P == P64) {
        dvec2 v;
        v.x = (double)x[0].re;
        v.y = (double)x[0].im;
        *reinterpret_cast<WL_GLOBAL dvec2 *>(plane + off) = v;
    } else if constexpr (P == P32) {
        fvec4 v;
        v.x = (float)x[0].re;
        v.y = (float)x[0].im;
        v.z = (float)x[1].re;
        v.w = (float)x[1].im;
        *reinterpret_cast<WL_GLOBAL fvec4 *>(plane + off) = v;
    } else {
        hvec4 v;
        v[0] = (_Float16)(float)x[0].re;
        v[1] = (_Float16)(float)x[0].im;
        v[2] = (_Float16)(float)x[1].re;
        v[3] = (_Float16)(float)x[1].im;
        *reinterpret_cast<WL_GLOBAL hvec4 *>(plane + off) = v;
    }
}

// Full site (12 complex) of rhs `r` of a parity field; FP16 values are rescaled.
template <int P, typename R, bool NT = false>
__device__ __forceinline__ void load_site(Cx<R> (&v)[12], const Spinor &f, int stride, int r, int i) {
    constexpr int CPE = SpinorPack<P>::CPE, NEL = SpinorPack<P>::NEL;
    const unsigned off = (unsigned)i * 16u;
#pragma unroll
    for (int e = 0; e < NEL; e++) ld_elem<P, R, NT>(&v[e * CPE], splane(f.data, r * NEL + e, stride), off);
    if constexpr (P == P16) {
        const R s = (R)(NT ? __builtin_nontemporal_load(gptr(f.scale) + (size_t)r * stride + i)
                           : gptr(f.scale)[(size_t)r * stride + i]);
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] = cscale(v[c], s);
    }
}

// FP16 encoding of a site: s = max |component| (FP32), h = fp16_rne(fp32(v / s)), s = 0 -> zeros.
template <int P, typename R, bool NT = false>
__device__ __forceinline__ void store_site(const Spinor &f, int stride, int r, int i, const Cx<R> (&v)[12]) {
    constexpr int CPE = SpinorPack<P>::CPE, NEL = SpinorPack<P>::NEL;
    const unsigned off = (unsigned)i * 16u;
    if constexpr (P == P16) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 12; c++) s = fmaxf(s, fmaxf(fabsf((float)v[c].re), fabsf((float)v[c].im)));
        const float sd = s > 0.f ? s : 1.f;
        Cx<float> q[12];
#pragma unroll
        for (int c = 0; c < 12; c++)
            q[c] = s > 0.f ? Cx<float>{(float)v[c].re / sd, (float)v[c].im / sd} : Cx<float>{0.f, 0.f};
#pragma unroll
        for (int e = 0; e < NEL; e++)
            st_elem<P, float, NT>(const_cast<gchar *>(splane(f.data, r * NEL + e, stride)), off, &q[e * CPE]);
        if constexpr (NT) __builtin_nontemporal_store(s, gptr_w(f.scale) + (size_t)r * stride + i);
        else gptr_w(f.scale)[(size_t)r * stride + i] = s;
    } else {
#pragma unroll
        for (int e = 0; e < NEL; e++)
            st_elem<P, R, NT>(const_cast<gchar *>(splane(f.data, r * NEL + e, stride)), off, &v[e * CPE]);
    }
}

// ---- clover site term -----------------------------------------------------------
// A site matrix T (12x12, commuting with gamma5) is kept as two Hermitian 6x6 blocks of
// the chiral basis.  In this Dirac basis gamma5 = -[[0,1],[1,0]] on spin pairs, so with
// d = v_up - v_lo and s = v_up + v_lo (spins (0,2) and (1,3), colour inner; the +
// and - chirality components up to 1/sqrt 2):
//     (T v)_up = (T+ d + T- s) / 2,   (T v)_lo = (T- s - T+ d) / 2.
// Packed block: reals 0..5 the diagonal, then (re, im) of the 15 entries above the
// diagonal in row-major order; element planes: block b, element e -> plane b*EPB + e.
template <int P>
struct ClovPack {
    static constexpr int EPB = P == P64 ? 18 : 9;  // 16-byte elements per block
};
__host__ __device__ constexpr int herm6_off(int i, int j) { return 6 + 2 * (i * (11 - i) / 2 + (j - i - 1)); }

template <int P, typename R>
__device__ __forceinline__ void clov_load_block(R (&m)[36], const void *base, int blk, int stride, int i) {
    constexpr int EPB = ClovPack<P>::EPB;
    const unsigned off = (unsigned)i * 16u;
#pragma unroll
    for (int e = 0; e < EPB; e++) {
        const gchar *pl = splane(base, blk * EPB + e, stride);
        if constexpr (P == P64) {
            const dvec2 v = ld_maybe_nt<dvec2, true>(pl + off);  // read once per launch
            m[2 * e] = (R)v.x;
            m[2 * e + 1] = (R)v.y;
        } else {
            const fvec4 v = ld_maybe_nt<fvec4, true>(pl + off);
            m[4 * e] = (R)v.x;
            m[4 * e + 1] = (R)v.y;
            m[4 * e + 2] = (R)v.z;
            m[4 * e + 3] = (R)v.w;
        }
    }
}

// y = M x for a packed Hermitian 6x6 block M
template <typename R>
__device__ __forceinline__ void herm6_apply(Cx<R> (&y)[6], const R (&m)[36], const Cx<R> (&x)[6]) {
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] = cscale(x[i], m[i]);
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i + 1; j < 6; j++) {
            const Cx<R> a = {m[herm6_off(i, j)], m[herm6_off(i, j) + 1]};
            y[i] = cfma(y[i], a, x[j]);       // M_ij x_j
            y[j] = cfma_conj(y[j], a, x[i]);  // M_ji x_i = conj(M_ij) x_i
        }
}

// v <- T v for the site matrix whose packed blocks (storage precision P) start at base
template <int P, typename R>
__device__ __forceinline__ void clov_apply(Cx<R> (&v)[12], const void *base, int stride, int i) {
    Cx<R> d[6], sm[6], yp[6], ym[6];
#pragma unroll
    for (int k = 0; k < 6; k++) {
        d[k] = csub(v[k], v[k + 6]);
        sm[k] = cadd(v[k], v[k + 6]);
    }
    {
        R m[36];
        clov_load_block<P, R>(m, base, 0, stride, i);
        herm6_apply(yp, m, d);
    }
    {
        R m[36];
        clov_load_block<P, R>(m, base, 1, stride, i);
        herm6_apply(ym, m, sm);
    }
    const R h = R(0.5);
#pragma unroll
    for (int k = 0; k < 6; k++) {
        v[k] = cscale(cadd(yp[k], ym[k]), h);
        v[k + 6] = cscale(csub(ym[k], yp[k]), h);
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

// ---- deterministic wave reduction of NV doubles; result written by lane 0 ----
template <int NV>
__device__ __forceinline__ void wave_reduce_to(double (&v)[NV], double *dst, size_t dst_stride) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) dst[(size_t)k * dst_stride] = v[k];
    }
}

// Site indexing: shared by the kernels and by the host replay of their index maps
// (wilson_index_check), so the host checks the code the kernels run.
//
// Site coordinates of checkerboard index i on output parity par.
struct SiteXY {
    int xh, b, y, z, t;
};
__host__ __device__ __forceinline__ SiteXY cb_coords(const Geom &g, int i, int par) {
    SiteXY c;
    const int q1 = (int)fdiv((uint32_t)i, g.dLxh);   // i / (Lx/2)
    c.xh = i - q1 * g.Lxh;
    const int q2 = (int)fdiv((uint32_t)q1, g.dLy);   // / Ly
    c.y = q1 - q2 * g.L[1];
    c.t = (int)fdiv((uint32_t)q2, g.dLz);            // / Lz
    c.z = q2 - c.t * g.L[2];
    c.b = (c.y + c.z + c.t + par) & 1;  // x = 2*xh + b
    return c;
}

// Checkerboard indices, in the fields of the other parity, of the eight neighbours of
// output site i (coordinates c): x+1, x-1, y+1, ..., t-1, periodic in every direction
// (the antiperiodic t sign is applied by the hop).  Along x the neighbour shares the
// site's row; whether x+1 is the same checkerboard column or the next depends on b.
struct SiteNbrs {
    int xp, xm, yp, ym, zp, zm, tp, tm;
};
__host__ __device__ __forceinline__ SiteNbrs site_nbrs(const Geom &g, int i, const SiteXY &c) {
    SiteNbrs n;
    const int row = i - c.xh;
    n.xp = row + ((c.xh + c.b == g.Lxh) ? 0 : c.xh + c.b);
    n.xm = row + ((c.xh + c.b == 0) ? g.Lxh - 1 : c.xh + c.b - 1);
    n.yp = (c.y == g.L[1] - 1) ? i - (g.L[1] - 1) * g.sy : i + g.sy;
    n.ym = (c.y == 0) ? i + (g.L[1] - 1) * g.sy : i - g.sy;
    n.zp = (c.z == g.L[2] - 1) ? i - (g.L[2] - 1) * g.sz : i + g.sz;
    n.zm = (c.z == 0) ? i + (g.L[2] - 1) * g.sz : i - g.sz;
    n.tp = (c.t == g.L[3] - 1) ? i - (g.L[3] - 1) * g.st : i + g.st;
    n.tm = (c.t == 0) ? i + (g.L[3] - 1) * g.st : i - g.st;
    return n;
}

// Processing order of sites.  zblk = 0: memory order (x, y, z, t).  zblk > 0: the
// (z, t) planes of Lxh*Ly sites are visited z-block by z-block, and within a block
// t-major then z, so that the spinor read by the +t and -t hops of neighbouring planes is
// still in L2 when the second hop needs it (in memory order the two uses lie 2*Lz planes
// apart).  Requires zblk | Lz; with Lxh*Ly a multiple of the block size every block stays
// inside one plane, so loads stay coalesced.  With zblk = Lz/8 and the XCD-contiguous block
// order below, each XCD walks one z-block through every t-slice.
struct VisitOrder {
    int zblk = 0;
    FastDiv plane, per_zb, zb;  // division by Lxh*Ly, zblk*Lt and zblk
};
inline VisitOrder make_visit_order(const Geom &g, int zblk) {
    VisitOrder vo;
    if (zblk > 0) {
        vo.zblk = zblk;
        vo.plane = make_fastdiv((uint32_t)(g.Lxh * g.L[1]));
        vo.per_zb = make_fastdiv((uint32_t)(zblk * g.L[3]));
        vo.zb = make_fastdiv((uint32_t)zblk);
    }
    return vo;
}
__host__ __device__ __forceinline__ int visit_order(int l, const Geom &g, const VisitOrder &v) {
    if (v.zblk <= 0) return l;
    const int S = (int)v.plane.d;
    const int pl = (int)fdiv((uint32_t)l, v.plane), within = l - pl * S;
    const int zb = (int)fdiv((uint32_t)pl, v.per_zb), rem = pl - zb * (int)v.per_zb.d;
    const int t = (int)fdiv((uint32_t)rem, v.zb), zi = rem - t * v.zblk;
    return ((zb * v.zblk + zi) + g.L[2] * t) * S + within;
}

// Block index remapped so that each XCD (blocks are dealt round-robin to 8 XCDs)
// processes one contiguous range of tiles: neighbouring tiles share an L2.
__host__ __device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n >> 3, rem = n & 7;
    const int k = b & 7, j = b >> 3;
    return (k < rem) ? k * (q + 1) + j : rem * (q + 1) + (k - rem) * q + j;
}

}  // namespace wl
