// Layout ablation of the parity hop.
//
// Sec. 4.1 of the paper folds lattice sites into SIMD vectors in two ways (consecutive
// x-sites in one vector, "layout 1"; one site from each of several sub-lattices, "layout 2",
// after Boyle et al.) and Sec. 5 finds the first faster and both far ahead of the
// array-of-structures base code.  On a GPU the vector is the wavefront.  One hop kernel is
// templated here on the storage layout of the spinor and link fields, everything else
// (arithmetic, spin projection, launch shape, tile order) being the same:
//   SOA    component planes over checkerboard sites: a wavefront of 64 consecutive sites
//          (consecutive in x, the GPU form of layout 1) reads one contiguous 1 KiB run per
//          16-byte component; the library's production layout;
//   AOS    every site's components contiguous (FP64: 192 B per spinor, 4 x 144 B of links);
//   AOSOA  tiles of 64 sites, component planes inside each tile;
//   VNODE  the lattice cut into 1 x 4 x 4 x 4 sub-lattices; lane l of a wavefront holds
//          sub-lattice l at the wavefront's local site (the GPU form of layout 2).  A
//          neighbour across a sub-lattice face sits in another lane's slot of the same
//          1 KiB run; a GPU lane gathers it directly, where a CPU vector needs a shuffle.
// Links are stored as 18 reals or as their first two rows (12 reals, third row rebuilt),
// in every layout.  One thread per output site, 256 threads per block, blocks assigned to
// the 8 XCDs in contiguous ranges.
#include "layout_lab.h"

#include "device.h"
#include "dslash_kernels.h"

namespace wl {

namespace {

struct LabArgs {
    void *out;
    const void *in;
    const void *U[2];
    LabGeom g;
    int par;
    double cH;
};

// Byte offset of 16-byte element e (of nel per site) of storage slot `slot`.
template <int LAY>
__device__ __forceinline__ size_t lab_off(int slot, int e, int nel, int pad) {
    if constexpr (LAY == LAB_AOS) return ((size_t)slot * nel + e) * 16u;
    else if constexpr (LAY == LAB_AOSOA) return (((size_t)(slot >> 6) * nel + e) << 10) + (size_t)(slot & 63) * 16u;
    else return ((size_t)e * pad + slot) * 16u;  // SOA and VNODE: planes of `pad` slots
}

struct LabSite {
    int xh, b;          // x = 2 xh + b
    int yl, zl, tl;     // coordinates inside the sub-lattice
    int by, bz, bt;     // sub-lattice coordinates
};

template <int LAY>
__device__ __forceinline__ LabSite lab_decode(const LabGeom &g, int slot, int par) {
    LabSite c;
    int j = slot;
    if constexpr (LAY == LAB_VNODE) {
        const int l = slot & 63;
        j = slot >> 6;
        c.by = l & 3;
        c.bz = (l >> 2) & 3;
        c.bt = l >> 4;
    } else {
        c.by = c.bz = c.bt = 0;
    }
    const int q1 = (int)fdiv((uint32_t)j, g.dnlxh);
    c.xh = j - q1 * g.nlxh;
    const int q2 = (int)fdiv((uint32_t)q1, g.dnl1);
    c.yl = q1 - q2 * g.nl[1];
    c.tl = (int)fdiv((uint32_t)q2, g.dnl2);
    c.zl = q2 - c.tl * g.nl[2];
    // sub-lattice extents are even, so the parity of the local and global coordinates agree
    c.b = (c.yl + c.zl + c.tl + par) & 1;
    return c;
}

template <int LAY>
__device__ __forceinline__ int lab_slot(const LabGeom &g, int xh, int yl, int zl, int tl, int by, int bz, int bt) {
    const int j = xh + g.nlxh * (yl + g.nl[1] * (zl + g.nl[2] * tl));
    if constexpr (LAY == LAB_VNODE) return (j << 6) + by + 4 * (bz + 4 * bt);
    else return j;
}

// one step of +-1 in a direction split into nb sub-lattices of extent n
__device__ __forceinline__ void lab_step(int &l, int &b, int n, int nb, int d) {
    l += d;
    if (l == n) {
        l = 0;
        b = b + 1 == nb ? 0 : b + 1;
    } else if (l < 0) {
        l = n - 1;
        b = b == 0 ? nb - 1 : b - 1;
    }
}

__device__ __forceinline__ int lab_global_site(const LabGeom &g, const LabSite &c) {
    const int x = 2 * c.xh + c.b, y = c.yl + c.by * g.nl[1], z = c.zl + c.bz * g.nl[2], t = c.tl + c.bt * g.nl[3];
    return x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
}

// One direction: link, neighbour gather, spin projection, SU(3) product, reconstruction.
template <int LAY, int P, int NE, int MU, bool FWD>
__device__ __forceinline__ void lab_dir(Cx<real_t<P>> (&acc)[4][3], const LabArgs &a, int nslot, int lslot,
                                        int lpar, real_t<P> sgn) {
    using R = real_t<P>;
    constexpr int CPE = P == P64 ? 1 : 2, NEL = 12 / CPE, NLE = (NE + CPE - 1) / CPE;
    const int pad = a.g.pad;
    Cx<R> U[3][3];
    {
        Cx<R> ue[NLE * CPE];
        const gchar *lb = gptr(static_cast<const char *>(a.U[lpar]));
#pragma unroll
        for (int e = 0; e < NLE; e++) ld_elem<P, R>(&ue[e * CPE], lb + lab_off<LAY>(lslot, MU * NLE + e, 4 * NLE, pad), 0u);
#pragma unroll
        for (int e = 0; e < NE; e++) U[e / 3][e % 3] = ue[e];
    }
    if constexpr (NE == 6) {
        const Cx<R> c0 = csub(cmul(U[0][1], U[1][2]), cmul(U[0][2], U[1][1]));
        const Cx<R> c1 = csub(cmul(U[0][2], U[1][0]), cmul(U[0][0], U[1][2]));
        const Cx<R> c2 = csub(cmul(U[0][0], U[1][1]), cmul(U[0][1], U[1][0]));
        U[2][0] = {c0.re, -c0.im};
        U[2][1] = {c1.re, -c1.im};
        U[2][2] = {c2.re, -c2.im};
    }
    // the t-hops need one spin half of the neighbour (upper forward, lower backward)
    constexpr int half = MU == 3 ? (FWD ? 1 : 0) : -1;
    Cx<R> comp[12];
    const gchar *sb = gptr(static_cast<const char *>(a.in));
#pragma unroll
    for (int e = 0; e < NEL; e++) {
        const bool need = half < 0 || (e * CPE >= 6 * half && e * CPE < 6 * half + 6);
        if (need) ld_elem<P, R>(&comp[e * CPE], sb + lab_off<LAY>(nslot, e, NEL, pad), 0u);
        else
#pragma unroll
            for (int k = 0; k < CPE; k++) comp[e * CPE + k] = {R(0), R(0)};
    }
    Cx<R> h[2][3];
    proj_in<P, MU, FWD, false>(comp, R(1), h);
    Cx<R> u[2][3];
#pragma unroll
    for (int k = 0; k < 2; k++)
#pragma unroll
        for (int r = 0; r < 3; r++) {
            Cx<R> t = {R(0), R(0)};
#pragma unroll
            for (int c = 0; c < 3; c++) {
                if constexpr (FWD) t = cfma(t, U[r][c], h[k][c]);       // U h
                else               t = cfma_conj(t, U[c][r], h[k][c]);  // U^dag h
            }
            u[k][r] = NE == 6 && MU == 3 ? cscale(t, sgn) : t;
        }
    reconstruct<MU, FWD, R>(acc, u);
    __builtin_amdgcn_sched_barrier(0);
}

template <int LAY, int P, int NE>
__global__ void __launch_bounds__(256) lab_hop_kernel(const LabArgs a, int xcd) {
    using R = real_t<P>;
    constexpr int CPE = P == P64 ? 1 : 2, NEL = 12 / CPE;
    const LabGeom &g = a.g;
    int blk = blockIdx.x;
    if (xcd) {  // blocks are dealt to the XCDs round-robin: give XCD k a contiguous range
        const int per = (int)gridDim.x >> 3;
        blk = (blk & 7) * per + (blk >> 3);
    }
    const int slot = blk * 256 + (int)threadIdx.x;
    if (slot >= g.Vh) return;
    const int par = a.par, opar = 1 - par;
    const LabSite c = lab_decode<LAY>(g, slot, par);
    const int x = 2 * c.xh + c.b;
    const int xp = x + 1 == g.L[0] ? 0 : x + 1, xm = x == 0 ? g.L[0] - 1 : x - 1;
    const int s_xp = lab_slot<LAY>(g, xp >> 1, c.yl, c.zl, c.tl, c.by, c.bz, c.bt);
    const int s_xm = lab_slot<LAY>(g, xm >> 1, c.yl, c.zl, c.tl, c.by, c.bz, c.bt);
    int l, b;
    l = c.yl; b = c.by; lab_step(l, b, g.nl[1], g.nsub[1], 1);
    const int s_yp = lab_slot<LAY>(g, c.xh, l, c.zl, c.tl, b, c.bz, c.bt);
    l = c.yl; b = c.by; lab_step(l, b, g.nl[1], g.nsub[1], -1);
    const int s_ym = lab_slot<LAY>(g, c.xh, l, c.zl, c.tl, b, c.bz, c.bt);
    l = c.zl; b = c.bz; lab_step(l, b, g.nl[2], g.nsub[2], 1);
    const int s_zp = lab_slot<LAY>(g, c.xh, c.yl, l, c.tl, c.by, b, c.bt);
    l = c.zl; b = c.bz; lab_step(l, b, g.nl[2], g.nsub[2], -1);
    const int s_zm = lab_slot<LAY>(g, c.xh, c.yl, l, c.tl, c.by, b, c.bt);
    l = c.tl; b = c.bt; lab_step(l, b, g.nl[3], g.nsub[3], 1);
    const int s_tp = lab_slot<LAY>(g, c.xh, c.yl, c.zl, l, c.by, c.bz, b);
    l = c.tl; b = c.bt; lab_step(l, b, g.nl[3], g.nsub[3], -1);
    const int s_tm = lab_slot<LAY>(g, c.xh, c.yl, c.zl, l, c.by, c.bz, b);
    const bool t_last = c.tl == g.nl[3] - 1 && c.bt == g.nsub[3] - 1, t_first = c.tl == 0 && c.bt == 0;
    const R one = R(1);
    const R sgn_tf = (NE == 6 && t_last) ? -one : one;   // forward hop across t = Lt-1 -> 0
    const R sgn_tb = (NE == 6 && t_first) ? -one : one;  // backward hop across t = 0 -> Lt-1

    Cx<R> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int k = 0; k < 3; k++) acc[s][k] = {R(0), R(0)};
    lab_dir<LAY, P, NE, 0, true>(acc, a, s_xp, slot, par, one);
    lab_dir<LAY, P, NE, 0, false>(acc, a, s_xm, s_xm, opar, one);
    lab_dir<LAY, P, NE, 1, true>(acc, a, s_yp, slot, par, one);
    lab_dir<LAY, P, NE, 1, false>(acc, a, s_ym, s_ym, opar, one);
    lab_dir<LAY, P, NE, 2, true>(acc, a, s_zp, slot, par, one);
    lab_dir<LAY, P, NE, 2, false>(acc, a, s_zm, s_zm, opar, one);
    lab_dir<LAY, P, NE, 3, true>(acc, a, s_tp, slot, par, sgn_tf);
    lab_dir<LAY, P, NE, 3, false>(acc, a, s_tm, s_tm, opar, sgn_tb);

    const R cH = (R)a.cH;
    Cx<R> o[12];
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int k = 0; k < 3; k++) o[s * 3 + k] = cscale(acc[s][k], cH);
    gchar *ob = gptr_w(static_cast<char *>(a.out));
#pragma unroll
    for (int e = 0; e < NEL; e++) st_elem<P, R>(ob + lab_off<LAY>(slot, e, NEL, g.pad), 0u, &o[e * CPE]);
}

template <int LAY, int P>
__global__ void lab_pack_spinor_kernel(void *dst, const double2 *canon, const LabGeom g, int par) {
    constexpr int CPE = P == P64 ? 1 : 2, NEL = 12 / CPE;
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= g.Vh) return;
    const int s = lab_global_site(g, lab_decode<LAY>(g, slot, par));
    Cx<double> v[12];
    for (int k = 0; k < 12; k++) v[k] = {canon[(size_t)s * 12 + k].x, canon[(size_t)s * 12 + k].y};
    for (int e = 0; e < NEL; e++)
        st_elem<P, double>(gptr_w(static_cast<char *>(dst)) + lab_off<LAY>(slot, e, NEL, g.pad), 0u, &v[e * CPE]);
}

template <int LAY, int P>
__global__ void lab_unpack_spinor_kernel(double2 *canon, const void *src, const LabGeom g, int par) {
    constexpr int CPE = P == P64 ? 1 : 2, NEL = 12 / CPE;
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= g.Vh) return;
    const int s = lab_global_site(g, lab_decode<LAY>(g, slot, par));
    Cx<double> v[12];
    for (int e = 0; e < NEL; e++)
        ld_elem<P, double>(&v[e * CPE], gptr(static_cast<const char *>(src)) + lab_off<LAY>(slot, e, NEL, g.pad), 0u);
    for (int k = 0; k < 12; k++) canon[(size_t)s * 12 + k] = make_double2(v[k].re, v[k].im);
}

template <int LAY, int P>
__global__ void lab_pack_links_kernel(void *dst, const double2 *canonU, const LabGeom g, int ne, int par) {
    constexpr int CPE = P == P64 ? 1 : 2;
    const int nle = (ne + CPE - 1) / CPE;
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= g.Vh) return;
    const LabSite c = lab_decode<LAY>(g, slot, par);
    const int s = lab_global_site(g, c);
    const bool t_last = c.tl == g.nl[3] - 1 && c.bt == g.nsub[3] - 1;
    for (int mu = 0; mu < 4; mu++) {
        // full storage carries the antiperiodic sign of the t-links leaving t = Lt-1
        const double sg = (ne == 9 && mu == 3 && t_last) ? -1.0 : 1.0;
        Cx<double> v[10];
        for (int k = 0; k < 10; k++) {
            const double2 u = k < ne ? canonU[((size_t)s * 4 + mu) * 9 + k] : make_double2(0.0, 0.0);
            v[k] = {sg * u.x, sg * u.y};
        }
        for (int e = 0; e < nle; e++)
            st_elem<P, double>(gptr_w(static_cast<char *>(dst)) + lab_off<LAY>(slot, mu * nle + e, 4 * nle, g.pad), 0u,
                               &v[e * CPE]);
    }
}

__global__ void lab_zero_kernel(double *p, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0.0;
}

// dispatch helpers: layout and precision (and link storage) as template arguments
template <template <int, int> class F, typename... A>
hipError_t lab_dispatch2(int layout, int prec, A... args) {
    switch (layout * 2 + (prec == P64 ? 0 : 1)) {
        case 0: F<LAB_SOA, P64>::run(args...); break;
        case 1: F<LAB_SOA, P32>::run(args...); break;
        case 2: F<LAB_AOS, P64>::run(args...); break;
        case 3: F<LAB_AOS, P32>::run(args...); break;
        case 4: F<LAB_AOSOA, P64>::run(args...); break;
        case 5: F<LAB_AOSOA, P32>::run(args...); break;
        case 6: F<LAB_VNODE, P64>::run(args...); break;
        case 7: F<LAB_VNODE, P32>::run(args...); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

unsigned lab_blocks(const LabGeom &g) { return (unsigned)((g.Vh + 255) / 256); }

template <int LAY, int P>
struct PackSpinor {
    static void run(void *dst, const double *canon, LabGeom g, int par, hipStream_t s) {
        hipLaunchKernelGGL((lab_pack_spinor_kernel<LAY, P>), dim3(lab_blocks(g)), dim3(256), 0, s, dst,
                           reinterpret_cast<const double2 *>(canon), g, par);
    }
};
template <int LAY, int P>
struct UnpackSpinor {
    static void run(double *canon, const void *src, LabGeom g, int par, hipStream_t s) {
        hipLaunchKernelGGL((lab_unpack_spinor_kernel<LAY, P>), dim3(lab_blocks(g)), dim3(256), 0, s,
                           reinterpret_cast<double2 *>(canon), src, g, par);
    }
};
template <int LAY, int P>
struct PackLinks {
    static void run(void *dst, const double *canonU, LabGeom g, int ne, int par, hipStream_t s) {
        hipLaunchKernelGGL((lab_pack_links_kernel<LAY, P>), dim3(lab_blocks(g)), dim3(256), 0, s, dst,
                           reinterpret_cast<const double2 *>(canonU), g, ne, par);
    }
};
template <int LAY, int P>
struct Hop {
    static void run(const LabArgs &a, int ne, hipStream_t s) {
        const unsigned nb = lab_blocks(a.g);
        const int xcd = nb % 8 == 0 ? 1 : 0;
        if (ne == 6) hipLaunchKernelGGL((lab_hop_kernel<LAY, P, 6>), dim3(nb), dim3(256), 0, s, a, xcd);
        else hipLaunchKernelGGL((lab_hop_kernel<LAY, P, 9>), dim3(nb), dim3(256), 0, s, a, xcd);
    }
};

}  // namespace

bool lab_geom(LabGeom &g, const int32_t dims[4], int layout) {
    for (int k = 0; k < 4; k++)
        if (dims[k] < 2 || dims[k] % 2) return false;
    const bool vn = layout == LAB_VNODE;
    for (int k = 0; k < 4; k++) {
        g.L[k] = dims[k];
        g.nsub[k] = vn && k > 0 ? 4 : 1;
        if (dims[k] % (2 * g.nsub[k])) return false;  // sub-lattice extents even
        g.nl[k] = dims[k] / g.nsub[k];
    }
    g.nlxh = g.nl[0] / 2;
    const long long vh = (long long)dims[0] * dims[1] * dims[2] * dims[3] / 2;
    if (vh >= (1LL << 30)) return false;
    g.Vh = (int)vh;
    g.pad = (g.Vh + 63) / 64 * 64;
    g.dnlxh = make_fastdiv((uint32_t)g.nlxh);
    g.dnl1 = make_fastdiv((uint32_t)g.nl[1]);
    g.dnl2 = make_fastdiv((uint32_t)g.nl[2]);
    return true;
}

size_t lab_spinor_bytes(const LabGeom &g, int prec) { return (size_t)g.pad * (prec == P64 ? 12 : 6) * 16; }
size_t lab_link_bytes(const LabGeom &g, int prec, int link_reals) {
    const int ne = link_reals / 2, nle = prec == P64 ? ne : (ne + 1) / 2;
    return (size_t)g.pad * 4 * nle * 16;
}

hipError_t launch_lab_pack_spinor(void *dst, const double *canon, const LabGeom &g, int layout, int prec, int par,
                                  hipStream_t s) {
    return lab_dispatch2<PackSpinor>(layout, prec, dst, canon, g, par, s);
}
hipError_t launch_lab_unpack_spinor(double *canon, const void *src, const LabGeom &g, int layout, int prec, int par,
                                    hipStream_t s) {
    return lab_dispatch2<UnpackSpinor>(layout, prec, canon, src, g, par, s);
}
hipError_t launch_lab_pack_links(void *dst, const double *canonU, const LabGeom &g, int layout, int prec,
                                 int link_reals, int par, hipStream_t s) {
    if (link_reals != 12 && link_reals != 18) return hipErrorInvalidValue;
    return lab_dispatch2<PackLinks>(layout, prec, dst, canonU, g, link_reals / 2, par, s);
}
hipError_t launch_lab_hop(void *out, const void *in, const void *U0, const void *U1, const LabGeom &g, int layout,
                          int prec, int link_reals, int par, double cH, hipStream_t s) {
    if (link_reals != 12 && link_reals != 18) return hipErrorInvalidValue;
    LabArgs a;
    a.out = out;
    a.in = in;
    a.U[0] = U0;
    a.U[1] = U1;
    a.g = g;
    a.par = par;
    a.cH = cH;
    return lab_dispatch2<Hop>(layout, prec, a, link_reals / 2, s);
}
hipError_t launch_lab_zero(double *p, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(lab_zero_kernel, dim3(1024), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace wl
