// Clover site term of the clover fermion matrix (Sec. 2.1.2): D_clov = D_W + F(x), with
// T(x) = 1 + F(x) the site-diagonal block.  F is Hermitian and, in a suitable basis, block
// diagonal with two 6x6 Hermitian blocks; here that basis is the chiral one (F commutes
// with gamma5).  This file packs T and T^-1 per site from the canonical 12x12 F and
// applies a packed site matrix to a spinor field.
#include "common.h"
#include "device.h"

namespace wl {

namespace {

typedef double2 z64;

__device__ __forceinline__ z64 zmul(z64 a, z64 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ z64 zsub(z64 a, z64 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ z64 zadd(z64 a, z64 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double zabs2(z64 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ z64 zdiv(z64 a, z64 b) {
    const double d = zabs2(b);
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Inverse of a 6x6 complex matrix in place (Gauss-Jordan, partial pivoting).  false when
// a pivot vanishes.
__device__ bool inv6(z64 (&a)[6][6]) {
    z64 b[6][6];
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 6; c++) b[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    for (int col = 0; col < 6; col++) {
        int piv = col;
        for (int r = col + 1; r < 6; r++)
            if (zabs2(a[r][col]) > zabs2(a[piv][col])) piv = r;
        if (zabs2(a[piv][col]) == 0.0) return false;
        if (piv != col)
            for (int c = 0; c < 6; c++) {
                z64 t = a[col][c]; a[col][c] = a[piv][c]; a[piv][c] = t;
                t = b[col][c]; b[col][c] = b[piv][c]; b[piv][c] = t;
            }
        const z64 d = a[col][col];
        for (int c = 0; c < 6; c++) {
            a[col][c] = zdiv(a[col][c], d);
            b[col][c] = zdiv(b[col][c], d);
        }
        for (int r = 0; r < 6; r++) {
            if (r == col) continue;
            const z64 f = a[r][col];
            for (int c = 0; c < 6; c++) {
                a[r][c] = zsub(a[r][c], zmul(f, a[col][c]));
                b[r][c] = zsub(b[r][c], zmul(f, b[col][c]));
            }
        }
    }
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 6; c++) a[r][c] = b[r][c];
    return true;
}

// Packed reals (diagonal real parts, then the upper triangle) of a Hermitian block.
__device__ void pack36(double (&m)[36], const z64 (&a)[6][6]) {
    for (int i = 0; i < 6; i++) m[i] = a[i][i].x;
    for (int i = 0; i < 6; i++)
        for (int j = i + 1; j < 6; j++) {
            m[herm6_off(i, j)] = a[i][j].x;
            m[herm6_off(i, j) + 1] = a[i][j].y;
        }
}

__device__ void store36(void *base, int prec, int blk, int stride, int i, const double (&m)[36]) {
    const unsigned off = (unsigned)i * 16u;
    if (prec == P64) {
        for (int e = 0; e < 18; e++) {
            dvec2 v;
            v.x = m[2 * e];
            v.y = m[2 * e + 1];
            *reinterpret_cast<WL_GLOBAL dvec2 *>(const_cast<gchar *>(splane(base, blk * 18 + e, stride)) + off) = v;
        }
    } else {
        for (int e = 0; e < 9; e++) {
            fvec4 v;
            v.x = (float)m[4 * e];
            v.y = (float)m[4 * e + 1];
            v.z = (float)m[4 * e + 2];
            v.w = (float)m[4 * e + 3];
            *reinterpret_cast<WL_GLOBAL fvec4 *>(const_cast<gchar *>(splane(base, blk * 9 + e, stride)) + off) = v;
        }
    }
}

// One thread per checkerboard site; blockIdx.y is the parity (the plane bases must be
// uniform over a wavefront).  F at canonical site s: 144 complex,
// row/column 3*spin + colour.  With F in 6x6 blocks over the spin pairs (up = spins
// 0,1; lo = spins 2,3), the chiral blocks are A+ = (Fuu - Ful - Flu + Fll)/2 and
// A- = (Fuu + Ful + Flu + Fll)/2, and the blocks coupling the two chiralities,
// (Fuu + Ful - Flu - Fll)/2 and (Fuu - Ful + Flu - Fll)/2, must vanish.
__global__ void clover_pack_kernel(void *t64, void *ti64, void *t32, void *ti32, const double *F, const Geom g,
                                   double tol, int *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    const SiteXY c = cb_coords(g, i, par);
    const long s = (long)(2 * c.xh + c.b) + (long)g.L[0] * (c.y + (long)g.L[1] * (c.z + (long)g.L[2] * c.t));
    const z64 *f = reinterpret_cast<const z64 *>(F) + s * 144;
    double fmax = 0.0, err = 0.0;
    for (int k = 0; k < 144; k++) fmax = fmax > zabs2(f[k]) ? fmax : zabs2(f[k]);
    fmax = sqrt(fmax);
    int bad = 0;
    for (int blk = 0; blk < 2; blk++) {
        const double sg = blk == 0 ? -1.0 : 1.0;  // + block: Fuu - Ful - Flu + Fll
        z64 T[6][6];
        for (int a = 0; a < 6; a++)
            for (int b = 0; b < 6; b++) {
                const z64 uu = f[a * 12 + b], ul = f[a * 12 + b + 6], lu = f[(a + 6) * 12 + b], ll = f[(a + 6) * 12 + b + 6];
                T[a][b] = make_double2(0.5 * (uu.x + sg * ul.x + sg * lu.x + ll.x) + (a == b ? 1.0 : 0.0),
                                       0.5 * (uu.y + sg * ul.y + sg * lu.y + ll.y));
                // coupling of the two chiralities
                const z64 cpl = make_double2(0.5 * (uu.x - sg * ul.x + sg * lu.x - ll.x),
                                             0.5 * (uu.y - sg * ul.y + sg * lu.y - ll.y));
                err = fmax > 0 ? (err > sqrt(zabs2(cpl)) ? err : sqrt(zabs2(cpl))) : err;
            }
        for (int a = 0; a < 6; a++)  // Hermiticity
            for (int b = a; b < 6; b++) {
                const double d = sqrt((T[a][b].x - T[b][a].x) * (T[a][b].x - T[b][a].x) +
                                      (T[a][b].y + T[b][a].y) * (T[a][b].y + T[b][a].y));
                err = err > d ? err : d;
            }
        double m[36];
        pack36(m, T);
        store36(static_cast<char *>(t64) + par * clover_parity_bytes(P64, g), P64, blk, g.stride, i, m);
        if (t32) store36(static_cast<char *>(t32) + par * clover_parity_bytes(P32, g), P32, blk, g.stride, i, m);
        if (!inv6(T)) bad |= 2;
        pack36(m, T);
        store36(static_cast<char *>(ti64) + par * clover_parity_bytes(P64, g), P64, blk, g.stride, i, m);
        if (ti32) store36(static_cast<char *>(ti32) + par * clover_parity_bytes(P32, g), P32, blk, g.stride, i, m);
    }
    if (err > tol * (1.0 + fmax)) bad |= 1;
    if (bad) atomicOr(flag, bad);
}

template <int SP>
__global__ void clover_apply_kernel(Spinor out, Spinor in, const void *blocks, const Geom g, int nrhs) {
    using R = real_t<SP>;
    constexpr int CP = SP == P64 ? P64 : P32;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= g.Vh || r >= nrhs) return;
    Cx<R> v[12];
    load_site<SP, R>(v, in, g.stride, r, i);
    clov_apply<CP, R>(v, blocks, g.stride, i);
    store_site<SP, R>(out, g.stride, r, i, v);
}

}  // namespace

hipError_t launch_clover_pack(void *t64, void *ti64, void *t32, void *ti32, const double *F, const Geom &g,
                              double tol, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(clover_pack_kernel, dim3((g.Vh + 127) / 128, 2), dim3(128), 0, s, t64, ti64, t32, ti32, F, g,
                       tol, flag);
    return hipGetLastError();
}

hipError_t launch_clover_apply(Spinor out, Spinor in, const void *blocks, const Geom &g, int nrhs, hipStream_t s) {
    if (out.prec != in.prec || nrhs < 1 || nrhs > 65535) return hipErrorInvalidValue;
    dim3 grid((g.Vh + 255) / 256, nrhs);
    switch (in.prec) {
        case P64: hipLaunchKernelGGL(clover_apply_kernel<P64>, grid, dim3(256), 0, s, out, in, blocks, g, nrhs); break;
        case P32: hipLaunchKernelGGL(clover_apply_kernel<P32>, grid, dim3(256), 0, s, out, in, blocks, g, nrhs); break;
        case P16: hipLaunchKernelGGL(clover_apply_kernel<P16>, grid, dim3(256), 0, s, out, in, blocks, g, nrhs); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wl
