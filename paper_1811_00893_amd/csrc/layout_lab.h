// Layout ablation of the parity hop: the same hop arithmetic under several storage layouts
// of the spinor and link fields (the comparison of data layouts of Sec. 4.1 and its
// result in Sec. 5, carried over to wavefronts).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "common.h"

namespace wl {

enum LabLayout : int {
    LAB_SOA = 0,    // component planes over checkerboard sites (the library's own layout)
    LAB_AOS = 1,    // each site's components contiguous
    LAB_AOSOA = 2,  // tiles of 64 sites, component planes inside a tile
    LAB_VNODE = 3,  // 64 sub-lattices, lane l of a wavefront holds sub-lattice l
    LAB_LAYOUT_COUNT = 4
};

// Lattice and storage geometry of one layout.  With LAB_VNODE the lattice is cut into
// 1 x 4 x 4 x 4 sub-lattices in (x, y, z, t) and a storage slot is (local cb index) * 64 +
// (sub-lattice); otherwise the slot is the checkerboard index and nsub[] = {1, 1, 1, 1}.
struct LabGeom {
    int L[4];      // global extents
    int nl[4];     // sub-lattice extents (L[k] / nsub[k])
    int nsub[4];   // sub-lattices per direction
    int nlxh;      // nl[0] / 2
    int Vh;        // slots (sites) per parity
    int pad;       // Vh rounded up to a multiple of 64: plane stride and tile count * 64
    FastDiv dnlxh, dnl1, dnl2;  // division by nl[0]/2, nl[1], nl[2]
};

// false when the extents do not allow the layout (every extent even and >= 2; LAB_VNODE
// also needs Ly, Lz and Lt to be multiples of 8 so that every sub-lattice extent is even)
bool lab_geom(LabGeom &g, const int32_t dims[4], int layout);

// Bytes of one parity field: a spinor (12 complex per site) or the links of one parity
// (4 links of `link_reals` reals per site) in precision prec (P64 or P32).
size_t lab_spinor_bytes(const LabGeom &g, int prec);
size_t lab_link_bytes(const LabGeom &g, int prec, int link_reals);

// Canonical complex128 field (site s = x + Lx*(y + Ly*(z + Lz*t)), 12 complex per site)
// -> the sites of parity par in the layout, and back (unpack writes only parity par).
hipError_t launch_lab_pack_spinor(void *dst, const double *canon, const LabGeom &g, int layout, int prec, int par,
                                  hipStream_t s);
hipError_t launch_lab_unpack_spinor(double *canon, const void *src, const LabGeom &g, int layout, int prec, int par,
                                    hipStream_t s);
// Canonical links (U_mu(s) at complex offset ((s*4+mu)*3+a)*3+b) of the sites of parity par.
// With 18 reals the antiperiodic sign of the t-links on t = Lt-1 is folded in; with 12 the
// first two rows are kept and the hop applies the sign.
hipError_t launch_lab_pack_links(void *dst, const double *canonU, const LabGeom &g, int layout, int prec,
                                 int link_reals, int par, hipStream_t s);
// out (parity par) = cH * H in (in: parity 1-par); U[p]: links of parity p.
hipError_t launch_lab_hop(void *out, const void *in, const void *U0, const void *U1, const LabGeom &g, int layout,
                          int prec, int link_reals, int par, double cH, hipStream_t s);
// Fill n doubles with zero.
hipError_t launch_lab_zero(double *p, size_t n, hipStream_t s);

}  // namespace wl
