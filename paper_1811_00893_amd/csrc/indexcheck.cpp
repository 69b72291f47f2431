// Host replay of the kernels' site indexing on one lattice (wilson_index_check).
//
// The kernels decode a checkerboard index into coordinates (cb_coords), form the eight
// neighbour indices of the hop (site_nbrs), permute sites in the plane-blocked visiting
// order (visit_order) and blocks in the XCD-contiguous order (xcd_tile).  The same
// functions (device.h, compiled for the host here) are checked against plain
// coordinate arithmetic: every index in range, coordinates and neighbours where the
// definition of the lattice puts them, neighbours on the other parity, and every map
// that should be a permutation a permutation.
#include <string>
#include <vector>

#include "common.h"
#include "device.h"
#include "runtime.h"

namespace wl {

namespace {

// checkerboard index of the site with coordinates (x, y, z, t) among the sites of its parity
long long plain_cb(const int L[4], int x, int y, int z, int t) {
    return ((long long)x + (long long)L[0] * (y + (long long)L[1] * (z + (long long)L[2] * t))) / 2;
}

struct Checker {
    long long bad = 0;
    std::string first;
    void fail(const std::string &m) {
        if (bad++ == 0) first = m;
    }
    // p[0..n) must be a permutation of [0, n)
    void permutation(const std::vector<int> &p, const std::string &what) {
        std::vector<char> seen(p.size(), 0);
        for (size_t k = 0; k < p.size(); k++) {
            if (p[k] < 0 || (size_t)p[k] >= p.size()) {
                fail(what + ": index " + std::to_string(p[k]) + " out of [0, " + std::to_string(p.size()) + ")");
                return;
            }
            if (seen[p[k]]++) {
                fail(what + ": index " + std::to_string(p[k]) + " visited twice");
                return;
            }
        }
    }
};

}  // namespace

long long index_check(const int32_t dims[4], std::string &first) {
    const Geom g = make_geom(dims);
    const int *L = g.L;
    Checker ck;
    for (int par = 0; par < 2; par++) {
        std::vector<std::vector<int>> nbr(8, std::vector<int>(g.Vh));
        for (int i = 0; i < g.Vh; i++) {
            const SiteXY c = cb_coords(g, i, par);
            // plain decode: i = xh + Lx/2 (y + Ly (z + Lz t)), x = 2 xh + (y + z + t + par) mod 2
            const int xh = i % g.Lxh, q1 = i / g.Lxh, y = q1 % L[1], q2 = q1 / L[1], z = q2 % L[2], t = q2 / L[2];
            const int x = 2 * xh + ((y + z + t + par) & 1);
            if (c.xh != xh || c.y != y || c.z != z || c.t != t || 2 * c.xh + c.b != x || t >= L[3]) {
                ck.fail("parity " + std::to_string(par) + " site " + std::to_string(i) + ": coordinates differ from the plain decode");
                continue;
            }
            const SiteNbrs n = site_nbrs(g, i, c);
            const int got[8] = {n.xp, n.xm, n.yp, n.ym, n.zp, n.zm, n.tp, n.tm};
            for (int d = 0; d < 8; d++) {
                const int mu = d / 2, step = (d % 2) ? -1 : 1;
                int X[4] = {x, y, z, t};
                X[mu] = (X[mu] + step + L[mu]) % L[mu];
                const long long want = plain_cb(L, X[0], X[1], X[2], X[3]);
                const int npar = (X[0] + X[1] + X[2] + X[3]) & 1;
                if (got[d] < 0 || got[d] >= g.Vh || got[d] != want || npar != 1 - par) {
                    ck.fail("parity " + std::to_string(par) + " site " + std::to_string(i) + " neighbour " +
                            std::to_string(d) + ": index " + std::to_string(got[d]) + ", expected " +
                            std::to_string(want) + " on the other parity");
                    continue;
                }
                nbr[d][i] = got[d];
            }
        }
        for (int d = 0; d < 8; d++) ck.permutation(nbr[d], "parity " + std::to_string(par) + " neighbour map " + std::to_string(d));
    }
    // plane-blocked visiting orders: every zblk a launch may use (a divisor of Lz)
    for (int zblk = 1; zblk <= L[2]; zblk++) {
        if (L[2] % zblk) continue;
        const VisitOrder vo = make_visit_order(g, zblk);
        std::vector<int> p(g.Vh);
        for (int l = 0; l < g.Vh; l++) p[l] = visit_order(l, g, vo);
        ck.permutation(p, "visiting order zblk " + std::to_string(zblk));
    }
    // XCD-contiguous block order: every grid of up to 4096 blocks, and the grid sizes of
    // this lattice's hop launches (site tiles of 64, 128 or 256 sites, or t-marching
    // segments, times the usual right-hand-side group counts)
    std::vector<int> sizes;
    for (int n = 1; n <= 4096; n++) sizes.push_back(n);
    for (int tile : {64, 128, 256}) {
        std::vector<int> base = {(g.Vh + tile - 1) / tile};
        for (int tm : {2, 4, 8})
            if (L[3] % (2 * tm) == 0) base.push_back((g.st + tile - 1) / tile * (L[3] / tm));
        for (int b : base)
            for (int groups : {1, 2, 3, 4, 6, 12, 64}) sizes.push_back(b * groups);
    }
    for (int n : sizes) {
        std::vector<int> p(n);
        for (int b = 0; b < n; b++) p[b] = xcd_tile(b, n);
        ck.permutation(p, "XCD block order over " + std::to_string(n) + " blocks");
    }
    first = ck.first;
    return ck.bad;
}

}  // namespace wl
