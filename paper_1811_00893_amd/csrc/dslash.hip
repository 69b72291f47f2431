// Launch dispatch of the parity hop: configuration checks and the precision pair switch.
// The kernels are in dslash_kernels.h, instantiated one precision pair per translation unit.
#include "common.h"
#include "device.h"

namespace wl {

template <int SP, int GP>
hipError_t launch_hop_r(const HopArgs &a, const LaunchCfg &c, hipStream_t s);

// ---------------------------------------------------------------------------------
bool hop_cfg_valid(const HopArgs &a, const LaunchCfg &c) {
    if (c.dsplit)  // one RHS per block, five waves, memory-order tiles of 64 sites
        return c.dsplit == 1 && c.block == 320 && c.rpt == 1 && !c.shx && !c.wsplit && c.zblk == 0 && c.lds_kb == 0 &&
               !c.ldsl && !c.tm;
    if (c.tm) {  // t-marching: whole t-chunks, segments of at least one wavefront per slice, no clover
        if (c.tm < 1 || a.g.L[3] % (2 * c.tm) != 0 || a.g.st < 64) return false;
        if (c.zblk != 0 || c.lds_kb != 0 || a.clov_mode != CLV_NONE) return false;
    }
    if (c.ldsl) {  // links in LDS: wave split, one or two RHS per lane, no clover epilogue
        if (c.ldsl < 1 || c.ldsl > 2 || !c.wsplit || c.lds_kb != 0 || c.rpt > 2 || (c.shx && c.rpt != 1)) return false;
        if (a.clov_mode != CLV_NONE || (a.gprec == P64 && a.recon == 18)) return false;
        // 2: two-row FP32 / FP16 links rebuilt to full links while staging (not with t-marching)
        if (c.ldsl == 2 && (a.gprec == P64 || a.recon != 12 || c.tm)) return false;
    }
    if (c.rpt < 1 || c.rpt > 4) return false;
    if (c.shx && c.rpt != 1) return false;  // with more RHS per lane the exchange spills
    if (a.clov_mode != CLV_NONE && (c.rpt != 1 || c.shx)) return false;  // clover kernels: one RHS per lane
    if (a.nrhs % c.rpt != 0) return false;
    if (c.wsplit) {
        // 2..4 waves, each on its own RHS group of one 64-site tile
        if (c.block != 128 && c.block != 192 && c.block != 256) return false;
        if ((a.nrhs / c.rpt) % (c.block / 64) != 0) return false;
    } else if (c.block != 64 && c.block != 128 && c.block != 256) {
        return false;
    }
    if (a.in.prec == P64 && c.rpt > 2) return false;
    if (c.zblk < 0 || (c.zblk > 0 && a.g.L[2] % c.zblk != 0)) return false;
    if (c.lds_kb < 0 || c.lds_kb > 56) return false;
    return true;
}

// Number of site tiles of a launch (the row length of the partial sums it writes).
int hop_nblocks(const HopArgs &a, const LaunchCfg &c) {
    const int tile = c.wsplit || c.dsplit ? 64 : c.block;
    if (c.tm) return (a.g.st + tile - 1) / tile * (a.g.L[3] / c.tm);
    return (a.g.Vh + tile - 1) / tile;
}

hipError_t launch_hop(const HopArgs &a, const LaunchCfg &c, hipStream_t s) {
    if (!hop_cfg_valid(a, c)) return hipErrorInvalidValue;
    const int sp = a.in.prec, gp = a.gprec;
    if (a.recon != 12 && a.recon != 18) return hipErrorInvalidValue;
    if (sp == P64 && gp == P64) return launch_hop_r<P64, P64>(a, c, s);
    if (sp == P32 && gp == P32) return launch_hop_r<P32, P32>(a, c, s);
    if (sp == P16 && gp == P16) return launch_hop_r<P16, P16>(a, c, s);
    if (sp == P16 && gp == P32) return launch_hop_r<P16, P32>(a, c, s);
    return hipErrorInvalidValue;
}

}  // namespace wl
