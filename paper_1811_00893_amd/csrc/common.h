// Internal declarations shared by the host runtime (.cpp) and the kernels (.hip).
//
// Data layout in HBM ("parity-split structure of arrays"):
//   * a lattice site (x,y,z,t) of parity p = (x+y+z+t)&1 has checkerboard index
//     cb = (x + Lx*(y + Ly*(z + Lz*t))) / 2 in [0, Vh), Vh = V/2;
//   * a spinor field of one parity is a set of planes of 16-byte elements; element plane e
//     holds components CPE*e .. CPE*e+CPE-1 (component c = 3*spin + colour; CPE = 1, 2, 4
//     complex for FP64, FP32, FP16) of every cb site: element (e, cb) at byte
//     (e*stride + cb)*16; nrhs fields are stacked with 12/CPE planes each.  FP16 fields add
//     one FP32 scale per site, [rhs*stride + cb];
//   * links: element plane (p, mu, e) holds entries of U_mu(x) of every parity-p site x
//     (row-major entries, 1 complex per 16-byte FP64 element, 2 per FP32 / FP16 element);
//     SU(3) fields keep rows 0 and 1 only, other fields all 9 entries with the
//     antiperiodic sign folded into U_t on the t = Lt-1 slice.
// One lane processes one site: every plane load of a wavefront is one contiguous,
// fully coalesced segment.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace wl {

constexpr int kMaxRhs = 64;

enum Prec : int { P64 = 0, P32 = 1, P16 = 2 };

inline size_t real_bytes(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }

// Division of a non-negative 31-bit n by a fixed d >= 1 with one multiply-high, an add
// and a shift (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
// n / d = (mulhi(m, n) + n) >> l; mulhi + n stays below 2^32 because n < 2^31.
struct FastDiv {
    uint32_t d = 1, m = 1, l = 0;
};
inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((1ull << l) < d) l++;
    f.l = l;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    return f;
}
__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv &f) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t hi = __umulhi(f.m, n);
#else
    const uint32_t hi = (uint32_t)(((uint64_t)f.m * n) >> 32);
#endif
    return (hi + n) >> f.l;
}

struct Geom {
    int L[4];     // Lx, Ly, Lz, Lt
    int Lxh;      // Lx / 2
    int Vh;       // sites per parity
    int stride;   // plane stride (Vh rounded up to a multiple of 64)
    int sy, sz, st;  // checkerboard-index strides of +y, +z, +t
    FastDiv dLxh, dLy, dLz;  // division by Lx/2, Ly, Lz (site-index decoding)
};

Geom make_geom(const int32_t dims[4]);

// A spinor field of one parity (possibly nrhs fields back to back).
struct Spinor {
    void *data = nullptr;   // planes: double2 / float2 / _Float16 x2 per complex
    float *scale = nullptr; // FP16 per-site scales, [rhs][stride]
    int prec = P64;
};

inline size_t spinor_plane_bytes(int prec, const Geom &g) { return (size_t)g.stride * 2 * real_bytes(prec); }
inline size_t spinor_field_bytes(int prec, const Geom &g) {
    return 12 * spinor_plane_bytes(prec, g) + (prec == P16 ? (size_t)g.stride * 4 : 0);
}

// Per-right-hand-side Krylov state, resident on the device.  The scalars of the
// iteration are computed on the device, so the host never has to wait for them.
enum Phase : int { PH_IDLE = 1, PH_RUN = 2, PH_SCONV = 4, PH_DONE = 8, PH_FAIL = 16 };
enum FailCode : int { FAIL_NONE = 0, FAIL_BREAKDOWN = 1, FAIL_NONFINITE = 2 };

constexpr int kStateRing = 4;  // host-mapped state mirrors of a solve in flight

struct alignas(16) RhsState {
    double rho_re, rho_im;      // <rhat, r>
    double alpha_re, alpha_im;
    double omega_re, omega_im;
    double beta_re, beta_im;
    double r2;                  // |r|^2 (iterated residual)
    double s2;                  // |s|^2
    double rhat2;               // |rhat|^2
    double stop2;               // (tol * |b|)^2
    double zz;                  // CGLS |z|^2
    double aux;                 // scratch (e.g. a norm returned to the host)
    int phase;
    int fail;
    int iter;
    int pad;
};

// Reduction kinds a kernel epilogue can produce (values per block).
enum RedKind : int { RED_NONE = 0, RED_NORM2 = 1, RED_DOT = 2, RED_TS = 3 };
__host__ __device__ inline int red_nvals(int kind) { return kind == RED_NONE ? 0 : (kind == RED_NORM2 ? 1 : (kind == RED_DOT ? 2 : 3)); }

// Scalar programs run by the finalize kernel after a reduction.
enum FinOp : int {
    FIN_STORE_AUX = 0,  // aux = value 0 (norms for the host)
    FIN_BICG_INIT,      // r2 = |r|^2, rho = r2, alpha = omega = 1, beta = 0
    FIN_BICG_ALPHA,     // alpha = rho / <rhat, v>
    FIN_BICG_S,         // s2 = |s|^2; s-convergence
    FIN_BICG_OMEGA,     // omega = <t,s> / |t|^2
    FIN_BICG_RHO,       // r2, rho' -> beta, rho; convergence
    FIN_CG_R2,          // r2 = |r|^2; convergence at start
    FIN_CG_ZZ,          // zz = |z|^2 (first)
    FIN_CG_ALPHA,       // alpha = zz / |w|^2
    FIN_CG_R,           // r2 after the update; iteration count; convergence
    FIN_CG_BETA,        // beta = |z'|^2 / zz; zz = |z'|^2
    FIN_ADD_AUX,        // aux += value 0
    FIN_BLOCK_TS        // omega = <t,s> (values 0, 1), aux = |t|^2 (value 2), summed over the block later
};

// Arguments of one parity-hop launch:  out = cH[rhs] * (G5out? g5:1) H (G5in? g5:1) in
//                                            (+ y) (+ cz * z), on output parity `par`.
struct HopArgs {
    Geom g;
    int par;           // output parity
    int nrhs;
    Spinor out, in, y, z, w;  // y, z: same parity as out (optional); w: dot partner
    const void *gauge; // links of the kernel's precision
    int gprec;
    int recon;         // 18: full links, sign folded; 12: two rows, third rebuilt, t-boundary sign applied here
    int has_y, has_z, g5in, g5out, nostore;
    int red;           // RedKind
    double cz;
    double cH[kMaxRhs];
    double *partials;  // [rhs][nvals][pstride]
    int pstride;       // stride between partial rows (0: the launch's block count)
    RhsState *state;   // optional: per-rhs phase gate
    int run_mask;
    // clover site term (see ClovMode): packed 6x6 blocks of the output parity, in the
    // precision of the arithmetic (FP64 for FP64 spinors, FP32 otherwise)
    const void *clov;
    int clov_mode;
};

// Where the clover site matrices (T = 1 + F or its inverse, packed per site as two
// Hermitian 6x6 blocks of the chiral basis) enter a hop's epilogue.
enum ClovMode {
    CLV_NONE = 0,
    CLV_Y = 1,    // out = cH H in + T y          (the reduction partner y stays y)
    CLV_Z = 2,    // out = cH H in + y + cz T z
    CLV_ALL = 3   // out = T (cH H in + y)        (T: the blocks passed, e.g. the inverse)
};

// Packed Hermitian 6x6 block: 6 real diagonal entries, then the 15 entries above the
// diagonal (row-major) as (re, im): 36 reals; two blocks (+, - chirality) per site.
constexpr int kClovReals = 72;
// bytes of one parity's packed clover blocks (planes of 16-byte elements)
__host__ __device__ inline size_t clover_parity_bytes(int prec, const Geom &g) {
    return (size_t)(prec == P64 ? 36 : 18) * g.stride * 16u;
}

// Launch configuration chosen by the tuner.
struct LaunchCfg {
    int block = 256;
    int rpt = 1;       // right-hand sides per thread (multi-RHS hop)
    int xcd = 1;       // XCD-contiguous tile order
    int zblk = 0;      // >0: visit (z,t) planes in blocks of zblk z-values, t inner (divides Lz)
    int lds_kb = 0;    // >0: reserve this much LDS per block to cap blocks per CU (waves in flight)
    int wsplit = 0;    // 1: the waves of a block take successive RHS groups of the same 64 sites
    int shx = 0;       // 1: x/y neighbours shuffled from the lanes that loaded them (RPT 1)
    int dsplit = 0;    // 1: five waves per 64-site tile, wave 1 + mu on direction mu (block 320, RPT 1)
    int ldsl = 0;      // 1: with wsplit, the tile's links loaded once into LDS for all waves of the block;
                       // 2: the same with two-row links rebuilt to nine entries while staging
    int tm = 0;        // >= 1: each block marches its segment of the (x,y,z) slices through tm t-slices (every second one)
};

// ---- block BiCGStab (several right-hand sides of one matrix share one Krylov space) ----
constexpr int kMaxBlock = 16;  // right-hand sides per block; larger sets are split into blocks
// Device-resident s x s matrices of one block iteration (complex, row-major [i][j]).
struct BlockState {
    double gram[2 * kMaxBlock * kMaxBlock * 2];  // one or two Gram matrices R~^H Y of the last reduction
    double lu[kMaxBlock * kMaxBlock * 2];        // LU factors of R~^H V (unit L below the diagonal)
    double alpha[kMaxBlock * kMaxBlock * 2];
    double beta[kMaxBlock * kMaxBlock * 2];
    double omega[2];
    int piv[kMaxBlock];                          // row exchanged with row k at step k
};
// Arguments of the block kernels (FP64 fields of s right-hand sides, parity-split planes).
struct BlockArgs {
    Geom g;
    int s;
    Spinor a, b, c, d, x;   // operand roles per kernel
    double *partials;       // [value][nblk]
    int nblk;               // partial row length (set by the launcher)
    BlockState *bs;
    RhsState *state;        // the s per-RHS states; all carry the block's phase
    RhsState *mirror;       // optional host-mapped copy written by the check step
};
enum BlockSolveOp : int {
    BS_INIT = 0,   // make the per-RHS phases after the initial norms one block phase
    BS_ALPHA,      // LU of G0 = R~^H V (kept), alpha = G0^-1 G1 with G1 = R~^H R
    BS_BETA,       // omega = sum <T_j,S_j> / sum |T_j|^2; beta = -G0^-1 (R~^H T)
    BS_CHECK       // |R_j|^2 from the update's partials; iteration count; convergence of all
};
enum BlockUpdateOp : int {
    BU_S = 0,   // S(a) = R(b) - V(c) alpha
    BU_XR,      // X += P(a) alpha + omega S(b); R(c) = S - omega T(d); |R_j|^2 partials
    BU_P        // P(a) = R(b) + (P - omega V(c)) beta
};
// Gram: G_p = A^H B_p (A = a, B_0 = b, B_1 = c when np = 2) reduced into bs->gram.
hipError_t launch_block_gram(BlockArgs a, int np, hipStream_t s);
hipError_t launch_block_solve(int op, BlockArgs a, hipStream_t s);
hipError_t launch_block_update(int op, BlockArgs a, hipStream_t s);
// partial sums the block kernels need (doubles)
size_t block_partials_doubles(const Geom &g);

// ---- kernel launchers (implemented in the .hip files) ----
int hop_nblocks(const HopArgs &a, const LaunchCfg &c);
hipError_t launch_hop(const HopArgs &a, const LaunchCfg &c, hipStream_t s);
bool hop_cfg_valid(const HopArgs &a, const LaunchCfg &c);

// A finalize run at the start of a vector kernel instead of a launch of its own (short
// partial rows only): the scalar step `op` on the `nv` values of each right-hand side's
// `nblocks` partials, applied to the states `src` (phases in run_mask) and stored, with
// every other field, to `dst`; the kernel then uses the new state.
struct PreFin {
    int on;
    int op;           // FinOp
    int nv;
    int nblocks;
    int run_mask;
    const double *partials;  // [rhs][nv][nblocks]; not the kernel's own partials buffer
    const RhsState *src;
    RhsState *dst;
};
// vector kernels run the finalize of their input only for partial rows up to this length
// (every block of the kernel sums the row again); the finalize kernel sums such rows with
// one wave, as they do
constexpr int kPreFinMax = 128;

// BLAS-1 on one parity, nrhs fields; all take the per-rhs state gate.
struct BlasArgs {
    Geom g;
    int nrhs;
    Spinor a, b, c, d, e;   // operand roles documented per op
    Spinor x;               // solution field (may differ in precision)
    double *partials;       // [rhs][nvals][pstride]
    int pstride;            // 0: the launch's block count
    RhsState *state;
    int run_mask;
    PreFin pre;             // optional finalize before the op (then the gate and the op use its state)
};
enum BlasOp : int {
    BL_P_UPDATE = 0,  // a = p: p = r(b) + beta (p - omega v(c))
    BL_S_UPDATE,      // a = s: s = r(b) - alpha v(c); |s|^2
    BL_XR_UPDATE,     // x += alpha p(a) + omega s(b); r(c) = s - omega t(d); |r|^2, <rhat(e), r>
    BL_COPY_NORM,     // a = copy of b; |b|^2
    BL_CG_XR,         // x += alpha p(a); r(b) -= alpha w(c); |r|^2
    BL_CG_P,          // p(a) = z(b) + beta p
    BL_NORM2          // |a|^2
};
// partial sums one BLAS launch leaves per RHS and value (prec: storage precision of its operands)
int blas_nblocks(const Geom &g, int prec);
hipError_t launch_blas(int op, const BlasArgs &a, hipStream_t s);
hipError_t launch_finalize(int op, const double *partials, int nvals, int nblocks, int nrhs, RhsState *state,
                           int run_mask, hipStream_t s, RhsState *mirror = nullptr);
hipError_t launch_zero(const Spinor &f, const Geom &g, int nrhs, hipStream_t s);

// Layout / precision conversion.
// canonical complex128 [rhs][V][4][3]  <->  parity field of precision f.prec.
hipError_t launch_to_parity(Spinor f, const double *canon, const Geom &g, int par, int nrhs, double scale,
                            hipStream_t s);
hipError_t launch_from_parity(double *canon, Spinor f, const Geom &g, int par, int nrhs, hipStream_t s);
// dst (prec) = scale * src (FP64 parity field); nrhs fields; scale per rhs from state->aux if use_state.
hipError_t launch_convert(Spinor dst, Spinor src, const Geom &g, int nrhs, const RhsState *state, int inv_sqrt_aux,
                          hipStream_t s);
// x64 += c[rhs] * e (any precision): c = sqrt(state[rhs].aux) with sqrt_aux, else 1.
hipError_t launch_axpy_f64(Spinor x64, Spinor e, const Geom &g, int nrhs, const RhsState *state, int sqrt_aux,
                           hipStream_t s);
// Gauge: canonical complex128 links -> parity-split planes in precision prec.
// recon 18: all 9 entries, t-boundary sign folded in; recon 12: rows 0 and 1 only, no sign.
hipError_t launch_gauge_pack(void *dst, int prec, const double *canon, const Geom &g, int recon, hipStream_t s);
// Sets *flag (device int) to 1 if any canonical link deviates from SU(3) by more than tol
// (max |U U^dag - 1|, |det U - 1|).
hipError_t launch_su3_check(const double *canon, size_t nlinks, double tol, int *flag, hipStream_t s);
// Link planes: 16-byte elements of 1 (FP64) or 2 (FP32) complex, 8-byte elements of 2
// complex (FP16); 6 or 9 complex entries per link.
inline size_t gauge_bytes(int prec, int recon, const Geom &g) {
    const int ne = recon == 12 ? 6 : 9;
    const int nl = prec == P64 ? ne : (ne + 1) / 2;
    return (size_t)2 * 4 * nl * g.stride * (prec == P16 ? 8 : 16);
}
hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
// Read-only bandwidth probe; sink needs 8192 unsigned words.
hipError_t launch_stream_read(const void *src, size_t bytes, unsigned *sink, hipStream_t s);
// Checks that canonical input is finite; sets *flag (device int) to 1 otherwise.
hipError_t launch_check_finite(const double *p, size_t n, int *flag, hipStream_t s);
// clover: canonical F (V x 12 x 12 complex, Dirac basis) -> packed T = 1 + F and T^-1 for
// both parities in FP64 (and FP32 when t32/ti32 are given); flag |= 1 when F is not
// Hermitian or does not commute with gamma5 (relative tolerance tol), |= 2 when a block
// of T is singular.
hipError_t launch_clover_pack(void *t64, void *ti64, void *t32, void *ti32, const double *F, const Geom &g,
                              double tol, int *flag, hipStream_t s);
// out = M in on one parity (M: packed blocks of that parity, in the spinors' precision
// family), for nrhs right-hand sides.
hipError_t launch_clover_apply(Spinor out, Spinor in, const void *blocks, const Geom &g, int nrhs, hipStream_t s);

}  // namespace wl
