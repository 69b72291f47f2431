// Parity hop of the Wilson operator (Eq. (1), Sec. 2.1):
//
//   out(x) = cH * sum_mu [ (1 - gamma_mu) U_mu(x) in(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag in(x-mu) ]
//            (+ y(x)) (+ cz * z(x)),   for every site x of the output parity,
//
// with optional gamma5 on the input and on the hop result (used for M^dag = g5 M g5),
// and an optional fused reduction of the result (|out|^2, <w,out>, or <out,y> and |out|^2).
//
// One lane owns one output site and `RPT` right-hand sides; every link is loaded once
// per site and reused for those right-hand sides.  The 4x4 spin structure is applied
// through spin projection: (1 -/+ gamma_mu) has rank 2, so only a two-spinor "half
// spinor" h is multiplied by the link (two SU(3) mat-vecs instead of four) and the
// other two spin rows are rebuilt from it.  In the Dirac basis (gamma_t diagonal)
// the t projections are (0, 0, 2psi2, 2psi3) forward and (2psi0, 2psi1, 0, 0) backward,
// so a t-hop reads only two spins of its neighbour.
//
// Links are stored either in full (18 reals, antiperiodic sign folded into the t-links of
// the t = Lt-1 slice) or, for SU(3) fields, as their first two rows (12 reals: a third
// less link traffic, the largest part of the kernel's bytes); the third row is then
// rebuilt as conj(row0 x row1) and the boundary sign is applied to the two t-hops that
// cross t = Lt-1 <-> 0.
#pragma once
// Kernel templates; each dslash_<precision>.hip instantiates one precision pair.
#include <cstdio>

#include "common.h"
#include "device.h"

namespace wl {

// --- spin projection / reconstruction tables (Dirac basis) ------------------------
// forward uses (1 - gamma_mu), backward (1 + gamma_mu).  psi: 4 spins x 3 colours.
template <int MU, bool FWD, typename R>
__device__ __forceinline__ void project(const Cx<R> (&p)[4][3], Cx<R> (&h)[2][3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if constexpr (MU == 0) {
            if constexpr (FWD) { h[0][c] = cadd_i(p[0][c], p[3][c]); h[1][c] = cadd_i(p[1][c], p[2][c]); }
            else               { h[0][c] = csub_i(p[0][c], p[3][c]); h[1][c] = csub_i(p[1][c], p[2][c]); }
        } else if constexpr (MU == 1) {
            if constexpr (FWD) { h[0][c] = cadd(p[0][c], p[3][c]); h[1][c] = csub(p[1][c], p[2][c]); }
            else               { h[0][c] = csub(p[0][c], p[3][c]); h[1][c] = cadd(p[1][c], p[2][c]); }
        } else if constexpr (MU == 2) {
            if constexpr (FWD) { h[0][c] = cadd_i(p[0][c], p[2][c]); h[1][c] = csub_i(p[1][c], p[3][c]); }
            else               { h[0][c] = csub_i(p[0][c], p[2][c]); h[1][c] = cadd_i(p[1][c], p[3][c]); }
        } else {
            if constexpr (FWD) { h[0][c] = cadd(p[2][c], p[2][c]); h[1][c] = cadd(p[3][c], p[3][c]); }
            else               { h[0][c] = cadd(p[0][c], p[0][c]); h[1][c] = cadd(p[1][c], p[1][c]); }
        }
    }
}

template <int MU, bool FWD, typename R>
__device__ __forceinline__ void reconstruct(Cx<R> (&acc)[4][3], const Cx<R> (&u)[2][3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if constexpr (MU == 3) {
            if constexpr (FWD) { acc[2][c] = cadd(acc[2][c], u[0][c]); acc[3][c] = cadd(acc[3][c], u[1][c]); }
            else               { acc[0][c] = cadd(acc[0][c], u[0][c]); acc[1][c] = cadd(acc[1][c], u[1][c]); }
        } else {
            acc[0][c] = cadd(acc[0][c], u[0][c]);
            acc[1][c] = cadd(acc[1][c], u[1][c]);
            if constexpr (MU == 0) {
                if constexpr (FWD) { acc[2][c] = csub_i(acc[2][c], u[1][c]); acc[3][c] = csub_i(acc[3][c], u[0][c]); }
                else               { acc[2][c] = cadd_i(acc[2][c], u[1][c]); acc[3][c] = cadd_i(acc[3][c], u[0][c]); }
            } else if constexpr (MU == 1) {
                if constexpr (FWD) { acc[2][c] = csub(acc[2][c], u[1][c]); acc[3][c] = cadd(acc[3][c], u[0][c]); }
                else               { acc[2][c] = cadd(acc[2][c], u[1][c]); acc[3][c] = csub(acc[3][c], u[0][c]); }
            } else {
                if constexpr (FWD) { acc[2][c] = csub_i(acc[2][c], u[0][c]); acc[3][c] = cadd_i(acc[3][c], u[1][c]); }
                else               { acc[2][c] = cadd_i(acc[2][c], u[0][c]); acc[3][c] = csub_i(acc[3][c], u[1][c]); }
            }
        }
    }
}

// Spins of the neighbour a direction needs: t forward reads 2,3; t backward 0,1.
template <int MU, bool FWD>
__device__ __forceinline__ constexpr bool spin_needed(int s) {
    return MU != 3 ? true : (FWD ? s >= 2 : s < 2);
}

// NE: stored complex entries per link (9, or 6 = the first two rows of an SU(3) matrix).
// sgn: boundary sign of this hop (only used with NE == 6; full links carry it folded in).
// Projected half spinor of one neighbour: gamma5 (when it acts on the input), the spin
// projection of direction MU/FWD, and the FP16 site scale.
template <int SP, int MU, bool FWD, bool G5>
__device__ __forceinline__ void proj_in(const Cx<real_t<SP>> (&comp)[12], real_t<SP> sc, Cx<real_t<SP>> (&h)[2][3]) {
    using R = real_t<SP>;
    Cx<R> p[4][3];
    // gamma5 on the input: (g5 psi)_s = -psi_{s^2} (a compile-time choice: the values
    // of both permutations would otherwise have to stay live across a branch)
#pragma unroll
    for (int sp = 0; sp < 4; sp++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            if constexpr (G5)
                p[sp][c] = spin_needed<MU, FWD>(sp) ? Cx<R>{-comp[(sp ^ 2) * 3 + c].re, -comp[(sp ^ 2) * 3 + c].im}
                                                    : Cx<R>{R(0), R(0)};
            else
                p[sp][c] = spin_needed<MU, FWD>(sp) ? comp[sp * 3 + c] : Cx<R>{R(0), R(0)};
        }
    project<MU, FWD, R>(p, h);
    if constexpr (SP == P16) {
#pragma unroll
        for (int k = 0; k < 2; k++)
#pragma unroll
            for (int c = 0; c < 3; c++) h[k][c] = cscale(h[k][c], sc);
    }
}

// SRC selects where the neighbour comes from: 0 = loaded here from the input field;
// 1 = its projected half spinors given in H.  LL: the link comes from the block's LDS copy
// `ll` (see stage_links) instead of global memory.
template <int SP, int GP, int RPT, int NE, bool G5, bool LNT, int MU, bool FWD, int SRC = 0, bool LL = false,
          int BAR = -1, int LNE = 0>
__device__ __forceinline__ void hop_dir(Cx<real_t<SP>> (&acc)[RPT][4][3], const HopArgs &a, const bool (&act)[RPT],
                                        int r0, int nbr, int link_par, int link_site, real_t<SP> sgn, int stride,
                                        const Cx<real_t<SP>> (*H)[2][3] = nullptr, const char *ll = nullptr) {
    using R = real_t<SP>;
    // link U_mu(x) (forward, at the output site) or U_mu(x - mu) (backward, at the neighbour)
    // LNE = 9: the block's LDS copy holds all nine entries, the boundary sign folded in
    constexpr bool FULL = LL && LNE == 9;
    Cx<R> U[3][3];
    {
        constexpr int NEU = FULL ? 9 : NE;
        constexpr int NL = LinkElems<GP, NEU>::N, CPL = LinkPack<GP>::CPL;
        Cx<R> ue[NL * CPL];
        if constexpr (LL) {
            constexpr int d = 2 * MU + (FWD ? 0 : 1);
            const unsigned lane = threadIdx.x & 63u;
#pragma unroll
            for (int e = 0; e < NL; e++)
                ld_link_elem_lds<GP, R>(&ue[e * CPL], ll, ((unsigned)(d * NL + e) * 64u + lane) * LinkPack<GP>::EB);
        } else {
            const unsigned loff = (unsigned)link_site * LinkPack<GP>::EB;
#pragma unroll
            for (int e = 0; e < NL; e++)
                ld_link_elem<GP, R, LNT>(&ue[e * CPL], lplane<GP>(a.gauge, (link_par * 4 + MU) * NL + e, stride), loff);
        }
#pragma unroll
        for (int e = 0; e < NEU; e++) U[e / 3][e % 3] = ue[e];
    }
    if constexpr (NE == 6 && !FULL) {
        // third row of an SU(3) matrix: complex conjugate of (row 0) x (row 1)
        const Cx<R> c0 = csub(cmul(U[0][1], U[1][2]), cmul(U[0][2], U[1][1]));
        const Cx<R> c1 = csub(cmul(U[0][2], U[1][0]), cmul(U[0][0], U[1][2]));
        const Cx<R> c2 = csub(cmul(U[0][0], U[1][1]), cmul(U[0][1], U[1][0]));
        U[2][0] = {c0.re, -c0.im};
        U[2][1] = {c1.re, -c1.im};
        U[2][2] = {c2.re, -c2.im};
    }

    constexpr int CPE = SpinorPack<SP>::CPE, NEL = SpinorPack<SP>::NEL;
    // the t-hops read one spin half of the neighbour (components 6h..6h+5): the upper half
    // forward, the lower half backward, swapped when gamma5 acts on the input
    constexpr int half = MU == 3 ? ((FWD ? 1 : 0) ^ (G5 ? 1 : 0)) : -1;
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        // with one RHS per lane the kernel has already returned when it is inactive
        if (RPT > 1 && !act[r]) continue;
        Cx<R> h[2][3];
        if constexpr (SRC == 0) {
            const unsigned soff = (unsigned)nbr * 16u;
            Cx<R> comp[12];
#pragma unroll
            for (int e = 0; e < NEL; e++) {
                const bool need = half < 0 || ((e + 1) * CPE > 6 * half && e * CPE < 6 * half + 6);
                if (need) ld_elem<SP, R>(&comp[e * CPE], splane(a.in.data, (r0 + r) * NEL + e, stride), soff);
                else
#pragma unroll
                    for (int k = 0; k < CPE; k++) comp[e * CPE + k] = {R(0), R(0)};
            }
            R sc = R(1);
            if constexpr (SP == P16) sc = (R)gptr(a.in.scale)[(size_t)(r0 + r) * stride + nbr];
            proj_in<SP, MU, FWD, G5>(comp, sc, h);
        } else {
#pragma unroll
            for (int k = 0; k < 2; k++)
#pragma unroll
                for (int c = 0; c < 3; c++) h[k][c] = H[r][k][c];
        }
        Cx<R> u[2][3];
#pragma unroll
        for (int k = 0; k < 2; k++)
#pragma unroll
            for (int a_ = 0; a_ < 3; a_++) {
                Cx<R> t = {R(0), R(0)};
#pragma unroll
                for (int b_ = 0; b_ < 3; b_++) {
                    if constexpr (FWD) t = cfma(t, U[a_][b_], h[k][b_]);       // U h
                    else               t = cfma_conj(t, U[b_][a_], h[k][b_]);  // U^dag h
                }
                u[k][a_] = NE == 6 && MU == 3 && !FULL ? cscale(t, sgn) : t;
            }
        reconstruct<MU, FWD, R>(acc[r], u);
    }
    // directions go in two groups (x and y, then z and t): the loads of a group may overlap,
    // and a barrier after each group keeps later gathers from being hoisted into it (all
    // eight directions in flight need more registers than the budget; one direction at a
    // time measured 1.5 % slower in FP64)
    // (BAR 0 / 1: no barrier / a barrier after this direction, for other orders)
    if constexpr (BAR == 1 || (BAR < 0 && (MU == 1 || MU == 3) && !FWD)) __builtin_amdgcn_sched_barrier(0);
}

// One output site i (all RPT right-hand sides of this lane): gather, project, multiply,
// reconstruct, epilogue, store; the site's reduction terms are added to red[r][*].
// Input components of site j (all RPT right-hand sides, raw: before gamma5 and FP16 scale).
template <int SP, int RPT>
__device__ __forceinline__ void load_raw(Cx<real_t<SP>> (&v)[RPT][12], real_t<SP> (&vs)[RPT], const HopArgs &a,
                                         const bool (&act)[RPT], int r0, int j, int stride) {
    using R = real_t<SP>;
    constexpr int CPE = SpinorPack<SP>::CPE, NEL = SpinorPack<SP>::NEL;
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        if (RPT > 1 && !act[r]) {  // defined values for the lanes' exchanges; never used
#pragma unroll
            for (int k = 0; k < 12; k++) v[r][k] = {R(0), R(0)};
            vs[r] = R(1);
            continue;
        }
#pragma unroll
        for (int e = 0; e < NEL; e++)
            ld_elem<SP, R>(&v[r][e * CPE], splane(a.in.data, (r0 + r) * NEL + e, stride), (unsigned)j * 16u);
        if constexpr (SP == P16) vs[r] = (R)gptr(a.in.scale)[(size_t)(r0 + r) * stride + j];
        else vs[r] = R(1);
    }
}

// Projected neighbour j (direction MU/FWD) of this lane's site i: every lane projects its
// own centre C, and the lane of the same wavefront that holds site j as its centre
// (lane + j - i) hands its result over; where no lane holds j (the neighbour belongs to
// another wavefront, or the visiting order is not contiguous there) it is loaded.
template <int SP, int RPT, int MU, bool FWD, bool G5>
__device__ __forceinline__ void lane_nbr(Cx<real_t<SP>> (&H)[RPT][2][3], const Cx<real_t<SP>> (&C)[RPT][12],
                                         const real_t<SP> (&Cs)[RPT], const HopArgs &a, const bool (&act)[RPT], int r0,
                                         int i, int j, int stride) {
    using R = real_t<SP>;
    const int lane = (int)threadIdx.x & 63;
    const int src = lane + (j - i);
    const int srcc = src < 0 ? 0 : (src > 63 ? 63 : src);
    const bool ok = src == srcc && __shfl(i, srcc, 64) == j;
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        Cx<R> own[2][3];
        proj_in<SP, MU, FWD, G5>(C[r], Cs[r], own);
#pragma unroll
        for (int k = 0; k < 2; k++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                H[r][k][c].re = __shfl(own[k][c].re, srcc, 64);
                H[r][k][c].im = __shfl(own[k][c].im, srcc, 64);
            }
    }
    if (!ok) {
        Cx<R> v[RPT][12];
        R vs[RPT];
        load_raw<SP, RPT>(v, vs, a, act, r0, j, stride);
#pragma unroll
        for (int r = 0; r < RPT; r++) proj_in<SP, MU, FWD, G5>(v[r], vs[r], H[r]);
    }
    // the direction's link loads stay after the exchange (registers)
    __builtin_amdgcn_sched_barrier(0);
}

// Epilogue of one output site and right-hand side: gamma5 on the hop result, the factor
// cH, the y and z terms (with the clover modes), the store and the site's reduction terms.
// PRE (bits 1, 2, 4): y, z, the dot partner w are already in yv, zv, wv (loaded by the
// caller); the others are loaded here.  NT: the output and the operands read here are
// streamed (non-temporal); the small-lattice kernel keeps them cached instead, since the
// next kernel finds its whole working set in L2.
template <int SP, bool CLV, int PRE, bool NT = true>
__device__ __forceinline__ void hop_finish(const HopArgs &a, int i, bool valid, int rhs,
                                           const Cx<real_t<SP>> (&acc)[4][3], Cx<real_t<SP>> (&yv)[12],
                                           Cx<real_t<SP>> (&zv)[12], Cx<real_t<SP>> (&wv)[12], double (&red)[3],
                                           int stride) {
    using R = real_t<SP>;
    constexpr int CP = SP == P64 ? P64 : P32;  // storage precision of clover blocks
    const R cH = (R)a.cH[rhs];
    Cx<R> o[12];
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            // gamma5 on the hop result: (g5 v)_s = -v_{s^2}
            Cx<R> v = a.g5out ? Cx<R>{-acc[s ^ 2][k].re, -acc[s ^ 2][k].im} : acc[s][k];
            o[s * 3 + k] = cscale(v, cH);
        }
    if (a.has_y) {
        if (!(PRE & 1)) load_site<SP, R, NT>(yv, a.y, stride, rhs, i);
        if (CLV && a.clov_mode == CLV_Y) {  // T y enters the sum; y itself stays the dot partner
            Cx<R> ty[12];
#pragma unroll
            for (int k = 0; k < 12; k++) ty[k] = yv[k];
            clov_apply<CP, R>(ty, a.clov, stride, i);
#pragma unroll
            for (int k = 0; k < 12; k++) o[k] = cadd(o[k], ty[k]);
        } else {
#pragma unroll
            for (int k = 0; k < 12; k++) o[k] = cadd(o[k], yv[k]);
        }
    }
    if (CLV && a.clov_mode == CLV_ALL) clov_apply<CP, R>(o, a.clov, stride, i);
    if (a.has_z) {
        if (!(PRE & 2)) load_site<SP, R, NT>(zv, a.z, stride, rhs, i);
        if (CLV && a.clov_mode == CLV_Z) clov_apply<CP, R>(zv, a.clov, stride, i);
        const R cz = (R)a.cz;
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = cadd(o[k], cscale(zv[k], cz));
    }
    if (valid && !a.nostore) store_site<SP, R, NT>(a.out, stride, rhs, i, o);
    if (!valid || a.red == RED_NONE) return;
    if (a.red == RED_NORM2) {
        for (int k = 0; k < 12; k++) red[0] += (double)o[k].re * o[k].re + (double)o[k].im * o[k].im;
    } else if (a.red == RED_DOT) {
        if (!(PRE & 4)) load_site<SP, R, NT>(wv, a.w, stride, rhs, i);
        for (int k = 0; k < 12; k++) {  // <w, o> = sum conj(w) o
            red[0] += (double)wv[k].re * o[k].re + (double)wv[k].im * o[k].im;
            red[1] += (double)wv[k].re * o[k].im - (double)wv[k].im * o[k].re;
        }
    } else {
        for (int k = 0; k < 12; k++) {  // <o, y> and |o|^2
            red[0] += (double)o[k].re * yv[k].re + (double)o[k].im * yv[k].im;
            red[1] += (double)o[k].re * yv[k].im - (double)o[k].im * yv[k].re;
            red[2] += (double)o[k].re * o[k].re + (double)o[k].im * o[k].im;
        }
    }
}

// With the wave split all waves of a block work on the same 64 sites, so each link of the
// tile is needed by every wave: the waves load it once into LDS, wave w the directions
// d = w, w + nw, ... (lane l for site l of the tile), and everyone reads it from there.
// Every wave of the block calls this (it holds a block barrier).
template <int GP, int NE>
__device__ __forceinline__ void stage_links(char *ll, const HopArgs &a, int par, const int (&lsite)[8], int stride) {
    constexpr int NL = LinkElems<GP, NE>::N;
    constexpr unsigned EB = LinkPack<GP>::EB;
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6, nw = (int)blockDim.x >> 6;
    for (int d = w; d < 8; d += nw) {
        const int mu = d >> 1, lpar = (d & 1) ? 1 - par : par;
        const int site = lsite[d];
#pragma unroll
        for (int e = 0; e < NL; e++) {
            const gchar *src = lplane<GP>(a.gauge, (lpar * 4 + mu) * NL + e, stride) + (unsigned)site * EB;
            char *dst = ll + ((unsigned)(d * NL + e) * 64u + lane) * EB;
            typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
            typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
            if constexpr (EB == 16) *reinterpret_cast<u32x4 *>(dst) = *reinterpret_cast<const WL_GLOBAL u32x4 *>(src);
            else *reinterpret_cast<u32x2 *>(dst) = *reinterpret_cast<const WL_GLOBAL u32x2 *>(src);
        }
    }
    __syncthreads();
}

// The same staging with the links stored as two rows: the staging waves rebuild the third
// row (once per link and block, not once per RHS group) and fold in the antiperiodic sign
// of the t-links on the slice t = Lt - 1 (lsgn), so the LDS copy holds full links of nine
// entries (FP32 / FP16: five elements of two complex, the last half unused).
template <int GP>
__device__ __forceinline__ void stage_links_full(char *ll, const HopArgs &a, int par, const int (&lsite)[8],
                                                 const float (&lsgn)[8], int stride) {
    using R = float;  // FP32 and FP16 links (FP64 links keep the stored form)
    constexpr int NL6 = LinkElems<GP, 6>::N, NL9 = LinkElems<GP, 9>::N, CPL = LinkPack<GP>::CPL;
    constexpr unsigned EB = LinkPack<GP>::EB;
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6, nw = (int)blockDim.x >> 6;
    for (int d = w; d < 8; d += nw) {
        const int mu = d >> 1, lpar = (d & 1) ? 1 - par : par;
        Cx<R> ue[NL9 * CPL];
        const unsigned loff = (unsigned)lsite[d] * EB;
#pragma unroll
        for (int e = 0; e < NL6; e++)
            ld_link_elem<GP, R, false>(&ue[e * CPL], lplane<GP>(a.gauge, (lpar * 4 + mu) * NL6 + e, stride), loff);
        // third row of an SU(3) matrix: complex conjugate of (row 0) x (row 1)
        const Cx<R> c0 = csub(cmul(ue[1], ue[5]), cmul(ue[2], ue[4]));
        const Cx<R> c1 = csub(cmul(ue[2], ue[3]), cmul(ue[0], ue[5]));
        const Cx<R> c2 = csub(cmul(ue[0], ue[4]), cmul(ue[1], ue[3]));
        ue[6] = {c0.re, -c0.im};
        ue[7] = {c1.re, -c1.im};
        ue[8] = {c2.re, -c2.im};
        if constexpr (NL9 * CPL > 9) ue[9] = {R(0), R(0)};
        const R sg = (R)lsgn[d];
#pragma unroll
        for (int k = 0; k < 9; k++) ue[k] = cscale(ue[k], sg);
#pragma unroll
        for (int e = 0; e < NL9; e++) {
            char *dst = ll + ((unsigned)(d * NL9 + e) * 64u + lane) * EB;
            if constexpr (GP == P32) {
                fvec4 v;
                v.x = ue[2 * e].re;
                v.y = ue[2 * e].im;
                v.z = ue[2 * e + 1].re;
                v.w = ue[2 * e + 1].im;
                *reinterpret_cast<fvec4 *>(dst) = v;
            } else {
                hvec4 v;
                v[0] = (_Float16)ue[2 * e].re;
                v[1] = (_Float16)ue[2 * e].im;
                v[2] = (_Float16)ue[2 * e + 1].re;
                v[3] = (_Float16)ue[2 * e + 1].im;
                *reinterpret_cast<hvec4 *>(dst) = v;
            }
        }
    }
    __syncthreads();
}

template <int SP, int GP, int RPT, int NE, bool G5, bool LNT, bool SHX, bool CLV, bool LL = false, int LNE = 0>
__device__ __forceinline__ void hop_site(const HopArgs &a, int i, bool valid, int r0, const bool (&act)[RPT],
                                         double (&red)[RPT][3]) {
    using R = real_t<SP>;
    const Geom &g = a.g;
    const int stride = g.stride;
    const int par = a.par, opar = 1 - par;
    const SiteXY c = cb_coords(g, i, par);
    const SiteNbrs nb = site_nbrs(g, i, c);
    const int xp = nb.xp, xm = nb.xm, yp = nb.yp, ym = nb.ym, zp = nb.zp, zm = nb.zm, tp = nb.tp, tm = nb.tm;

    const char *ll = nullptr;
    if constexpr (LL) {
        constexpr int NES = LNE == 9 ? 9 : NE;
        __shared__ __align__(16) char ll_buf[8 * LinkElems<GP, NES>::N * 64 * LinkPack<GP>::EB];
        const int lsite[8] = {i, xm, i, ym, i, zm, i, tm};
        if constexpr (LNE == 9) {
            const float lsgn[8] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, c.t == g.L[3] - 1 ? -1.f : 1.f, c.t == 0 ? -1.f : 1.f};
            stage_links_full<GP>(ll_buf, a, par, lsite, lsgn, stride);
        } else {
            stage_links<GP, NE>(ll_buf, a, par, lsite, stride);
        }
        ll = ll_buf;
        bool any = false;
#pragma unroll
        for (int r = 0; r < RPT; r++) any |= act[r];
        if (!any) return;  // after the barrier: this wave's RHS group has finished
    }

    Cx<R> acc[RPT][4][3];
#pragma unroll
    for (int r = 0; r < RPT; r++)
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int k = 0; k < 3; k++) acc[r][s][k] = {R(0), R(0)};

    const R one = R(1);
    const R sgn_tf = (NE == 6 && c.t == g.L[3] - 1) ? -one : one;  // forward hop across t = Lt-1 -> 0
    const R sgn_tb = (NE == 6 && c.t == 0) ? -one : one;            // backward hop across t = 0 -> Lt-1
    if constexpr (SHX) {
        // the x-neighbours (one of them has this site's own index) and the y-neighbours
        // are mostly the centres of lanes of the same wavefront
        Cx<R> C[RPT][12];
        R Cs[RPT];
        load_raw<SP, RPT>(C, Cs, a, act, r0, i, stride);
        Cx<R> H[RPT][2][3];
        lane_nbr<SP, RPT, 0, true, G5>(H, C, Cs, a, act, r0, i, xp, stride);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 0, true, 1, LL, -1, LNE>(acc, a, act, r0, xp, par, i, one, stride, H, ll);
        lane_nbr<SP, RPT, 0, false, G5>(H, C, Cs, a, act, r0, i, xm, stride);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 0, false, 1, LL, -1, LNE>(acc, a, act, r0, xm, opar, xm, one, stride, H, ll);
        lane_nbr<SP, RPT, 1, true, G5>(H, C, Cs, a, act, r0, i, yp, stride);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 1, true, 1, LL, -1, LNE>(acc, a, act, r0, yp, par, i, one, stride, H, ll);
        lane_nbr<SP, RPT, 1, false, G5>(H, C, Cs, a, act, r0, i, ym, stride);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 1, false, 1, LL, -1, LNE>(acc, a, act, r0, ym, opar, ym, one, stride, H, ll);
    } else {
        hop_dir<SP, GP, RPT, NE, G5, LNT, 0, true, 0, LL, -1, LNE>(acc, a, act, r0, xp, par, i, one, stride, nullptr, ll);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 0, false, 0, LL, -1, LNE>(acc, a, act, r0, xm, opar, xm, one, stride, nullptr, ll);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 1, true, 0, LL, -1, LNE>(acc, a, act, r0, yp, par, i, one, stride, nullptr, ll);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 1, false, 0, LL, -1, LNE>(acc, a, act, r0, ym, opar, ym, one, stride, nullptr, ll);
    }
    hop_dir<SP, GP, RPT, NE, G5, LNT, 2, true, 0, LL, -1, LNE>(acc, a, act, r0, zp, par, i, one, stride, nullptr, ll);
    hop_dir<SP, GP, RPT, NE, G5, LNT, 2, false, 0, LL, -1, LNE>(acc, a, act, r0, zm, opar, zm, one, stride, nullptr, ll);
    hop_dir<SP, GP, RPT, NE, G5, LNT, 3, true, 0, LL, -1, LNE>(acc, a, act, r0, tp, par, i, sgn_tf, stride, nullptr, ll);
    hop_dir<SP, GP, RPT, NE, G5, LNT, 3, false, 0, LL, -1, LNE>(acc, a, act, r0, tm, opar, tm, sgn_tb, stride, nullptr, ll);

#pragma unroll
    for (int r = 0; r < RPT; r++) {
        if (RPT > 1 && !act[r]) continue;
        Cx<R> yv[12], zv[12], wv[12];
        hop_finish<SP, CLV, 0>(a, i, valid, r0 + r, acc[r], yv, zv, wv, red[r], stride);
    }
}

// Block b (in XCD-contiguous order when xcd_remap) covers site tile b / ngroups and
// right-hand-side group b % ngroups: the groups that share a tile's links run next to
// each other on one XCD, so the links come from HBM once and from L2 after that.
// A tile is `blockDim` consecutive checkerboard indices, optionally permuted plane-wise
// (zblk); one lane processes one site.
// With wsplit, a tile is 64 sites and the waves of a block take successive RHS groups of
// it: the block's waves read the same links at the same time on one CU, so a link is
// requested from L2 once per block instead of once per group.  Each wave then reduces
// its own partial sums (no block barrier).
// Register budget: waves per SIMD the compiler must fit (FP64: 2, else 4 up to two RHS
// per lane, 3 beyond); without it the scheduler hoists the gathers of all eight
// directions and the single-RHS kernels spill.
template <int SP, int RPT>
struct HopOcc {
    static constexpr int value = SP == P64 ? 2 : (RPT <= 2 ? 4 : 3);
};

template <int SP, int GP, int RPT, int NE, bool G5, bool LNT, bool SHX, bool CLV, bool LL = false, int LNE = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HopOcc<SP, RPT>::value)))
hop_kernel(const HopArgs a, int xcd_remap, const VisitOrder vo, int wsplit) {
    const Geom &g = a.g;
    const int ngroups = a.nrhs / RPT;
    const int lb = xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const int nw = (int)blockDim.x >> 6;
    const int bpt = wsplit ? ngroups / nw : ngroups;  // blocks per tile
    const int tile = lb / bpt;
    int r0, l;
    if (wsplit) {
        r0 = __builtin_amdgcn_readfirstlane(((lb - tile * bpt) * nw + ((int)threadIdx.x >> 6)) * RPT);
        l = tile * 64 + ((int)threadIdx.x & 63);
    } else {
        r0 = (lb - tile * bpt) * RPT;
        l = tile * (int)blockDim.x + (int)threadIdx.x;
    }
    bool act[RPT];
    bool any = false;
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        act[r] = (r0 + r < a.nrhs) && (a.state == nullptr || (a.state[r0 + r].phase & a.run_mask));
        any |= act[r];
    }
    // uniform over the block (over the wave with wsplit); with the links in LDS every wave
    // takes part in loading them first
    if (!any && !LL) return;

    double red[RPT][3];
#pragma unroll
    for (int r = 0; r < RPT; r++) red[r][0] = red[r][1] = red[r][2] = 0.0;

    const bool valid = l < g.Vh;
    const int i = valid ? visit_order(l, g, vo) : g.Vh - 1;
    hop_site<SP, GP, RPT, NE, G5, LNT, SHX, CLV, LL, LNE>(a, i, valid, r0, act, red);
    if (LL && !any) return;

    const int nv = red_nvals(a.red);
    if (nv == 0) return;
    const int ntiles = (int)gridDim.x / bpt;
    const int ps = a.pstride ? a.pstride : ntiles;
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        if (!act[r]) continue;
        double *dst = a.partials + (size_t)(r0 + r) * nv * ps + tile;
        if (nv == 1) {
            double v[1] = {red[r][0]};
            if (wsplit) wave_reduce_to<1>(v, dst, ps);
            else block_reduce_to<1>(v, dst, ps);
        } else if (nv == 2) {
            double v[2] = {red[r][0], red[r][1]};
            if (wsplit) wave_reduce_to<2>(v, dst, ps);
            else block_reduce_to<2>(v, dst, ps);
        } else {
            double v[3] = {red[r][0], red[r][1], red[r][2]};
            if (wsplit) wave_reduce_to<3>(v, dst, ps);
            else block_reduce_to<3>(v, dst, ps);
        }
    }
}

// t-marching: the sites of a launch are cut into segments of `tile` consecutive positions
// of the (x, y, z) slices (a position p is the checkerboard index within a slice; the site
// of slice t is i = t * st + p), and a block marches one segment through nt t-slices of
// one parity of t: t = t0, t0 + 2, ..., t0 + 2 (nt - 1).  In the Dirac basis a t-hop reads
// one spin half of its neighbour, and the input at (t + 1, p) is the forward t-neighbour of
// output (t, p) and the backward t-neighbour of output (t + 2, p), the block's next step:
// it is loaded once, its forward half used at once and its projected backward half kept
// in registers for the next step.  The two blocks of a segment and 2 nt slices (t0 even
// and odd) load each input of those slices once between them, plus one half-slice of halo
// each; the plain kernel loads the two t-neighbour halves of every site separately, 2 Lz
// planes apart in memory and far beyond the L2 of an XCD.  Blocks are ordered t-chunk
// major, then segment, then the slice parity, so an XCD's contiguous range of blocks
// covers neighbouring segments (the z-neighbours) of the same slices.  Links come from
// global memory, or (LL, with the wave split) are staged in LDS per step for all waves.
// No clover epilogue.
// Register budget of the marching kernels: the loop keeps one projected half per RHS and
// the per-step plane bases beyond the plain kernel's (FP64: 2 waves per SIMD; FP32/FP16:
// 3 up to two RHS per lane, 2 beyond).
template <int SP, int RPT>
struct TmOcc {
    static constexpr int value = SP == P64 ? 2 : (RPT <= 2 ? 3 : 2);
};
template <int SP, int GP, int RPT, int NE, bool G5, bool LNT, bool SHX, bool LL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TmOcc<SP, RPT>::value)))
hop_kernel_tm(const HopArgs a, int xcd_remap, int nt, int wsplit) {
    using R = real_t<SP>;
    const Geom &g = a.g;
    const int stride = g.stride;
    const int par = a.par, opar = 1 - par;
    const int ngroups = a.nrhs / RPT;
    const int nw = (int)blockDim.x >> 6;
    const int bpt = wsplit ? ngroups / nw : ngroups;  // blocks per tile
    const int tile = wsplit ? 64 : (int)blockDim.x;
    const int nseg = (g.st + tile - 1) / tile;
    const int lb = xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tid = lb / bpt;  // tile: (t-chunk, segment, slice parity), the last fastest
    const int q = tid & 1, cs = tid >> 1;
    const int chunk = cs / nseg, seg = cs - chunk * nseg;
    int r0, pos;
    if (wsplit) {
        r0 = __builtin_amdgcn_readfirstlane(((lb - tid * bpt) * nw + ((int)threadIdx.x >> 6)) * RPT);
        pos = seg * 64 + ((int)threadIdx.x & 63);
    } else {
        r0 = (lb - tid * bpt) * RPT;
        pos = seg * tile + (int)threadIdx.x;
    }
    const bool valid = pos < g.st;
    const int p = valid ? pos : g.st - 1;  // ragged last segment: computed, not stored
    bool act[RPT];
    bool any = false;
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        act[r] = (r0 + r < a.nrhs) && (a.state == nullptr || (a.state[r0 + r].phase & a.run_mask));
        any |= act[r];
    }
    if (!any && !LL) return;  // uniform over the block (the wave with wsplit)

    const int Lt = g.L[3];
    const int t0 = chunk * 2 * nt + q;
    double red[RPT][3];
#pragma unroll
    for (int r = 0; r < RPT; r++) red[r][0] = red[r][1] = red[r][2] = 0.0;

    // the projected backward half of the input at (t0 - 1, p), for the first step
    Cx<R> pb[RPT][2][3];
    {
        Cx<R> v[RPT][12];
        R vs[RPT];
        load_raw<SP, RPT>(v, vs, a, act, r0, (t0 == 0 ? Lt - 1 : t0 - 1) * g.st + p, stride);
#pragma unroll
        for (int r = 0; r < RPT; r++) proj_in<SP, 3, false, G5>(v[r], vs[r], pb[r]);
    }
    const char *ll = nullptr;
    __shared__ __align__(16) char ll_buf[LL ? 8 * LinkElems<GP, NE>::N * 64 * LinkPack<GP>::EB : 16];
    if constexpr (LL) ll = ll_buf;

    for (int j = 0; j < nt; j++) {
        // the plane stride, opaque to the compiler on every step: the forty-odd plane base
        // addresses derived from it are then formed in scalar registers per step instead of
        // being hoisted out of the loop (which spills the scalar registers)
        int ls = stride;
        asm volatile("" : "+s"(ls));

        const int t = t0 + 2 * j;
        const int i = t * g.st + p;
        const SiteXY c = cb_coords(g, i, par);
        const SiteNbrs nb = site_nbrs(g, i, c);
        const int xp = nb.xp, xm = nb.xm, yp = nb.yp, ym = nb.ym, zp = nb.zp, zm = nb.zm;
        const int tp = (t == Lt - 1) ? p : i + g.st;  // = nb.tp, with t known here
        const int tm = (t == 0) ? (Lt - 1) * g.st + p : i - g.st;
        if constexpr (LL) {
            if (j > 0) __syncthreads();  // every wave has read the previous step's links
            const int lsite[8] = {i, xm, i, ym, i, zm, i, tm};
            stage_links<GP, NE>(ll_buf, a, par, lsite, ls);
        }
        if (!any) continue;  // (LL) this wave's RHS group has finished; it only helps staging

        Cx<R> acc[RPT][4][3];
#pragma unroll
        for (int r = 0; r < RPT; r++)
#pragma unroll
            for (int s_ = 0; s_ < 4; s_++)
#pragma unroll
                for (int k = 0; k < 3; k++) acc[r][s_][k] = {R(0), R(0)};
        const R one = R(1);
        if constexpr (SHX) {
            Cx<R> C[RPT][12];
            R Cs[RPT];
            load_raw<SP, RPT>(C, Cs, a, act, r0, i, ls);
            Cx<R> H[RPT][2][3];
            lane_nbr<SP, RPT, 0, true, G5>(H, C, Cs, a, act, r0, i, xp, ls);
            hop_dir<SP, GP, RPT, NE, G5, LNT, 0, true, 1, LL>(acc, a, act, r0, xp, par, i, one, ls, H, ll);
            lane_nbr<SP, RPT, 0, false, G5>(H, C, Cs, a, act, r0, i, xm, ls);
            hop_dir<SP, GP, RPT, NE, G5, LNT, 0, false, 1, LL>(acc, a, act, r0, xm, opar, xm, one, ls, H, ll);
            lane_nbr<SP, RPT, 1, true, G5>(H, C, Cs, a, act, r0, i, yp, ls);
            hop_dir<SP, GP, RPT, NE, G5, LNT, 1, true, 1, LL>(acc, a, act, r0, yp, par, i, one, ls, H, ll);
            lane_nbr<SP, RPT, 1, false, G5>(H, C, Cs, a, act, r0, i, ym, ls);
            hop_dir<SP, GP, RPT, NE, G5, LNT, 1, false, 1, LL>(acc, a, act, r0, ym, opar, ym, one, ls, H, ll);
        } else {
            hop_dir<SP, GP, RPT, NE, G5, LNT, 0, true, 0, LL>(acc, a, act, r0, xp, par, i, one, ls, nullptr, ll);
            hop_dir<SP, GP, RPT, NE, G5, LNT, 0, false, 0, LL>(acc, a, act, r0, xm, opar, xm, one, ls, nullptr, ll);
            hop_dir<SP, GP, RPT, NE, G5, LNT, 1, true, 0, LL>(acc, a, act, r0, yp, par, i, one, ls, nullptr, ll);
            hop_dir<SP, GP, RPT, NE, G5, LNT, 1, false, 0, LL>(acc, a, act, r0, ym, opar, ym, one, ls, nullptr, ll);
        }
        // backward t-hop from the half kept since the last step (its registers are free after it)
        const R sgn_tb = (NE == 6 && t == 0) ? -one : one;
        hop_dir<SP, GP, RPT, NE, G5, LNT, 3, false, 1, LL, 0>(acc, a, act, r0, tm, opar, tm, sgn_tb, ls, pb, ll);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 2, true, 0, LL, 0>(acc, a, act, r0, zp, par, i, one, ls, nullptr, ll);
        hop_dir<SP, GP, RPT, NE, G5, LNT, 2, false, 0, LL, 1>(acc, a, act, r0, zm, opar, zm, one, ls, nullptr, ll);
        {
            // the input at (t + 1, p): forward half now, backward half for the next step
            Cx<R> H[RPT][2][3];
            {
                Cx<R> v[RPT][12];
                R vs[RPT];
                load_raw<SP, RPT>(v, vs, a, act, r0, tp, ls);
#pragma unroll
                for (int r = 0; r < RPT; r++) {
                    proj_in<SP, 3, true, G5>(v[r], vs[r], H[r]);
                    proj_in<SP, 3, false, G5>(v[r], vs[r], pb[r]);
                }
            }
            const R sgn_tf = (NE == 6 && t == Lt - 1) ? -one : one;
            hop_dir<SP, GP, RPT, NE, G5, LNT, 3, true, 1, LL, 0>(acc, a, act, r0, tp, par, i, sgn_tf, ls, H, ll);
        }
#pragma unroll
        for (int r = 0; r < RPT; r++) {
            if (RPT > 1 && !act[r]) continue;
            Cx<R> yv[12], zv[12], wv[12];
            hop_finish<SP, false, 0>(a, i, valid, r0 + r, acc[r], yv, zv, wv, red[r], ls);
        }
    }
    if (!any) return;

    const int nv = red_nvals(a.red);
    if (nv == 0) return;
    const int ntiles = (int)gridDim.x / bpt;
    const int ps = a.pstride ? a.pstride : ntiles;
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        if (!act[r]) continue;
        double *dst = a.partials + (size_t)(r0 + r) * nv * ps + tid;
        if (nv == 1) {
            double v[1] = {red[r][0]};
            if (wsplit) wave_reduce_to<1>(v, dst, ps);
            else block_reduce_to<1>(v, dst, ps);
        } else if (nv == 2) {
            double v[2] = {red[r][0], red[r][1]};
            if (wsplit) wave_reduce_to<2>(v, dst, ps);
            else block_reduce_to<2>(v, dst, ps);
        } else {
            double v[3] = {red[r][0], red[r][1], red[r][2]};
            if (wsplit) wave_reduce_to<3>(v, dst, ps);
            else block_reduce_to<3>(v, dst, ps);
        }
    }
}

template <int SP, int GP, int NE, bool G5, bool LNT, bool SHX, bool LL>
static hipError_t launch_hop_tm(const HopArgs &a, const LaunchCfg &c, hipStream_t s) {
    const int ngroups = a.nrhs / c.rpt;
    const dim3 grid(hop_nblocks(a, c) * (c.wsplit ? ngroups / (c.block / 64) : ngroups)), block(c.block);
    switch (c.rpt) {
        case 1:
            hipLaunchKernelGGL((hop_kernel_tm<SP, GP, 1, NE, G5, LNT, SHX, LL>), grid, block, 0, s, a, c.xcd, c.tm,
                               c.wsplit);
            break;
        case 2:
            if constexpr (!SHX)
                hipLaunchKernelGGL((hop_kernel_tm<SP, GP, 2, NE, G5, LNT, false, LL>), grid, block, 0, s, a, c.xcd,
                                   c.tm, c.wsplit);
            else return hipErrorInvalidValue;
            break;
        case 3:
        case 4:
            if constexpr (SP != P64 && !SHX && !LL) {
                if (c.rpt == 3)
                    hipLaunchKernelGGL((hop_kernel_tm<SP, GP, 3, NE, G5, LNT, false, false>), grid, block, 0, s, a,
                                       c.xcd, c.tm, c.wsplit);
                else
                    hipLaunchKernelGGL((hop_kernel_tm<SP, GP, 4, NE, G5, LNT, false, false>), grid, block, 0, s, a,
                                       c.xcd, c.tm, c.wsplit);
            } else {
                return hipErrorInvalidValue;
            }
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Lattices too small to fill the GPU: with one wave per 64 sites most of it idles, and a
// wave's time is its chain of dependent gathers.  Here five waves share a tile of 64
// sites (one right-hand side per block): wave 1 + mu does the two hops along mu and leaves
// its sum in LDS, while wave 0 loads the epilogue's y; after the barrier wave 0
// adds the four sums in a fixed order (x, y, z, t) and finishes the sites.  Partial sums
// of the reductions: one per tile, from wave 0.
template <int SP, int GP, int NE, bool G5, bool LNT, bool CLV>
__global__ void __launch_bounds__(320) hop_kernel_ds(const HopArgs a, int xcd_remap) {
    using R = real_t<SP>;
    const Geom &g = a.g;
    const int stride = g.stride;
    const int lb = xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tile = lb / a.nrhs, rhs = lb - tile * a.nrhs;
    const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    if (a.state != nullptr && !(a.state[rhs].phase & a.run_mask)) return;  // uniform over the block
    const int l = tile * 64 + lane;
    const bool valid = l < g.Vh;
    const int i = valid ? l : g.Vh - 1;
    __shared__ R part[4][24][64];
    Cx<R> yv[12], zv[12], wd[12];
    if (wv > 0) {
        const bool act[1] = {true};
        Cx<R> acc[1][4][3];
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int k = 0; k < 3; k++) acc[0][s][k] = {R(0), R(0)};
        const int par = a.par, opar = 1 - par;
        const SiteXY c = cb_coords(g, i, par);
        const R one = R(1);
        // each wave forms only the pair of neighbours of its direction
        if (wv == 1) {
            const SiteNbrs nb = site_nbrs(g, i, c);
            hop_dir<SP, GP, 1, NE, G5, LNT, 0, true>(acc, a, act, rhs, nb.xp, par, i, one, stride);
            hop_dir<SP, GP, 1, NE, G5, LNT, 0, false>(acc, a, act, rhs, nb.xm, opar, nb.xm, one, stride);
        } else if (wv == 2) {
            const SiteNbrs nb = site_nbrs(g, i, c);
            hop_dir<SP, GP, 1, NE, G5, LNT, 1, true>(acc, a, act, rhs, nb.yp, par, i, one, stride);
            hop_dir<SP, GP, 1, NE, G5, LNT, 1, false>(acc, a, act, rhs, nb.ym, opar, nb.ym, one, stride);
        } else if (wv == 3) {
            const SiteNbrs nb = site_nbrs(g, i, c);
            hop_dir<SP, GP, 1, NE, G5, LNT, 2, true>(acc, a, act, rhs, nb.zp, par, i, one, stride);
            hop_dir<SP, GP, 1, NE, G5, LNT, 2, false>(acc, a, act, rhs, nb.zm, opar, nb.zm, one, stride);
        } else {
            const SiteNbrs nb = site_nbrs(g, i, c);
            const int tp = nb.tp, tm = nb.tm;
            const R sgn_tf = (NE == 6 && c.t == g.L[3] - 1) ? -one : one;
            const R sgn_tb = (NE == 6 && c.t == 0) ? -one : one;
            hop_dir<SP, GP, 1, NE, G5, LNT, 3, true>(acc, a, act, rhs, tp, par, i, sgn_tf, stride);
            hop_dir<SP, GP, 1, NE, G5, LNT, 3, false>(acc, a, act, rhs, tm, opar, tm, sgn_tb, stride);
        }
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                part[wv - 1][2 * (s * 3 + k)][lane] = acc[0][s][k].re;
                part[wv - 1][2 * (s * 3 + k) + 1][lane] = acc[0][s][k].im;
            }
    } else if (a.has_y) {  // z and w are loaded after the barrier (registers)
        load_site<SP, R, false>(yv, a.y, stride, rhs, i);
    }
    __syncthreads();
    if (wv != 0) return;
    Cx<R> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int e = 2 * (s * 3 + k);
            acc[s][k] = {((part[0][e][lane] + part[1][e][lane]) + part[2][e][lane]) + part[3][e][lane],
                         ((part[0][e + 1][lane] + part[1][e + 1][lane]) + part[2][e + 1][lane]) + part[3][e + 1][lane]};
        }
    double red[3] = {0.0, 0.0, 0.0};
    hop_finish<SP, CLV, 1, false>(a, i, valid, rhs, acc, yv, zv, wd, red, stride);
    const int nv = red_nvals(a.red);
    if (nv == 0) return;
    const int ntiles = (int)gridDim.x / a.nrhs;
    const int ps = a.pstride ? a.pstride : ntiles;
    double *dst = a.partials + (size_t)rhs * nv * ps + tile;
    if (nv == 1) {
        double v[1] = {red[0]};
        wave_reduce_to<1>(v, dst, ps);
    } else if (nv == 2) {
        double v[2] = {red[0], red[1]};
        wave_reduce_to<2>(v, dst, ps);
    } else {
        double v[3] = {red[0], red[1], red[2]};
        wave_reduce_to<3>(v, dst, ps);
    }
}

template <int SP, int GP, int NE, bool G5, bool LNT, bool CLV>
static hipError_t launch_hop_ds(const HopArgs &a, const LaunchCfg &c, hipStream_t s) {
    const dim3 grid(hop_nblocks(a, c) * a.nrhs), block(320);
    hipLaunchKernelGGL((hop_kernel_ds<SP, GP, NE, G5, LNT, CLV>), grid, block, 0, s, a, c.xcd);
    return hipGetLastError();
}

template <int SP, int GP, int NE, bool G5, bool LNT, bool SHX, bool CLV>
static hipError_t launch_hop_k(const HopArgs &a, const LaunchCfg &c, hipStream_t s) {
    const int ngroups = a.nrhs / c.rpt;
    dim3 grid(hop_nblocks(a, c) * (c.wsplit ? ngroups / (c.block / 64) : ngroups));
    dim3 block(c.block);
    const int remap = c.xcd;
    // Unused dynamic LDS caps the blocks resident per CU (160 KB of LDS per CU), so fewer
    // sites are in flight per XCD and their neighbour data stays in L2.
    const size_t lds = (size_t)c.lds_kb * 1024;
    const VisitOrder vo = make_visit_order(a.g, c.zblk);
    switch (c.rpt) {
        case 1: hipLaunchKernelGGL((hop_kernel<SP, GP, 1, NE, G5, LNT, SHX, CLV>), grid, block, lds, s, a, remap, vo, c.wsplit); break;
        case 2:
            if constexpr (!CLV && !SHX)
                hipLaunchKernelGGL((hop_kernel<SP, GP, 2, NE, G5, LNT, SHX, CLV>), grid, block, lds, s, a, remap, vo, c.wsplit);
            else return hipErrorInvalidValue;
            break;
        case 3:
            if constexpr (SP != P64 && !SHX && !CLV)
                hipLaunchKernelGGL((hop_kernel<SP, GP, 3, NE, G5, LNT, SHX, CLV>), grid, block, lds, s, a, remap, vo, c.wsplit);
            else return hipErrorInvalidValue;
            break;
        case 4:
            if constexpr (SP != P64 && !SHX && !CLV)
                hipLaunchKernelGGL((hop_kernel<SP, GP, 4, NE, G5, LNT, SHX, CLV>), grid, block, lds, s, a, remap, vo, c.wsplit);
            else return hipErrorInvalidValue;
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Wave split with the tile's links staged in LDS (one or two RHS per lane, no clover
// epilogue; links through L2 since several RHS groups read them).
template <int SP, int GP, int NE, bool G5, bool SHX>
static hipError_t launch_hop_ll(const HopArgs &a, const LaunchCfg &c, hipStream_t s) {
    const int ngroups = a.nrhs / c.rpt;
    const dim3 grid(hop_nblocks(a, c) * (ngroups / (c.block / 64))), block(c.block);
    const VisitOrder vo = make_visit_order(a.g, c.zblk);
    if (c.ldsl == 2) {  // two-row links rebuilt to full links while staging (FP32 / FP16 links)
        if constexpr (NE == 6 && GP != P64) {
            if (c.rpt == 1)
                hipLaunchKernelGGL((hop_kernel<SP, GP, 1, NE, G5, false, SHX, false, true, 9>), grid, block, 0, s, a,
                                   c.xcd, vo, 1);
            else if (c.rpt == 2 && !SHX)
                hipLaunchKernelGGL((hop_kernel<SP, GP, 2, NE, G5, false, false, false, true, 9>), grid, block, 0, s, a,
                                   c.xcd, vo, 1);
            else
                return hipErrorInvalidValue;
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (c.rpt == 1)
        hipLaunchKernelGGL((hop_kernel<SP, GP, 1, NE, G5, false, SHX, false, true>), grid, block, 0, s, a, c.xcd, vo, 1);
    else if (c.rpt == 2 && !SHX)
        hipLaunchKernelGGL((hop_kernel<SP, GP, 2, NE, G5, false, false, false, true>), grid, block, 0, s, a, c.xcd, vo, 1);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Links are loaded non-temporally when one group covers every right-hand side (each link
// is read once per launch) and through L2 otherwise.
template <int SP, int GP, int NE, bool G5>
static hipError_t launch_hop_t(const HopArgs &a, const LaunchCfg &c, hipStream_t s) {
    const bool lnt = a.nrhs == c.rpt;
    if (c.tm) {
        if (c.ldsl == 2) return hipErrorInvalidValue;
        if (c.ldsl) {
            if constexpr (GP == P64 && NE == 9) return hipErrorInvalidValue;
            else return c.shx ? launch_hop_tm<SP, GP, NE, G5, false, true, true>(a, c, s)
                              : launch_hop_tm<SP, GP, NE, G5, false, false, true>(a, c, s);
        }
        if (c.shx)
            return lnt ? launch_hop_tm<SP, GP, NE, G5, true, true, false>(a, c, s)
                       : launch_hop_tm<SP, GP, NE, G5, false, true, false>(a, c, s);
        return lnt ? launch_hop_tm<SP, GP, NE, G5, true, false, false>(a, c, s)
                   : launch_hop_tm<SP, GP, NE, G5, false, false, false>(a, c, s);
    }
    if (c.ldsl) {
        if constexpr (GP == P64 && NE == 9) return hipErrorInvalidValue;  // 72 KB of links per tile
        else return c.shx ? launch_hop_ll<SP, GP, NE, G5, true>(a, c, s) : launch_hop_ll<SP, GP, NE, G5, false>(a, c, s);
    }
    if (c.dsplit) {
        if (a.clov_mode != CLV_NONE)
            return lnt ? launch_hop_ds<SP, GP, NE, G5, true, true>(a, c, s) : launch_hop_ds<SP, GP, NE, G5, false, true>(a, c, s);
        return lnt ? launch_hop_ds<SP, GP, NE, G5, true, false>(a, c, s) : launch_hop_ds<SP, GP, NE, G5, false, false>(a, c, s);
    }
    if (a.clov_mode != CLV_NONE)  // clover epilogue: its own instantiations (one RHS per lane)
        return lnt ? launch_hop_k<SP, GP, NE, G5, true, false, true>(a, c, s)
                   : launch_hop_k<SP, GP, NE, G5, false, false, true>(a, c, s);
    if (c.shx)
        return lnt ? launch_hop_k<SP, GP, NE, G5, true, true, false>(a, c, s)
                   : launch_hop_k<SP, GP, NE, G5, false, true, false>(a, c, s);
    return lnt ? launch_hop_k<SP, GP, NE, G5, true, false, false>(a, c, s)
               : launch_hop_k<SP, GP, NE, G5, false, false, false>(a, c, s);
}

template <int SP, int GP>
hipError_t launch_hop_r(const HopArgs &a, const LaunchCfg &c, hipStream_t s) {
    if (a.g5in) return a.recon == 12 ? launch_hop_t<SP, GP, 6, true>(a, c, s) : launch_hop_t<SP, GP, 9, true>(a, c, s);
    return a.recon == 12 ? launch_hop_t<SP, GP, 6, false>(a, c, s) : launch_hop_t<SP, GP, 9, false>(a, c, s);
}

}  // namespace wl
