// Block BiCGStab kernels: s right-hand sides of one matrix share one Krylov space
// (Guennouni, Jbilou and Sadok, "A block version of BiCGSTAB for linear systems with
// multiple right-hand sides", 2003).  The scalars alpha and beta of BiCGStab become
// s x s matrices from small solves against the shadow block R~ = R_0; omega stays one
// scalar of Frobenius inner products:
//     V = A P;  alpha = (R~^H V)^-1 R~^H R;  S = R - V alpha;  T = A S;
//     omega = <T,S>_F / <T,T>_F;  X += P alpha + omega S;  R = S - omega T;
//     beta = -(R~^H V)^-1 R~^H T;  P = R + (P - omega V) beta.
// A = M_ee runs through the parity hops; this file holds the rest, in FP64:
//   * gram: the s x s (or two) products R~^H Y, a tall-skinny contraction over all sites
//     and components, with per-block partials and a fixed-order reduction;
//   * solve: one workgroup factors R~^H V (partial pivoting, kept for beta), solves for
//     alpha and beta, forms omega, and runs the convergence check of the whole block;
//   * update: the three block combinations, one site-component element per thread with
//     all s right-hand sides in registers (s^2 complex multiply-adds against LDS).
// Every kernel reads the block's phase first (all s per-RHS states carry it), so
// iterations enqueued ahead of the host's poll turn into no-ops once the block is done.
#include <algorithm>

#include "common.h"
#include "device.h"

namespace wl {

using dcx = Cx<double>;

__device__ __forceinline__ bool block_running(const BlockArgs &a) { return a.state[0].phase == PH_RUN; }

// plane address shared by the whole wavefront (kept in scalar registers)
typedef const WL_GLOBAL dvec2 *gdvec2p;
__device__ __forceinline__ gdvec2p fplane(const void *base, int plane, int stride) {
    return reinterpret_cast<gdvec2p>(splane(base, plane, stride));
}
// plane address that differs between the lanes of a wavefront (no scalar promotion)
__device__ __forceinline__ gdvec2p fplane_lane(const void *base, int plane, int stride) {
    return gptr(reinterpret_cast<const dvec2 *>(static_cast<const char *>(base) + (size_t)plane * stride * 16u));
}
template <bool NT = false>
__device__ __forceinline__ dcx ldc(gdvec2p p, int i) {
    const dvec2 v = NT ? __builtin_nontemporal_load(p + i) : p[i];
    return {v.x, v.y};
}
template <bool NT = false>
__device__ __forceinline__ void stc(gdvec2p p, int i, dcx v) {
    dvec2 w;
    w.x = v.re;
    w.y = v.im;
    if constexpr (NT) __builtin_nontemporal_store(w, const_cast<WL_GLOBAL dvec2 *>(p) + i);
    else const_cast<WL_GLOBAL dvec2 *>(p)[i] = w;
}

// ---------------------------------------------------------------------------------
// Gram products G_p[i][j] = sum over sites and components of conj(A_i) B_p,j.
// Register tiles of 4 rows x 4 columns: the wave (rg, cg) of a block owns rows
// 4rg..4rg+3 and columns 4cg..4cg+3, its 64 lanes 64 consecutive sites of one component
// plane, so every load of a wave is one contiguous 1 KB run.  A lane loads 4 elements of
// A and 4 of B per tile and does 16 complex multiply-adds with them; the ceil(s/4)^2 waves
// of a block share each A and B run through L1 (each is loaded by ceil(s/4) waves).  With
// two operands B_0, B_1, blockIdx.y picks one (a block holding both would need more than
// the registers of 9 waves).  At the end each wave sums its 64 lanes and writes one
// partial per value.
constexpr int kGramSites = 64;

template <int NW>
__global__ void __launch_bounds__(64 * NW) block_gram_kernel(const BlockArgs a) {
    if (!block_running(a)) return;
    const int s = a.s, Vh = a.g.Vh, stride = a.g.stride;
    const int p = blockIdx.y;
    const void *bdata = p == 0 ? a.b.data : a.c.data;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ng = (s + 3) >> 2;
    const int rg = w / ng, cg = w - (w / ng) * ng;
    const int tps = (Vh + kGramSites - 1) / kGramSites;
    const int ntiles = 12 * tps;
    dcx acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = {0.0, 0.0};
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int c = tile / tps;
        const int site = (tile - c * tps) * kGramSites + lane;
        const bool ok = site < Vh;
        const int si = ok ? site : Vh - 1;
        dcx av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int row = 4 * rg + i < s ? 4 * rg + i : s - 1;
            av[i] = ldc(fplane(a.a.data, row * 12 + c, stride), si);
            if (!ok) av[i] = {0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int col = 4 * cg + j < s ? 4 * cg + j : s - 1;
            bv[j] = ldc(fplane(bdata, col * 12 + c, stride), si);
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[i][j] = cfma_conj(acc[i][j], av[i], bv[j]);
    }
    // sum the 64 lanes (fixed butterfly order) and write the wave's entries
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                acc[i][j].re += __shfl_xor(acc[i][j].re, off, 64);
                acc[i][j].im += __shfl_xor(acc[i][j].im, off, 64);
            }
        }
    if (lane == 0) {
        const size_t nb = a.nblk;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int row = 4 * rg + i, col = 4 * cg + j;
                if (row < s && col < s) {
                    const size_t v = ((size_t)(p * s + row) * s + col) * 2;
                    a.partials[v * nb + blockIdx.x] = acc[i][j].re;
                    a.partials[(v + 1) * nb + blockIdx.x] = acc[i][j].im;
                }
            }
    }
}

// One block per value: its row of partials summed in a fixed order.
__global__ void __launch_bounds__(256) block_gram_reduce_kernel(const BlockArgs a) {
    if (!block_running(a)) return;
    const double *p = a.partials + (size_t)blockIdx.x * a.nblk;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int j = threadIdx.x;
    for (; j + 3 * (int)blockDim.x < a.nblk; j += 4 * blockDim.x) {
#pragma unroll
        for (int u = 0; u < 4; u++) acc[u] += p[j + u * blockDim.x];
    }
    for (int u = 0; u < 4; u++)
        if (j + u * (int)blockDim.x < a.nblk) acc[u] += p[j + u * blockDim.x];
    double v[1] = {(acc[0] + acc[1]) + (acc[2] + acc[3])};
    block_reduce_to<1>(v, &a.bs->gram[blockIdx.x], 1);
}

constexpr int kGramBlocks = 512;

hipError_t launch_block_gram(BlockArgs a, int np, hipStream_t s) {
    if (a.s < 1 || a.s > kMaxBlock || (np != 1 && np != 2)) return hipErrorInvalidValue;
    const int ntiles = 12 * ((a.g.Vh + kGramSites - 1) / kGramSites);
    a.nblk = std::min(ntiles, kGramBlocks);
    const int ng = (a.s + 3) / 4;
    const dim3 grid(a.nblk, np), block(64 * ng * ng);
    switch (ng) {
        case 1: hipLaunchKernelGGL(block_gram_kernel<1>, grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL(block_gram_kernel<4>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(block_gram_kernel<9>, grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL(block_gram_kernel<16>, grid, block, 0, s, a); break;
    }
    hipLaunchKernelGGL(block_gram_reduce_kernel, dim3(np * a.s * a.s * 2), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Small dense algebra in one workgroup (s <= 16: one thread per matrix entry).
__device__ __forceinline__ dcx cdiv(dcx x, dcx d) {
    const double n = d.re * d.re + d.im * d.im;
    return {(x.re * d.re + x.im * d.im) / n, (x.im * d.re - x.re * d.im) / n};
}
__device__ __forceinline__ double cabs2(dcx v) { return v.re * v.re + v.im * v.im; }
__device__ __forceinline__ bool cfinite(dcx v) { return isfinite(v.re) && isfinite(v.im); }

__device__ __forceinline__ dcx gram_at(const BlockState *bs, int p, int i, int j, int s) {
    const int v = ((p * s + i) * s + j) * 2;
    return {bs->gram[v], bs->gram[v + 1]};
}

// X <- M^-1 X for the factors of P G = L U held in M (unit L below the diagonal, U on and
// above it; rows exchanged as recorded in piv, full rows, so L is the final one): every
// exchange is applied first, then L and U are solved.  Thread t owns column t of X.
__device__ void lu_solve_lds(dcx (*M)[kMaxBlock], const int *piv, dcx (*X)[kMaxBlock], int s) {
    const int t = threadIdx.x;
    if (t < s) {
        for (int k = 0; k < s; k++) {
            const int p = piv[k];
            if (p != k) {
                const dcx tmp = X[k][t];
                X[k][t] = X[p][t];
                X[p][t] = tmp;
            }
        }
        for (int k = 0; k < s; k++) {
            const dcx xk = X[k][t];
            for (int i = k + 1; i < s; i++) {
                const dcx l = M[i][k];
                X[i][t] = {X[i][t].re - (l.re * xk.re - l.im * xk.im), X[i][t].im - (l.re * xk.im + l.im * xk.re)};
            }
        }
        for (int k = s - 1; k >= 0; k--) {
            dcx x = X[k][t];
            for (int m = k + 1; m < s; m++) {
                const dcx u = M[k][m], xm = X[m][t];
                x = {x.re - (u.re * xm.re - u.im * xm.im), x.im - (u.re * xm.im + u.im * xm.re)};
            }
            X[k][t] = cdiv(x, M[k][k]);
        }
    }
    __syncthreads();
}

__device__ void block_fail(const BlockArgs &a, int code) {
    for (int j = 0; j < a.s; j++) {
        a.state[j].phase = PH_FAIL;
        a.state[j].fail = code;
    }
}

template <int OP>
__global__ void __launch_bounds__(256) block_solve_kernel(const BlockArgs a) {
    const int s = a.s, t = threadIdx.x;
    BlockState *bs = a.bs;
    __shared__ dcx M[kMaxBlock][kMaxBlock];
    __shared__ dcx X[kMaxBlock][kMaxBlock];
    __shared__ int piv[kMaxBlock];
    __shared__ int flag;
    __shared__ double red[kMaxBlock];
    if constexpr (OP == BS_INIT) {
        // FIN_BICG_INIT left a per-RHS phase; the block runs while any column runs
        if (t == 0) {
            int any_fail = 0, all_done = 1;
            for (int j = 0; j < s; j++) {
                any_fail |= a.state[j].phase == PH_FAIL;
                all_done &= a.state[j].phase == PH_DONE;
            }
            for (int j = 0; j < s; j++) {
                a.state[j].iter = 0;
                if (any_fail) {
                    a.state[j].phase = PH_FAIL;
                    a.state[j].fail = FAIL_NONFINITE;
                } else {
                    a.state[j].phase = all_done ? PH_DONE : PH_RUN;
                }
            }
        }
        return;
    } else if constexpr (OP == BS_ALPHA) {
        if (!block_running(a)) return;
        if (t < s * s) {
            const int i = t / s, j = t - (t / s) * s;
            M[i][j] = gram_at(bs, 0, i, j, s);
            X[i][j] = gram_at(bs, 1, i, j, s);
        }
        __syncthreads();
        if (t == 0) {  // scale of the matrix for the pivot test; finiteness of both
            double mx = 0.0;
            int bad = 0;
            for (int i = 0; i < s; i++)
                for (int j = 0; j < s; j++) {
                    mx = fmax(mx, cabs2(M[i][j]));
                    bad |= !cfinite(M[i][j]) || !cfinite(X[i][j]);
                }
            red[0] = mx;
            flag = bad ? FAIL_NONFINITE : FAIL_NONE;
        }
        __syncthreads();
        // LU with partial pivoting (largest modulus), full rows exchanged
        for (int k = 0; k < s && flag == FAIL_NONE; k++) {
            if (t == 0) {
                int p = k;
                double best = cabs2(M[k][k]);
                for (int i = k + 1; i < s; i++) {
                    const double v = cabs2(M[i][k]);
                    if (v > best) { best = v; p = i; }
                }
                piv[k] = p;
                if (!(best > 1e-26 * red[0])) flag = FAIL_BREAKDOWN;  // |pivot| <= 1e-13 max |G|
            }
            __syncthreads();
            if (flag != FAIL_NONE) break;
            const int p = piv[k];
            if (t < s && p != k) {
                const dcx tm = M[k][t];
                M[k][t] = M[p][t];
                M[p][t] = tm;
            }
            __syncthreads();
            if (t < s && t > k) M[t][k] = cdiv(M[t][k], M[k][k]);  // multipliers
            __syncthreads();
            if (t < s * s) {
                const int i = t / s, j = t - (t / s) * s;
                if (i > k && j > k) {
                    const dcx l = M[i][k], u = M[k][j];
                    M[i][j] = {M[i][j].re - (l.re * u.re - l.im * u.im), M[i][j].im - (l.re * u.im + l.im * u.re)};
                }
            }
            __syncthreads();
        }
        if (flag != FAIL_NONE) {
            if (t == 0) block_fail(a, flag);
            return;
        }
        lu_solve_lds(M, piv, X, s);
        if (t < s * s) {
            const int i = t / s, j = t - (t / s) * s;
            const int v = (i * kMaxBlock + j) * 2;
            bs->lu[v] = M[i][j].re;
            bs->lu[v + 1] = M[i][j].im;
            bs->alpha[v] = X[i][j].re;
            bs->alpha[v + 1] = X[i][j].im;
        }
        if (t < s) bs->piv[t] = piv[t];
    } else if constexpr (OP == BS_BETA) {
        if (!block_running(a)) return;
        if (t == 0) {
            double tr = 0.0, ti = 0.0, tt = 0.0;
            for (int j = 0; j < s; j++) {
                tr += a.state[j].omega_re;
                ti += a.state[j].omega_im;
                tt += a.state[j].aux;
            }
            int bad = !isfinite(tr) || !isfinite(ti) || !isfinite(tt);
            for (int i = 0; i < s * s && !bad; i++) bad |= !cfinite(gram_at(bs, 0, i / s, i % s, s));
            flag = bad ? FAIL_NONFINITE : FAIL_NONE;
            bs->omega[0] = tt > 0.0 ? tr / tt : 0.0;
            bs->omega[1] = tt > 0.0 ? ti / tt : 0.0;
        }
        if (t < s * s) {
            const int i = t / s, j = t - (t / s) * s;
            const int v = (i * kMaxBlock + j) * 2;
            M[i][j] = {bs->lu[v], bs->lu[v + 1]};
            const dcx g = gram_at(bs, 0, i, j, s);
            X[i][j] = {-g.re, -g.im};
        }
        if (t < s) piv[t] = bs->piv[t];
        __syncthreads();
        if (flag != FAIL_NONE) {
            if (t == 0) block_fail(a, flag);
            return;
        }
        lu_solve_lds(M, piv, X, s);
        if (t < s * s) {
            const int i = t / s, j = t - (t / s) * s;
            const int v = (i * kMaxBlock + j) * 2;
            bs->beta[v] = X[i][j].re;
            bs->beta[v + 1] = X[i][j].im;
        }
    } else if constexpr (OP == BS_CHECK) {
        if (block_running(a)) {
            // |R_j|^2: wave w sums rows j = w, w + 4, ... of the update's partials
            const int lane = t & 63, w = t >> 6;
            for (int j = w; j < s; j += 4) {
                const double *p = a.partials + (size_t)j * a.nblk;
                double acc = 0.0;
                for (int k = lane; k < a.nblk; k += 64) acc += p[k];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
                if (lane == 0) red[j] = acc;
            }
            __syncthreads();
            if (t == 0) {
                int bad = 0, all = 1;
                for (int j = 0; j < s; j++) {
                    bad |= !isfinite(red[j]);
                    all &= red[j] <= a.state[j].stop2;
                }
                for (int j = 0; j < s; j++) {
                    RhsState *st = &a.state[j];
                    st->r2 = red[j];
                    st->iter += 1;
                    if (bad) {
                        st->phase = PH_FAIL;
                        st->fail = FAIL_NONFINITE;
                    } else if (all) {
                        st->phase = PH_DONE;
                    }
                }
            }
        }
        __syncthreads();
        if (a.mirror && t < s) a.mirror[t] = a.state[t];
    }
}

constexpr int kUpdBlock = 256;
constexpr int kUpdMaxBlocks = 2048;  // the update with a reduction loops over tiles
static int xr_nblocks(const Geom &g) { return std::min(12 * ((g.Vh + kUpdBlock - 1) / kUpdBlock), kUpdMaxBlocks); }

hipError_t launch_block_solve(int op, BlockArgs a, hipStream_t s) {
    if (a.s < 1 || a.s > kMaxBlock) return hipErrorInvalidValue;
    a.nblk = xr_nblocks(a.g);  // the check sums the partials the X/R update left
    switch (op) {
        case BS_INIT: hipLaunchKernelGGL(block_solve_kernel<BS_INIT>, dim3(1), dim3(64), 0, s, a); break;
        case BS_ALPHA: hipLaunchKernelGGL(block_solve_kernel<BS_ALPHA>, dim3(1), dim3(256), 0, s, a); break;
        case BS_BETA: hipLaunchKernelGGL(block_solve_kernel<BS_BETA>, dim3(1), dim3(256), 0, s, a); break;
        case BS_CHECK: hipLaunchKernelGGL(block_solve_kernel<BS_CHECK>, dim3(1), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Block combinations.  A thread takes one 16-byte element (one component of one site)
// of every right-hand side: it loads the s elements of the operand that is multiplied by
// the s x s matrix (staged in LDS and read as broadcasts), then produces the s outputs.
template <int OP, bool NT>
__global__ void __launch_bounds__(kUpdBlock) block_update_kernel(const BlockArgs a) {
    if (!block_running(a)) return;
    const int s = a.s, Vh = a.g.Vh, stride = a.g.stride;
    __shared__ dcx C[kMaxBlock * kMaxBlock];
    const double *src = OP == BU_P ? a.bs->beta : a.bs->alpha;
    for (int k = threadIdx.x; k < kMaxBlock * kMaxBlock; k += blockDim.x) C[k] = {src[2 * k], src[2 * k + 1]};
    const dcx omega = {a.bs->omega[0], a.bs->omega[1]};
    __syncthreads();
    const int tps = (Vh + kUpdBlock - 1) / kUpdBlock;
    const int ntiles = 12 * tps;
    double r2[kMaxBlock];
#pragma unroll
    for (int j = 0; j < kMaxBlock; j++) r2[j] = 0.0;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // C is read from LDS in every tile: without this compiler fence the whole s x s
        // matrix (up to 256 complex doubles) is hoisted out of the loop into registers and
        // spilled, since stores through global pointers cannot touch LDS
        __asm__ volatile("" ::: "memory");
        const int c = tile / tps;
        const int site = (tile - c * tps) * kUpdBlock + threadIdx.x;
        if (site >= Vh) continue;
        dcx m[kMaxBlock];  // the operand multiplied by C
#pragma unroll
        for (int i = 0; i < kMaxBlock; i++) {
            if (i < s) {
                if constexpr (OP == BU_S) {
                    m[i] = ldc<NT>(fplane(a.c.data, i * 12 + c, stride), site);          // V_i
                } else if constexpr (OP == BU_XR) {
                    m[i] = ldc<NT>(fplane(a.a.data, i * 12 + c, stride), site);          // P_i
                } else {
                    const dcx p = ldc<NT>(fplane(a.a.data, i * 12 + c, stride), site);   // P_i - omega V_i
                    const dcx v = ldc<NT>(fplane(a.c.data, i * 12 + c, stride), site);
                    m[i] = csub(p, cmul(omega, v));
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kMaxBlock; j++) {
            if (j < s) {
                dcx acc = {0.0, 0.0};
#pragma unroll
                for (int i = 0; i < kMaxBlock; i++)
                    if (i < s) acc = cfma(acc, m[i], C[i * kMaxBlock + j]);
                if constexpr (OP == BU_S) {
                    const dcx r = ldc<NT>(fplane(a.b.data, j * 12 + c, stride), site);
                    stc<NT>(fplane(a.a.data, j * 12 + c, stride), site, csub(r, acc));
                } else if constexpr (OP == BU_XR) {
                    const dcx sj = ldc<NT>(fplane(a.b.data, j * 12 + c, stride), site);
                    const dcx tj = ldc<NT>(fplane(a.d.data, j * 12 + c, stride), site);
                    gdvec2p xp = fplane(a.x.data, j * 12 + c, stride);
                    const dcx x = ldc<NT>(xp, site);
                    stc<NT>(xp, site, cadd(x, cadd(acc, cmul(omega, sj))));
                    const dcx r = csub(sj, cmul(omega, tj));
                    stc<NT>(fplane(a.c.data, j * 12 + c, stride), site, r);
                    r2[j] += cabs2(r);
                } else {
                    const dcx r = ldc<NT>(fplane(a.b.data, j * 12 + c, stride), site);
                    stc<NT>(fplane(a.a.data, j * 12 + c, stride), site, cadd(r, acc));
                }
            }
        }
    }
    if constexpr (OP == BU_XR) block_reduce_to<kMaxBlock>(r2, a.partials + blockIdx.x, a.nblk);
}

hipError_t launch_block_update(int op, BlockArgs a, hipStream_t s) {
    if (a.s < 1 || a.s > kMaxBlock) return hipErrorInvalidValue;
    const int ntiles = 12 * ((a.g.Vh + kUpdBlock - 1) / kUpdBlock);
    // block vectors beyond 32 MB stream through the caches: non-temporal loads and stores
    const bool nt = (size_t)a.s * spinor_field_bytes(P64, a.g) > ((size_t)32 << 20);
    switch (op) {
        case BU_S:
            a.nblk = ntiles;
            if (nt) hipLaunchKernelGGL((block_update_kernel<BU_S, true>), dim3(ntiles), dim3(kUpdBlock), 0, s, a);
            else hipLaunchKernelGGL((block_update_kernel<BU_S, false>), dim3(ntiles), dim3(kUpdBlock), 0, s, a);
            break;
        case BU_XR:
            a.nblk = xr_nblocks(a.g);
            if (nt) hipLaunchKernelGGL((block_update_kernel<BU_XR, true>), dim3(a.nblk), dim3(kUpdBlock), 0, s, a);
            else hipLaunchKernelGGL((block_update_kernel<BU_XR, false>), dim3(a.nblk), dim3(kUpdBlock), 0, s, a);
            break;
        case BU_P:
            a.nblk = ntiles;
            if (nt) hipLaunchKernelGGL((block_update_kernel<BU_P, true>), dim3(ntiles), dim3(kUpdBlock), 0, s, a);
            else hipLaunchKernelGGL((block_update_kernel<BU_P, false>), dim3(ntiles), dim3(kUpdBlock), 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t block_partials_doubles(const Geom &g) {
    const size_t gram = (size_t)2 * kMaxBlock * kMaxBlock * 2 * kGramBlocks;
    const size_t upd = (size_t)kMaxBlock * kUpdMaxBlocks;
    (void)g;
    return std::max(gram, upd);
}

}  // namespace wl
