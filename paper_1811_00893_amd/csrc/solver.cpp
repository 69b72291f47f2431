// Even-odd Krylov solvers (BiCGStab, CGLS), FP64 defect correction, and the Dslash call.
// See solver.h for the scheme.
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <sstream>

namespace wl {

void FieldBuf::make(int prec, const Geom &g, int nrhs) {
    const size_t data = (size_t)nrhs * 12 * spinor_plane_bytes(prec, g);
    const size_t scl = prec == P16 ? (size_t)nrhs * g.stride * sizeof(float) : 0;
    buf.alloc(data + scl);
    f.data = buf.get();
    f.scale = prec == P16 ? reinterpret_cast<float *>(static_cast<char *>(buf.get()) + data) : nullptr;
    f.prec = prec;
}

void FieldBuf::place(int prec, const Geom &g, int nrhs, Arena &A) {
    const size_t data = (size_t)nrhs * 12 * spinor_plane_bytes(prec, g);
    const size_t scl = prec == P16 ? (size_t)nrhs * g.stride * sizeof(float) : 0;
    char *p = static_cast<char *>(A.take(data + scl));
    f.data = p;
    f.scale = prec == P16 && p ? reinterpret_cast<float *>(p + data) : nullptr;
    f.prec = prec;
}

static inline int inner_prec(int precision) {
    switch (precision) {
        case WILSON_FP64: return P64;
        case WILSON_FP32: return P32;
        default: return P16;
    }
}
static inline int inner_gauge_prec(int precision) {
    switch (precision) {
        case WILSON_FP64: return P64;
        case WILSON_FP32: return P32;
        case WILSON_FP16: return P16;
        default: return P32;  // WILSON_FP16_L32
    }
}

constexpr int kRing = kStateRing;  // host-mapped state mirrors in flight
// Iteration chunks captured as HIP graphs: lattices up to this many sites per parity (where
// the kernels are short and the gaps between launches a large part of an iteration), this
// many iterations per graph.
constexpr int kGraphMaxVh = 1 << 16;
constexpr int kGraphChunk = 4;
// Graph replay of iteration chunks is opt-in (WILSON_GRAPHS=1, read per solve): on ROCm 7.2
// a replayed chunk took longer than the same kernels launched one by one (8^4 FP64 solves
// 1.30 ms against 1.26 ms), since the host already runs ahead of the device and a graph
// does not shorten the gaps between dependent kernels on the device.
static bool graphs_enabled() {
    const char *e = std::getenv("WILSON_GRAPHS");
    return e && std::strcmp(e, "1") == 0;
}
constexpr int kAllPhases = PH_IDLE | PH_RUN | PH_SCONV | PH_DONE | PH_FAIL;
// The BiCGStab iteration lets its s and x/r vector kernels run the finalize of the hop
// before them (alpha, omega) when the hop's partial rows are short (small lattices, where
// every launch is short and the gaps between dependent launches dominate): two launches
// fewer per iteration, the same sums in the same order.  WILSON_FUSE_FIN=0 turns it off.
static bool prefin_enabled() {
    const char *e = std::getenv("WILSON_FUSE_FIN");
    return !(e && std::strcmp(e, "0") == 0);
}

size_t EoMem::carve(char *base, const Geom &g, int n, int precision, int method) {
    const int P = inner_prec(precision), PX = P == P16 ? P32 : P;
    const bool mixed = precision != WILSON_FP64;
    Arena A;
    A.base = base;
    for (FieldBuf *f : {&b_e, &b_o, &x_e, &x_o, &bp}) f->place(P64, g, n, A);
    if (mixed) {
        r64.place(P64, g, n, A);
        tmp64.place(P64, g, n, A);
        rf.place(P, g, n, A);
        xin.place(PX, g, n, A);
    }
    for (FieldBuf *f : {&r, &rh, &p, &v, &s, &t, &tmp}) f->place(P, g, n, A);
    size_t npart = partials_doubles(g, n);
    if (method == WILSON_SOLVER_BLOCK_BICGSTAB_EO) {
        npart = std::max(npart, block_partials_doubles(g));
        bstate = static_cast<BlockState *>(A.take(sizeof(BlockState)));
    }
    partials = static_cast<double *>(A.take(npart * sizeof(double)));
    partials2 = static_cast<double *>(A.take(partials_doubles(g, n) * sizeof(double)));
    st_in = static_cast<RhsState *>(A.take(sizeof(RhsState) * n));
    st_out = static_cast<RhsState *>(A.take(sizeof(RhsState) * n));
    st_alt = static_cast<RhsState *>(A.take(sizeof(RhsState) * n));
    bytes = (A.used + 255) & ~size_t(255);
    return bytes;
}

// Fields, states and primitive operations of one even-odd problem with nrhs RHS.
// Device memory: one region holding every buffer (EoMem), either allocated here or the
// caller's (a workspace, or the static scratch array of the no-allocation solve).  Host
// resources (pinned state mirrors, ring events): owned, or lent by the context.
class EoCore : public EoMem {
   public:
    wilson_ctx *ctx;
    const wilson_gauge *G;
    Geom g;
    int nrhs;
    int P, PX, GP;  // inner spinor, inner solution and inner link precisions
    bool mixed;
    int method;
    std::vector<double> kappa;
    // RHS range [k0, k0 + nk) that primitive launches act on (the batch engine narrows it
    // to one slot for per-slot bookkeeping; solves use the full range).
    int k0 = 0, nk = 0;

    DevBuf own;                             // the region, when the library allocates it
    std::unique_ptr<SolveHostRes> own_host; // host resources, when not lent
    SolveHostRes *host = nullptr;
    const hipEvent_t *ring_ev = nullptr;
    // captured iteration chunks: one executable graph per solution field, gauge field
    // addresses, RHS range, kappa values and mirror slot (the kernels' arguments), with the
    // bookkeeping of one replay
    bool graphs = false;  // set per call
    bool prefin = false;  // vector kernels may run the finalize before them (set per call)
    // device addresses a captured chunk reads from the gauge field (links of every
    // precision, clover blocks) and its link storage: a cached workspace may be bound to
    // another field, or to a field loaded again at the same host address
    struct GaugeSig {
        const void *p[7];
        int recon;
        bool operator==(const GaugeSig &o) const {
            for (int k = 0; k < 7; k++)
                if (p[k] != o.p[k]) return false;
            return recon == o.recon;
        }
    };
    GaugeSig gauge_sig() const {
        return {{G->links(P64), G->links(P32), G->links(P16), G->clovT[0].get(), G->clovT[1].get(),
                 G->clovTi[0].get(), G->clovTi[1].get()},
                G->recon};
    }
    struct Chunk {
        const void *x;
        GaugeSig gauge;
        int k0, nk, method, slot, iters;
        bool prefin;
        std::vector<double> kappa;
        hipGraphExec_t exec;
        int64_t hops;
        double bytes, flops;
    };
    std::vector<Chunk> chunks;

    // ws / ws_bytes: the caller's device region (null: allocate one); lent: host resources
    // to use instead of allocating (at least n right-hand sides)
    EoCore(wilson_ctx *c, const wilson_gauge *gauge, int n, int precision, int meth, void *ws = nullptr,
           size_t ws_bytes = 0, SolveHostRes *lent = nullptr)
        : ctx(c), G(gauge), g(gauge->g), nrhs(n), method(meth), nk(n) {
        P = inner_prec(precision);
        GP = inner_gauge_prec(precision);
        PX = P == P16 ? P32 : P;
        mixed = precision != WILSON_FP64;
        if (!G->links(GP)) throw Error(WILSON_INVALID_ARG, "gauge field lacks the link precision requested");
        const size_t need = carve(nullptr, g, n, precision, method);
        char *base;
        if (ws) {
            if (ws_bytes < need)
                throw Error(WILSON_INVALID_ARG, "workspace of " + std::to_string(ws_bytes) + " bytes is smaller than the " +
                                                    std::to_string(need) + " bytes this solve needs");
            if (reinterpret_cast<uintptr_t>(ws) % 256) throw Error(WILSON_INVALID_ARG, "workspace must be 256-byte aligned");
            base = static_cast<char *>(ws);
        } else {
            own.alloc(need);
            base = own.as<char>();
        }
        carve(base, g, n, precision, method);
        if (lent) {
            if (lent->cap < n) throw Error(WILSON_INVALID_ARG, "lent host resources too small");
            host = lent;
        } else {
            own_host = std::make_unique<SolveHostRes>();
            own_host->create(n);
            host = own_host.get();
        }
        ring_ev = host->ring;
        // the Krylov fields start at zero (a workspace holds whatever its last user left)
        std::vector<Spinor> all = {r.f, rh.f, p.f, v.f, s.f, t.f, tmp.f};
        for (auto &f : all) WL_HIP(launch_zero(f, g, n, ctx->stream));
    }
    // use another gauge field of the same shape
    void bind(const wilson_gauge *gauge) {
        if (!gauge->links(GP)) throw Error(WILSON_INVALID_ARG, "gauge field lacks the link precision requested");
        G = gauge;
    }

    ~EoCore() {
        for (auto &c : chunks) (void)hipGraphExecDestroy(c.exec);
    }
    size_t footprint() const { return bytes; }

    Spinor V(Spinor f) const {
        if (!f.data) return f;
        Spinor v = f;
        v.data = static_cast<char *>(f.data) + (size_t)k0 * 12 * spinor_plane_bytes(f.prec, g);
        if (f.scale) v.scale = f.scale + (size_t)k0 * g.stride;
        return v;
    }
    RhsState *S(RhsState *st) const { return st ? st + k0 : nullptr; }
    double kap(int k) const { return kappa[k0 + k]; }
    void select(int first, int count) { k0 = first; nk = count; }
    void select_all() { k0 = 0; nk = nrhs; }

    RhsState *sin() const { return st_in; }
    RhsState *sout() const { return st_out; }
    RhsState *mirror_dev(int slot) const { return reinterpret_cast<RhsState *>(host->mirror.dev()) + (size_t)slot * nrhs; }
    RhsState *mirror_host(int slot) const { return reinterpret_cast<RhsState *>(host->mirror.host()) + (size_t)slot * nrhs; }
    double *part() const { return partials; }
    double *part2() const { return partials2; }
    RhsState *salt() const { return st_alt; }
    const void *links(int prec) const { return G->links(prec == P64 ? P64 : GP); }
    int lprec(int prec) const { return prec == P64 ? P64 : GP; }

    // ---- primitives ----
    HopArgs hop_args(int par, Spinor out, Spinor in) const {
        HopArgs a;
        std::memset(&a, 0, sizeof a);
        a.g = g;
        a.par = par;
        a.nrhs = nk;
        a.out = V(out);
        a.in = V(in);
        a.gauge = links(in.prec);
        a.gprec = lprec(in.prec);
        a.recon = G->recon;
        a.partials = part();
        return a;
    }
    int run_hop(HopArgs &a) { return hop(ctx, a, hop_bytes(a)); }

    // from: the partials to sum (null: the common buffer)
    void finalize(int op, int nv, int nblocks, RhsState *st, int mask, RhsState *mir = nullptr,
                  const double *from = nullptr) {
        WL_HIP(launch_finalize(op, from ? from : part(), nv, nblocks, nk, S(st), mask, ctx->stream,
                               mir ? mir + k0 : nullptr));
    }
    // the finalize `op` of partials `from` run by the vector kernel of `a`, from states src to dst
    void attach_prefin(BlasArgs &a, int op, int nv, int nblocks, const double *from, RhsState *src, RhsState *dst) const {
        a.pre.on = 1;
        a.pre.op = op;
        a.pre.nv = nv;
        a.pre.nblocks = nblocks;
        a.pre.run_mask = PH_RUN;
        a.pre.partials = from;
        a.pre.src = S(src);
        a.pre.dst = S(dst);
    }

    // out_e = in_e - k^2 H_eo H_oe in_e  (dag: g5 M g5), optional reduction (finalized by caller)
    // bmx: out_e = b_e - M in_e
    // red_part: where the reduction's partials go (null: the common buffer)
    int apply_M(Spinor out, Spinor in, Spinor tmpo, bool dag, int red, Spinor w, RhsState *st, int mask,
                const Spinor *bmx = nullptr, double *red_part = nullptr) {
        HopArgs h1 = hop_args(1, tmpo, in);
        h1.g5in = dag;
        for (int k = 0; k < nk; k++) h1.cH[k] = 1.0;
        h1.state = S(st);
        h1.run_mask = mask;
        if (G->has_clover()) {  // tmp_o = T_oo^-1 H_oe in
            h1.clov = G->clover(true, in.prec, 1);
            h1.clov_mode = CLV_ALL;
        }
        run_hop(h1);
        HopArgs h2 = hop_args(0, out, tmpo);
        if (bmx) {
            h2.has_y = 1; h2.y = V(*bmx);
            h2.has_z = 1; h2.z = V(in); h2.cz = -1.0;
            for (int k = 0; k < nk; k++) h2.cH[k] = kap(k) * kap(k);
            if (G->has_clover()) h2.clov_mode = CLV_Z;  // b_e - T_ee in + k^2 H tmp
        } else {
            h2.has_y = 1; h2.y = V(in);
            h2.g5out = dag;
            for (int k = 0; k < nk; k++) h2.cH[k] = -kap(k) * kap(k);
            if (G->has_clover()) h2.clov_mode = CLV_Y;  // T_ee in - k^2 H tmp (T commutes with g5)
        }
        if (G->has_clover()) h2.clov = G->clover(false, in.prec, 0);
        h2.red = red;
        h2.w = V(w);
        h2.state = S(st);
        h2.run_mask = mask;
        if (red_part) h2.partials = red_part;
        return run_hop(h2);
    }

    BlasArgs blas_args(RhsState *st, int mask) const {
        BlasArgs a;
        std::memset(&a, 0, sizeof a);
        a.g = g;
        a.nrhs = nk;
        a.partials = part();
        a.state = S(st);
        a.run_mask = mask;
        return a;
    }
    // launch a BLAS op with its operand fields narrowed to the selected range
    void run_blas(int op, BlasArgs a, double bytes) {
        a.a = V(a.a); a.b = V(a.b); a.c = V(a.c); a.d = V(a.d); a.e = V(a.e); a.x = V(a.x);
        blas(ctx, op, a, bytes);
    }
    // block BiCGStab kernels on the selected range (s = nk right-hand sides)
    enum { BK_GRAM, BK_SOLVE, BK_UPDATE };
    BlockArgs block_args(RhsState *st, RhsState *mir = nullptr) const {
        BlockArgs a;
        std::memset(&a, 0, sizeof a);
        a.g = g;
        a.s = nk;
        a.partials = part();
        a.bs = bstate;
        a.state = S(st);
        a.mirror = mir ? mir + k0 : nullptr;
        return a;
    }
    void run_block(int kind, int op, BlockArgs a, double bytes) {
        a.a = V(a.a); a.b = V(a.b); a.c = V(a.c); a.d = V(a.d); a.x = V(a.x);
        timed_launch(ctx, WILSON_KERNEL_BLAS, bytes, [&]() {
            if (kind == BK_GRAM) return launch_block_gram(a, op, ctx->stream);
            if (kind == BK_SOLVE) return launch_block_solve(op, a, ctx->stream);
            return launch_block_update(op, a, ctx->stream);
        });
    }

    double vec_bytes(int prec, int nvec) const {
        return (double)nvec * g.Vh * nk * (24.0 * real_bytes(prec) + (prec == P16 ? 4.0 : 0.0));
    }

    // |e|^2 + |o|^2 of FP64 fields into st[].aux
    void norm2_full(Spinor e, Spinor o, RhsState *st) {
        BlasArgs a = blas_args(nullptr, 0);
        a.a = e;
        run_blas(BL_NORM2, a, vec_bytes(e.prec, 1));
        finalize(FIN_STORE_AUX, 1, blas_nblocks(g, e.prec), st, kAllPhases);
        a.a = o;
        run_blas(BL_NORM2, a, vec_bytes(o.prec, 1));
        finalize(FIN_ADD_AUX, 1, blas_nblocks(g, o.prec), st, kAllPhases);
    }

    // host <-> device copies of the states of the selected range
    void upload_states(RhsState *dst, const std::vector<RhsState> &h) {
        WL_HIP(hipStreamSynchronize(ctx->stream));  // hinit may still be the source of a copy
        std::memcpy(host->hinit.host(), h.data(), sizeof(RhsState) * nk);
        WL_HIP(hipMemcpyAsync(S(dst), host->hinit.host(), sizeof(RhsState) * nk, hipMemcpyHostToDevice, ctx->stream));
    }
    std::vector<RhsState> read_states(RhsState *src) {
        WL_HIP(hipMemcpyAsync(host->hread.host(), S(src), sizeof(RhsState) * nk, hipMemcpyDeviceToHost, ctx->stream));
        WL_HIP(hipStreamSynchronize(ctx->stream));
        ctx->drain_timing();
        std::vector<RhsState> h(nk);
        std::memcpy(h.data(), host->hread.host(), sizeof(RhsState) * nk);
        return h;
    }

    // b' = b_e + k H_eo b_o
    // (clover: b'_e = b_e + k H_eo T_oo^-1 b_o)
    void prepare_bprime() {
        Spinor src = b_o.f;
        if (G->has_clover()) {
            Spinor t = tmp64_or_scratch();
            WL_HIP(launch_clover_apply(V(t), V(b_o.f), G->clover(true, P64, 1), g, nk, ctx->stream));
            src = t;
        }
        HopArgs a = hop_args(0, bp.f, src);
        a.has_y = 1; a.y = V(b_e.f);
        for (int k = 0; k < nk; k++) a.cH[k] = kap(k);
        run_hop(a);
    }
    // x_o = b_o + k H_oe x_e  (clover: x_o = T_oo^-1 (b_o + k H_oe x_e))
    void reconstruct() {
        HopArgs a = hop_args(1, x_o.f, x_e.f);
        a.has_y = 1; a.y = V(b_o.f);
        for (int k = 0; k < nk; k++) a.cH[k] = kap(k);
        if (G->has_clover()) {
            a.clov = G->clover(true, P64, 1);
            a.clov_mode = CLV_ALL;
        }
        run_hop(a);
    }
    // |b - D x|^2 of the full system into sout()[].aux (nothing stored)
    void true_residual2() {
        for (int par = 0; par < 2; par++) {
            HopArgs a = hop_args(par, par ? tmp64_or_scratch() : tmp64_or_scratch(), par ? x_e.f : x_o.f);
            a.nostore = 1;
            a.has_y = 1; a.y = V(par ? b_o.f : b_e.f);
            a.has_z = 1; a.z = V(par ? x_o.f : x_e.f); a.cz = -1.0;
            for (int k = 0; k < nk; k++) a.cH[k] = kap(k);
            if (G->has_clover()) {  // b - T x + k H x
                a.clov = G->clover(false, P64, par);
                a.clov_mode = CLV_Z;
            }
            a.red = RED_NORM2;
            const int nb = run_hop(a);
            finalize(par ? FIN_ADD_AUX : FIN_STORE_AUX, 1, nb, sout(), kAllPhases);
        }
    }
    Spinor tmp64_or_scratch() {
        // output of a no-store hop is never written; any distinct FP64 field serves as the descriptor
        return mixed ? tmp64.f : (P == P64 ? tmp.f : tmp64.f);
    }

    // ---- inner Krylov solve on M_ee x = rhs (rhs in P, x in PX) ----
    // active[k]: which RHS take part; stop2[k]: (tol * norm)^2 of the iterated residual.
    // Returns per-RHS final states.
    // resume (BiCGStab only): the states to continue from, with phase, stop2 and iter set by
    // the caller, who has also replaced the iterated residual r; no initialisation runs and
    // the recurrence (p, v, rhat, rho, alpha, omega, beta) carries on.
    std::vector<RhsState> inner_solve(Spinor rhs, Spinor x, bool use_x0, const std::vector<char> &active,
                                      const std::vector<double> &stop2, int maxiter, int poll_every,
                                      const std::vector<RhsState> *resume = nullptr) {
        std::vector<RhsState> h(nk);
        for (int k = 0; k < nk; k++) {
            std::memset(&h[k], 0, sizeof(RhsState));
            h[k].phase = active[k] ? PH_RUN : PH_IDLE;
            h[k].stop2 = stop2[k];
        }
        if (resume) h = *resume;
        upload_states(sin(), h);
        const int nb = blas_nblocks(g, P);
        Spinor none;
        if (resume) {
            if (method != WILSON_SOLVER_BICGSTAB_EO) throw Error(WILSON_INVALID_ARG, "only BiCGStab resumes");
        } else if (method == WILSON_SOLVER_BICGSTAB_EO) {
            // r = rhs - M x  (or rhs), rhat = r
            if (use_x0) {
                apply_M(r.f, x, tmp.f, false, RED_NONE, none, sin(), PH_RUN, &rhs);
                BlasArgs a = blas_args(sin(), PH_RUN);
                a.a = rh.f; a.b = r.f;
                run_blas(BL_COPY_NORM, a, vec_bytes(P, 2));
            } else {
                BlasArgs a = blas_args(sin(), PH_RUN);
                a.a = r.f; a.b = rhs;
                run_blas(BL_COPY_NORM, a, vec_bytes(P, 2));
                a.a = rh.f; a.b = rhs;
                run_blas(BL_COPY_NORM, a, vec_bytes(P, 2));
            }
            finalize(FIN_BICG_INIT, 1, nb, sin(), PH_RUN);
            for (Spinor f : {p.f, v.f, t.f}) WL_HIP(launch_zero(V(f), g, nk, ctx->stream));
        } else if (method == WILSON_SOLVER_BLOCK_BICGSTAB_EO) {
            // R = rhs - A X (or rhs), P = R, R~ = R with the column norms, then one phase
            // for the whole block (it runs while any column misses its threshold)
            BlasArgs a = blas_args(sin(), PH_RUN);
            if (use_x0) {
                apply_M(r.f, x, tmp.f, false, RED_NONE, none, sin(), PH_RUN, &rhs);
            } else {
                a.a = r.f; a.b = rhs;
                run_blas(BL_COPY_NORM, a, vec_bytes(P, 2));
            }
            a.a = p.f; a.b = r.f;
            run_blas(BL_COPY_NORM, a, vec_bytes(P, 2));
            a.a = rh.f; a.b = r.f;
            run_blas(BL_COPY_NORM, a, vec_bytes(P, 2));
            finalize(FIN_BICG_INIT, 1, nb, sin(), PH_RUN);
            run_block(BK_SOLVE, BS_INIT, block_args(sin()), 0.0);
        } else {
            // CGLS: r = rhs - M x, z = M^dag r, p = z
            if (use_x0) {
                const int hb = apply_M(r.f, x, tmp.f, false, RED_NORM2, none, sin(), PH_RUN, &rhs);
                finalize(FIN_CG_R2, 1, hb, sin(), PH_RUN);
            } else {
                BlasArgs a = blas_args(sin(), PH_RUN);
                a.a = r.f; a.b = rhs;
                run_blas(BL_COPY_NORM, a, vec_bytes(P, 2));
                finalize(FIN_CG_R2, 1, nb, sin(), PH_RUN);
            }
            const int hb = apply_M(s.f, r.f, tmp.f, true, RED_NORM2, none, sin(), PH_RUN);
            finalize(FIN_CG_ZZ, 1, hb, sin(), PH_RUN);
            BlasArgs a = blas_args(sin(), PH_RUN);
            a.a = p.f; a.b = s.f;
            run_blas(BL_COPY_NORM, a, vec_bytes(P, 2));
        }
        // enqueue iterations ahead of the host; poll `lag` iterations behind
        const int lag = 2;
        int it = 0;
        std::vector<RhsState> init = read_states(sin());
        bool any_run = false;
        for (auto &st : init) any_run |= (st.phase == PH_RUN);
        if (!any_run) return init;
        poll_every = std::max(1, poll_every);
        int enq = 0;
        // with graphs: after one ordinary iteration (which settles every launch shape), chunks
        // of kGraphChunk iterations replayed from a captured graph, polled at their end; the
        // device runs the same kernels with the same arguments, so the result is the same
        const bool chunked = graphs && method != WILSON_SOLVER_BLOCK_BICGSTAB_EO && !ctx->timing;
        for (it = 0; it < maxiter;) {
            const int slot = enq % kRing;
            bool poll_here;
            if (chunked && it >= 1 && it + kGraphChunk <= maxiter) {
                replay_chunk(x, slot);
                it += kGraphChunk;
                poll_here = true;
            } else {
                poll_here = ((it + 1) % poll_every == 0) || it + 1 == maxiter;
                iterate(x, poll_here ? mirror_dev(slot) : nullptr);
                it++;
            }
            if (!poll_here) continue;
            WL_HIP(hipEventRecord(ring_ev[slot], ctx->stream));
            enq++;
            if (enq > lag) {
                const int ps = (enq - 1 - lag) % kRing;
                WL_HIP(hipEventSynchronize(ring_ev[ps]));
                const RhsState *m = mirror_host(ps) + k0;
                bool running = false;
                for (int k = 0; k < nk; k++) running |= (m[k].phase == PH_RUN || m[k].phase == PH_SCONV);
                if (!running) break;
            }
        }
        return read_states(sin());
    }

    void iterate(Spinor x, RhsState *mir) {
        if (method == WILSON_SOLVER_BICGSTAB_EO) bicg_iter(x, mir);
        else if (method == WILSON_SOLVER_BLOCK_BICGSTAB_EO) block_iter(x, mir);
        else cg_iter(x, mir);
    }

    // kGraphChunk iterations from a graph captured on the context's capture stream (kernel
    // nodes only: the iterations launch nothing else) and replayed on its stream; the last
    // one writes the state mirror of `slot`.
    void replay_chunk(Spinor x, int slot) {
        const std::vector<double> kap(kappa.begin() + k0, kappa.begin() + k0 + nk);
        Chunk *c = nullptr;
        const GaugeSig gs = gauge_sig();
        for (auto &e : chunks)
            if (e.x == x.data && e.gauge == gs && e.k0 == k0 && e.nk == nk && e.method == method && e.slot == slot &&
                e.iters == kGraphChunk && e.prefin == prefin && e.kappa == kap) {
                c = &e;
                break;
            }
        if (!c) {
            if (!ctx->capture_stream) WL_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
            const int64_t h0 = ctx->hop_launch_count;
            const double b0 = ctx->bytes_issued, f0 = ctx->flops_issued;
            hipStream_t run = ctx->stream;
            hipGraph_t gph = nullptr;
            ctx->stream = ctx->capture_stream;  // every launch of the iterations goes to the capture
            WL_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            try {
                for (int i = 0; i < kGraphChunk; i++) iterate(x, i == kGraphChunk - 1 ? mirror_dev(slot) : nullptr);
            } catch (...) {
                (void)hipStreamEndCapture(ctx->stream, &gph);
                if (gph) (void)hipGraphDestroy(gph);
                ctx->stream = run;
                throw;
            }
            const hipError_t e = hipStreamEndCapture(ctx->stream, &gph);
            ctx->stream = run;
            WL_HIP(e);
            hipGraphExec_t ex = nullptr;
            const hipError_t ei = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gph);
            WL_HIP(ei);
            if (chunks.size() >= 16) {  // keep the most recent graphs
                (void)hipGraphExecDestroy(chunks.front().exec);
                chunks.erase(chunks.begin());
            }
            // the capture ran nothing: its bookkeeping belongs to each replay
            chunks.push_back({x.data, gs, k0, nk, method, slot, kGraphChunk, prefin, kap, ex, ctx->hop_launch_count - h0,
                              ctx->bytes_issued - b0, ctx->flops_issued - f0});
            ctx->hop_launch_count = h0;
            ctx->bytes_issued = b0;
            ctx->flops_issued = f0;
            c = &chunks.back();
        }
        WL_HIP(hipGraphLaunch(c->exec, ctx->stream));
        ctx->hop_launch_count += c->hops;
        ctx->bytes_issued += c->bytes;
        ctx->flops_issued += c->flops;
    }

    void bicg_iter(Spinor x, RhsState *mir) {
        const int nb = blas_nblocks(g, P);
        Spinor none;
        {   // p = r + beta (p - omega v)
            BlasArgs a = blas_args(sin(), PH_RUN);
            a.a = p.f; a.b = r.f; a.c = v.f;
            run_blas(BL_P_UPDATE, a, vec_bytes(P, 4));
        }
        // With prefin, the two hops' partials go to their own buffer and the vector kernels
        // after them run the alpha and omega steps: states sin() -> salt() -> sin().
        double *hp = prefin ? part2() : part();
        // v = M p, <rhat, v> -> alpha
        int hb = apply_M(v.f, p.f, tmp.f, false, RED_DOT, rh.f, sin(), PH_RUN, nullptr, hp);
        const bool pa = prefin && hb <= kPreFinMax;
        if (!pa) finalize(FIN_BICG_ALPHA, 2, hb, sin(), PH_RUN, nullptr, hp);
        RhsState *st = pa ? salt() : sin();
        {   // s = r - alpha v, |s|^2
            BlasArgs a = blas_args(sin(), PH_RUN);
            a.a = s.f; a.b = r.f; a.c = v.f;
            if (pa) attach_prefin(a, FIN_BICG_ALPHA, 2, hb, hp, sin(), salt());
            run_blas(BL_S_UPDATE, a, vec_bytes(P, 3));
            finalize(FIN_BICG_S, 1, nb, st, PH_RUN);
        }
        // t = M s, <t, s>, |t|^2 -> omega
        hb = apply_M(t.f, s.f, tmp.f, false, RED_TS, none, st, PH_RUN, nullptr, hp);
        const bool po = pa && hb <= kPreFinMax;  // the hops of one iteration share their launch shape
        if (!po) finalize(FIN_BICG_OMEGA, 3, hb, st, PH_RUN, nullptr, hp);
        {   // x += alpha p + omega s; r = s - omega t; |r|^2, <rhat, r> -> beta, rho
            BlasArgs a = blas_args(st, PH_RUN | PH_SCONV);
            a.a = p.f; a.b = s.f; a.c = r.f; a.d = t.f; a.e = rh.f; a.x = x;
            if (po) attach_prefin(a, FIN_BICG_OMEGA, 3, hb, hp, salt(), sin());
            run_blas(BL_XR_UPDATE, a, vec_bytes(P, 5) + vec_bytes(x.prec, 2));
            if (po) st = sin();
            finalize(FIN_BICG_RHO, 3, nb, st, PH_RUN | PH_SCONV, mir);
        }
        if (st != sin())  // (only if the two hops' partial rows differed) the states back to sin()
            WL_HIP(hipMemcpyAsync(S(sin()), S(st), sizeof(RhsState) * nk, hipMemcpyDeviceToDevice, ctx->stream));
    }

    // One block BiCGStab iteration (block.hip has the recurrence); x in FP64.
    void block_iter(Spinor x, RhsState *mir) {
        Spinor none;
        const double u = vec_bytes(P64, 1);  // one field of every right-hand side
        apply_M(v.f, p.f, tmp.f, false, RED_NONE, none, sin(), PH_RUN);  // V = A P
        BlockArgs a = block_args(sin());
        a.a = rh.f; a.b = v.f; a.c = r.f;
        run_block(BK_GRAM, 2, a, 3 * u);                                  // R~^H V, R~^H R
        run_block(BK_SOLVE, BS_ALPHA, block_args(sin()), 0.0);
        a = block_args(sin());
        a.a = s.f; a.b = r.f; a.c = v.f;
        run_block(BK_UPDATE, BU_S, a, 3 * u);                             // S = R - V alpha
        const int hb = apply_M(t.f, s.f, tmp.f, false, RED_TS, none, sin(), PH_RUN);  // T = A S
        finalize(FIN_BLOCK_TS, 3, hb, sin(), PH_RUN);
        a = block_args(sin());
        a.a = rh.f; a.b = t.f;
        run_block(BK_GRAM, 1, a, 2 * u);                                  // R~^H T
        run_block(BK_SOLVE, BS_BETA, block_args(sin()), 0.0);             // omega, beta
        a = block_args(sin());
        a.a = p.f; a.b = s.f; a.c = r.f; a.d = t.f; a.x = x;
        run_block(BK_UPDATE, BU_XR, a, 6 * u);                            // X, R, |R_j|^2
        run_block(BK_SOLVE, BS_CHECK, block_args(sin(), mir), 0.0);
        a = block_args(sin());
        a.a = p.f; a.b = r.f; a.c = v.f;
        run_block(BK_UPDATE, BU_P, a, 4 * u);                             // P = R + (P - omega V) beta
    }

    void cg_iter(Spinor x, RhsState *mir) {
        const int nb = blas_nblocks(g, P);
        Spinor none;
        // w = M p, |w|^2 -> alpha
        int hb = apply_M(v.f, p.f, tmp.f, false, RED_NORM2, none, sin(), PH_RUN);
        finalize(FIN_CG_ALPHA, 1, hb, sin(), PH_RUN);
        {   // x += alpha p; r -= alpha w; |r|^2
            BlasArgs a = blas_args(sin(), PH_RUN);
            a.a = p.f; a.b = r.f; a.c = v.f; a.x = x;
            run_blas(BL_CG_XR, a, vec_bytes(P, 4) + vec_bytes(x.prec, 2));
            finalize(FIN_CG_R, 1, nb, sin(), PH_RUN, mir);
        }
        // z = M^dag r, |z|^2 -> beta
        hb = apply_M(s.f, r.f, tmp.f, true, RED_NORM2, none, sin(), PH_RUN);
        finalize(FIN_CG_BETA, 1, hb, sin(), PH_RUN);
        {   // p = z + beta p
            BlasArgs a = blas_args(sin(), PH_RUN);
            a.a = p.f; a.b = s.f;
            run_blas(BL_CG_P, a, vec_bytes(P, 3));
        }
    }

    // r64 = b' - M x_e (FP64), |r64|^2 -> sout().aux
    void outer_residual() {
        Spinor none;
        const int hb = apply_M(r64.f, x_e.f, tmp64.f, false, RED_NORM2, none, nullptr, 0, &bp.f);
        finalize(FIN_STORE_AUX, 1, hb, sout(), kAllPhases);
    }
};

static std::string solve_key(const wilson_gauge *G, const SolveParams &p) {
    std::ostringstream os;
    os << G->dims[0] << "x" << G->dims[1] << "x" << G->dims[2] << "x" << G->dims[3] << " " << p.precision << " "
       << p.method;
    return os.str();
}

// Workspaces depend on the lattice shape, precision and method only (the gauge field is
// bound per call); a cached one with room for at least nrhs right-hand sides is reused.
static std::shared_ptr<EoCore> get_core(wilson_ctx *ctx, const wilson_gauge *G, int nrhs, const SolveParams &p) {
    const std::string key = solve_key(G, p);
    auto &cache = ctx->solve_cache;
    for (size_t k = 0; k < cache.size(); k++) {
        if (cache[k].first != key) continue;
        auto core = std::static_pointer_cast<EoCore>(cache[k].second);
        if (core->nrhs >= nrhs) {
            auto hit = cache[k];
            cache.erase(cache.begin() + k);
            cache.push_back(hit);  // most recently used last
            core->bind(G);
            return core;
        }
        WL_HIP(hipStreamSynchronize(ctx->stream));
        cache.erase(cache.begin() + k);
        break;
    }
    WL_HIP(hipStreamSynchronize(ctx->stream));
    if (cache.size() >= 4) cache.erase(cache.begin());
    auto core = std::make_shared<EoCore>(ctx, G, nrhs, p.precision, p.method);
    cache.emplace_back(key, core);
    return core;
}

size_t solve_footprint(const Geom &g, int nrhs, const SolveParams &p) {
    EoMem m;
    return m.carve(nullptr, g, nrhs, p.precision, p.method);
}

// Sets the context's no-tuning flag for the lifetime of a call.
struct NoTuneScope {
    wilson_ctx *ctx;
    bool prev;
    NoTuneScope(wilson_ctx *c, bool on) : ctx(c), prev(c->no_tune) { c->no_tune = prev || on; }
    ~NoTuneScope() { ctx->no_tune = prev; }
};

int solve_device(wilson_ctx *ctx, const wilson_gauge *G, double *x_canon, const double *b_canon, int nrhs,
                 const double *kappa, const double *tol, const SolveParams &prm, wilson_solve_info *info) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t hop0 = ctx->hop_launch_count;
    const double bytes0 = ctx->bytes_issued, flops0 = ctx->flops_issued;
    NoTuneScope nts(ctx, prm.no_tune);
    // a caller's region holds the device buffers of this call only (built per call, with
    // the context's host resources); otherwise a cached workspace of the context
    auto core = prm.workspace ? std::make_shared<EoCore>(ctx, G, nrhs, prm.precision, prm.method, prm.workspace,
                                                         prm.workspace_bytes, &ctx->lend)
                              : get_core(ctx, G, nrhs, prm);
    EoCore &C = *core;
    const Geom &g = C.g;
    C.graphs = prm.graphs && !prm.no_tune && graphs_enabled() && g.Vh <= kGraphMaxVh;
    C.prefin = prefin_enabled();
    C.select(0, nrhs);
    C.kappa.assign(C.nrhs, 0.0);
    std::copy(kappa, kappa + nrhs, C.kappa.begin());

    // b -> parity fields; |b|^2
    WL_HIP(launch_to_parity(C.b_e.f, b_canon, g, 0, nrhs, 1.0, ctx->stream));
    WL_HIP(launch_to_parity(C.b_o.f, b_canon, g, 1, nrhs, 1.0, ctx->stream));
    {
        std::vector<RhsState> h(nrhs);
        std::memset(h.data(), 0, sizeof(RhsState) * nrhs);
        for (auto &s : h) s.phase = PH_RUN;
        C.upload_states(C.sout(), h);
    }
    C.norm2_full(C.b_e.f, C.b_o.f, C.sout());
    std::vector<RhsState> hs = C.read_states(C.sout());
    std::vector<double> bn2(nrhs), stop2(nrhs);
    std::vector<int> status(nrhs, WILSON_NOT_CONVERGED), iters(nrhs, 0), cycles(nrhs, 0), restarts(nrhs, 0);
    std::vector<char> done(nrhs, 0);
    for (int k = 0; k < nrhs; k++) {
        bn2[k] = hs[k].aux;
        if (!std::isfinite(bn2[k])) throw Error(WILSON_NONFINITE, "right-hand side contains NaN or Inf");
        stop2[k] = tol[k] * tol[k] * bn2[k];
    }
    if (prm.use_x0) {
        WL_HIP(launch_to_parity(C.x_e.f, x_canon, g, 0, nrhs, 1.0, ctx->stream));
    } else {
        WL_HIP(launch_zero(C.x_e.f, g, nrhs, ctx->stream));
    }
    C.prepare_bprime();
    int used = 0;  // inner iterations consumed (max over RHS: they run in lockstep)
    std::vector<double> res2(nrhs, 0.0);
    bool checked = false;

    auto true_check = [&]() {
        checked = true;
        C.reconstruct();
        C.true_residual2();
        std::vector<RhsState> h = C.read_states(C.sout());
        for (int k = 0; k < nrhs; k++) res2[k] = h[k].aux;
    };

    if (prm.method == WILSON_SOLVER_BLOCK_BICGSTAB_EO) {
        // Blocks of up to kMaxBlock consecutive non-zero right-hand sides, one after the
        // other; a zero right-hand side has the solution 0 and stays out of every block.
        std::vector<int> fail(nrhs, FAIL_NONE);
        for (int k = 0; k < nrhs; k++)
            if (bn2[k] == 0.0) {
                C.select(k, 1);
                WL_HIP(launch_zero(C.V(C.x_e.f), g, 1, ctx->stream));
            }
        int k = 0;
        while (k < nrhs) {
            if (bn2[k] == 0.0) { k++; continue; }
            const int c0 = k;
            while (k < nrhs && bn2[k] > 0.0 && k - c0 < kMaxBlock) k++;
            const int cn = k - c0;
            C.select(c0, cn);
            const std::vector<double> st2(stop2.begin() + c0, stop2.begin() + c0 + cn);
            std::vector<char> act(cn, 1);
            bool use_x0 = prm.use_x0, single = false;
            int used_c = 0;
            for (int attempt = 0;; attempt++) {
                const int budget = prm.maxiter - used_c;
                if (budget <= 0) break;
                // after a breakdown of the block: one recurrence per right-hand side
                C.method = single ? WILSON_SOLVER_BICGSTAB_EO : WILSON_SOLVER_BLOCK_BICGSTAB_EO;
                std::vector<RhsState> fin;
                try {
                    fin = C.inner_solve(C.bp.f, C.x_e.f, use_x0, act, st2, budget, prm.poll_every);
                } catch (...) {
                    C.method = WILSON_SOLVER_BLOCK_BICGSTAB_EO;
                    throw;
                }
                C.method = WILSON_SOLVER_BLOCK_BICGSTAB_EO;
                int mx = 0;
                for (int j = 0; j < cn; j++)
                    if (act[j]) {
                        iters[c0 + j] += fin[j].iter;
                        mx = std::max(mx, fin[j].iter);
                    }
                used_c += std::max(mx, 1);
                C.reconstruct();
                C.true_residual2();
                std::vector<RhsState> h = C.read_states(C.sout());
                bool all_ok = true, broke = false, nonfinite = false;
                for (int j = 0; j < cn; j++) {
                    res2[c0 + j] = h[j].aux;
                    if (act[j]) fail[c0 + j] = fin[j].phase == PH_FAIL ? fin[j].fail : FAIL_NONE;
                    broke |= fail[c0 + j] == FAIL_BREAKDOWN;
                    nonfinite |= fail[c0 + j] == FAIL_NONFINITE;
                    all_ok &= res2[c0 + j] <= st2[j];
                }
                if (all_ok || nonfinite) break;
                if (attempt >= prm.max_restarts || used_c >= prm.maxiter) break;
                if (broke) single = true;
                for (int j = 0; j < cn; j++) {
                    if (single) act[j] = res2[c0 + j] > st2[j];
                    if (act[j]) restarts[c0 + j]++;
                }
                use_x0 = true;
            }
        }
        C.select_all();
        true_check();
        for (int j = 0; j < nrhs; j++) {
            if (bn2[j] == 0.0) continue;
            if (fail[j] == FAIL_NONFINITE) status[j] = WILSON_NONFINITE;
            else if (res2[j] <= stop2[j]) status[j] = WILSON_OK;
            else if (fail[j] == FAIL_BREAKDOWN) status[j] = WILSON_BREAKDOWN;
            else status[j] = WILSON_NOT_CONVERGED;
        }
    } else if (!C.mixed) {
        bool use_x0 = prm.use_x0;
        for (int attempt = 0;; attempt++) {
            std::vector<char> active(nrhs);
            for (int k = 0; k < nrhs; k++) active[k] = !done[k] && bn2[k] > 0.0;
            if (std::none_of(active.begin(), active.end(), [](char c) { return c; })) break;
            const int budget = prm.maxiter - used;
            if (budget <= 0) break;
            std::vector<RhsState> fin = C.inner_solve(C.bp.f, C.x_e.f, use_x0, active, stop2, budget, prm.poll_every);
            int mx = 0;
            for (int k = 0; k < nrhs; k++)
                if (active[k]) {
                    iters[k] += fin[k].iter;
                    mx = std::max(mx, fin[k].iter);
                }
            used += std::max(mx, 1);
            true_check();
            bool again = false;
            for (int k = 0; k < nrhs; k++) {
                if (!active[k]) continue;
                if (fin[k].phase == PH_FAIL && fin[k].fail == FAIL_NONFINITE) {
                    status[k] = WILSON_NONFINITE;
                    done[k] = 1;
                } else if (res2[k] <= stop2[k]) {
                    status[k] = WILSON_OK;
                    done[k] = 1;
                } else if (attempt >= prm.max_restarts || used >= prm.maxiter) {
                    status[k] = fin[k].phase == PH_FAIL ? WILSON_BREAKDOWN : WILSON_NOT_CONVERGED;
                    done[k] = 1;
                } else {
                    restarts[k]++;
                    again = true;
                }
            }
            if (!again) break;
            use_x0 = true;
            checked = false;
        }
    } else if (prm.reliable) {
        // Reliable updates (Sleijpen and van der Vorst, 1996): one low-precision BiCGStab
        // recurrence runs through every cycle.  A cycle ends when the iterated residual has
        // dropped by delta; then the low-precision solution increment is added to the FP64
        // solution, the FP64 residual b' - M x is recomputed and replaces the iterated
        // residual, and the recurrence goes on with its search directions and scalars.  The
        // fields are not rescaled between cycles (FP32 and per-site-scaled FP16 keep the
        // range of a 1e-10 relative residual).
        const double delta = prm.inner_tol > 0 ? prm.inner_tol : (C.P == P32 ? 1e-5 : 1e-2);
        C.outer_residual();
        std::vector<RhsState> h = C.read_states(C.sout());
        std::vector<double> prev(nrhs, 0.0), inner_stop(nrhs, 0.0);
        std::vector<int> stall(nrhs, 0);
        for (int k = 0; k < nrhs; k++) prev[k] = h[k].aux;
        std::vector<RhsState> rec;  // the recurrence to resume (empty: start one)
        const int max_cycles = 400;
        for (int cyc = 0; cyc < max_cycles; cyc++) {
            std::vector<char> active(nrhs);
            for (int k = 0; k < nrhs; k++) {
                if (done[k]) { active[k] = 0; continue; }
                const double rr = h[k].aux;
                if (!std::isfinite(rr)) { status[k] = WILSON_NONFINITE; done[k] = 1; active[k] = 0; continue; }
                if (rr <= stop2[k]) { done[k] = 2; active[k] = 0; continue; }  // confirmed below
                active[k] = 1;
                inner_stop[k] = std::max(delta * delta * rr, 0.25 * stop2[k]);
            }
            if (std::none_of(active.begin(), active.end(), [](char c) { return c; })) break;
            const int budget = prm.maxiter - used;
            if (budget <= 0) break;
            // a recurrence that ended on a failure, or on |s| (omega = 0), cannot go on
            bool fresh = rec.empty();
            for (int k = 0; k < nrhs && !fresh; k++)
                if (active[k] && (rec[k].phase == PH_FAIL || (rec[k].omega_re == 0.0 && rec[k].omega_im == 0.0)))
                    fresh = true;
            WL_HIP(launch_zero(C.xin.f, g, nrhs, ctx->stream));
            std::vector<RhsState> fin;
            if (fresh) {
                WL_HIP(launch_convert(C.rf.f, C.r64.f, g, nrhs, C.sout(), 0, ctx->stream));
                fin = C.inner_solve(C.rf.f, C.xin.f, false, active, inner_stop, budget, prm.poll_every);
            } else {
                WL_HIP(launch_convert(C.r.f, C.r64.f, g, nrhs, C.sout(), 0, ctx->stream));  // r <- true residual
                for (int k = 0; k < nrhs; k++) {
                    rec[k].phase = active[k] ? PH_RUN : PH_IDLE;
                    rec[k].stop2 = inner_stop[k];
                    rec[k].r2 = h[k].aux;
                    rec[k].iter = 0;
                    rec[k].fail = FAIL_NONE;
                }
                fin = C.inner_solve(C.rf.f, C.xin.f, false, active, inner_stop, budget, prm.poll_every, &rec);
            }
            rec = fin;
            int mx = 0;
            for (int k = 0; k < nrhs; k++)
                if (active[k]) {
                    iters[k] += fin[k].iter;
                    cycles[k] += 1;
                    mx = std::max(mx, fin[k].iter);
                    if (fin[k].phase == PH_FAIL && fin[k].fail == FAIL_NONFINITE) {
                        status[k] = WILSON_NONFINITE;
                        done[k] = 1;
                    }
                }
            used += std::max(mx, 1);
            WL_HIP(launch_axpy_f64(C.x_e.f, C.xin.f, g, nrhs, C.sout(), 0, ctx->stream));
            C.outer_residual();
            h = C.read_states(C.sout());
            for (int k = 0; k < nrhs; k++) {
                if (!active[k] || done[k]) continue;
                // no progress over 8 cycles in a row: give up
                stall[k] = h[k].aux > 0.9 * prev[k] ? stall[k] + 1 : 0;
                if (stall[k] >= 8) { status[k] = WILSON_NOT_CONVERGED; done[k] = 1; }
                prev[k] = h[k].aux;
            }
        }
        true_check();
        for (int k = 0; k < nrhs; k++) {
            if (status[k] == WILSON_NONFINITE) continue;
            if (bn2[k] == 0.0 || res2[k] <= stop2[k]) status[k] = WILSON_OK;
            else status[k] = WILSON_NOT_CONVERGED;
        }
    } else {
        // FP64 defect correction on the even system around low-precision inner solves
        const double delta = prm.inner_tol > 0 ? prm.inner_tol : (C.P == P32 ? 1e-5 : 1e-2);
        std::vector<double> inner_stop(nrhs, delta * delta);  // inner rhs has unit norm
        std::vector<double> prev(nrhs, 0.0);
        std::vector<int> stall(nrhs, 0);
        C.outer_residual();
        std::vector<RhsState> h = C.read_states(C.sout());
        for (int k = 0; k < nrhs; k++) prev[k] = h[k].aux;
        const int max_cycles = 200;
        for (int cyc = 0; cyc < max_cycles; cyc++) {
            std::vector<char> active(nrhs);
            for (int k = 0; k < nrhs; k++) {
                if (done[k]) { active[k] = 0; continue; }
                const double rr = h[k].aux;
                if (!std::isfinite(rr)) { status[k] = WILSON_NONFINITE; done[k] = 1; active[k] = 0; continue; }
                if (rr <= stop2[k]) { done[k] = 2; active[k] = 0; continue; }  // candidate, confirmed below
                active[k] = 1;
            }
            if (std::none_of(active.begin(), active.end(), [](char c) { return c; })) break;
            const int budget = prm.maxiter - used;
            if (budget <= 0) break;
            WL_HIP(launch_convert(C.rf.f, C.r64.f, g, nrhs, C.sout(), 1, ctx->stream));
            WL_HIP(launch_zero(C.xin.f, g, nrhs, ctx->stream));
            std::vector<RhsState> fin = C.inner_solve(C.rf.f, C.xin.f, false, active, inner_stop, budget,
                                                      prm.poll_every);
            int mx = 0;
            for (int k = 0; k < nrhs; k++)
                if (active[k]) {
                    iters[k] += fin[k].iter;
                    cycles[k] += 1;
                    mx = std::max(mx, fin[k].iter);
                }
            used += std::max(mx, 1);
            WL_HIP(launch_axpy_f64(C.x_e.f, C.xin.f, g, nrhs, C.sout(), 1, ctx->stream));
            C.outer_residual();
            h = C.read_states(C.sout());
            for (int k = 0; k < nrhs; k++) {
                if (!active[k]) continue;
                if (h[k].aux > 0.25 * prev[k]) stall[k]++;
                if (stall[k] >= 4) { status[k] = WILSON_NOT_CONVERGED; done[k] = 1; }
                prev[k] = h[k].aux;
            }
        }
        true_check();
        for (int k = 0; k < nrhs; k++) {
            if (status[k] == WILSON_NONFINITE) continue;
            if (bn2[k] == 0.0 || res2[k] <= stop2[k]) status[k] = WILSON_OK;
            else if (status[k] != WILSON_NOT_CONVERGED) status[k] = WILSON_NOT_CONVERGED;
        }
    }
    if (!checked) true_check();  // x_o for every RHS (also those that never ran)
    for (int k = 0; k < nrhs; k++)
        if (bn2[k] == 0.0) { status[k] = WILSON_OK; res2[k] = 0.0; }

    // x -> canonical
    WL_HIP(launch_from_parity(x_canon, C.x_e.f, g, 0, nrhs, ctx->stream));
    WL_HIP(launch_from_parity(x_canon, C.x_o.f, g, 1, nrhs, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    ctx->drain_timing();
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = WILSON_OK;
    for (int k = 0; k < nrhs; k++) {
        const int st = status[k];
        if (st < 0 && (worst >= 0 || st < worst)) worst = st;
        else if (worst == WILSON_OK && st > 0) worst = st;
        if (info) {
            info[k].iterations = iters[k];
            info[k].outer_cycles = cycles[k];
            info[k].restarts = restarts[k];
            info[k].converged = st == WILSON_OK;
            info[k].true_residual = bn2[k] > 0 ? std::sqrt(res2[k] / bn2[k]) : 0.0;
            info[k].ms = ms;
            info[k].hop_launches = (double)(ctx->hop_launch_count - hop0);
            info[k].bytes = ctx->bytes_issued - bytes0;
            info[k].flops = ctx->flops_issued - flops0;
        }
    }
    return worst;
}

// ---------------------------------------------------------------------------------
struct DslashWs {
    FieldBuf in_e, in_o, out_e, out_o;
};

void dslash_device(wilson_ctx *ctx, const wilson_gauge *G, double *out, const double *in, double kappa, int parity,
                   int precision, int nrhs) {
    const Geom &g = G->g;
    const int P = inner_prec(precision), GP = inner_gauge_prec(precision);
    if (!G->links(GP)) throw Error(WILSON_INVALID_ARG, "gauge field lacks the link precision requested");
    std::ostringstream os;
    os << (const void *)G << " " << P << " " << nrhs;
    std::shared_ptr<DslashWs> ws;
    if (ctx->dslash_ws && ctx->dslash_key == os.str()) {
        ws = std::static_pointer_cast<DslashWs>(ctx->dslash_ws);
    } else {
        ctx->dslash_ws.reset();
        WL_HIP(hipStreamSynchronize(ctx->stream));
        ws = std::make_shared<DslashWs>();
        ws->in_e.make(P, g, nrhs); ws->in_o.make(P, g, nrhs);
        ws->out_e.make(P, g, nrhs); ws->out_o.make(P, g, nrhs);
        ctx->dslash_ws = ws;
        ctx->dslash_key = os.str();
    }
    WL_HIP(launch_to_parity(ws->in_e.f, in, g, 0, nrhs, 1.0, ctx->stream));
    WL_HIP(launch_to_parity(ws->in_o.f, in, g, 1, nrhs, 1.0, ctx->stream));
    for (int par = 0; par < 2; par++) {
        if (parity != 2 && parity != par) continue;
        HopArgs a;
        std::memset(&a, 0, sizeof a);
        a.g = g;
        a.par = par;
        a.nrhs = nrhs;
        a.out = par ? ws->out_o.f : ws->out_e.f;
        a.in = par ? ws->in_e.f : ws->in_o.f;
        a.gauge = G->links(P == P64 ? P64 : GP);
        a.gprec = P == P64 ? P64 : GP;
        a.recon = G->recon;
        for (int k = 0; k < nrhs; k++) a.cH[k] = -kappa;
        if (parity == 2) {  // D psi = T psi - k H psi (T = 1 without a clover term)
            a.has_y = 1;
            a.y = par ? ws->in_o.f : ws->in_e.f;
            if (G->has_clover()) {
                a.clov = G->clover(false, P, par);
                a.clov_mode = CLV_Y;
            }
        }
        hop(ctx, a, hop_bytes(a));
        WL_HIP(launch_from_parity(out, a.out, g, par, nrhs, ctx->stream));
    }
}

// ---------------------------------------------------------------------------------
// Continuous batching: nslots independent solves on one resident gauge field.  All
// running slots advance together in every batched iteration (each with its own
// scalars, kappa and tolerance); per-slot transitions (start, outer correction,
// finish) are launched on that slot alone when the host polls.  A slot's arithmetic
// never depends on the other slots (the reductions are per slot and the partial sums
// are combined in a fixed order), so a result is the same alone and in any mix.
class BatchEngine {
   public:
    enum SlotState { FREE = 0, RUNNING = 1, FINISHED = 2 };
    struct Slot {
        int state = FREE;
        int status = WILSON_OK;
        double kappa = 0, tol = 0, bn2 = 0, stop2 = 0, res2 = 0, prev = 0;
        int maxiter = 0, iters = 0, cycles = 0, restarts = 0, stall = 0;
        std::chrono::steady_clock::time_point t0;
        double ms = 0;
    };
    wilson_ctx *ctx;
    const wilson_gauge *G;
    SolveParams prm;
    int n;
    std::unique_ptr<EoCore> C;
    std::vector<Slot> slots;
    double delta;

    BatchEngine(wilson_ctx *c, const wilson_gauge *g, int nslots, const SolveParams &p)
        : ctx(c), G(g), prm(p), n(nslots), slots(nslots) {
        // a caller's workspace holds the batch's device buffers until the batch is destroyed
        C = std::make_unique<EoCore>(c, g, nslots, p.precision, p.method, p.workspace, p.workspace_bytes);
        C->prefin = prefin_enabled();
        C->kappa.assign(nslots, 0.0);
        delta = p.inner_tol > 0 ? p.inner_tol : (C->P == P32 ? 1e-5 : (C->P == P16 ? 1e-2 : 0.0));
        std::vector<RhsState> h(n);
        std::memset(h.data(), 0, sizeof(RhsState) * n);
        for (auto &s : h) s.phase = PH_IDLE;
        C->select_all();
        C->upload_states(C->sin(), h);
        C->upload_states(C->sout(), h);
        WL_HIP(hipStreamSynchronize(ctx->stream));
    }

    // start a Krylov cycle for slot k on rhs (inner precision) and solution x
    void start_inner(int k, Spinor rhs, Spinor x, bool use_x0, double stop2) {
        C->select(k, 1);
        std::vector<RhsState> h(1);
        std::memset(h.data(), 0, sizeof(RhsState));
        h[0].phase = PH_RUN;
        h[0].stop2 = stop2;
        C->upload_states(C->sin(), h);
        const int nb = blas_nblocks(C->g, C->P);
        Spinor none;
        if (C->method == WILSON_SOLVER_BICGSTAB_EO) {
            BlasArgs a = C->blas_args(C->sin(), PH_RUN);
            if (use_x0) {
                C->apply_M(C->r.f, x, C->tmp.f, false, RED_NONE, none, C->sin(), PH_RUN, &rhs);
                a.a = C->rh.f; a.b = C->r.f;
                C->run_blas(BL_COPY_NORM, a, 0);
            } else {
                a.a = C->r.f; a.b = rhs;
                C->run_blas(BL_COPY_NORM, a, 0);
                a.a = C->rh.f; a.b = rhs;
                C->run_blas(BL_COPY_NORM, a, 0);
            }
            C->finalize(FIN_BICG_INIT, 1, nb, C->sin(), PH_RUN);
            for (Spinor f : {C->p.f, C->v.f, C->t.f}) WL_HIP(launch_zero(C->V(f), C->g, 1, ctx->stream));
        } else {
            if (use_x0) {
                const int hb = C->apply_M(C->r.f, x, C->tmp.f, false, RED_NORM2, none, C->sin(), PH_RUN, &rhs);
                C->finalize(FIN_CG_R2, 1, hb, C->sin(), PH_RUN);
            } else {
                BlasArgs a = C->blas_args(C->sin(), PH_RUN);
                a.a = C->r.f; a.b = rhs;
                C->run_blas(BL_COPY_NORM, a, 0);
                C->finalize(FIN_CG_R2, 1, nb, C->sin(), PH_RUN);
            }
            const int hb = C->apply_M(C->s.f, C->r.f, C->tmp.f, true, RED_NORM2, none, C->sin(), PH_RUN);
            C->finalize(FIN_CG_ZZ, 1, hb, C->sin(), PH_RUN);
            BlasArgs a = C->blas_args(C->sin(), PH_RUN);
            a.a = C->p.f; a.b = C->s.f;
            C->run_blas(BL_COPY_NORM, a, 0);
        }
        C->select_all();
    }

    void begin_cycle(int k) {
        if (C->mixed) {
            C->select(k, 1);
            WL_HIP(launch_convert(C->V(C->rf.f), C->V(C->r64.f), C->g, 1, C->S(C->sout()), 1, ctx->stream));
            WL_HIP(launch_zero(C->V(C->xin.f), C->g, 1, ctx->stream));
            C->select_all();
            start_inner(k, C->rf.f, C->xin.f, false, delta * delta);
        } else {
            start_inner(k, C->bp.f, C->x_e.f, slots[k].restarts > 0, slots[k].stop2);
        }
    }

    // true residual of slot k: reconstruct x_o, |b - D x|^2 -> res2 (waits)
    double true_res2(int k) {
        C->select(k, 1);
        C->reconstruct();
        C->true_residual2();
        const double r2 = C->read_states(C->sout())[0].aux;
        C->select_all();
        return r2;
    }

    void finish(int k, int status) {
        Slot &s = slots[k];
        s.status = status;
        s.state = FINISHED;
        s.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s.t0).count();
        C->select(k, 1);
        std::vector<RhsState> h(1);
        std::memset(h.data(), 0, sizeof(RhsState));
        h[0].phase = PH_IDLE;
        C->upload_states(C->sin(), h);
        C->select_all();
    }

    int attach(int k, const double *b_dev, double kappa, double tol, int maxiter) {
        if (k < 0 || k >= n) throw Error(WILSON_INVALID_ARG, "slot out of range");
        Slot &s = slots[k];
        if (s.state != FREE) return WILSON_BUSY;
        s = Slot();
        s.kappa = kappa;
        s.tol = tol;
        s.maxiter = maxiter;
        s.t0 = std::chrono::steady_clock::now();
        C->kappa[k] = kappa;
        C->select(k, 1);
        WL_HIP(launch_to_parity(C->V(C->b_e.f), b_dev, C->g, 0, 1, 1.0, ctx->stream));
        WL_HIP(launch_to_parity(C->V(C->b_o.f), b_dev, C->g, 1, 1, 1.0, ctx->stream));
        C->norm2_full(C->b_e.f, C->b_o.f, C->sout());
        s.bn2 = C->read_states(C->sout())[0].aux;
        C->select_all();
        if (!std::isfinite(s.bn2)) {
            s.state = FINISHED;
            s.status = WILSON_NONFINITE;
            return WILSON_OK;
        }
        s.stop2 = tol * tol * s.bn2;
        s.state = RUNNING;
        C->select(k, 1);
        WL_HIP(launch_zero(C->V(C->x_e.f), C->g, 1, ctx->stream));
        C->prepare_bprime();
        if (C->mixed) {
            C->outer_residual();
            s.prev = C->read_states(C->sout())[0].aux;
        }
        C->select_all();
        if (s.bn2 == 0.0) {
            C->select(k, 1);
            C->reconstruct();
            C->select_all();
            s.res2 = 0.0;
            finish(k, WILSON_OK);
            return WILSON_OK;
        }
        begin_cycle(k);
        return WILSON_OK;
    }

    void step(int iters) {
        bool any = false;
        for (auto &s : slots) any |= s.state == RUNNING;
        if (!any) return;
        C->select_all();
        for (int it = 0; it < iters; it++) {
            if (C->method == WILSON_SOLVER_BICGSTAB_EO) C->bicg_iter(C->mixed ? C->xin.f : C->x_e.f, nullptr);
            else C->cg_iter(C->mixed ? C->xin.f : C->x_e.f, nullptr);
        }
    }

    // Advance the host-side state machine of every running slot whose inner cycle ended.
    void poll(int32_t *state, int32_t *status) {
        C->select_all();
        std::vector<RhsState> h = C->read_states(C->sin());
        for (int k = 0; k < n; k++) {
            Slot &s = slots[k];
            if (s.state != RUNNING) continue;
            const RhsState &st = h[k];
            const bool ended = st.phase == PH_DONE || st.phase == PH_FAIL || st.phase == PH_IDLE;
            const int used = s.iters + st.iter;
            if (!ended && used < s.maxiter) continue;
            s.iters += st.iter;
            if (st.phase == PH_FAIL && st.fail == FAIL_NONFINITE) {
                true_res2(k);
                finish(k, WILSON_NONFINITE);
                continue;
            }
            if (!C->mixed) {
                s.res2 = true_res2(k);
                if (s.res2 <= s.stop2) finish(k, WILSON_OK);
                else if (s.restarts >= prm.max_restarts || s.iters >= s.maxiter)
                    finish(k, st.phase == PH_FAIL ? WILSON_BREAKDOWN : WILSON_NOT_CONVERGED);
                else {
                    s.restarts++;
                    begin_cycle(k);
                }
                continue;
            }
            // mixed: fold the correction into x (FP64), new FP64 residual
            s.cycles++;
            C->select(k, 1);
            WL_HIP(launch_axpy_f64(C->V(C->x_e.f), C->V(C->xin.f), C->g, 1, C->S(C->sout()), 1, ctx->stream));
            C->outer_residual();
            const double r2 = C->read_states(C->sout())[0].aux;
            C->select_all();
            if (r2 > 0.25 * s.prev) s.stall++;
            s.prev = r2;
            if (!std::isfinite(r2)) {
                finish(k, WILSON_NONFINITE);
            } else if (r2 <= s.stop2) {
                s.res2 = true_res2(k);
                finish(k, s.res2 <= s.stop2 ? WILSON_OK : WILSON_NOT_CONVERGED);
            } else if (s.iters >= s.maxiter || s.stall >= 4) {
                s.res2 = true_res2(k);
                finish(k, WILSON_NOT_CONVERGED);
            } else {
                begin_cycle(k);
            }
        }
        for (int k = 0; k < n; k++) {
            state[k] = slots[k].state;
            status[k] = slots[k].status;
        }
    }

    int detach(int k, double *x_dev, wilson_solve_info *info) {
        if (k < 0 || k >= n) throw Error(WILSON_INVALID_ARG, "slot out of range");
        Slot &s = slots[k];
        if (s.state != FINISHED) return WILSON_BUSY;
        C->select(k, 1);
        WL_HIP(launch_from_parity(x_dev, C->V(C->x_e.f), C->g, 0, 1, ctx->stream));
        WL_HIP(launch_from_parity(x_dev, C->V(C->x_o.f), C->g, 1, 1, ctx->stream));
        C->select_all();
        if (info) {
            info->iterations = s.iters;
            info->outer_cycles = s.cycles;
            info->restarts = s.restarts;
            info->converged = s.status == WILSON_OK;
            info->true_residual = s.bn2 > 0 ? std::sqrt(s.res2 / s.bn2) : 0.0;
            info->ms = s.ms;
            info->hop_launches = 0;
            info->bytes = 0;
            info->flops = 0;
        }
        const int st = s.status;
        s.state = FREE;
        return st;
    }
};

BatchEngine *batch_create(wilson_ctx *ctx, const wilson_gauge *G, int nslots, const SolveParams &p) {
    return new BatchEngine(ctx, G, nslots, p);
}
void batch_destroy(BatchEngine *b) {
    (void)hipStreamSynchronize(b->ctx->stream);
    delete b;
}
int batch_attach(BatchEngine *b, int slot, const double *b_canon_dev, double kappa, double tol, int maxiter) {
    return b->attach(slot, b_canon_dev, kappa, tol, maxiter);
}
void batch_step(BatchEngine *b, int iters) { b->step(iters); }
void batch_poll(BatchEngine *b, int32_t *state, int32_t *status) { b->poll(state, status); }
int batch_detach(BatchEngine *b, int slot, double *x_canon_dev, wilson_solve_info *info) {
    return b->detach(slot, x_canon_dev, info);
}
wilson_ctx *batch_ctx(BatchEngine *b) { return b->ctx; }
size_t batch_spinor_bytes(BatchEngine *b) { return (size_t)b->C->g.Vh * 2 * 24 * sizeof(double); }

}  // namespace wl
