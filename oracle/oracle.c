/*
 * FP64 CPU oracle for the Wilson fermion matrix and its Krylov solvers.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes (Kanamori & Matsufuru, "Practical Implementation of Lattice
 * QCD Simulation on SIMD Machines with Intel AVX-512", Sec. 2):
 *
 *   D(x,y) = delta_{x,y} - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) delta_{x+mu,y}
 *                                         + (1 + gamma_mu) U_mu(x-mu)^dag delta_{x-mu,y} ]
 *
 * (Eq. (1), Sec. 2.1 "Wilson Fermion Matrix").  The bracketed sum is the
 * hopping term H, so D = 1 - kappa*H.  The operator is written out literally:
 * the 3x3 link multiplies every spin component, then the dense 4x4 spin matrix
 * (1 -/+ gamma_mu) is applied.  No spin projection, no checkerboard storage,
 * no blocking.
 *
 * Conventions (readings of the paper where it is silent):
 *   - 0-based coordinates, x fastest: site s = x + Lx*(y + Ly*(z + Lz*t));
 *     mu = 0..3 <-> x, y, z, t (the paper numbers them 1..4 with t fourth).
 *   - spinor element (s, spin, colour) at complex offset (s*4 + spin)*3 + colour.
 *   - link U_mu(s)[a][b] at complex offset ((s*4 + mu)*3 + a)*3 + b.
 *   - gamma matrices in the Dirac basis (gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 *     gamma_4 = diag(1,1,-1,-1)); Eq. (1) only says "a 4x4 matrix".
 *   - boundaries periodic in x, y, z and antiperiodic in t (Sec. 2.1 allows
 *     either).  The sign -1 multiplies a hop exactly when it is a t-hop that
 *     crosses the t = Lt-1 <-> 0 wrap, in both directions.  The link array
 *     passed in is periodic; the sign is applied here, at the hop.
 *   - extents of 2: x+mu and x-mu are the same site and both terms are added.
 *
 * Build: gcc -O2 -fopenmp -fcx-limited-range -shared -fPIC (see build.py).
 * -fcx-limited-range only drops the NaN/Inf recovery of complex multiply.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* gamma[0..3] = gamma_1..gamma_4 (x, y, z, t), gamma[4] = gamma_5 = g1 g2 g3 g4 */
static cplx GAMMA[5][4][4];

static void matmul4(cplx c[4][4], cplx a[4][4], cplx b[4][4]) {
    cplx r[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx acc = 0;
            for (int k = 0; k < 4; k++) acc += a[i][k] * b[k][j];
            r[i][j] = acc;
        }
    memcpy(c, r, sizeof r);
}

__attribute__((constructor)) static void oracle_init_gamma(void) {
    /* Pauli matrices sigma_1, sigma_2, sigma_3 */
    cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAMMA, 0, sizeof GAMMA);
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                GAMMA[k][a][2 + b] = -I * sig[k][a][b]; /* upper-right block: -i sigma_k */
                GAMMA[k][2 + a][b] = I * sig[k][a][b];  /* lower-left block:  +i sigma_k */
            }
    GAMMA[3][0][0] = 1;
    GAMMA[3][1][1] = 1;
    GAMMA[3][2][2] = -1;
    GAMMA[3][3][3] = -1;
    matmul4(GAMMA[4], GAMMA[0], GAMMA[1]);
    matmul4(GAMMA[4], GAMMA[4], GAMMA[2]);
    matmul4(GAMMA[4], GAMMA[4], GAMMA[3]);
}

/* Copy of the gamma matrix table, for tests (idx 0..3 = gamma_1..4, 4 = gamma_5). */
void oracle_gamma(int idx, double *out32) {
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            out32[2 * (a * 4 + b)] = creal(GAMMA[idx][a][b]);
            out32[2 * (a * 4 + b) + 1] = cimag(GAMMA[idx][a][b]);
        }
}

static inline long site_index(const int c[4], const int L[4]) {
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static inline void site_coords(long s, const int L[4], int c[4]) {
    c[0] = (int)(s % L[0]); s /= L[0];
    c[1] = (int)(s % L[1]); s /= L[1];
    c[2] = (int)(s % L[2]); s /= L[2];
    c[3] = (int)s;
}

static inline long volume(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

/* (H psi)(s) for one site s, written to res[4][3]. */
static void hop_at_site(cplx res[4][3], const cplx *psi, const cplx *U, const int L[4], long s) {
    int c[4];
    site_coords(s, L, c);
    memset(res, 0, sizeof(cplx) * 12);
    for (int mu = 0; mu < 4; mu++) {
        /* forward neighbour x+mu and its boundary sign */
        int cf[4] = {c[0], c[1], c[2], c[3]};
        cf[mu] = (c[mu] + 1) % L[mu];
        double sgn_f = (mu == 3 && c[3] == L[3] - 1) ? -1.0 : 1.0;
        long sf = site_index(cf, L);
        /* backward neighbour x-mu and its boundary sign */
        int cb[4] = {c[0], c[1], c[2], c[3]};
        cb[mu] = (c[mu] + L[mu] - 1) % L[mu];
        double sgn_b = (mu == 3 && c[3] == 0) ? -1.0 : 1.0;
        long sb = site_index(cb, L);

        /* forward: (1 - gamma_mu) (x) U_mu(x) psi(x+mu) */
        const cplx *Uf = U + (s * 4 + mu) * 9;
        cplx w[4][3];
        for (int sp = 0; sp < 4; sp++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int b = 0; b < 3; b++) acc += Uf[a * 3 + b] * psi[(sf * 4 + sp) * 3 + b];
                w[sp][a] = acc;
            }
        for (int sp = 0; sp < 4; sp++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int sq = 0; sq < 4; sq++) {
                    cplx m = (sp == sq ? 1.0 : 0.0) - GAMMA[mu][sp][sq];
                    acc += m * w[sq][a];
                }
                res[sp][a] += sgn_f * acc;
            }

        /* backward: (1 + gamma_mu) (x) U_mu(x-mu)^dagger psi(x-mu) */
        const cplx *Ub = U + (sb * 4 + mu) * 9;
        for (int sp = 0; sp < 4; sp++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int b = 0; b < 3; b++) acc += conj(Ub[b * 3 + a]) * psi[(sb * 4 + sp) * 3 + b];
                w[sp][a] = acc;
            }
        for (int sp = 0; sp < 4; sp++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int sq = 0; sq < 4; sq++) {
                    cplx m = (sp == sq ? 1.0 : 0.0) + GAMMA[mu][sp][sq];
                    acc += m * w[sq][a];
                }
                res[sp][a] += sgn_b * acc;
            }
    }
}

static inline int site_parity(long s, const int L[4]) {
    int c[4];
    site_coords(s, L, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/*
 * out(s) = alpha*(H psi)(s) + beta*y(s) on every site s whose parity is in
 * `which` (0 even, 1 odd, 2 both); other sites of out are left untouched.
 * y may be NULL (treated as zero).  out must not alias psi.
 */
static void hop_axpy(cplx *out, const cplx *psi, const cplx *U, const int L[4], int which, cplx alpha,
                     const cplx *y, cplx beta) {
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        if (which != 2 && site_parity(s, L) != which) continue;
        cplx res[4][3];
        hop_at_site(res, psi, U, L, s);
        for (int k = 0; k < 12; k++) {
            cplx v = alpha * ((cplx *)res)[k];
            if (y) v += beta * y[s * 12 + k];
            out[s * 12 + k] = v;
        }
    }
}

/* (H psi) on all sites: Eq. (1)'s bracketed sum. */
void oracle_hop(double *out, const double *psi, const double *U, const int32_t dims[4]) {
    int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    hop_axpy((cplx *)out, (const cplx *)psi, (const cplx *)U, L, 2, 1.0, NULL, 0.0);
}

/* D psi = psi - kappa H psi on all sites (Eq. (1)). */
void oracle_apply_D(double *out, const double *psi, const double *U, double kappa, const int32_t dims[4]) {
    int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    hop_axpy((cplx *)out, (const cplx *)psi, (const cplx *)U, L, 2, -kappa, (const cplx *)psi, 1.0);
}

/*
 * Library-call semantics of the Dslash entry point.
 *   parity p in {0,1}: out = -kappa * H psi on parity-p sites only; parity-(1-p)
 *                      sites of out keep their previous contents.  H maps
 *                      parity 1-p to parity p, so psi is read only there.
 *   parity 2:          out = D psi on every site.
 */
void oracle_dslash(double *out, const double *psi, const double *U, double kappa, const int32_t dims[4],
                   int32_t parity) {
    int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    if (parity == 2)
        hop_axpy((cplx *)out, (const cplx *)psi, (const cplx *)U, L, 2, -kappa, (const cplx *)psi, 1.0);
    else
        hop_axpy((cplx *)out, (const cplx *)psi, (const cplx *)U, L, parity, -kappa, NULL, 0.0);
}

/* (H psi) evaluated at a list of sites only: out[i*24 ..] for sites[i]. */
void oracle_hop_sites(double *out, const double *psi, const double *U, const int32_t dims[4], const int64_t *sites,
                      int64_t n) {
    int L[4] = {dims[0], dims[1], dims[2], dims[3]};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        cplx res[4][3];
        hop_at_site(res, (const cplx *)psi, (const cplx *)U, L, sites[i]);
        memcpy(out + i * 24, res, sizeof res);
    }
}

/* out = gamma_5 psi, site by site (dense 4x4). */
void oracle_gamma5(double *out, const double *psi, int64_t V) {
    const cplx *p = (const cplx *)psi;
    cplx *o = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; s++) {
        cplx r[4][3];
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) {
                cplx acc = 0;
                for (int b = 0; b < 4; b++) acc += GAMMA[4][a][b] * p[(s * 4 + b) * 3 + c];
                r[a][c] = acc;
            }
        memcpy(o + s * 12, r, sizeof r);
    }
}

/* ------------------------------------------------------------------------- */
/* Even-odd (Schur complement) form.  D = [[1, -k H_eo], [-k H_oe, 1]] in     */
/* (even, odd) blocks, so with M_ee = 1 - k^2 H_eo H_oe:                      */
/*     b'_e = b_e + k H_eo b_o,   M_ee x_e = b'_e,   x_o = b_o + k H_oe x_e.  */
/* Vectors are full-lattice arrays; "even-supported" means odd sites are 0.  */
/* ------------------------------------------------------------------------- */

typedef struct {
    const cplx *U;
    int L[4];
    double kappa;
    cplx *tmp; /* full-lattice scratch */
    int dagger; /* apply M_ee^dagger = gamma5 M_ee gamma5 instead */
} eo_ctx;

static void zero_parity(cplx *v, const int L[4], int p) {
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++)
        if (site_parity(s, L) == p) memset(v + s * 12, 0, sizeof(cplx) * 12);
}

/* out_e = M_ee in_e (odd sites of out set to 0).  in must be even-supported. */
static void apply_Mee(cplx *out, const cplx *in, eo_ctx *c) {
    long V = volume(c->L);
    /* tmp_o = H_oe in_e */
    memset(c->tmp, 0, sizeof(cplx) * 12 * V);
    hop_axpy(c->tmp, in, c->U, c->L, 1, 1.0, NULL, 0.0);
    /* out_e = in_e - k^2 H_eo tmp_o */
    hop_axpy(out, c->tmp, c->U, c->L, 0, -c->kappa * c->kappa, in, 1.0);
    zero_parity(out, c->L, 1);
}

static void apply_Mee_dagger(cplx *out, const cplx *in, eo_ctx *c) {
    long V = volume(c->L);
    cplx *g = malloc(sizeof(cplx) * 12 * V);
    oracle_gamma5((double *)g, (const double *)in, V);
    apply_Mee(out, g, c);
    oracle_gamma5((double *)g, (const double *)out, V);
    memcpy(out, g, sizeof(cplx) * 12 * V);
    free(g);
}

void oracle_eo_prepare(double *bprime, const double *b, const double *U, double kappa, const int32_t dims[4]) {
    int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    long V = volume(L);
    memset(bprime, 0, sizeof(cplx) * 12 * V);
    /* b'_e = b_e + k H_eo b_o  (H at even sites reads only odd sites of b) */
    hop_axpy((cplx *)bprime, (const cplx *)b, (const cplx *)U, L, 0, kappa, (const cplx *)b, 1.0);
}

void oracle_eo_reconstruct(double *x, const double *b, const double *U, double kappa, const int32_t dims[4]) {
    /* x holds x_e on even sites; writes x_o = b_o + k H_oe x_e on odd sites */
    int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    long V = volume(L);
    cplx *xe = malloc(sizeof(cplx) * 12 * V);
    memcpy(xe, x, sizeof(cplx) * 12 * V);
    zero_parity(xe, L, 1);
    hop_axpy((cplx *)x, xe, (const cplx *)U, L, 1, kappa, (const cplx *)b, 1.0);
    free(xe);
}

void oracle_apply_Mee(double *out, const double *in, const double *U, double kappa, const int32_t dims[4],
                      int32_t dagger) {
    eo_ctx c;
    c.U = (const cplx *)U;
    memcpy(c.L, dims, sizeof c.L);
    c.kappa = kappa;
    c.tmp = malloc(sizeof(cplx) * 12 * volume(c.L));
    c.dagger = dagger;
    long V = volume(c.L);
    cplx *ine = malloc(sizeof(cplx) * 12 * V);
    memcpy(ine, in, sizeof(cplx) * 12 * V);
    zero_parity(ine, c.L, 1);
    if (dagger)
        apply_Mee_dagger((cplx *)out, ine, &c);
    else
        apply_Mee((cplx *)out, ine, &c);
    free(ine);
    free(c.tmp);
}

/* ------------------------------------------------------------------------- */
/* Krylov solvers on a generic operator.                                      */
/* ------------------------------------------------------------------------- */

typedef void (*op_fn)(cplx *out, const cplx *in, void *ctx);

static cplx dotc(const cplx *a, const cplx *b, long n) { /* <a,b> = sum conj(a) b */
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; i++) {
        cplx v = conj(a[i]) * b[i];
        re += creal(v);
        im += cimag(v);
    }
    return re + I * im;
}

static double norm2(const cplx *a, long n) { return creal(dotc(a, a, n)); }

/*
 * BiCGStab (van der Vorst 1992; the paper names the algorithm in Sec. 2 but
 * does not print it), in its textbook order:
 *   x0 = 0 (or the given guess), r = b - A x0, rhat = r, rho = alpha = omega = 1, v = p = 0;
 *   loop: rho' = <rhat,r>; beta = (rho'/rho)(alpha/omega); p = r + beta (p - omega v);
 *         v = A p; alpha = rho'/<rhat,v>; s = r - alpha v;
 *         if |s| <= tol*bnorm: x += alpha p, stop;
 *         t = A s; omega = <t,s>/<t,t>; x += alpha p + omega s; r = s - omega t;
 *         stop if |r| <= tol*bnorm; rho = rho'.
 * Returns the number of iterations, or -1 if maxiter was reached, -2 on breakdown.
 */
static int bicgstab(cplx *x, const cplx *b, long n, op_fn A, void *ctx, double tol, double bnorm, int maxiter,
                    double *res_out) {
    cplx *r = calloc(n, sizeof(cplx)), *rh = calloc(n, sizeof(cplx)), *p = calloc(n, sizeof(cplx));
    cplx *v = calloc(n, sizeof(cplx)), *s = calloc(n, sizeof(cplx)), *t = calloc(n, sizeof(cplx));
    A(r, x, ctx);
    for (long i = 0; i < n; i++) r[i] = b[i] - r[i];
    memcpy(rh, r, sizeof(cplx) * n);
    cplx rho = 1, alpha = 1, omega = 1;
    int it = 0, ret = -1;
    double rn = sqrt(norm2(r, n));
    if (rn <= tol * bnorm) {
        ret = 0;
        goto done;
    }
    for (it = 1; it <= maxiter; it++) {
        cplx rho1 = dotc(rh, r, n);
        if (cabs(rho1) == 0.0) { ret = -2; break; }
        cplx beta = (rho1 / rho) * (alpha / omega);
        for (long i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        A(v, p, ctx);
        cplx rv = dotc(rh, v, n);
        if (cabs(rv) == 0.0) { ret = -2; break; }
        alpha = rho1 / rv;
        for (long i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
        double sn = sqrt(norm2(s, n));
        if (sn <= tol * bnorm) {
            for (long i = 0; i < n; i++) x[i] += alpha * p[i];
            rn = sn;
            ret = it;
            break;
        }
        A(t, s, ctx);
        double tt = norm2(t, n);
        omega = dotc(t, s, n) / tt;
        for (long i = 0; i < n; i++) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rn = sqrt(norm2(r, n));
        rho = rho1;
        if (rn <= tol * bnorm) { ret = it; break; }
    }
done:
    if (res_out) *res_out = rn;
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return ret;
}

/*
 * CG on the normal equations in its CGLS form (Hestenes-Stiefel):
 *   r = b - A x; z = A^dag r; p = z;
 *   loop: w = A p; alpha = |z|^2/|w|^2; x += alpha p; r -= alpha w;
 *         stop if |r| <= tol*bnorm; z' = A^dag r; beta = |z'|^2/|z|^2; p = z' + beta p.
 */
static int cgls(cplx *x, const cplx *b, long n, op_fn A, op_fn Adag, void *ctx, double tol, double bnorm,
                int maxiter, double *res_out) {
    cplx *r = calloc(n, sizeof(cplx)), *z = calloc(n, sizeof(cplx)), *p = calloc(n, sizeof(cplx));
    cplx *w = calloc(n, sizeof(cplx));
    A(r, x, ctx);
    for (long i = 0; i < n; i++) r[i] = b[i] - r[i];
    double rn = sqrt(norm2(r, n));
    int ret = -1, it = 0;
    if (rn <= tol * bnorm) { ret = 0; goto done; }
    Adag(z, r, ctx);
    memcpy(p, z, sizeof(cplx) * n);
    double zz = norm2(z, n);
    for (it = 1; it <= maxiter; it++) {
        A(w, p, ctx);
        double ww = norm2(w, n);
        if (ww == 0.0) { ret = -2; break; }
        double alpha = zz / ww;
        for (long i = 0; i < n; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * w[i];
        }
        rn = sqrt(norm2(r, n));
        if (rn <= tol * bnorm) { ret = it; break; }
        Adag(z, r, ctx);
        double zz1 = norm2(z, n);
        double beta = zz1 / zz;
        zz = zz1;
        for (long i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    }
done:
    if (res_out) *res_out = rn;
    free(r); free(z); free(p); free(w);
    return ret;
}

static void op_D(cplx *out, const cplx *in, void *vctx) {
    eo_ctx *c = vctx;
    hop_axpy(out, in, c->U, c->L, 2, -c->kappa, in, 1.0);
}
static void op_Mee(cplx *out, const cplx *in, void *vctx) { apply_Mee(out, in, vctx); }
static void op_Mee_dag(cplx *out, const cplx *in, void *vctx) { apply_Mee_dagger(out, in, vctx); }

/*
 * Solve D x = b.
 *   method 0: BiCGStab on the full D.
 *   method 1: even-odd BiCGStab on M_ee, then reconstruct x_o.
 *   method 2: even-odd CGLS (CG on M_ee^dag M_ee), then reconstruct x_o.
 * Stops on the iterated residual |r| <= tol*|b| with |b| of the full system,
 * x starts from the contents of x (pass zeros for x0 = 0).  Returns iterations
 * (>= 0), -1 not converged, -2 breakdown.  *true_res gets |b - D x| / |b|.
 */
int oracle_solve(double *x, const double *b, const double *U, double kappa, const int32_t dims[4], double tol,
                 int32_t maxiter, int32_t method, double *true_res) {
    eo_ctx c;
    c.U = (const cplx *)U;
    memcpy(c.L, dims, sizeof c.L);
    c.kappa = kappa;
    long V = volume(c.L);
    long n = 12 * V;
    c.tmp = malloc(sizeof(cplx) * n);
    c.dagger = 0;
    const cplx *bb = (const cplx *)b;
    cplx *xx = (cplx *)x;
    double bnorm = sqrt(norm2(bb, n));
    int ret;
    double res;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        if (true_res) *true_res = 0.0;
        free(c.tmp);
        return 0;
    }
    if (method == 0) {
        ret = bicgstab(xx, bb, n, op_D, &c, tol, bnorm, maxiter, &res);
    } else {
        cplx *bp = malloc(sizeof(cplx) * n);
        oracle_eo_prepare((double *)bp, b, U, kappa, dims);
        zero_parity(xx, c.L, 1);
        if (method == 1)
            ret = bicgstab(xx, bp, n, op_Mee, &c, tol, bnorm, maxiter, &res);
        else
            ret = cgls(xx, bp, n, op_Mee, op_Mee_dag, &c, tol, bnorm, maxiter, &res);
        oracle_eo_reconstruct(x, b, U, kappa, dims);
        free(bp);
    }
    if (true_res) {
        cplx *r = malloc(sizeof(cplx) * n);
        op_D(r, xx, &c);
        for (long i = 0; i < n; i++) r[i] = bb[i] - r[i];
        *true_res = sqrt(norm2(r, n)) / bnorm;
        free(r);
    }
    free(c.tmp);
    return ret;
}

/*
 * Run exactly `iters` BiCGStab iterations of method 0/1 from x = 0 with no
 * stopping test (tol = 0): used to time a bounded sample of a solve.
 */
int oracle_bicgstab_fixed(double *x, const double *b, const double *U, double kappa, const int32_t dims[4],
                          int32_t iters, int32_t method) {
    double tr;
    return oracle_solve(x, b, U, kappa, dims, 0.0, iters, method, &tr);
}

/* ------------------------------------------------------------------------- */
/* Clover fermion matrix (Sec. 2.1.2):  D_clov = D_W + F(x) delta_{x,y},        */
/* F(x) a Hermitian 12x12 site matrix made of link variables and stored as an  */
/* array like U; the paper does not give its construction, so F is an input:   */
/* F[s][a][b], a, b = 3*spin + colour (Dirac basis), complex.  With            */
/* T(x) = 1 + F(x) the site-diagonal block, D_clov psi = T psi - kappa H psi.  */
/* Even-odd: D_clov = [[T_ee, -k H_eo], [-k H_oe, T_oo]] gives                 */
/*   M_ee = T_ee - k^2 H_eo T_oo^-1 H_oe,  b'_e = b_e + k H_eo T_oo^-1 b_o,     */
/*   x_o = T_oo^-1 (b_o + k H_oe x_e).                                          */
/* Written literally: dense 12x12 products and a dense inverse per site.      */
/* ------------------------------------------------------------------------- */

/* out = M v for a dense 12x12 M (row-major) and a 12-vector v. */
static void mat12_vec(cplx *out, const cplx *M, const cplx *v) {
    for (int a = 0; a < 12; a++) {
        cplx acc = 0;
        for (int b = 0; b < 12; b++) acc += M[a * 12 + b] * v[b];
        out[a] = acc;
    }
}

/* Inverse of a 12x12 complex matrix by Gauss-Jordan elimination with partial
   pivoting.  Returns 0, or -1 if a pivot is zero. */
static int mat12_inverse(cplx *inv, const cplx *M) {
    cplx a[12][24];
    for (int r = 0; r < 12; r++)
        for (int c = 0; c < 24; c++) a[r][c] = c < 12 ? M[r * 12 + c] : (c - 12 == r ? 1.0 : 0.0);
    for (int col = 0; col < 12; col++) {
        int piv = col;
        for (int r = col + 1; r < 12; r++)
            if (cabs(a[r][col]) > cabs(a[piv][col])) piv = r;
        if (cabs(a[piv][col]) == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < 24; c++) {
                cplx t = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = t;
            }
        cplx d = a[col][col];
        for (int c = 0; c < 24; c++) a[col][c] /= d;
        for (int r = 0; r < 12; r++) {
            if (r == col) continue;
            cplx f = a[r][col];
            if (f == 0) continue;
            for (int c = 0; c < 24; c++) a[r][c] -= f * a[col][c];
        }
    }
    for (int r = 0; r < 12; r++)
        for (int c = 0; c < 12; c++) inv[r * 12 + c] = a[r][12 + c];
    return 0;
}

/* Tinv[s] = (1 + F[s])^-1 on every site.  Returns -1 if some T is singular. */
int oracle_clover_inverse(double *Tinv, const double *F, int64_t V) {
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long s = 0; s < V; s++) {
        cplx T[144];
        const cplx *f = (const cplx *)F + s * 144;
        for (int k = 0; k < 144; k++) T[k] = f[k] + ((k / 12 == k % 12) ? 1.0 : 0.0);
        bad |= mat12_inverse((cplx *)Tinv + s * 144, T) != 0;
    }
    return bad ? -1 : 0;
}

/* out(s) = M(s) in(s) on sites of parity `which` (2: all); M = T (inv = 0), with
   T = 1 + F, or the given inverses (inv = 1, M = Tinv).  out may alias in. */
static void site_apply(cplx *out, const cplx *in, const cplx *F, const cplx *Tinv, int inv, const int L[4],
                       int which) {
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        if (which != 2 && site_parity(s, L) != which) continue;
        cplx v[12], r[12];
        memcpy(v, in + s * 12, sizeof v);
        if (inv) {
            mat12_vec(r, Tinv + s * 144, v);
        } else {
            mat12_vec(r, F + s * 144, v);
            for (int k = 0; k < 12; k++) r[k] += v[k];
        }
        memcpy(out + s * 12, r, sizeof r);
    }
}

/* D_clov psi = (1 + F) psi - kappa H psi on all sites. */
void oracle_apply_Dclov(double *out, const double *psi, const double *U, const double *F, double kappa,
                        const int32_t dims[4]) {
    int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    long V = volume(L);
    cplx *tp = malloc(sizeof(cplx) * 12 * V);
    site_apply(tp, (const cplx *)psi, (const cplx *)F, NULL, 0, L, 2);
    hop_axpy((cplx *)out, (const cplx *)psi, (const cplx *)U, L, 2, -kappa, tp, 1.0);
    free(tp);
}

typedef struct {
    const cplx *U, *F, *Tinv;
    int L[4];
    double kappa;
    cplx *tmp, *tmp2;
} clov_ctx;

/* out_e = M_ee in_e = T_ee in_e - k^2 H_eo T_oo^-1 H_oe in_e (odd sites of out = 0). */
static void apply_Mee_clov(cplx *out, const cplx *in, clov_ctx *c) {
    long V = volume(c->L);
    memset(c->tmp, 0, sizeof(cplx) * 12 * V);
    hop_axpy(c->tmp, in, c->U, c->L, 1, 1.0, NULL, 0.0);          /* H_oe in_e */
    site_apply(c->tmp, c->tmp, c->F, c->Tinv, 1, c->L, 1);          /* T_oo^-1 */
    memset(c->tmp2, 0, sizeof(cplx) * 12 * V);
    site_apply(c->tmp2, in, c->F, NULL, 0, c->L, 0);                /* T_ee in_e */
    hop_axpy(out, c->tmp, c->U, c->L, 0, -c->kappa * c->kappa, c->tmp2, 1.0);
    zero_parity(out, c->L, 1);
}

/* M_ee^dag = gamma5 M_ee gamma5, valid when F commutes with gamma5 (F block diagonal
   in the chiral basis, as the inputs are built). */
static void apply_Mee_clov_dagger(cplx *out, const cplx *in, clov_ctx *c) {
    long V = volume(c->L);
    cplx *g = malloc(sizeof(cplx) * 12 * V);
    oracle_gamma5((double *)g, (const double *)in, V);
    apply_Mee_clov(out, g, c);
    oracle_gamma5((double *)g, (const double *)out, V);
    memcpy(out, g, sizeof(cplx) * 12 * V);
    free(g);
}

static void clov_prepare(cplx *bp, const cplx *b, clov_ctx *c) {
    long V = volume(c->L);
    memset(c->tmp, 0, sizeof(cplx) * 12 * V);
    site_apply(c->tmp, b, c->F, c->Tinv, 1, c->L, 1);                 /* T_oo^-1 b_o */
    memset(bp, 0, sizeof(cplx) * 12 * V);
    hop_axpy(bp, c->tmp, c->U, c->L, 0, c->kappa, b, 1.0);            /* b_e + k H_eo (.) */
}

static void clov_reconstruct(cplx *x, const cplx *b, clov_ctx *c) {
    long V = volume(c->L);
    cplx *xe = malloc(sizeof(cplx) * 12 * V);
    memcpy(xe, x, sizeof(cplx) * 12 * V);
    zero_parity(xe, c->L, 1);
    hop_axpy(x, xe, c->U, c->L, 1, c->kappa, b, 1.0);                 /* b_o + k H_oe x_e */
    site_apply(x, x, c->F, c->Tinv, 1, c->L, 1);                      /* T_oo^-1 */
    free(xe);
}

static int clov_ctx_init(clov_ctx *c, const double *U, const double *F, double kappa, const int32_t dims[4]) {
    c->U = (const cplx *)U;
    c->F = (const cplx *)F;
    memcpy(c->L, dims, sizeof c->L);
    c->kappa = kappa;
    long V = volume(c->L);
    c->tmp = malloc(sizeof(cplx) * 12 * V);
    c->tmp2 = malloc(sizeof(cplx) * 12 * V);
    cplx *ti = malloc(sizeof(cplx) * 144 * V);
    c->Tinv = ti;
    return oracle_clover_inverse((double *)ti, F, V);
}

static void clov_ctx_free(clov_ctx *c) {
    free(c->tmp);
    free(c->tmp2);
    free((void *)c->Tinv);
}

void oracle_clov_eo_prepare(double *bprime, const double *b, const double *U, const double *F, double kappa,
                            const int32_t dims[4]) {
    clov_ctx c;
    clov_ctx_init(&c, U, F, kappa, dims);
    clov_prepare((cplx *)bprime, (const cplx *)b, &c);
    clov_ctx_free(&c);
}

void oracle_clov_eo_reconstruct(double *x, const double *b, const double *U, const double *F, double kappa,
                                const int32_t dims[4]) {
    clov_ctx c;
    clov_ctx_init(&c, U, F, kappa, dims);
    clov_reconstruct((cplx *)x, (const cplx *)b, &c);
    clov_ctx_free(&c);
}

void oracle_apply_Mee_clov(double *out, const double *in, const double *U, const double *F, double kappa,
                           const int32_t dims[4], int32_t dagger) {
    clov_ctx c;
    clov_ctx_init(&c, U, F, kappa, dims);
    long V = volume(c.L);
    cplx *ine = malloc(sizeof(cplx) * 12 * V);
    memcpy(ine, in, sizeof(cplx) * 12 * V);
    zero_parity(ine, c.L, 1);
    if (dagger)
        apply_Mee_clov_dagger((cplx *)out, ine, &c);
    else
        apply_Mee_clov((cplx *)out, ine, &c);
    free(ine);
    clov_ctx_free(&c);
}

static void op_Dclov(cplx *out, const cplx *in, void *vctx) {
    clov_ctx *c = vctx;
    long V = volume(c->L);
    site_apply(c->tmp2, in, c->F, NULL, 0, c->L, 2);
    hop_axpy(out, in, c->U, c->L, 2, -c->kappa, c->tmp2, 1.0);
    (void)V;
}
static void op_Mee_clov(cplx *out, const cplx *in, void *vctx) { apply_Mee_clov(out, in, vctx); }
static void op_Mee_clov_dag(cplx *out, const cplx *in, void *vctx) { apply_Mee_clov_dagger(out, in, vctx); }

/* Solve D_clov x = b; methods and return values as oracle_solve.  Returns -3 if
   some site matrix 1 + F is singular. */
int oracle_solve_clov(double *x, const double *b, const double *U, const double *F, double kappa,
                      const int32_t dims[4], double tol, int32_t maxiter, int32_t method, double *true_res) {
    clov_ctx c;
    if (clov_ctx_init(&c, U, F, kappa, dims) != 0) {
        clov_ctx_free(&c);
        return -3;
    }
    long V = volume(c.L);
    long n = 12 * V;
    const cplx *bb = (const cplx *)b;
    cplx *xx = (cplx *)x;
    double bnorm = sqrt(norm2(bb, n));
    int ret;
    double res;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        if (true_res) *true_res = 0.0;
        clov_ctx_free(&c);
        return 0;
    }
    if (method == 0) {
        ret = bicgstab(xx, bb, n, op_Dclov, &c, tol, bnorm, maxiter, &res);
    } else {
        cplx *bp = malloc(sizeof(cplx) * n);
        clov_prepare(bp, bb, &c);
        zero_parity(xx, c.L, 1);
        if (method == 1)
            ret = bicgstab(xx, bp, n, op_Mee_clov, &c, tol, bnorm, maxiter, &res);
        else
            ret = cgls(xx, bp, n, op_Mee_clov, op_Mee_clov_dag, &c, tol, bnorm, maxiter, &res);
        clov_reconstruct(xx, bb, &c);
        free(bp);
    }
    if (true_res) {
        cplx *r = malloc(sizeof(cplx) * n);
        op_Dclov(r, xx, &c);
        for (long i = 0; i < n; i++) r[i] = bb[i] - r[i];
        *true_res = sqrt(norm2(r, n)) / bnorm;
        free(r);
    }
    clov_ctx_free(&c);
    return ret;
}

/* |a - b| relative helpers for tests */
double oracle_norm(const double *a, int64_t n_complex) { return sqrt(norm2((const cplx *)a, n_complex)); }

/* Host memory triad a = b + s*c over n doubles, `reps` times; returns seconds. */
#include <omp.h>
double oracle_triad(int64_t n, int32_t reps) {
    double *a = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) { a[i] = 0; b[i] = 1; c[i] = 2; }
    double t0 = omp_get_wtime();
    for (int r = 0; r < reps; r++) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) a[i] = b[i] + 0.5 * c[i];
    }
    double t1 = omp_get_wtime();
    volatile double sink = a[n / 2];
    (void)sink;
    free(a); free(b); free(c);
    return t1 - t0;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }

/* OpenMP threads of later calls (for timing).  The operators write disjoint sites and do
   not depend on it; the solver's OpenMP dot products may round differently. */
void oracle_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
