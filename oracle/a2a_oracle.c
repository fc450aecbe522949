/*
 * a2a_oracle.c -- plain FP64 CPU oracle for the stochastic all-to-all propagator path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls
 * this file; it is loaded by the test-suite, by the smoke check and by the benchmark's
 * CPU-baseline leg, and it shares no code, header or table with the HIP kernels.
 *
 * Everything is the plain definition, written with std C99 complex doubles on the
 * canonical lexicographic layout, one site at a time, no blocking or fusion:
 *
 *   site index      s = ((t*Z + z)*Y + y)*X + x        (x fastest)
 *   links  U        [site][mu][row][col]  complex, mu = 0..3 <-> x, y, z, t
 *   spinor psi      [site][spin][colour]   complex
 *
 * Conventions (the paper never writes the operator; these are the readings used
 * throughout, stated once here):
 *   gamma basis     chiral, Hermitian:  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
 *                   gamma_4 = [[0, 1], [1, 0]];  gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4.
 *   hopping         (H psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                       + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *                   with the fermion time boundary sign t_bc on hops that wrap in t.
 *   clover          F_munu(x) = (Q_munu(x) - Q_munu(x)^dag) / 8, Q the sum of the four
 *                   plaquette leaves around x in the (mu,nu) plane, counter-clockwise;
 *                   A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_munu (x) F_munu(x),
 *                   sigma_munu = (i/2)[gamma_mu, gamma_nu].
 *   Dirac operator  D = A - kappa H   (Wilson-clover in the hopping-parameter form; the
 *                   paper's "lattice fermion matrix", Sec. 7, with c_SW as in Sec. 8).
 *
 * Sec. 7 (eq. of the stochastic estimator) needs X_i = D^{-1} eta_i; the oracle solves
 * the full (un-preconditioned) system with textbook BiCGStab (van der Vorst 1992) and
 * restarts from the current iterate until the true residual ||eta - D X|| / ||eta||
 * meets the tolerance; CG on the normal equations (CGNR) is the alternative solver.  The
 * even-odd Schur operator is provided as its plain definition
 * (full-lattice operators restricted to a parity) so the GPU's Schur kernels can be
 * checked against it.
 *
 * Sec. 7 (eq. stoop): O_ij(t) = sum_{y in t} eta_i(y)^dag gamma_5 X_j(y) and the pion
 * correlator C(t - t0) from sum_ij O_ij(t) O_ji(t0).  Sec. 5 / Sec. 8 diagrams 0-3 at
 * zero momentum are built from blocks of O with independent noise groups (Sec. 7: one
 * independent noise set per propagator).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cx;

typedef struct {
    int L[4]; /* X, Y, Z, T */
    long V;
    int tbc;
} geom_t;

static int geom_init(geom_t *g, const int *dims, int tbc)
{
    g->V = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 1) return -1;
        g->L[m] = dims[m];
        g->V *= dims[m];
    }
    g->tbc = tbc;
    return 0;
}

static void coords(const geom_t *g, long s, int c[4])
{
    for (int m = 0; m < 4; ++m) {
        c[m] = (int)(s % g->L[m]);
        s /= g->L[m];
    }
}

static long index_of(const geom_t *g, const int c[4])
{
    return ((long)((long)c[3] * g->L[2] + c[2]) * g->L[1] + c[1]) * g->L[0] + c[0];
}

/* site x + dir * mu-hat, periodic; *wrap_t is set when the step crosses the t boundary */
static long shift(const geom_t *g, long s, int mu, int dir, int *wrap_t)
{
    int c[4];
    coords(g, s, c);
    int v = c[mu] + dir;
    int w = 0;
    if (v >= g->L[mu]) { v -= g->L[mu]; w = 1; }
    if (v < 0) { v += g->L[mu]; w = 1; }
    c[mu] = v;
    if (wrap_t) *wrap_t = (mu == 3) && w;
    return index_of(g, c);
}

static int parity_of(const geom_t *g, long s)
{
    int c[4];
    coords(g, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* ------------------------------------------------------------------------------------ */
/* gamma matrices                                                                        */
/* ------------------------------------------------------------------------------------ */
static cx GAM[4][4][4];  /* gamma_mu[row][col], mu = 0..3 <-> x, y, z, t */
static cx GAM5[4][4];
static cx SIG[4][4][4][4]; /* sigma_munu[row][col] */
static int gamma_ready = 0;

static void mat4_mul(cx a[4][4], cx b[4][4], cx out[4][4])
{
    cx t[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cx acc = 0;
            for (int k = 0; k < 4; ++k) acc += a[i][k] * b[k][j];
            t[i][j] = acc;
        }
    memcpy(out, t, sizeof(t));
}

static void gamma_init(void)
{
    if (gamma_ready) return;
    /* Pauli matrices */
    cx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAM, 0, sizeof(GAM));
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                GAM[k][i][2 + j] = -I * pauli[k][i][j];
                GAM[k][2 + i][j] = I * pauli[k][i][j];
            }
    for (int i = 0; i < 2; ++i) {
        GAM[3][i][2 + i] = 1;
        GAM[3][2 + i][i] = 1;
    }
    cx t[4][4];
    mat4_mul(GAM[0], GAM[1], t);
    mat4_mul(t, GAM[2], t);
    mat4_mul(t, GAM[3], GAM5);
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            cx ab[4][4], ba[4][4];
            mat4_mul(GAM[m], GAM[n], ab);
            mat4_mul(GAM[n], GAM[m], ba);
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) SIG[m][n][i][j] = 0.5 * I * (ab[i][j] - ba[i][j]);
        }
    gamma_ready = 1;
}

/* ------------------------------------------------------------------------------------ */
/* SU(3) helpers                                                                          */
/* ------------------------------------------------------------------------------------ */
typedef struct { cx m[3][3]; } m3;

static m3 m3_mul(m3 a, m3 b)
{
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cx acc = 0;
            for (int k = 0; k < 3; ++k) acc += a.m[i][k] * b.m[k][j];
            r.m[i][j] = acc;
        }
    return r;
}

static m3 m3_dag(m3 a)
{
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.m[i][j] = conj(a.m[j][i]);
    return r;
}

static m3 link(const cx *U, long s, int mu)
{
    m3 r;
    memcpy(r.m, U + ((size_t)s * 4 + mu) * 9, sizeof(r.m));
    return r;
}

/* ------------------------------------------------------------------------------------ */
/* public: gamma matrices (for tests)                                                     */
/* ------------------------------------------------------------------------------------ */
int orc_gamma(int mu, double *out /* 4x4 complex; mu = 0..3, 4 = gamma_5 */)
{
    gamma_init();
    if (mu < 0 || mu > 4) return -1;
    cx *o = (cx *)out;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) o[i * 4 + j] = (mu == 4) ? GAM5[i][j] : GAM[mu][i][j];
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* hopping term, full lattice                                                             */
/* ------------------------------------------------------------------------------------ */
static void hop_site(const geom_t *g, const cx *U, const cx *in, long s, cx out[12])
{
    for (int k = 0; k < 12; ++k) out[k] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        /* forward: (1 - gamma_mu) U_mu(x) psi(x + mu) */
        int wf;
        long sf = shift(g, s, mu, +1, &wf);
        double phf = wf ? (double)g->tbc : 1.0;
        m3 u = link(U, s, mu);
        cx up[4][3];
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                cx acc = 0;
                for (int b = 0; b < 3; ++b) acc += u.m[a][b] * in[(size_t)sf * 12 + sp * 3 + b];
                up[sp][a] = acc;
            }
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                cx acc = 0;
                for (int sq = 0; sq < 4; ++sq) acc += ((sp == sq ? 1.0 : 0.0) - GAM[mu][sp][sq]) * up[sq][a];
                out[sp * 3 + a] += phf * acc;
            }
        /* backward: (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) */
        int wb;
        long sb = shift(g, s, mu, -1, &wb);
        double phb = wb ? (double)g->tbc : 1.0;
        m3 ud = m3_dag(link(U, sb, mu));
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                cx acc = 0;
                for (int b = 0; b < 3; ++b) acc += ud.m[a][b] * in[(size_t)sb * 12 + sp * 3 + b];
                up[sp][a] = acc;
            }
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                cx acc = 0;
                for (int sq = 0; sq < 4; ++sq) acc += ((sp == sq ? 1.0 : 0.0) + GAM[mu][sp][sq]) * up[sq][a];
                out[sp * 3 + a] += phb * acc;
            }
    }
}

static void hop(const geom_t *g, const cx *U, const cx *in, cx *out)
{
    gamma_init();
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g->V; ++s) hop_site(g, U, in, s, out + (size_t)s * 12);
}

int orc_hop(const int *dims, int tbc, const double *U, const double *in, double *out)
{
    geom_t g;
    if (geom_init(&g, dims, tbc)) return -1;
    hop(&g, (const cx *)U, (const cx *)in, (cx *)out);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* clover                                                                                 */
/* ------------------------------------------------------------------------------------ */
/* F_munu(x) for mu < nu, planes ordered (01, 02, 03, 12, 13, 23) */
static void field_strength_site(const geom_t *g, const cx *U, long x, int mu, int nu, m3 *F)
{
    long xpm = shift(g, x, mu, +1, NULL);
    long xpn = shift(g, x, nu, +1, NULL);
    long xmm = shift(g, x, mu, -1, NULL);
    long xmn = shift(g, x, nu, -1, NULL);
    long xmm_pn = shift(g, xmm, nu, +1, NULL);
    long xmm_mn = shift(g, xmm, nu, -1, NULL);
    long xmn_pm = shift(g, xmn, mu, +1, NULL);

    m3 l1 = m3_mul(m3_mul(link(U, x, mu), link(U, xpm, nu)), m3_mul(m3_dag(link(U, xpn, mu)), m3_dag(link(U, x, nu))));
    m3 l2 = m3_mul(m3_mul(link(U, x, nu), m3_dag(link(U, xmm_pn, mu))), m3_mul(m3_dag(link(U, xmm, nu)), link(U, xmm, mu)));
    m3 l3 = m3_mul(m3_mul(m3_dag(link(U, xmm, mu)), m3_dag(link(U, xmm_mn, nu))), m3_mul(link(U, xmm_mn, mu), link(U, xmn, nu)));
    m3 l4 = m3_mul(m3_mul(m3_dag(link(U, xmn, nu)), link(U, xmn, mu)), m3_mul(link(U, xmn_pm, nu), m3_dag(link(U, x, mu))));
    m3 q;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) q.m[i][j] = l1.m[i][j] + l2.m[i][j] + l3.m[i][j] + l4.m[i][j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F->m[i][j] = (q.m[i][j] - conj(q.m[j][i])) / 8.0;
}

int orc_field_strength(const int *dims, const double *U, double *F /* [V][6][3][3] complex */)
{
    geom_t g;
    if (geom_init(&g, dims, 1)) return -1;
    const cx *u = (const cx *)U;
    cx *f = (cx *)F;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < g.V; ++x) {
        int p = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu, ++p) {
                m3 Fm;
                field_strength_site(&g, u, x, mu, nu, &Fm);
                memcpy(f + ((size_t)x * 6 + p) * 9, Fm.m, sizeof(Fm.m));
            }
    }
    return 0;
}

/* A(x) as a dense 12x12 matrix, index (spin*3 + colour) */
int orc_clover(const int *dims, const double *U, double kappa, double csw, double *A /* [V][12][12] complex */)
{
    geom_t g;
    if (geom_init(&g, dims, 1)) return -1;
    gamma_init();
    const cx *u = (const cx *)U;
    cx *a = (cx *)A;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < g.V; ++x) {
        cx *ax = a + (size_t)x * 144;
        for (int i = 0; i < 144; ++i) ax[i] = 0;
        for (int i = 0; i < 12; ++i) ax[i * 12 + i] = 1;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                m3 F;
                field_strength_site(&g, u, x, mu, nu, &F);
                for (int s1 = 0; s1 < 4; ++s1)
                    for (int s2 = 0; s2 < 4; ++s2) {
                        cx sg = SIG[mu][nu][s1][s2];
                        if (sg == 0) continue;
                        for (int c1 = 0; c1 < 3; ++c1)
                            for (int c2 = 0; c2 < 3; ++c2)
                                ax[(s1 * 3 + c1) * 12 + s2 * 3 + c2] += I * kappa * csw * sg * F.m[c1][c2];
                    }
            }
    }
    return 0;
}

/* per-site inverse of a dense 12x12 matrix: Gauss-Jordan elimination, partial pivoting */
static int inv12(const cx *m, cx *out)
{
    cx a[12][24];
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
            a[i][j] = m[i * 12 + j];
            a[i][12 + j] = (i == j) ? 1 : 0;
        }
    for (int c = 0; c < 12; ++c) {
        int piv = c;
        for (int r = c + 1; r < 12; ++r)
            if (cabs(a[r][c]) > cabs(a[piv][c])) piv = r;
        if (cabs(a[piv][c]) == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < 24; ++j) {
                cx t = a[c][j];
                a[c][j] = a[piv][j];
                a[piv][j] = t;
            }
        cx d = 1.0 / a[c][c];
        for (int j = 0; j < 24; ++j) a[c][j] *= d;
        for (int r = 0; r < 12; ++r) {
            if (r == c) continue;
            cx f = a[r][c];
            if (f == 0) continue;
            for (int j = 0; j < 24; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) out[i * 12 + j] = a[i][12 + j];
    return 0;
}

int orc_invert_sites(long n, const double *A, double *Ainv)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long x = 0; x < n; ++x)
        bad |= inv12((const cx *)A + (size_t)x * 144, (cx *)Ainv + (size_t)x * 144) ? 1 : 0;
    return bad ? -2 : 0;
}

static void site_matvec(const cx *A, const cx *in, cx *out, long V)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        const cx *a = A + (size_t)x * 144;
        for (int i = 0; i < 12; ++i) {
            cx acc = 0;
            for (int j = 0; j < 12; ++j) acc += a[i * 12 + j] * in[(size_t)x * 12 + j];
            out[(size_t)x * 12 + i] = acc;
        }
    }
}

int orc_site_matvec(long V, const double *A, const double *in, double *out)
{
    site_matvec((const cx *)A, (const cx *)in, (cx *)out, V);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* full operator D = A - kappa H                                                          */
/* ------------------------------------------------------------------------------------ */
static void apply_D(const geom_t *g, const cx *U, const cx *A, double kappa, const cx *in, cx *out, cx *tmp)
{
    hop(g, U, in, tmp);
    site_matvec(A, in, out, g->V);
    size_t n = (size_t)g->V * 12;
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) out[i] -= kappa * tmp[i];
}

int orc_apply_D(const int *dims, int tbc, const double *U, const double *A, double kappa, const double *in,
                double *out)
{
    geom_t g;
    if (geom_init(&g, dims, tbc)) return -1;
    cx *tmp = malloc(sizeof(cx) * 12 * (size_t)g.V);
    if (!tmp) return -3;
    apply_D(&g, (const cx *)U, (const cx *)A, kappa, (const cx *)in, (cx *)out, tmp);
    free(tmp);
    return 0;
}

/* Schur complement on the odd sites, plain definition with full-lattice vectors:
 *   out_o = A_oo x_o - kappa^2 H_oe A_ee^{-1} H_eo x_o, out_e = 0.
 * `in` is read on odd sites only. */
int orc_schur(const int *dims, int tbc, const double *U, const double *A, const double *Ainv, double kappa,
              const double *in, double *out)
{
    geom_t g;
    if (geom_init(&g, dims, tbc)) return -1;
    size_t n = (size_t)g.V * 12;
    cx *xo = calloc(n, sizeof(cx)), *t1 = malloc(n * sizeof(cx)), *t2 = malloc(n * sizeof(cx));
    cx *o = (cx *)out;
    const cx *x = (const cx *)in;
    if (!xo || !t1 || !t2) return -3;
    for (long s = 0; s < g.V; ++s)
        if (parity_of(&g, s) == 1) memcpy(xo + s * 12, x + s * 12, 12 * sizeof(cx));
    hop(&g, (const cx *)U, xo, t1); /* H x_o, keep even part */
    for (long s = 0; s < g.V; ++s)
        if (parity_of(&g, s) == 1) memset(t1 + s * 12, 0, 12 * sizeof(cx));
    site_matvec((const cx *)Ainv, t1, t2, g.V); /* A_ee^{-1} (.)_e */
    hop(&g, (const cx *)U, t2, t1);            /* H_oe (.) */
    site_matvec((const cx *)A, xo, o, g.V);     /* A_oo x_o */
    for (long s = 0; s < g.V; ++s) {
        if (parity_of(&g, s) == 1)
            for (int k = 0; k < 12; ++k) o[s * 12 + k] -= kappa * kappa * t1[s * 12 + k];
        else
            memset(o + s * 12, 0, 12 * sizeof(cx));
    }
    free(xo);
    free(t1);
    free(t2);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* solver: BiCGStab on the full D with true-residual restarts                            */
/* ------------------------------------------------------------------------------------ */
static cx dotc(const cx *a, const cx *b, size_t n) /* sum conj(a) b, sequential order */
{
    cx acc = 0;
    for (size_t i = 0; i < n; ++i) acc += conj(a[i]) * b[i];
    return acc;
}

static double norm2(const cx *a, size_t n)
{
    double acc = 0;
    for (size_t i = 0; i < n; ++i) acc += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return acc;
}

typedef struct {
    int iters;
    int restarts;
    int converged;
    double true_rel_residual;
} orc_info;

static int solve_one(const geom_t *g, const cx *U, const cx *A, double kappa, const cx *b, cx *x, double tol,
                     int maxit, orc_info *info)
{
    size_t n = (size_t)g->V * 12;
    cx *r = malloc(n * sizeof(cx)), *rh = malloc(n * sizeof(cx)), *p = malloc(n * sizeof(cx)),
       *v = malloc(n * sizeof(cx)), *s = malloc(n * sizeof(cx)), *t = malloc(n * sizeof(cx)),
       *tmp = malloc(n * sizeof(cx));
    if (!r || !rh || !p || !v || !s || !t || !tmp) return -3;
    double bn = sqrt(norm2(b, n));
    info->iters = 0;
    info->restarts = 0;
    info->converged = 0;
    memset(x, 0, n * sizeof(cx));
    if (bn == 0.0) {
        info->converged = 1;
        info->true_rel_residual = 0.0;
        goto done;
    }
    for (;;) {
        /* true residual */
        apply_D(g, U, A, kappa, x, r, tmp);
        for (size_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double rn = sqrt(norm2(r, n));
        info->true_rel_residual = rn / bn;
        if (rn <= tol * bn) {
            info->converged = 1;
            break;
        }
        if (info->iters >= maxit || info->restarts > 50) break;
        info->restarts++;
        memcpy(rh, r, n * sizeof(cx));
        memset(p, 0, n * sizeof(cx));
        memset(v, 0, n * sizeof(cx));
        cx rho_prev = 1, alpha = 1, omega = 1;
        double target = 0.5 * tol * bn;
        while (info->iters < maxit) {
            cx rho = dotc(rh, r, n);
            if (cabs(rho) == 0.0) break;
            cx beta = (rho / rho_prev) * (alpha / omega);
            for (size_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            apply_D(g, U, A, kappa, p, v, tmp);
            cx rv = dotc(rh, v, n);
            if (cabs(rv) == 0.0) break;
            alpha = rho / rv;
            for (size_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
            info->iters++;
            if (sqrt(norm2(s, n)) <= target) {
                for (size_t i = 0; i < n; ++i) x[i] += alpha * p[i];
                break;
            }
            apply_D(g, U, A, kappa, s, t, tmp);
            double tt = norm2(t, n);
            if (tt == 0.0) break;
            omega = dotc(t, s, n) / tt;
            for (size_t i = 0; i < n; ++i) {
                x[i] += alpha * p[i] + omega * s[i];
                r[i] = s[i] - omega * t[i];
            }
            rho_prev = rho;
            if (sqrt(norm2(r, n)) <= target) break;
            if (cabs(omega) == 0.0) break;
        }
    }
done:
    free(r); free(rh); free(p); free(v); free(s); free(t); free(tmp);
    return info->converged ? 0 : 1;
}

/* Solve D X_i = eta_i for nrhs sources; info is [nrhs][4] doubles
 * (iterations, restarts, converged, true relative residual).  Returns the number of
 * unconverged sources (0 on success) or a negative error. */
int orc_solve(const int *dims, int tbc, const double *U, const double *A, double kappa, int nrhs,
              const double *eta, double *X, double tol, int maxit, double *info)
{
    geom_t g;
    if (geom_init(&g, dims, tbc)) return -1;
    gamma_init();
    size_t n = (size_t)g.V * 12;
    int bad = 0;
    for (int i = 0; i < nrhs; ++i) {
        orc_info inf;
        int rc = solve_one(&g, (const cx *)U, (const cx *)A, kappa, (const cx *)eta + i * n, (cx *)X + i * n, tol,
                           maxit, &inf);
        if (rc < 0) return rc;
        bad += rc;
        if (info) {
            info[i * 4 + 0] = inf.iters;
            info[i * 4 + 1] = inf.restarts;
            info[i * 4 + 2] = inf.converged;
            info[i * 4 + 3] = inf.true_rel_residual;
        }
    }
    return bad;
}

/* Run exactly `iters` BiCGStab iterations on one source from x = 0 (no restarts) and
 * report the iterated relative residual after each; used to time a bounded sample. */
int orc_bicgstab_fixed(const int *dims, int tbc, const double *U, const double *A, double kappa,
                       const double *eta, double *X, int iters, double *resid_hist)
{
    geom_t g;
    if (geom_init(&g, dims, tbc)) return -1;
    gamma_init();
    size_t n = (size_t)g.V * 12;
    const cx *b = (const cx *)eta;
    cx *x = (cx *)X;
    cx *r = malloc(n * sizeof(cx)), *rh = malloc(n * sizeof(cx)), *p = calloc(n, sizeof(cx)),
       *v = calloc(n, sizeof(cx)), *s = malloc(n * sizeof(cx)), *t = malloc(n * sizeof(cx)),
       *tmp = malloc(n * sizeof(cx));
    if (!r || !rh || !p || !v || !s || !t || !tmp) return -3;
    double bn = sqrt(norm2(b, n));
    memset(x, 0, n * sizeof(cx));
    memcpy(r, b, n * sizeof(cx));
    memcpy(rh, b, n * sizeof(cx));
    cx rho_prev = 1, alpha = 1, omega = 1;
    for (int it = 0; it < iters; ++it) {
        cx rho = dotc(rh, r, n);
        cx beta = (rho / rho_prev) * (alpha / omega);
        for (size_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        apply_D(&g, (const cx *)U, (const cx *)A, kappa, p, v, tmp);
        alpha = rho / dotc(rh, v, n);
        for (size_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        apply_D(&g, (const cx *)U, (const cx *)A, kappa, s, t, tmp);
        omega = dotc(t, s, n) / norm2(t, n);
        for (size_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rho_prev = rho;
        if (resid_hist) resid_hist[it] = sqrt(norm2(r, n)) / bn;
    }
    free(r); free(rh); free(p); free(v); free(s); free(t); free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* solver: CG on the normal equations                                                    */
/* ------------------------------------------------------------------------------------ */
/* gamma_5 applied to every site of a spinor field, from the matrix built in gamma_init */
static void apply_g5(const geom_t *g, const cx *in, cx *out)
{
    for (long s = 0; s < g->V; ++s)
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) {
                cx acc = 0;
                for (int b = 0; b < 4; ++b) acc += GAM5[a][b] * in[s * 12 + b * 3 + c];
                out[s * 12 + a * 3 + c] = acc;
            }
}

/* D^dag in = gamma_5 D gamma_5 in.  That D is gamma_5-hermitian is itself a checked
 * property of the operator (the dense D against its conjugate transpose). */
static void apply_Ddag(const geom_t *g, const cx *U, const cx *A, double kappa, const cx *in, cx *out, cx *tmp,
                       cx *tmp2)
{
    apply_g5(g, in, tmp2);
    apply_D(g, U, A, kappa, tmp2, out, tmp);
    apply_g5(g, out, tmp2);
    memcpy(out, tmp2, sizeof(cx) * 12 * (size_t)g->V);
}

/* CG applied to D^dag D x = D^dag b, in the form that carries the residual r = b - D x of
 * the original system (CGNR; Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
 * Sec. 8.3):
 *   r = b - D x,  z = D^dag r,  p = z
 *   repeat:  w = D p;  alpha = |z|^2 / |w|^2;  x += alpha p;  r -= alpha w;
 *            z' = D^dag r;  beta = |z'|^2 / |z|^2;  p = z' + beta p
 * `iters` steps from the given x (no restart); returns the iterations taken, stopping
 * early when |r| <= target. */
static int cgnr_steps(const geom_t *g, const cx *U, const cx *A, double kappa, const cx *b, cx *x, int iters,
                      double target, double *resid_hist, double bn)
{
    size_t n = (size_t)g->V * 12;
    cx *r = malloc(n * sizeof(cx)), *z = malloc(n * sizeof(cx)), *p = malloc(n * sizeof(cx)),
       *w = malloc(n * sizeof(cx)), *tmp = malloc(n * sizeof(cx)), *tmp2 = malloc(n * sizeof(cx));
    if (!r || !z || !p || !w || !tmp || !tmp2) return -3;
    apply_D(g, U, A, kappa, x, r, tmp);
    for (size_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    apply_Ddag(g, U, A, kappa, r, z, tmp, tmp2);
    memcpy(p, z, n * sizeof(cx));
    double zz = norm2(z, n);
    int it = 0;
    while (it < iters && zz > 0.0) {
        apply_D(g, U, A, kappa, p, w, tmp);
        double ww = norm2(w, n);
        if (ww == 0.0) break;
        double alpha = zz / ww;
        for (size_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * w[i];
        }
        ++it;
        double rn = sqrt(norm2(r, n));
        if (resid_hist) resid_hist[it - 1] = rn / bn;
        if (rn <= target) break;
        apply_Ddag(g, U, A, kappa, r, z, tmp, tmp2);
        double zz_new = norm2(z, n);
        double beta = zz_new / zz;
        for (size_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        zz = zz_new;
    }
    free(r); free(z); free(p); free(w); free(tmp); free(tmp2);
    return it;
}

/* X_i = D^{-1} eta_i by CGNR, restarted from the current iterate on the true residual
 * until ||eta - D X|| <= tol ||eta||; info as for orc_solve. */
int orc_solve_cgnr(const int *dims, int tbc, const double *U, const double *A, double kappa, int nrhs,
                   const double *eta, double *X, double tol, int maxit, double *info)
{
    geom_t g;
    if (geom_init(&g, dims, tbc)) return -1;
    gamma_init();
    size_t n = (size_t)g.V * 12;
    cx *tmp = malloc(n * sizeof(cx)), *r = malloc(n * sizeof(cx));
    if (!tmp || !r) return -3;
    int bad = 0;
    for (int i = 0; i < nrhs; ++i) {
        const cx *b = (const cx *)eta + i * n;
        cx *x = (cx *)X + i * n;
        memset(x, 0, n * sizeof(cx));
        double bn = sqrt(norm2(b, n)), rel = 0.0;
        int iters = 0, restarts = 0, conv = 0;
        for (;;) {
            apply_D(&g, (const cx *)U, (const cx *)A, kappa, x, r, tmp);
            for (size_t k = 0; k < n; ++k) r[k] = b[k] - r[k];
            rel = bn > 0 ? sqrt(norm2(r, n)) / bn : 0.0;
            if (rel <= tol) {
                conv = 1;
                break;
            }
            if (iters >= maxit || restarts > 50) break;
            ++restarts;
            int k = cgnr_steps(&g, (const cx *)U, (const cx *)A, kappa, b, x, maxit - iters, 0.5 * tol * bn, NULL, bn);
            if (k < 0) return k;
            iters += k;
        }
        bad += !conv;
        if (info) {
            info[i * 4 + 0] = iters;
            info[i * 4 + 1] = restarts;
            info[i * 4 + 2] = conv;
            info[i * 4 + 3] = rel;
        }
    }
    free(tmp);
    free(r);
    return bad;
}

/* Exactly `iters` CGNR steps on one source from x = 0; the relative residual after each
 * goes to resid_hist. */
int orc_cgnr_fixed(const int *dims, int tbc, const double *U, const double *A, double kappa, const double *eta,
                   double *X, int iters, double *resid_hist)
{
    geom_t g;
    if (geom_init(&g, dims, tbc)) return -1;
    gamma_init();
    size_t n = (size_t)g.V * 12;
    memset(X, 0, n * sizeof(cx));
    double bn = sqrt(norm2((const cx *)eta, n));
    int k = cgnr_steps(&g, (const cx *)U, (const cx *)A, kappa, (const cx *)eta, (cx *)X, iters, -1.0, resid_hist, bn);
    return k < 0 ? k : 0;
}

/* ------------------------------------------------------------------------------------ */
/* contractions                                                                           */
/* ------------------------------------------------------------------------------------ */
/* O[t][a][b] = sum_{y in timeslice t} sum_{s,s',c} conj(eta_a(y,s,c)) gamma5[s][s'] X_b(y,s',c) */
int orc_stochastic_operators(const int *dims, int nrhs, const double *eta, const double *X, double *O)
{
    geom_t g;
    if (geom_init(&g, dims, 1)) return -1;
    gamma_init();
    const cx *e = (const cx *)eta, *x = (const cx *)X;
    cx *o = (cx *)O;
    int T = g.L[3];
    long V3 = g.V / T;
    size_t n = (size_t)g.V * 12;
#pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < T; ++t)
        for (int a = 0; a < nrhs; ++a)
            for (int b = 0; b < nrhs; ++b) {
                cx acc = 0;
                for (long y = (long)t * V3; y < (long)(t + 1) * V3; ++y)
                    for (int s = 0; s < 4; ++s)
                        for (int sp = 0; sp < 4; ++sp) {
                            if (GAM5[s][sp] == 0) continue;
                            for (int c = 0; c < 3; ++c)
                                acc += conj(e[a * n + y * 12 + s * 3 + c]) * GAM5[s][sp] * x[b * n + y * 12 + sp * 3 + c];
                        }
                o[((size_t)t * nrhs + a) * nrhs + b] = acc;
            }
    return 0;
}

/* Pion correlator from the stochastic operators.
 *   mode 0 (unbiased): C(dt) = 1/(T N (N-1)) sum_t0 sum_{a != b} O_ab(t0+dt) O_ba(t0)
 *   mode 1 (all pairs, as printed in Sec. 7): C(dt) = 1/(T N^2) sum_t0 sum_{a,b} ...
 *   mode 2 (raw sum over a != b, no normalisation)
 *   mode 3 (raw sum over all a, b, no normalisation) */
int orc_pion_from_O(int T, int nrhs, const double *O, int mode, double *corr)
{
    const cx *o = (const cx *)O;
    cx *c = (cx *)corr;
    int N = nrhs;
    for (int dt = 0; dt < T; ++dt) {
        cx acc = 0;
        for (int t0 = 0; t0 < T; ++t0) {
            int t1 = (t0 + dt) % T;
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) {
                    if ((mode == 0 || mode == 2) && a == b) continue;
                    acc += o[((size_t)t1 * N + a) * N + b] * o[((size_t)t0 * N + b) * N + a];
                }
        }
        double norm = 1.0;
        if (mode == 0) norm = (double)T * N * (N - 1);
        if (mode == 1) norm = (double)T * N * N;
        c[dt] = acc / norm;
    }
    return 0;
}

int orc_contract_pion(const int *dims, int nrhs, const double *eta, const double *X, int mode, double *corr,
                      double *O_or_null)
{
    if (nrhs < 1 || (mode == 0 && nrhs < 2)) return -1;
    int T = dims[3];
    double *O = O_or_null ? O_or_null : malloc(sizeof(cx) * (size_t)T * nrhs * nrhs);
    if (!O) return -3;
    int rc = orc_stochastic_operators(dims, nrhs, eta, X, O);
    if (!rc) rc = orc_pion_from_O(T, nrhs, O, mode, corr);
    if (!O_or_null) free(O);
    return rc;
}

/* pi-pi zero-momentum pieces from four disjoint noise groups g1..g4 of n = N/4 sources.
 * B^{gh}(t) is the n x n block of O with rows in group g and columns in group h.
 *   L^{gh}(t1, t2) = tr[B^{gh}(t1) B^{hg}(t2)] / n^2           (one pion line, two noise sets)
 *   D0(dt) = 1/T sum_t0 L^{12}(t0+dt, t0) L^{34}(t0+dt, t0)     (direct)
 *   D1(dt) = 1/T sum_t0 L^{12}(t0+dt, t0+dt) L^{34}(t0, t0)     (vacuum, unsubtracted)
 *   D2(dt) = 1/T sum_t0 tr[B^{12}(t0) B^{23}(t1) B^{34}(t1) B^{41}(t0)] / n^4,  t1 = t0+dt
 *   D3(dt) = 1/T sum_t0 tr[B^{12}(t1) B^{23}(t1) B^{34}(t0) B^{41}(t0)] / n^4
 *   vac(t) = L^{12}(t, t)
 * With normalise = 0 the 1/n^2, 1/n^4 and 1/T factors are dropped (raw sums). */
static cx Oblk(const cx *o, int N, int n, int t, int g, int h, int i, int j)
{
    return o[((size_t)t * N + g * n + i) * N + h * n + j];
}

static cx loop2(const cx *o, int N, int n, int g, int h, int t1, int t2)
{
    cx acc = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) acc += Oblk(o, N, n, t1, g, h, i, j) * Oblk(o, N, n, t2, h, g, j, i);
    return acc;
}

static cx loop4(const cx *o, int N, int n, int ta, int tb, int tc, int td)
{
    /* tr[B^{12}(ta) B^{23}(tb) B^{34}(tc) B^{41}(td)]: two plain matrix products, then the trace */
    cx *m1 = malloc(sizeof(cx) * (size_t)n * n), *m2 = malloc(sizeof(cx) * (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            cx acc = 0;
            for (int j = 0; j < n; ++j) acc += Oblk(o, N, n, ta, 0, 1, i, j) * Oblk(o, N, n, tb, 1, 2, j, k);
            m1[i * n + k] = acc;
        }
    for (int i = 0; i < n; ++i)
        for (int l = 0; l < n; ++l) {
            cx acc = 0;
            for (int k = 0; k < n; ++k) acc += m1[i * n + k] * Oblk(o, N, n, tc, 2, 3, k, l);
            m2[i * n + l] = acc;
        }
    cx acc = 0;
    for (int i = 0; i < n; ++i)
        for (int l = 0; l < n; ++l) acc += m2[i * n + l] * Oblk(o, N, n, td, 3, 0, l, i);
    free(m1);
    free(m2);
    return acc;
}

int orc_pipi_from_O(int T, int nrhs, const double *O, int normalise, double *diagrams /* [4][T] */,
                    double *vac /* [T] */)
{
    if (nrhs < 4 || nrhs % 4) return -1;
    const cx *o = (const cx *)O;
    int N = nrhs, n = N / 4;
    cx *d = (cx *)diagrams, *v = (cx *)vac;
    double n2 = normalise ? (double)n * n : 1.0, n4 = n2 * n2, nt = normalise ? (double)T : 1.0;
    for (int dt = 0; dt < T; ++dt) {
        cx d0 = 0, d1 = 0, d2 = 0, d3 = 0;
        for (int t0 = 0; t0 < T; ++t0) {
            int t1 = (t0 + dt) % T;
            d0 += (loop2(o, N, n, 0, 1, t1, t0) / n2) * (loop2(o, N, n, 2, 3, t1, t0) / n2);
            d1 += (loop2(o, N, n, 0, 1, t1, t1) / n2) * (loop2(o, N, n, 2, 3, t0, t0) / n2);
            d2 += loop4(o, N, n, t0, t1, t1, t0) / n4;
            d3 += loop4(o, N, n, t1, t1, t0, t0) / n4;
        }
        d[0 * T + dt] = d0 / nt;
        d[1 * T + dt] = d1 / nt;
        d[2 * T + dt] = d2 / nt;
        d[3 * T + dt] = d3 / nt;
    }
    if (v)
        for (int t = 0; t < T; ++t) v[t] = loop2(o, N, n, 0, 1, t, t) / n2;
    return 0;
}

int orc_contract_pipi(const int *dims, int nrhs, const double *eta, const double *X, double *diagrams, double *vac)
{
    if (nrhs < 4 || nrhs % 4) return -1;
    int T = dims[3];
    double *O = malloc(sizeof(cx) * (size_t)T * nrhs * nrhs);
    if (!O) return -3;
    int rc = orc_stochastic_operators(dims, nrhs, eta, X, O);
    if (!rc) rc = orc_pipi_from_O(T, nrhs, O, 1, diagrams, vac);
    free(O);
    return rc;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops that follow (n >= 1); for timing the oracle on one core. */
int orc_set_num_threads(int n)
{
    if (n < 1) return -1;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return 0;
}
