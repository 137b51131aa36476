/*
 * mdx_oracle.c -- plain, slow, CPU reference for McMurchie-Davidson (MD)
 * electron-repulsion integrals over contracted Gaussian shells.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * never links, loads or calls it, and the two share no code or tables.
 *
 * It follows Asadchev & Valeev, "Implementation of McMurchie-Davidson
 * algorithm for Gaussian AO integrals suited for SIMD processors"
 * (arXiv:2506.12501), Section 2.1, in the paper's order:
 *
 *   Eq. (1)/(5)      primitive / contracted Cartesian Gaussians
 *   Eqs. (10),(11)   E recursion for a product of two Gaussians, bootstrapped
 *                    by Eq. (14); zero outside 0 <= t <= a+b.  The parity
 *                    clause printed in Eq. (15) is NOT applied: it is false
 *                    for two distinct centres (E^0_{10} = X_PA E^0_{00} != 0).
 *   Eqs. (27),(28)   [0]^(m) from the Boys function
 *   Eq. (31)         Hermite recursion [r+1_i]^(m) -> [r]^(0)
 *   Eq. (25)         [p|q] = (-1)^{l_q} [p+q]^(0)
 *   Eqs. (32),(33)   ket transform, then bra transform (here with the plain
 *                    Cartesian E matrices in place of H)
 *   Eqs. (24),(26),(30),(34)  1-particle Coulomb integrals of point charges,
 *                    transformed charge by charge (no early summation)
 *   Eq. (8)          overlap; kinetic energy from the same 1-D overlaps
 *   Eq. (5) / Sec. 2.1 text: primitives are accumulated into contracted ints
 *   Eqs. (18),(19)   Cartesian -> real solid harmonics, with the coefficient
 *                    C^a_{lm} built from the closed-form expansion of the
 *                    real solid harmonics (Schlegel & Frisch; Helgaker,
 *                    Jorgensen & Olsen ch. 6.4), Racah normalisation
 *                    (each solid harmonic has the norm of x^l).
 *
 * Boys function (Eq. (28)): for x <= 50 the all-positive Kummer series
 *   F_m(x) = exp(-x) sum_k (2x)^k / ((2m+1)(2m+3)...(2m+2k+1)),
 * which is exact term by term from the definition; for x > 50
 *   F_0 = sqrt(pi/(4x)) erf(sqrt x)   (Sec. 3.2.1; the factor 1/2 missing
 * from the printed Eq. (41) restored) and the upward recursion of Eq. (42),
 * keeping the exp(-x) term.
 *
 * 3-centre (X|cd) and 2-centre (a|c) integrals (Eq. (4)) use a unit s shell
 * (exponent 0, coefficient 1, same centre) as the missing partner, which the
 * 2-centre E recursion handles exactly (P = A, zeta_p = zeta_a).
 *
 * Gradients differentiate Eq. (1) directly:
 *   d/dA_i phi_a = 2 zeta_a phi_{a+1_i} - a_i phi_{a-1_i}
 * for each of the four centres (no translational-invariance shortcut).
 *
 * Conventions (shared with the library's public header, but not its code):
 *   Cartesian order within a shell: (l,0,0),(l-1,1,0),(l-1,0,1),(l-2,2,0),...
 *   Solid order m = -l..l.  Coefficients are applied as given (no
 *   normalisation).  Atomic units.
 *   Dense output: out[ij + nbra*(ab + nab*(cd + ncd*kl))].
 *
 * REAL is double, or __float128 (libquadmath) when built with -DORACLE_QUAD.
 * The exported functions take and return double in both builds.
 */
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#include <math.h>

#ifdef ORACLE_QUAD
#include <quadmath.h>
typedef __float128 REAL;
#define R_EXP expq
#define R_SQRT sqrtq
#define R_ERF erfq
#define R_FABS fabsq
#define R_PI M_PIq
#define R_EPS 1e-34Q
#else
#include <math.h>
typedef double REAL;
#define R_EXP exp
#define R_SQRT sqrt
#define R_ERF erf
#define R_FABS fabs
#define R_PI 3.14159265358979323846264338327950288
#define R_EPS 1e-17
#endif

#define OR_LMAX 8          /* per shell, including the +1 of a derivative */
#define OR_MAXCART 45      /* n_c(8) */

/* ------------------------------------------------------------------ */
/* Cartesian components of a shell                                     */
/* ------------------------------------------------------------------ */
static int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static int nsph(int l) { return 2 * l + 1; }

static void cart_list(int l, int c[][3])
{
    int n = 0;
    for (int ax = l; ax >= 0; --ax)
        for (int ay = l - ax; ay >= 0; --ay) {
            c[n][0] = ax; c[n][1] = ay; c[n][2] = l - ax - ay; ++n;
        }
}

static int cart_index(int ax, int ay, int az)
{
    /* position of (ax,ay,az) in cart_list(ax+ay+az) */
    int l = ax + ay + az;
    int s = l - ax;               /* = ay + az */
    return s * (s + 1) / 2 + az;
}

/* ------------------------------------------------------------------ */
/* Real solid harmonics: closed-form coefficients                      */
/* C[m+l][cart] = coefficient of x^ax y^ay z^az in S_lm (Racah norm.)  */
/* ------------------------------------------------------------------ */
/* Built in REAL: the __float128 build then checks the fp64 build's
 * Cartesian -> solid step too (its coefficients carry no double rounding). */
static REAL fact(int n) { REAL r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }
static REAL binom(int n, int k)
{
    if (k < 0 || k > n) return 0;
    return fact(n) / (fact(k) * fact(n - k));
}
static REAL ipow(REAL x, int n) { REAL r = 1; for (int i = 0; i < n; ++i) r *= x; return r; }

static void solid_coefs(int l, REAL C[][OR_MAXCART])
{
    int nc = ncart(l);
    for (int i = 0; i < 2 * l + 1; ++i)
        for (int j = 0; j < nc; ++j) C[i][j] = 0;
    for (int m = -l; m <= l; ++m) {
        int am = m < 0 ? -m : m;
        int wm = m < 0 ? 1 : 0;                     /* 2 v_m */
        REAL N = 1 / (ipow(2, am) * fact(l)) *
                 R_SQRT(2 * fact(l + am) * fact(l - am) / (REAL)(m == 0 ? 2 : 1));
        for (int t = 0; t <= (l - am) / 2; ++t)
            for (int u = 0; u <= t; ++u)
                for (int w = wm; w <= am; w += 2) {  /* w = 2v */
                    int sgn_exp = t + (w - wm) / 2;
                    REAL c = ((sgn_exp & 1) ? -1 : 1) * ipow((REAL)0.25, t) *
                             binom(l, t) * binom(l - t, am + t) * binom(t, u) * binom(am, w);
                    int ax = 2 * t + am - 2 * u - w;
                    int ay = 2 * u + w;
                    int az = l - 2 * t - am;
                    C[m + l][cart_index(ax, ay, az)] += N * c;
                }
    }
}

/* ------------------------------------------------------------------ */
/* Boys function, Eq. (28)                                             */
/* ------------------------------------------------------------------ */
static void boys_all(int mmax, REAL x, REAL *F)
{
    if (x <= 50) {
        REAL ex = R_EXP(-x);
        for (int m = 0; m <= mmax; ++m) {
            REAL term = 1 / (REAL)(2 * m + 1);
            REAL sum = term;
            for (int k = 1; k < 2000; ++k) {
                term *= 2 * x / (REAL)(2 * m + 2 * k + 1);
                sum += term;
                if (term < R_EPS * sum) break;
            }
            F[m] = ex * sum;
        }
    } else {
        REAL ex = R_EXP(-x);
        F[0] = R_SQRT(R_PI / (4 * x)) * R_ERF(R_SQRT(x));
        for (int m = 0; m < mmax; ++m)
            F[m + 1] = ((2 * m + 1) * F[m] - ex) / (2 * x);
    }
}

/* ------------------------------------------------------------------ */
/* 1-D Hermite expansion coefficients, Eqs. (10), (11), (14)           */
/* E[i][j][t], i <= la, j <= lb, 0 <= t <= i+j                         */
/* ------------------------------------------------------------------ */
#define EDIM (OR_LMAX + 1)
#define ETDIM (2 * OR_LMAX + 1)
typedef REAL Etab[EDIM][EDIM][ETDIM];

static REAL eget(Etab E, int i, int j, int t)
{
    if (t < 0 || t > i + j) return 0;
    return E[i][j][t];
}

static void ecoef(int la, int lb, REAL za, REAL zb, REAL A, REAL B, Etab E)
{
    REAL p = za + zb;
    REAL P = (za * A + zb * B) / p;
    REAL XPA = P - A, XPB = P - B;
    REAL i2p = 1 / (2 * p);
    memset(E, 0, sizeof(Etab));
    E[0][0][0] = R_EXP(-za * zb * (A - B) * (A - B) / p);     /* Eq. (14) */
    for (int i = 0; i <= la; ++i) {
        if (i > 0) {                                            /* Eq. (10) */
            for (int t = 0; t <= i; ++t)
                E[i][0][t] = i2p * eget(E, i - 1, 0, t - 1) + XPA * eget(E, i - 1, 0, t) +
                             (t + 1) * eget(E, i - 1, 0, t + 1);
        }
        for (int j = 1; j <= lb; ++j)                           /* Eq. (11) */
            for (int t = 0; t <= i + j; ++t)
                E[i][j][t] = i2p * eget(E, i, j - 1, t - 1) + XPB * eget(E, i, j - 1, t) +
                             (t + 1) * eget(E, i, j - 1, t + 1);
    }
}

/* ------------------------------------------------------------------ */
/* Hermite auxiliary integrals, Eqs. (27), (31)                        */
/* R0[(t*(L+1)+u)*(L+1)+v] = [tuv]^(0), t+u+v <= L                     */
/* ------------------------------------------------------------------ */
static void rints(int L, REAL p, REAL q, const REAL P[3], const REAL Q[3], REAL *R0)
{
    int D = L + 1;
    REAL rho = p * q / (p + q);
    REAL X[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
    REAL T = rho * (X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    REAL F[64];
    boys_all(L, T, F);
    /* Rm[m][t][u][v] */
    size_t cube = (size_t)D * D * D;
    REAL *Rm = (REAL *)calloc((size_t)D * cube, sizeof(REAL));
#define RM(m, t, u, v) Rm[(size_t)(m) * cube + ((size_t)(t) * D + (u)) * D + (v)]
    REAL pref = 2 * R_PI * R_PI * R_SQRT(R_PI) / (p * q * R_SQRT(p + q));
    REAL fac = 1;
    for (int m = 0; m <= L; ++m) {                 /* Eq. (27) */
        RM(m, 0, 0, 0) = pref * fac * F[m];
        fac *= -2 * rho;
    }
    /* Eq. (31): raise one index at a time, level by level */
    for (int n = 1; n <= L; ++n)
        for (int t = 0; t <= n; ++t)
            for (int u = 0; u <= n - t; ++u) {
                int v = n - t - u;
                for (int m = 0; m <= L - n; ++m) {
                    REAL val;
                    if (t > 0)
                        val = (t > 1 ? (t - 1) * RM(m + 1, t - 2, u, v) : 0) + X[0] * RM(m + 1, t - 1, u, v);
                    else if (u > 0)
                        val = (u > 1 ? (u - 1) * RM(m + 1, t, u - 2, v) : 0) + X[1] * RM(m + 1, t, u - 1, v);
                    else
                        val = (v > 1 ? (v - 1) * RM(m + 1, t, u, v - 2) : 0) + X[2] * RM(m + 1, t, u, v - 1);
                    RM(m, t, u, v) = val;
                }
            }
    memcpy(R0, Rm, cube * sizeof(REAL));
#undef RM
    free(Rm);
}

/* ------------------------------------------------------------------ */
/* 1-particle Hermite auxiliary integrals of one point I, Eqs. (26),   */
/* (30): [0]_I^(m) = (2 pi/p) (-2p)^m F_m(p |P-I|^2), then the same     */
/* one-index raising as Eq. (31) with P - I in place of P - Q.          */
/* R0[(t*(L+1)+u)*(L+1)+v] = [tuv]_I^(0), t+u+v <= L                    */
/* ------------------------------------------------------------------ */
static void rints_point(int L, REAL p, const REAL P[3], const REAL I[3], REAL *R0)
{
    int D = L + 1;
    REAL X[3] = {P[0] - I[0], P[1] - I[1], P[2] - I[2]};
    REAL T = p * (X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    REAL F[64];
    boys_all(L, T, F);
    size_t cube = (size_t)D * D * D;
    REAL *Rm = (REAL *)calloc((size_t)D * cube, sizeof(REAL));
#define RM(m, t, u, v) Rm[(size_t)(m) * cube + ((size_t)(t) * D + (u)) * D + (v)]
    REAL fac = 2 * R_PI / p;
    for (int m = 0; m <= L; ++m) {                 /* Eq. (26) */
        RM(m, 0, 0, 0) = fac * F[m];
        fac *= -2 * p;
    }
    for (int n = 1; n <= L; ++n)                    /* Eq. (30) */
        for (int t = 0; t <= n; ++t)
            for (int u = 0; u <= n - t; ++u) {
                int v = n - t - u;
                for (int m = 0; m <= L - n; ++m) {
                    REAL val;
                    if (t > 0)
                        val = (t > 1 ? (t - 1) * RM(m + 1, t - 2, u, v) : 0) + X[0] * RM(m + 1, t - 1, u, v);
                    else if (u > 0)
                        val = (u > 1 ? (u - 1) * RM(m + 1, t, u - 2, v) : 0) + X[1] * RM(m + 1, t, u - 1, v);
                    else
                        val = (v > 1 ? (v - 1) * RM(m + 1, t, u, v - 2) : 0) + X[2] * RM(m + 1, t, u, v - 1);
                    RM(m, t, u, v) = val;
                }
            }
    memcpy(R0, Rm, cube * sizeof(REAL));
#undef RM
    free(Rm);
}

/* ------------------------------------------------------------------ */
/* Shell description and one contracted shell quartet                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int l, K;
    REAL A[3];
    const double *z, *c;
} shell_t;

static const double unit_z = 0.0, unit_c = 1.0;

static shell_t make_shell(int idx, const double *xyz, const int *l, const int *nprim,
                          const int *poff, const double *ex, const double *co)
{
    shell_t s;
    s.l = l[idx]; s.K = nprim[idx];
    for (int i = 0; i < 3; ++i) s.A[i] = xyz[3 * idx + i];
    s.z = ex + poff[idx]; s.c = co + poff[idx];
    return s;
}

static shell_t unit_shell(const shell_t *partner)
{
    shell_t s;
    s.l = 0; s.K = 1;
    for (int i = 0; i < 3; ++i) s.A[i] = partner->A[i];
    s.z = &unit_z; s.c = &unit_c;
    return s;
}

/* Pair Hermite matrix: Epair[ab][(t*(D)+u)*D+v] = E^t_x E^u_y E^v_z
 * for Cartesian a (of la) and b (of lb), hermite index dims D = lmax_t+1. */
static void pair_E(int la, int lb, REAL za, REAL zb, const REAL A[3], const REAL B[3],
                   int D, REAL *Ep /* [ncart(la)*ncart(lb)][D^3] */)
{
    Etab Ex, Ey, Ez;
    ecoef(la, lb, za, zb, A[0], B[0], Ex);
    ecoef(la, lb, za, zb, A[1], B[1], Ey);
    ecoef(la, lb, za, zb, A[2], B[2], Ez);
    int ca[OR_MAXCART][3], cb[OR_MAXCART][3];
    cart_list(la, ca); cart_list(lb, cb);
    int na = ncart(la), nb = ncart(lb);
    size_t cube = (size_t)D * D * D;
    memset(Ep, 0, (size_t)na * nb * cube * sizeof(REAL));
    for (int a = 0; a < na; ++a)
        for (int b = 0; b < nb; ++b) {
            REAL *e = Ep + (size_t)(a * nb + b) * cube;
            for (int t = 0; t <= ca[a][0] + cb[b][0]; ++t)
                for (int u = 0; u <= ca[a][1] + cb[b][1]; ++u)
                    for (int v = 0; v <= ca[a][2] + cb[b][2]; ++v)
                        e[(t * D + u) * D + v] = Ex[ca[a][0]][cb[b][0]][t] *
                                                 Ey[ca[a][1]][cb[b][1]][u] *
                                                 Ez[ca[a][2]][cb[b][2]][v];
        }
}

/*
 * Primitive Cartesian quartet through Eqs. (25), (32), (33):
 *   [p|q] = (-1)^{l_q} R_{p+q};  [p|cd] = sum_q [p|q] E_cd^q;
 *   [ab|cd] = sum_p E_ab^p [p|cd]
 * Eab: [nab][Db^3] (hermite dims Db), Ecd: [ncd][Dk^3]; lb_t/lk_t: max
 * hermite order on each side.  Accumulates w * [ab|cd] into out[ab*ncd+cd].
 */
static void prim_quartet(int lbt, int lkt, int nab, int ncd, const REAL *Eab, const REAL *Ecd,
                         REAL p, REAL q, const REAL P[3], const REAL Q[3], REAL w, REAL *out,
                         REAL *R0, REAL *pket)
{
    int L = lbt + lkt;
    int D = L + 1, Db = lbt + 1, Dk = lkt + 1;
    size_t cb = (size_t)Db * Db * Db, ck = (size_t)Dk * Dk * Dk;
    rints(L, p, q, P, Q, R0);
    /* ket transform, Eq. (32) */
    for (size_t i = 0; i < cb * ncd; ++i) pket[i] = 0;
    for (int t = 0; t <= lbt; ++t)
        for (int u = 0; u <= lbt - t; ++u)
            for (int v = 0; v <= lbt - t - u; ++v) {
                size_t ip = (t * Db + u) * Db + v;
                for (int tq = 0; tq <= lkt; ++tq)
                    for (int uq = 0; uq <= lkt - tq; ++uq)
                        for (int vq = 0; vq <= lkt - tq - uq; ++vq) {
                            REAL sgn = ((tq + uq + vq) & 1) ? -1 : 1;
                            REAL pq = sgn * R0[((size_t)(t + tq) * D + (u + uq)) * D + (v + vq)];
                            size_t iq = (tq * Dk + uq) * Dk + vq;
                            for (int cd = 0; cd < ncd; ++cd)
                                pket[ip * ncd + cd] += pq * Ecd[(size_t)cd * ck + iq];
                        }
            }
    /* bra transform, Eq. (33) */
    for (int ab = 0; ab < nab; ++ab)
        for (int cd = 0; cd < ncd; ++cd) {
            REAL s = 0;
            for (int t = 0; t <= lbt; ++t)
                for (int u = 0; u <= lbt - t; ++u)
                    for (int v = 0; v <= lbt - t - u; ++v) {
                        size_t ip = (t * Db + u) * Db + v;
                        s += Eab[(size_t)ab * cb + ip] * pket[ip * ncd + cd];
                    }
            out[ab * ncd + cd] += w * s;
        }
}

/*
 * Hermite matrix of d/dX_i [phi_a phi_b] for X the first (which = 0) or the
 * second (which = 1) centre of the pair, from the differentiated Eq. (1):
 *   d/dX_i phi_n = 2 zeta phi_{n+1_i} - n_i phi_{n-1_i}.
 * Eout: [ncart(la)*ncart(lb)][D^3], D >= la+lb+2.
 */
static void pair_E_deriv(int la, int lb, REAL za, REAL zb, const REAL A[3], const REAL B[3],
                         int which, int di, int D, REAL *Eout)
{
    size_t cube = (size_t)D * D * D;
    int na = ncart(la), nb = ncart(lb);
    int ca[OR_MAXCART][3], cb[OR_MAXCART][3];
    cart_list(la, ca); cart_list(lb, cb);
    memset(Eout, 0, (size_t)na * nb * cube * sizeof(REAL));
    int la1 = la + (which == 0), lb1 = lb + (which == 1);
    int nb1 = ncart(lb1);
    REAL *Eup = (REAL *)malloc((size_t)ncart(la1) * nb1 * cube * sizeof(REAL));
    pair_E(la1, lb1, za, zb, A, B, D, Eup);
    int la0 = la - (which == 0), lb0 = lb - (which == 1);
    REAL *Edn = NULL;
    int nb0 = 0;
    if (la0 >= 0 && lb0 >= 0) {
        nb0 = ncart(lb0);
        Edn = (REAL *)malloc((size_t)ncart(la0) * nb0 * cube * sizeof(REAL));
        pair_E(la0, lb0, za, zb, A, B, D, Edn);
    }
    REAL zeta = which == 0 ? za : zb;
    for (int a = 0; a < na; ++a)
        for (int b = 0; b < nb; ++b) {
            int qa[3] = {ca[a][0], ca[a][1], ca[a][2]};
            int qb[3] = {cb[b][0], cb[b][1], cb[b][2]};
            int *q = which == 0 ? qa : qb;
            REAL *dst = Eout + (size_t)(a * nb + b) * cube;
            q[di] += 1;
            const REAL *up = Eup + (size_t)(cart_index(qa[0], qa[1], qa[2]) * nb1 +
                                            cart_index(qb[0], qb[1], qb[2])) * cube;
            for (size_t h = 0; h < cube; ++h) dst[h] += 2 * zeta * up[h];
            q[di] -= 1;
            if (q[di] > 0) {
                REAL n = q[di];
                q[di] -= 1;
                const REAL *dn = Edn + (size_t)(cart_index(qa[0], qa[1], qa[2]) * nb0 +
                                                cart_index(qb[0], qb[1], qb[2])) * cube;
                for (size_t h = 0; h < cube; ++h) dst[h] -= n * dn[h];
            }
        }
    free(Eup);
    free(Edn);
}

/*
 * Contracted Cartesian shell quartet (ab|cd), or one centre derivative.
 *   deriv = -1 : plain integrals
 *   deriv = 3*X + i (X in 0..3 = A,B,C,D; i = x,y,z): d/dX_i (ab|cd)
 * out[ab*ncd + cd] (Cartesian, ab = a*ncart(lb)+b).
 */
static void cart_quartet(const shell_t *sa, const shell_t *sb, const shell_t *sc, const shell_t *sd,
                         int deriv, REAL *out)
{
    int la = sa->l, lb = sb->l, lc = sc->l, ld = sd->l;
    int nab = ncart(la) * ncart(lb), ncd = ncart(lc) * ncart(ld);
    int dX = deriv >= 0 ? deriv / 3 : -1, di = deriv >= 0 ? deriv % 3 : -1;
    /* Hermite ranges; a derivative raises one side by one */
    int lbt = la + lb + (dX == 0 || dX == 1 ? 1 : 0);
    int lkt = lc + ld + (dX == 2 || dX == 3 ? 1 : 0);
    int Db = lbt + 1, Dk = lkt + 1, D = lbt + lkt + 1;
    size_t cb = (size_t)Db * Db * Db, ck = (size_t)Dk * Dk * Dk;
    REAL *Eab = (REAL *)malloc((size_t)nab * cb * sizeof(REAL));
    REAL *Ecd = (REAL *)malloc((size_t)ncd * ck * sizeof(REAL));
    REAL *R0 = (REAL *)malloc((size_t)D * D * D * sizeof(REAL));
    REAL *pket = (REAL *)malloc(cb * ncd * sizeof(REAL));
    for (int i = 0; i < nab * ncd; ++i) out[i] = 0;

    for (int ka = 0; ka < sa->K; ++ka)
        for (int kb = 0; kb < sb->K; ++kb) {
            REAL za = sa->z[ka], zb = sb->z[kb];
            REAL p = za + zb;
            REAL P[3];
            for (int i = 0; i < 3; ++i) P[i] = (za * sa->A[i] + zb * sb->A[i]) / p;
            if (dX == 0 || dX == 1)
                pair_E_deriv(la, lb, za, zb, sa->A, sb->A, dX, di, Db, Eab);
            else
                pair_E(la, lb, za, zb, sa->A, sb->A, Db, Eab);
            REAL wab = (REAL)sa->c[ka] * (REAL)sb->c[kb];
            for (int kc = 0; kc < sc->K; ++kc)
                for (int kd = 0; kd < sd->K; ++kd) {
                    REAL zc = sc->z[kc], zd = sd->z[kd];
                    REAL q = zc + zd;
                    REAL Q[3];
                    for (int i = 0; i < 3; ++i) Q[i] = (zc * sc->A[i] + zd * sd->A[i]) / q;
                    if (dX == 2 || dX == 3)
                        pair_E_deriv(lc, ld, zc, zd, sc->A, sd->A, dX - 2, di, Dk, Ecd);
                    else
                        pair_E(lc, ld, zc, zd, sc->A, sd->A, Dk, Ecd);
                    REAL w = wab * (REAL)sc->c[kc] * (REAL)sd->c[kd];
                    prim_quartet(lbt, lkt, nab, ncd, Eab, Ecd, p, q, P, Q, w, out, R0, pket);
                }
        }
    free(Eab); free(Ecd); free(R0); free(pket);
}

/* Cartesian -> solid on all four indices, Eqs. (18), (19) */
static void to_solid(int la, int lb, int lc, int ld, const REAL *cart, REAL *sph)
{
    /* built per call: no shared mutable state between OpenMP threads */
    REAL Cs[4][2 * OR_LMAX + 1][OR_MAXCART];
    int l4[4] = {la, lb, lc, ld};
    for (int i = 0; i < 4; ++i) solid_coefs(l4[i], Cs[i]);
    int nc4[4], ns4[4];
    for (int i = 0; i < 4; ++i) { nc4[i] = ncart(l4[i]); ns4[i] = nsph(l4[i]); }
    /* transform one index at a time; tensor index order (a,b,c,d), d fastest */
    size_t maxn = 1;
    for (int i = 0; i < 4; ++i) maxn *= nc4[i];
    REAL *cur = (REAL *)malloc(maxn * sizeof(REAL));
    REAL *nxt = (REAL *)malloc(maxn * sizeof(REAL));
    memcpy(cur, cart, maxn * sizeof(REAL));
    int dims[4] = {nc4[0], nc4[1], nc4[2], nc4[3]};
    for (int ax = 0; ax < 4; ++ax) {
        size_t outer = 1, inner = 1;
        for (int i = 0; i < ax; ++i) outer *= dims[i];
        for (int i = ax + 1; i < 4; ++i) inner *= dims[i];
        int nin = dims[ax], nout = ns4[ax];
        for (size_t o = 0; o < outer; ++o)
            for (int m = 0; m < nout; ++m)
                for (size_t r = 0; r < inner; ++r) {
                    REAL s = 0;
                    for (int k = 0; k < nin; ++k)
                        s += Cs[ax][m][k] * cur[(o * nin + k) * inner + r];
                    nxt[(o * nout + m) * inner + r] = s;
                }
        dims[ax] = nout;
        REAL *t = cur; cur = nxt; nxt = t;
    }
    size_t n = (size_t)ns4[0] * ns4[1] * ns4[2] * ns4[3];
    memcpy(sph, cur, n * sizeof(REAL));
    free(cur); free(nxt);
}

static int nfunc(int l, int cartesian) { return cartesian ? ncart(l) : nsph(l); }

/* One shell quartet in the requested basis, value (deriv<0) or derivative.
 * res[ab*ncd+cd], ab = a*nb + b in the output basis. */
static void shellset(const shell_t *sa, const shell_t *sb, const shell_t *sc, const shell_t *sd,
                     int cartesian, int deriv, REAL *res)
{
    int ncart4 = ncart(sa->l) * ncart(sb->l) * ncart(sc->l) * ncart(sd->l);
    REAL *cart = (REAL *)malloc(ncart4 * sizeof(REAL));
    cart_quartet(sa, sb, sc, sd, deriv, cart);
    if (cartesian)
        memcpy(res, cart, ncart4 * sizeof(REAL));
    else
        to_solid(sa->l, sb->l, sc->l, sd->l, cart, res);
    free(cart);
}

/* ------------------------------------------------------------------ */
/* Exported C API (ctypes)                                             */
/* ------------------------------------------------------------------ */
#ifdef ORACLE_QUAD
#define EXPORT(name) mdx_oracle_q_##name
#else
#define EXPORT(name) mdx_oracle_##name
#endif

/* F[m*n + i] = F_m(x[i]), m = 0..mmax */
void EXPORT(boys)(int n, const double *x, int mmax, double *F)
{
    REAL f[256];
    for (int i = 0; i < n; ++i) {
        boys_all(mmax, (REAL)x[i], f);
        for (int m = 0; m <= mmax; ++m) F[(size_t)m * n + i] = (double)f[m];
    }
}

/* solid-harmonic coefficients C[(m+l)*ncart(l) + cart] (closed form) */
void EXPORT(solid_coefs)(int l, double *C)
{
    REAL Cs[2 * OR_LMAX + 1][OR_MAXCART];
    solid_coefs(l, Cs);
    for (int m = 0; m < 2 * l + 1; ++m)
        for (int k = 0; k < ncart(l); ++k) C[m * ncart(l) + k] = (double)Cs[m][k];
}

/* 1-D Hermite coefficients E[(i*(lb+1)+j)*(la+lb+1)+t] for one axis */
void EXPORT(ecoef_1d)(int la, int lb, double za, double zb, double A, double B, double *out)
{
    Etab E;
    ecoef(la, lb, za, zb, A, B, E);
    int T = la + lb + 1;
    for (int i = 0; i <= la; ++i)
        for (int j = 0; j <= lb; ++j)
            for (int t = 0; t < T; ++t) out[(i * (lb + 1) + j) * T + t] = (double)E[i][j][t];
}

/* Cartesian (or solid) overlap of two contracted shells via Eq. (8):
 * S_ab = sum_prims c_a c_b E^0_x E^0_y E^0_z (pi/p)^{3/2} */
void EXPORT(overlap)(int la, int lb, const double *A, const double *B, int Ka, int Kb,
                     const double *za, const double *ca, const double *zb, const double *cb,
                     int cartesian, double *out)
{
    int na = ncart(la), nb = ncart(lb);
    int qa[OR_MAXCART][3], qb[OR_MAXCART][3];
    cart_list(la, qa); cart_list(lb, qb);
    REAL S[OR_MAXCART * OR_MAXCART];
    for (int i = 0; i < na * nb; ++i) S[i] = 0;
    for (int ka = 0; ka < Ka; ++ka)
        for (int kb = 0; kb < Kb; ++kb) {
            Etab Ex, Ey, Ez;
            REAL a = za[ka], b = zb[kb], p = a + b;
            ecoef(la, lb, a, b, A[0], B[0], Ex);
            ecoef(la, lb, a, b, A[1], B[1], Ey);
            ecoef(la, lb, a, b, A[2], B[2], Ez);
            REAL f = (REAL)ca[ka] * (REAL)cb[kb] * R_PI / p * R_SQRT(R_PI / p);
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j)
                    S[i * nb + j] += f * Ex[qa[i][0]][qb[j][0]][0] * Ey[qa[i][1]][qb[j][1]][0] *
                                     Ez[qa[i][2]][qb[j][2]][0];
        }
    if (cartesian) {
        for (int i = 0; i < na * nb; ++i) out[i] = (double)S[i];
        return;
    }
    REAL Ca[2 * OR_LMAX + 1][OR_MAXCART], Cb[2 * OR_LMAX + 1][OR_MAXCART];
    solid_coefs(la, Ca); solid_coefs(lb, Cb);
    for (int m = 0; m < nsph(la); ++m)
        for (int n = 0; n < nsph(lb); ++n) {
            REAL s = 0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) s += Ca[m][i] * Cb[n][j] * S[i * nb + j];
            out[m * nsph(lb) + n] = (double)s;
        }
}

/* Cartesian (or solid) kinetic-energy integrals of two contracted shells,
 * T_ab = -1/2 <a| nabla^2 |b>.  The Laplacian acts on the ket Gaussian: along
 * one axis d^2/dx^2 of x_B^j exp(-b x_B^2) is
 *   j(j-1) x_B^{j-2} - 2b(2j+1) x_B^j + 4b^2 x_B^{j+2}   (times the Gaussian),
 * so each 1-D factor is a combination of 1-D overlaps E^{i,j'}_0 (Eq. (8)),
 * T_ab = sum_prims c_a c_b (pi/p)^{3/2} (t_x s_y s_z + s_x t_y s_z + s_x s_y t_z). */
void EXPORT(kinetic)(int la, int lb, const double *A, const double *B, int Ka, int Kb,
                     const double *za, const double *ca, const double *zb, const double *cb,
                     int cartesian, double *out)
{
    int na = ncart(la), nb = ncart(lb);
    int qa[OR_MAXCART][3], qb[OR_MAXCART][3];
    cart_list(la, qa); cart_list(lb, qb);
    REAL T[OR_MAXCART * OR_MAXCART];
    for (int i = 0; i < na * nb; ++i) T[i] = 0;
    for (int ka = 0; ka < Ka; ++ka)
        for (int kb = 0; kb < Kb; ++kb) {
            Etab E[3];
            REAL a = za[ka], b = zb[kb], p = a + b;
            for (int ax = 0; ax < 3; ++ax) ecoef(la, lb + 2, a, b, A[ax], B[ax], E[ax]);
            REAL f = (REAL)ca[ka] * (REAL)cb[kb] * R_PI / p * R_SQRT(R_PI / p);
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    REAL s1[3], t1[3];
                    for (int ax = 0; ax < 3; ++ax) {
                        int ia = qa[i][ax], jb = qb[j][ax];
                        s1[ax] = E[ax][ia][jb][0];
                        REAL d2 = 4 * b * b * E[ax][ia][jb + 2][0] - 2 * b * (2 * jb + 1) * E[ax][ia][jb][0];
                        if (jb >= 2) d2 += (REAL)(jb * (jb - 1)) * E[ax][ia][jb - 2][0];
                        t1[ax] = -d2 / 2;
                    }
                    T[i * nb + j] += f * (t1[0] * s1[1] * s1[2] + s1[0] * t1[1] * s1[2] + s1[0] * s1[1] * t1[2]);
                }
        }
    if (cartesian) {
        for (int i = 0; i < na * nb; ++i) out[i] = (double)T[i];
        return;
    }
    REAL Ca[2 * OR_LMAX + 1][OR_MAXCART], Cb[2 * OR_LMAX + 1][OR_MAXCART];
    solid_coefs(la, Ca); solid_coefs(lb, Cb);
    for (int m = 0; m < nsph(la); ++m)
        for (int n = 0; n < nsph(lb); ++n) {
            REAL s = 0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) s += Ca[m][i] * Cb[n][j] * T[i * nb + j];
            out[m * nsph(lb) + n] = (double)s;
        }
}

/* Cartesian (or solid) 1-particle Coulomb integrals of two contracted
 * shells in the field of ncharge point charges (charges[4I..4I+2] = position,
 * charges[4I+3] = q_I):
 *   V_ab = - sum_I q_I sum_p [p]_I^(0) H^p_ab                 Eqs. (24), (34)
 * with H^p_ab = c_a c_b E^{ab}_p (Eqs. (10)-(11), (14)), evaluated charge by
 * charge -- the order before the early summation of Eq. (37). */
void EXPORT(nuclear)(int la, int lb, const double *A, const double *B, int Ka, int Kb,
                     const double *za, const double *ca, const double *zb, const double *cb,
                     int ncharge, const double *charges, int cartesian, double *out)
{
    int na = ncart(la), nb = ncart(lb), L = la + lb, D = L + 1;
    int qa[OR_MAXCART][3], qb[OR_MAXCART][3];
    cart_list(la, qa); cart_list(lb, qb);
    REAL V[OR_MAXCART * OR_MAXCART];
    REAL *R0 = (REAL *)malloc((size_t)D * D * D * sizeof(REAL));
    for (int i = 0; i < na * nb; ++i) V[i] = 0;
    for (int ka = 0; ka < Ka; ++ka)
        for (int kb = 0; kb < Kb; ++kb) {
            Etab E[3];
            REAL a = za[ka], b = zb[kb], p = a + b, P[3];
            for (int ax = 0; ax < 3; ++ax) {
                ecoef(la, lb, a, b, A[ax], B[ax], E[ax]);
                P[ax] = (a * (REAL)A[ax] + b * (REAL)B[ax]) / p;
            }
            REAL cc = (REAL)ca[ka] * (REAL)cb[kb];
            for (int I = 0; I < ncharge; ++I) {
                REAL C[3] = {charges[4 * I], charges[4 * I + 1], charges[4 * I + 2]};
                rints_point(L, p, P, C, R0);
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j) {
                        REAL s = 0;
                        for (int t = 0; t <= qa[i][0] + qb[j][0]; ++t)
                            for (int u = 0; u <= qa[i][1] + qb[j][1]; ++u)
                                for (int v = 0; v <= qa[i][2] + qb[j][2]; ++v)
                                    s += E[0][qa[i][0]][qb[j][0]][t] * E[1][qa[i][1]][qb[j][1]][u] *
                                         E[2][qa[i][2]][qb[j][2]][v] * R0[((size_t)t * D + u) * D + v];
                        V[i * nb + j] -= (REAL)charges[4 * I + 3] * cc * s;
                    }
            }
        }
    free(R0);
    if (cartesian) {
        for (int i = 0; i < na * nb; ++i) out[i] = (double)V[i];
        return;
    }
    REAL Ca[2 * OR_LMAX + 1][OR_MAXCART], Cb[2 * OR_LMAX + 1][OR_MAXCART];
    solid_coefs(la, Ca); solid_coefs(lb, Cb);
    for (int m = 0; m < nsph(la); ++m)
        for (int n = 0; n < nsph(lb); ++n) {
            REAL s = 0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) s += Ca[m][i] * Cb[n][j] * V[i * nb + j];
            out[m * nsph(lb) + n] = (double)s;
        }
}

/*
 * Batched shell quartets.
 *   ncentre = 4: bra[2*ij], bra[2*ij+1] shell indices; same for ket.
 *   ncentre = 3: bra[2*ij+1] ignored (unit shell); ket is a pair.
 *   ncentre = 2: both sides single shells.
 * nquart < 0 : dense outer product, out[ij + nbra*(ab + nab*(cd + ncd*kl))]
 * nquart >= 0: explicit list, quartet q = (bra[qidx[2q]], ket[qidx[2q+1]]),
 *              out[q*nab*ncd + ab*ncd + cd]
 * deriv  < 0 : integrals.  deriv = 12: all 12 centre derivatives,
 *              dense: out[((ij + nbra*(d + 12*kl))*nab + ab)*ncd + cd]  (see below)
 *              list : out[((q*12 + d)*nab + ab)*ncd + cd]
 * The derivative layouts keep each shellset's [ab][cd] block contiguous.
 * Returns 0 on success, -1 on bad arguments.
 */
int EXPORT(eri)(int ncentre, int nshell, const double *xyz, const int *l, const int *nprim,
                const int *poff, const double *ex, const double *co, int nbra, const int *bra,
                int nket, const int *ket, int nquart, const int *qidx, int cartesian, int deriv,
                double *out)
{
    if (ncentre < 2 || ncentre > 4) return -1;
    for (int s = 0; s < nshell; ++s)
        if (l[s] < 0 || l[s] > OR_LMAX - 1 || nprim[s] < 1) return -1;
    if (nbra <= 0 || nket <= 0) return 0;
    int l0a = l[bra[0]], l0b = ncentre == 4 ? l[bra[1]] : 0;
    int l0c = l[ket[0]], l0d = ncentre >= 3 ? l[ket[1]] : 0;
    int nab = nfunc(l0a, cartesian) * nfunc(l0b, cartesian);
    int ncd = nfunc(l0c, cartesian) * nfunc(l0d, cartesian);
    long long ntask = nquart >= 0 ? nquart : (long long)nbra * nket;
    int nd = deriv >= 0 ? 12 : 1;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (long long task = 0; task < ntask; ++task) {
        int ij, kl;
        if (nquart >= 0) { ij = qidx[2 * task]; kl = qidx[2 * task + 1]; }
        else { ij = (int)(task % nbra); kl = (int)(task / nbra); }
        shell_t sa = make_shell(bra[2 * ij], xyz, l, nprim, poff, ex, co);
        shell_t sb = ncentre == 4 ? make_shell(bra[2 * ij + 1], xyz, l, nprim, poff, ex, co) : unit_shell(&sa);
        shell_t sc = make_shell(ket[2 * kl], xyz, l, nprim, poff, ex, co);
        shell_t sd = ncentre >= 3 ? make_shell(ket[2 * kl + 1], xyz, l, nprim, poff, ex, co) : unit_shell(&sc);
        if (sa.l != l0a || sb.l != l0b || sc.l != l0c || sd.l != l0d) { err = 1; continue; }
        REAL *res = (REAL *)malloc((size_t)nab * ncd * sizeof(REAL));
        for (int d = 0; d < nd; ++d) {
            shellset(&sa, &sb, &sc, &sd, cartesian, deriv >= 0 ? d : -1, res);
            for (int ab = 0; ab < nab; ++ab)
                for (int cd = 0; cd < ncd; ++cd) {
                    size_t o;
                    if (nquart >= 0)
                        o = (((size_t)task * nd + d) * nab + ab) * ncd + cd;
                    else if (deriv < 0)
                        o = (size_t)ij + (size_t)nbra * (ab + (size_t)nab * (cd + (size_t)ncd * kl));
                    else
                        o = (((size_t)ij + (size_t)nbra * (d + 12 * (size_t)kl)) * nab + ab) * ncd + cd;
                    out[o] = (double)res[ab * ncd + cd];
                }
        }
        free(res);
    }
    return err ? -1 : 0;
}
