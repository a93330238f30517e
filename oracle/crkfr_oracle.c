/*
 * crkfr_oracle.c -- plain FP64 CPU oracle of one cRKFR step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU baseline; never by the product path.  It shares no code
 * with the HIP library.
 *
 * The step follows the paper's statement of the scheme in its order:
 *   local cRK procedure (Sec. 3, eqs. crkfr, disc.avg.flux, crk22/33/44,
 *   time.avg.sol; sources per App. B, eq. crk33.source),
 *   time-averaged numerical flux with EA central part and D2 dissipation
 *   (Sec. 3.1, eqs. numflux.general, D2, evaluate), boundary ghost values
 *   (Sec. 3.3), the FR update (eq. crkfr.avg), the subcell blending scheme
 *   (Sec. 4, eqs. blended.scheme, subcell.defn, low.order.update, Fblend,
 *   fo.at.face, mh.at.face), the flux limiter for admissibility in means
 *   (Sec. 4.3) and the Zhang-Shu scaling limiter (Sec. 3.2).
 * Parts the paper defers to other work (indicator, MUSCL-Hancock details,
 * flux-limiter algorithm, scaling root) follow the readings listed in the
 * repository's design notes; each is marked "reading" below.
 */
#include "crkfr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ND REF_MAXND
#define NP REF_MAXNP
#define MM REF_MAXM

/* ------------------------------------------------------------------ */
/* Reference element on [0,1] (Sec. 2, eqs. soln.points, defn.lagrange,
 * diff.matrix).                                                        */
/* ------------------------------------------------------------------ */

/* Legendre polynomial P_n(x) and its derivative by the three-term recurrence */
static void legendre(int n, double x, double* P, double* dP)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = pk;
    }
    *P = p1;
    *dP = n * (x * p1 - p0) / (x * x - 1.0);
}

/* Gauss-Legendre nodes and weights mapped to [0,1]; exact to degree 2N+1 */
void ref_gl(int N, double* xi, double* w)
{
    int n = N + 1;
    for (int i = 0; i < n; ++i) {
        double x = -cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, x, &P, &dP);
            double dx = P / dP;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double P, dP;
        legendre(n, x, &P, &dP);
        xi[i] = 0.5 * (x + 1.0);
        w[i] = 0.5 * 2.0 / ((1.0 - x * x) * dP * dP);
    }
}

/* Gauss-Legendre-Lobatto nodes and weights mapped to [0,1]: the end points
 * and the roots of P_N' (Newton with P_N'' from Legendre's equation
 * (1 - x^2) P'' = 2 x P' - N (N+1) P); weights 2 / (N (N+1) P_N(x)^2) on
 * [-1,1]; exact to degree 2N-1 */
void ref_gll(int N, double* xi, double* w)
{
    for (int i = 0; i <= N; ++i) {
        double x = -cos(M_PI * i / N);
        if (i > 0 && i < N)
            for (int it = 0; it < 100; ++it) {
                double P, dP;
                legendre(N, x, &P, &dP);
                double d2P = (2.0 * x * dP - N * (N + 1.0) * P) / (1.0 - x * x);
                double dx = dP / d2P;
                x -= dx;
                if (fabs(dx) < 1e-16) break;
            }
        double P, dP;
        if (i == 0 || i == N) P = (i == 0 && N % 2 == 1) ? -1.0 : 1.0;
        else legendre(N, x, &P, &dP);
        xi[i] = 0.5 * (x + 1.0);
        w[i] = 0.5 * 2.0 / (N * (N + 1.0) * P * P);
    }
}

/* l_q(x) = prod_{p != q} (x - xi_p)/(xi_q - xi_p) */
void ref_lagrange_at(int N, const double* xi, double x, double* l)
{
    for (int q = 0; q <= N; ++q) {
        double v = 1.0;
        for (int p = 0; p <= N; ++p)
            if (p != q) v *= (x - xi[p]) / (xi[q] - xi[p]);
        l[q] = v;
    }
}

/* D[i][j] = l_j'(xi_i), from the derivative of the product form */
void ref_diff_matrix(int N, const double* xi, double* D)
{
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N; ++j) {
            double s = 0.0;
            for (int m = 0; m <= N; ++m) {
                if (m == j) continue;
                double t = 1.0 / (xi[j] - xi[m]);
                for (int k = 0; k <= N; ++k) {
                    if (k == j || k == m) continue;
                    t *= (xi[i] - xi[k]) / (xi[j] - xi[k]);
                }
                s += t;
            }
            D[i * (N + 1) + j] = s;
        }
}

/* orthonormal Legendre polynomials on [0,1]: L_k = sqrt(2k+1) P_k(2 xi - 1) */
void ref_legendre_orthonormal(int N, const double* xi, double* L)
{
    for (int k = 0; k <= N; ++k)
        for (int p = 0; p <= N; ++p) {
            double P, dP;
            double x = 2.0 * xi[p] - 1.0;
            if (k == 0) P = 1.0; else legendre(k, x, &P, &dP);
            L[k * (N + 1) + p] = sqrt(2.0 * k + 1.0) * P;
        }
}

/* Butcher tableaux of cRK22, cRK33, cRK44 (eqs. crk22, crk33, crk44) */
void ref_tableau(int s, double* a, double* b, double* c)
{
    for (int i = 0; i < 16; ++i) a[i] = 0.0;
    for (int i = 0; i < 4; ++i) { b[i] = 0.0; c[i] = 0.0; }
    if (s == 2) {
        a[1 * 4 + 0] = 0.5;
        b[0] = 0.0; b[1] = 1.0;
    } else if (s == 3) {
        a[1 * 4 + 0] = 1.0 / 3.0;
        a[2 * 4 + 1] = 2.0 / 3.0;
        b[0] = 0.25; b[1] = 0.0; b[2] = 0.75;
    } else {
        a[1 * 4 + 0] = 0.5;
        a[2 * 4 + 1] = 0.5;
        a[3 * 4 + 2] = 1.0;
        b[0] = 1.0 / 6.0; b[1] = 1.0 / 3.0; b[2] = 1.0 / 3.0; b[3] = 1.0 / 6.0;
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) c[i] += a[i * 4 + j];
}

typedef struct {
    int N, nd;
    double xi[ND], w[ND], D[ND * ND], l0[ND], l1[ND];
    double sub[ND + 1];   /* subfaces xi_{p-1/2}, p = 0..N+1 (eq. subcell.defn) */
    double Pm[ND * ND];   /* Pm[k][p]: coefficient k of the orthonormal Legendre
                             expansion of the interpolant of nodal values */
} refel;

/* Solution points GL or GLL (eq. soln.points).  The FR correction enters
 * through g_R'(xi_p) = l_p(1)/w_p and g_L'(xi_p) = -l_p(0)/w_p, which hold
 * for the Radau correction with GL points and for g2 with GLL points
 * (eq. fr.equiv).  Modal coefficients: exact projection of the interpolant
 * onto the orthonormal Legendre basis by GL quadrature of N+1 points (for GL
 * solution points the nodal quadrature itself). */
static void refel_init(refel* r, int N, int points)
{
    r->N = N; r->nd = N + 1;
    if (points == REF_POINTS_GLL) ref_gll(N, r->xi, r->w);
    else ref_gl(N, r->xi, r->w);
    ref_lagrange_at(N, r->xi, 0.0, r->l0);
    ref_lagrange_at(N, r->xi, 1.0, r->l1);
    ref_diff_matrix(N, r->xi, r->D);
    double xg[ND], wg[ND], Lg[ND * ND];
    ref_gl(N, xg, wg);
    ref_legendre_orthonormal(N, xg, Lg);
    for (int k = 0; k <= N; ++k)
        for (int p = 0; p <= N; ++p) r->Pm[k * (N + 1) + p] = 0.0;
    for (int j = 0; j <= N; ++j) {
        double lj[ND];
        ref_lagrange_at(N, r->xi, xg[j], lj);
        for (int k = 0; k <= N; ++k)
            for (int p = 0; p <= N; ++p) r->Pm[k * (N + 1) + p] += wg[j] * Lg[k * (N + 1) + j] * lj[p];
    }
    r->sub[0] = 0.0;
    for (int p = 0; p <= N; ++p) r->sub[p + 1] = r->sub[p] + r->w[p];
    r->sub[N + 1] = 1.0;
}

/* ------------------------------------------------------------------ */
/* Physics: linear advection, 1D/2D Euler (eqs. 1deuler, state, 2deuler,
 * 2dstate, spectral radii) and the ten-moment system (eqs. tmp,
 * tenmom.source).                                                       */
/* ------------------------------------------------------------------ */

int ref_nvar(int eq)
{
    switch (eq) {
    case REF_LINADV1D: return 1;
    case REF_EULER1D: return 3;
    case REF_EULER2D: return 4;
    case REF_TENMOM2D: return 6;
    case REF_BURGERS1D: return 1;
    case REF_TENMOM1D: return 6;
    }
    return 0;
}

int ref_nadm(int eq)
{
    switch (eq) {
    case REF_LINADV1D: return 0;
    case REF_EULER1D: return 2;
    case REF_EULER2D: return 2;
    case REF_TENMOM2D: return 3;
    case REF_TENMOM1D: return 3;
    }
    return 0;
}

static int eq_dim(int eq) { return eq == REF_EULER2D || eq == REF_TENMOM2D ? 2 : 1; }

static double euler_p(int eq, double gamma, const double* u)
{
    if (eq == REF_EULER1D) return (gamma - 1.0) * (u[2] - 0.5 * u[1] * u[1] / u[0]);
    return (gamma - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
}

void ref_flux(int eq, double gamma, double adv, const double* u, double* f, double* g)
{
    if (eq == REF_LINADV1D) {
        f[0] = adv * u[0];
    } else if (eq == REF_BURGERS1D) {
        f[0] = 0.5 * u[0] * u[0];
    } else if (eq == REF_EULER1D) {
        double v = u[1] / u[0], p = euler_p(eq, gamma, u);
        f[0] = u[1];
        f[1] = u[1] * v + p;
        f[2] = (u[2] + p) * v;
    } else if (eq == REF_EULER2D) {
        double v1 = u[1] / u[0], v2 = u[2] / u[0], p = euler_p(eq, gamma, u);
        f[0] = u[1];
        f[1] = u[1] * v1 + p;
        f[2] = u[2] * v1;
        f[3] = (u[3] + p) * v1;
        if (g) {
            g[0] = u[2];
            g[1] = u[1] * v2;
            g[2] = u[2] * v2 + p;
            g[3] = (u[3] + p) * v2;
        }
    } else {
        double r = u[0], v1 = u[1] / r, v2 = u[2] / r;
        double E11 = u[3], E12 = u[4], E22 = u[5];
        double P11 = 2.0 * E11 - r * v1 * v1;
        double P12 = 2.0 * E12 - r * v1 * v2;
        double P22 = 2.0 * E22 - r * v2 * v2;
        f[0] = r * v1;
        f[1] = P11 + r * v1 * v1;
        f[2] = P12 + r * v1 * v2;
        f[3] = (E11 + P11) * v1;
        f[4] = E12 * v1 + 0.5 * (P11 * v2 + P12 * v1);
        f[5] = E22 * v1 + P12 * v2;
        if (g) {
            g[0] = r * v2;
            g[1] = P12 + r * v1 * v2;
            g[2] = P22 + r * v2 * v2;
            g[3] = E11 * v2 + P12 * v1;
            g[4] = E12 * v2 + 0.5 * (P12 * v2 + P22 * v1);
            g[5] = (E22 + P22) * v2;
        }
    }
}

/* spectral radii of the flux Jacobians; ten-moment per the standard
 * eigen-structure of the system (reading) */
void ref_sigma(int eq, double gamma, double adv, const double* u, double* sx, double* sy)
{
    if (eq == REF_LINADV1D) {
        *sx = fabs(adv); *sy = 0.0;
    } else if (eq == REF_BURGERS1D) {
        *sx = fabs(u[0]); *sy = 0.0;
    } else if (eq == REF_EULER1D) {
        double p = euler_p(eq, gamma, u);
        *sx = fabs(u[1] / u[0]) + sqrt(gamma * p / u[0]);
        *sy = 0.0;
    } else if (eq == REF_EULER2D) {
        double p = euler_p(eq, gamma, u), c = sqrt(gamma * p / u[0]);
        *sx = fabs(u[1] / u[0]) + c;
        *sy = fabs(u[2] / u[0]) + c;
    } else {
        double r = u[0], v1 = u[1] / r, v2 = u[2] / r;
        double P11 = 2.0 * u[3] - r * v1 * v1;
        double P22 = 2.0 * u[5] - r * v2 * v2;
        *sx = fabs(v1) + sqrt(3.0 * P11 / r);
        *sy = fabs(v2) + sqrt(3.0 * P22 / r);
    }
}

/* admissibility functions P_k (eq. uad.form); ten-moment: rho, P11, det P */
double ref_adm(int eq, int k, double gamma, const double* u)
{
    if (k == 0) return u[0];
    if (eq == REF_EULER1D || eq == REF_EULER2D) return euler_p(eq, gamma, u);
    double r = u[0], v1 = u[1] / r, v2 = u[2] / r;
    double P11 = 2.0 * u[3] - r * v1 * v1;
    if (k == 1) return P11;
    double P12 = 2.0 * u[4] - r * v1 * v2;
    double P22 = 2.0 * u[5] - r * v2 * v2;
    return P11 * P22 - P12 * P12;
}

/* P_k concave once P_j > 0 for j < k: true for all but the determinant */
static int is_tenmom(int eq) { return eq == REF_TENMOM2D || eq == REF_TENMOM1D; }

/* admissibility margins of the limiter chain: relative (flux limiter and
 * subcell reconstruction, default 0.1) and absolute (scaling, default 1e-13) */
static double eps_rel(const ref_config* c) { return c->eps_rel > 0.0 ? c->eps_rel : 0.1; }
static double eps_abs(const ref_config* c) { return c->eps_abs > 0.0 ? c->eps_abs : 1e-13; }
static int adm_concave(int eq, int k) { return !(is_tenmom(eq) && k == 2); }

/* ten-moment source s^x + s^y (eq. tenmom.source) with the potential
 * W = A exp(-kappa ((x-xc)^2 + (y-yc)^2)) + gx x + gy y */
static void source_at(const ref_config* c, double x, double y, const double* u, double* s)
{
    int M = ref_nvar(c->eq);
    for (int v = 0; v < M; ++v) s[v] = 0.0;
    if (!c->source || !is_tenmom(c->eq)) return;
    /* the 1D system: W depends on x only */
    double dx = x - c->src_xc, dy = c->eq == REF_TENMOM2D ? y - c->src_yc : 0.0;
    double W = c->src_amp * exp(-c->src_kappa * (dx * dx + dy * dy));
    double Wx = -2.0 * c->src_kappa * dx * W + c->src_gx;
    double Wy = -2.0 * c->src_kappa * dy * W + c->src_gy;
    double r = u[0], v1 = u[1] / r, v2 = u[2] / r;
    s[1] = -0.5 * r * Wx;
    s[2] = -0.5 * r * Wy;
    s[3] = -0.5 * r * v1 * Wx;
    s[4] = -0.25 * r * v2 * Wx - 0.25 * r * v1 * Wy;
    s[5] = -0.5 * r * v2 * Wy;
}

/* wave speed of a trace value for the D2 dissipation (reading): the
 * spectral radius with the pressure clipped at zero, since an interpolant of
 * admissible nodes need not be admissible; a non-positive density falls back
 * to the face-adjacent solution point */
static double sigma_trace(const ref_config* c, int dir, const double* tr, const double* node)
{
    int eq = c->eq;
    const double* u = tr[0] > 0.0 || eq == REF_LINADV1D || eq == REF_BURGERS1D ? tr : node;
    if (eq == REF_LINADV1D) return fabs(c->adv);
    if (eq == REF_BURGERS1D) return fabs(u[0]);
    double r = u[0], v1 = u[1] / r;
    if (eq == REF_EULER1D || eq == REF_EULER2D) {
        double p = euler_p(eq, c->gamma, u);
        double cs = sqrt(c->gamma * fmax(p, 0.0) / r);
        if (eq == REF_EULER1D || dir == 0) return fabs(v1) + cs;
        return fabs(u[2] / r) + cs;
    }
    double v2 = u[2] / r;
    if (dir == 0) return fabs(v1) + sqrt(3.0 * fmax(2.0 * u[3] - r * v1 * v1, 0.0) / r);
    return fabs(v2) + sqrt(3.0 * fmax(2.0 * u[5] - r * v2 * v2, 0.0) / r);
}

static void rusanov(const ref_config* c, int dir, const double* a, const double* b, double* out)
{
    int M = ref_nvar(c->eq);
    double fa[MM], ga[MM], fb[MM], gb[MM], sxa, sya, sxb, syb;
    ref_flux(c->eq, c->gamma, c->adv, a, fa, ga);
    ref_flux(c->eq, c->gamma, c->adv, b, fb, gb);
    ref_sigma(c->eq, c->gamma, c->adv, a, &sxa, &sya);
    ref_sigma(c->eq, c->gamma, c->adv, b, &sxb, &syb);
    double lam = dir == 0 ? fmax(sxa, sxb) : fmax(sya, syb);
    for (int v = 0; v < M; ++v) {
        double fl = dir == 0 ? fa[v] : ga[v], fr = dir == 0 ? fb[v] : gb[v];
        out[v] = 0.5 * (fl + fr) - 0.5 * lam * (b[v] - a[v]);
    }
}

static void phys_flux(const ref_config* c, int dir, const double* u, double* out)
{
    double f[MM], g[MM];
    ref_flux(c->eq, c->gamma, c->adv, u, f, g);
    int M = ref_nvar(c->eq);
    for (int v = 0; v < M; ++v) out[v] = dir == 0 ? f[v] : g[v];
}

/* all constraints P_j >= eps_j hold (checked in order) */
static int admissible_eps(const ref_config* c, const double* u, const double* eps)
{
    int K = ref_nadm(c->eq);
    for (int k = 0; k < K; ++k)
        if (!(ref_adm(c->eq, k, c->gamma, u) >= eps[k])) return 0;
    return 1;
}

/* largest t in [0,1] found by 60 bisection steps with P_k(a + t(b-a)) >= eps,
 * given P_k(a) >= eps */
static double bisect_root(const ref_config* c, int k, const double* a, const double* b, double eps)
{
    int M = ref_nvar(c->eq);
    double lo = 0.0, hi = 1.0, z[MM];
    for (int it = 0; it < 60; ++it) {
        double mid = 0.5 * (lo + hi);
        for (int v = 0; v < M; ++v) z[v] = a[v] + mid * (b[v] - a[v]);
        if (ref_adm(c->eq, k, c->gamma, z) >= eps) lo = mid; else hi = mid;
    }
    return lo;
}

/* fraction t of the segment a -> b keeping P_k >= eps (reading): the
 * concavity bound (P(a)-eps)/(P(a)-P(b)) where P_k is concave, else bisection */
static double segment_fraction(const ref_config* c, int k, const double* a, const double* b, double eps)
{
    double Pa = ref_adm(c->eq, k, c->gamma, a);
    double Pb = ref_adm(c->eq, k, c->gamma, b);
    if (Pb >= eps) return 1.0;
    if (adm_concave(c->eq, k)) {
        double t = (Pa - eps) / (Pa - Pb);
        return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    }
    return bisect_root(c, k, a, b, eps);
}

/* ------------------------------------------------------------------ */
/* Local cRK procedure on one element (Sec. 3, eq. crkfr first line with
 * the local operator; time averages eqs. disc.avg.flux, time.avg.sol; the
 * source treatment of App. B).  Written for a general strictly lower
 * triangular tableau.                                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    double F[NP][MM], G[NP][MM], U[NP][MM], S[NP][MM];
    /* EA traces (eq. evaluate): x faces per row q, y faces per column p */
    double FxL[ND][MM], FxR[ND][MM], GyB[ND][MM], GyT[ND][MM];
    double UxL[ND][MM], UxR[ND][MM], UyB[ND][MM], UyT[ND][MM];
    double unxL[ND][MM], unxR[ND][MM], unyB[ND][MM], unyT[ND][MM];
    /* extrapolated discontinuous time-averaged flux F^delta(0), F^delta(1) */
    double FhL[ND][MM], FhR[ND][MM], GhB[ND][MM], GhT[ND][MM];
    /* stage values at the faces, u^(i)(x^+-) (D-CSX dissipation, eq. dcsx) */
    double uixL[4][ND][MM], uixR[4][ND][MM], uiyB[4][ND][MM], uiyT[4][ND][MM];
} local_out;

static void local_crk(const ref_config* c, const refel* r, const double* ue, double dt,
                      double dx, double dy, double xe0, double ye0, local_out* o)
{
    int M = ref_nvar(c->eq), nd = r->nd, dim = eq_dim(c->eq);
    int nq = dim == 2 ? nd : 1, np = nd * nq;
    int s = c->stages;
    double a[16], b[4], cc[4];
    ref_tableau(s, a, b, cc);
    double stage_rhs[4][NP][MM];   /* d_loc f/dx + d_loc g/dy - s, per stage */
    double ui[NP][MM], fi[NP][MM], gi[NP][MM], si[NP][MM];

    memset(o, 0, sizeof(*o));
    for (int i = 0; i < s; ++i) {
        /* stage value u^(i) = u^n - dt sum_{j<i} a_ij rhs_j */
        for (int k = 0; k < np; ++k)
            for (int v = 0; v < M; ++v) {
                double val = ue[v * np + k];
                for (int j = 0; j < i; ++j) val -= dt * a[i * 4 + j] * stage_rhs[j][k][v];
                ui[k][v] = val;
            }
        for (int q = 0; q < nq; ++q)
            for (int p = 0; p < nd; ++p) {
                int k = q * nd + p;
                double dummy[MM];
                ref_flux(c->eq, c->gamma, c->adv, ui[k], fi[k], dim == 2 ? gi[k] : dummy);
                if (dim == 1) for (int v = 0; v < M; ++v) gi[k][v] = 0.0;
                source_at(c, xe0 + r->xi[p] * dx, dim == 2 ? ye0 + r->xi[q] * dy : 0.0, ui[k], si[k]);
            }
        /* local derivative operator: D applied along x and along y */
        for (int q = 0; q < nq; ++q)
            for (int p = 0; p < nd; ++p) {
                int k = q * nd + p;
                for (int v = 0; v < M; ++v) {
                    double dfx = 0.0, dgy = 0.0;
                    for (int m = 0; m < nd; ++m) dfx += r->D[p * nd + m] * fi[q * nd + m][v];
                    if (dim == 2)
                        for (int m = 0; m < nd; ++m) dgy += r->D[q * nd + m] * gi[m * nd + p][v];
                    stage_rhs[i][k][v] = dfx / dx + (dim == 2 ? dgy / dy : 0.0) - si[k][v];
                }
            }
        /* time averages */
        for (int k = 0; k < np; ++k)
            for (int v = 0; v < M; ++v) {
                o->F[k][v] += b[i] * fi[k][v];
                o->G[k][v] += b[i] * gi[k][v];
                o->U[k][v] += b[i] * ui[k][v];
                o->S[k][v] += b[i] * si[k][v];
            }
        /* EA traces: evaluate the flux of the interpolated stage value */
        for (int q = 0; q < nq; ++q) {
            double uL[MM], uR[MM], fL[MM], fR[MM];
            for (int v = 0; v < M; ++v) {
                uL[v] = 0.0; uR[v] = 0.0;
                for (int p = 0; p < nd; ++p) {
                    uL[v] += r->l0[p] * ui[q * nd + p][v];
                    uR[v] += r->l1[p] * ui[q * nd + p][v];
                }
            }
            phys_flux(c, 0, uL, fL);
            phys_flux(c, 0, uR, fR);
            for (int v = 0; v < M; ++v) {
                o->FxL[q][v] += b[i] * fL[v];
                o->FxR[q][v] += b[i] * fR[v];
                o->uixL[i][q][v] = uL[v];
                o->uixR[i][q][v] = uR[v];
                if (i == 0) { o->unxL[q][v] = uL[v]; o->unxR[q][v] = uR[v]; }
            }
        }
        if (dim == 2)
            for (int p = 0; p < nd; ++p) {
                double uB[MM], uT[MM], gB[MM], gT[MM];
                for (int v = 0; v < M; ++v) {
                    uB[v] = 0.0; uT[v] = 0.0;
                    for (int q = 0; q < nd; ++q) {
                        uB[v] += r->l0[q] * ui[q * nd + p][v];
                        uT[v] += r->l1[q] * ui[q * nd + p][v];
                    }
                }
                phys_flux(c, 1, uB, gB);
                phys_flux(c, 1, uT, gT);
                for (int v = 0; v < M; ++v) {
                    o->GyB[p][v] += b[i] * gB[v];
                    o->GyT[p][v] += b[i] * gT[v];
                    o->uiyB[i][p][v] = uB[v];
                    o->uiyT[i][p][v] = uT[v];
                    if (i == 0) { o->unyB[p][v] = uB[v]; o->unyT[p][v] = uT[v]; }
                }
            }
    }
    /* traces of U and extrapolations of the averaged flux */
    for (int q = 0; q < nq; ++q)
        for (int v = 0; v < M; ++v)
            for (int p = 0; p < nd; ++p) {
                o->UxL[q][v] += r->l0[p] * o->U[q * nd + p][v];
                o->UxR[q][v] += r->l1[p] * o->U[q * nd + p][v];
                o->FhL[q][v] += r->l0[p] * o->F[q * nd + p][v];
                o->FhR[q][v] += r->l1[p] * o->F[q * nd + p][v];
            }
    if (dim == 2)
        for (int p = 0; p < nd; ++p)
            for (int v = 0; v < M; ++v)
                for (int q = 0; q < nd; ++q) {
                    o->UyB[p][v] += r->l0[q] * o->U[q * nd + p][v];
                    o->UyT[p][v] += r->l1[q] * o->U[q * nd + p][v];
                    o->GhB[p][v] += r->l0[q] * o->G[q * nd + p][v];
                    o->GhT[p][v] += r->l1[q] * o->G[q * nd + p][v];
                }
}

void ref_local_crk(const ref_config* c, const double* ue, double dt, double xe0, double ye0,
                   double* F, double* G, double* U, double* S)
{
    refel r;
    refel_init(&r, c->N, c->points);
    double dx = (c->x1 - c->x0) / c->nx, dy = (c->y1 - c->y0) / c->ny;
    local_out* o = (local_out*)malloc(sizeof(local_out));
    local_crk(c, &r, ue, dt, dx, dy, xe0, ye0, o);
    int M = ref_nvar(c->eq), nd = c->N + 1, np = eq_dim(c->eq) == 2 ? nd * nd : nd;
    for (int v = 0; v < M; ++v)
        for (int k = 0; k < np; ++k) {
            F[v * np + k] = o->F[k][v];
            G[v * np + k] = o->G[k][v];
            U[v * np + k] = o->U[k][v];
            S[v * np + k] = o->S[k][v];
        }
    free(o);
}

/* ------------------------------------------------------------------ */
/* Smoothness indicator (Sec. 4, blended.scheme; details are a reading of
 * the Hennemann et al. indicator the paper refers to).                  */
/* ------------------------------------------------------------------ */

static double indicator_quantity(const ref_config* c, const double* u)
{
    if (c->eq == REF_LINADV1D || c->eq == REF_BURGERS1D) return u[0];
    if (c->eq == REF_EULER1D || c->eq == REF_EULER2D) return u[0] * euler_p(c->eq, c->gamma, u);
    double r = u[0], v1 = u[1] / r, v2 = u[2] / r;
    double P11 = 2.0 * u[3] - r * v1 * v1;
    double P22 = 2.0 * u[5] - r * v2 * v2;
    return r * 0.5 * (P11 + P22);
}

/* energy_out[k], k = 0..N: energy of the modes whose highest index is k */
static double indicator_raw(const ref_config* c, const refel* r, const double* ue, double* energy_out)
{
    int M = ref_nvar(c->eq), nd = r->nd, N = r->N, dim = eq_dim(c->eq);
    int nq = dim == 2 ? nd : 1, np = nd * nq;
    double eps[NP], u[MM];
    for (int k = 0; k < np; ++k) {
        for (int v = 0; v < M; ++v) u[v] = ue[v * np + k];
        eps[k] = indicator_quantity(c, u);
    }
    /* orthonormal Legendre coefficients of the interpolant */
    double e[ND];
    for (int k = 0; k <= N; ++k) e[k] = 0.0;
    if (dim == 1) {
        for (int i = 0; i <= N; ++i) {
            double m = 0.0;
            for (int p = 0; p <= N; ++p) m += r->Pm[i * nd + p] * eps[p];
            e[i] += m * m;
        }
    } else {
        for (int j = 0; j <= N; ++j)
            for (int i = 0; i <= N; ++i) {
                double m = 0.0;
                for (int q = 0; q <= N; ++q)
                    for (int p = 0; p <= N; ++p)
                        m += r->Pm[i * nd + p] * r->Pm[j * nd + q] * eps[q * nd + p];
                e[i > j ? i : j] += m * m;
            }
    }
    if (energy_out) for (int k = 0; k <= N; ++k) energy_out[k] = e[k];
    double tot_N = 0.0, tot_Nm1 = 0.0;
    for (int k = 0; k <= N; ++k) tot_N += e[k];
    for (int k = 0; k < N; ++k) tot_Nm1 += e[k];
    double E1 = tot_N > 0.0 ? e[N] / tot_N : 0.0;
    double E2 = tot_Nm1 > 0.0 ? e[N - 1] / tot_Nm1 : 0.0;
    double E = E1 > E2 ? E1 : E2;
    double T = 0.5 * pow(10.0, -1.8 * pow(N + 1.0, 0.25));
    double sharp = log(9999.0);
    double a = 1.0 / (1.0 + exp(-(sharp / T) * (E - T)));
    if (a < c->alpha_min) a = 0.0;
    if (a > c->alpha_max) a = c->alpha_max;
    return a;
}

double ref_indicator_raw(const ref_config* c, const double* ue, double* energy_out)
{
    refel r;
    refel_init(&r, c->N, c->points);
    return indicator_raw(c, &r, ue, energy_out);
}

/* ------------------------------------------------------------------ */
/* Learned troubled-cell indicator: a small network maps the element's
 * modal energies (the quantities the indicator above compares) to the
 * blending coefficient; outside the box of features it was trained on,
 * the indicator above is used instead.                                 */
/* ------------------------------------------------------------------ */

static void features_from_energies(int N, const double* en, double* feat)
{
    double cum = en[0];
    for (int k = 1; k <= N; ++k) {
        cum += en[k];
        double r = cum > 0.0 ? en[k] / cum : 0.0;
        if (r < 1e-12) r = 1e-12;
        double v = log10(r) / 6.0 + 1.0;
        feat[k - 1] = v < -1.0 ? -1.0 : v;   /* the floor is exactly -1 */
    }
}

void ref_indicator_features(const ref_config* c, const double* ue, double* feat)
{
    refel r;
    refel_init(&r, c->N, c->points);
    double en[ND];
    indicator_raw(c, &r, ue, en);
    features_from_energies(c->N, en, feat);
}

static double learned_alpha(const ref_config* c, const refel* r, const double* ue, int* fallback)
{
    double en[ND], feat[ND];
    double a_ind = indicator_raw(c, r, ue, en);
    features_from_energies(c->N, en, feat);
    *fallback = 0;
    for (int k = 0; k < c->N; ++k)
        if (!(feat[k] >= c->mlp_lo[k] && feat[k] <= c->mlp_hi[k])) { *fallback = 1; return a_ind; }
    double y;
    ref_mlp_forward(c->mlp_nl, c->mlp_dims, c->mlp_params, 1, feat, &y, NULL);
    if (y < c->alpha_min) y = 0.0;
    if (y > c->alpha_max) y = c->alpha_max;
    return y;
}

double ref_learned_alpha(const ref_config* c, const double* ue, int* fallback)
{
    refel r;
    refel_init(&r, c->N, c->points);
    int fb = 0;
    double a = learned_alpha(c, &r, ue, &fb);
    if (fallback) *fallback = fb;
    return a;
}

/* ------------------------------------------------------------------ */
/* Zhang-Shu scaling limiter of one element (Sec. 3.2; reading: eps_k =
 * min(1e-13, P_k(mean)); linear root for density, 60-step bisection for
 * the other constraints).                                               */
/* ------------------------------------------------------------------ */

static double scale_element(const ref_config* c, const refel* r, double* ue, int* mean_bad)
{
    int M = ref_nvar(c->eq), nd = r->nd, dim = eq_dim(c->eq);
    int nq = dim == 2 ? nd : 1, np = nd * nq, K = ref_nadm(c->eq);
    double ubar[MM], theta_all = 1.0;
    *mean_bad = 0;
    for (int v = 0; v < M; ++v) {
        double s = 0.0;
        for (int q = 0; q < nq; ++q)
            for (int p = 0; p < nd; ++p)
                s += r->w[p] * (dim == 2 ? r->w[q] : 1.0) * ue[v * np + q * nd + p];
        ubar[v] = s;
    }
    for (int k = 0; k < K; ++k) {
        double Pbar = ref_adm(c->eq, k, c->gamma, ubar);
        if (!(Pbar > 0.0)) { *mean_bad = 1; return 0.0; }
        double eps = Pbar < eps_abs(c) ? Pbar : eps_abs(c);
        double theta = 1.0;
        for (int n = 0; n < np; ++n) {
            double un[MM];
            for (int v = 0; v < M; ++v) un[v] = ue[v * np + n];
            if (ref_adm(c->eq, k, c->gamma, un) >= eps) continue;
            double t;
            if (k == 0) t = (ubar[0] - eps) / (ubar[0] - un[0]);
            else t = bisect_root(c, k, ubar, un, eps);
            if (t < theta) theta = t;
        }
        if (theta < 1.0) {
            for (int v = 0; v < M; ++v)
                for (int n = 0; n < np; ++n)
                    ue[v * np + n] = ubar[v] + theta * (ue[v * np + n] - ubar[v]);
        }
        if (theta < theta_all) theta_all = theta;
    }
    return theta_all;
}

double ref_scale_element(const ref_config* c, double* ue, int* mean_bad)
{
    refel r;
    refel_init(&r, c->N, c->points);
    return scale_element(c, &r, ue, mean_bad);
}

/* ------------------------------------------------------------------ */
/* Means and time step (eqs. upmean, time.step.2d)                      */
/* ------------------------------------------------------------------ */

/* ------------------------------------------------------------------ */
/* The scheme in its stage form (eq. crkfr): the inner stages are the local
 * evolutions, the final stage applies the FR derivative (with a Rusanov
 * flux per stage at every face, eq. num.flux.fr) to each stage's flux and
 * combines them with b_i.  Periodic boundaries, no limiter, no source.    */
/* ------------------------------------------------------------------ */

static size_t sidx(int M, int np, int e, int k, int v) { return ((size_t)e * np + k) * M + v; }

void ref_step_crkfr_form(const ref_config* c, const double* u_in, double* u_out, double dt)
{
    refel r;
    refel_init(&r, c->N, c->points);
    const int M = ref_nvar(c->eq), nd = r.nd, dim = eq_dim(c->eq), N = c->N;
    const int nq = dim == 2 ? nd : 1, np = nd * nq, nx = c->nx, ny = c->ny, ne = nx * ny;
    const double dx = (c->x1 - c->x0) / nx, dy = dim == 2 ? (c->y1 - c->y0) / ny : 1.0;
    const int S = c->stages;
    double ta[16], tb[4], tc[4];
    ref_tableau(S, ta, tb, tc);
    const size_t tot = (size_t)ne * np * M;
    double* st = (double*)calloc((size_t)S * tot, sizeof(double));    /* stage values [i][e][k][v] */
    double* loc = (double*)calloc((size_t)S * tot, sizeof(double));   /* local derivative [i][e][k][v] */
    double* un = (double*)malloc(tot * sizeof(double));
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < np; ++k)
            for (int v = 0; v < M; ++v) un[sidx(M, np, e, k, v)] = u_in[((size_t)v * ne + e) * np + k];
    for (int i = 0; i < S; ++i) {
        double* si = st + (size_t)i * tot;
        for (size_t z = 0; z < tot; ++z) {
            double val = un[z];
            for (int j = 0; j < i; ++j) val -= dt * ta[i * 4 + j] * loc[(size_t)j * tot + z];
            si[z] = val;
        }
        double* li = loc + (size_t)i * tot;
        for (int e = 0; e < ne; ++e)
            for (int q = 0; q < nq; ++q)
                for (int p = 0; p < nd; ++p) {
                    double dfx[MM] = {0}, dgy[MM] = {0}, f[MM], g[MM];
                    for (int m = 0; m < nd; ++m) {
                        ref_flux(c->eq, c->gamma, c->adv, &si[sidx(M, np, e, q * nd + m, 0)], f, g);
                        for (int v = 0; v < M; ++v) dfx[v] += r.D[p * nd + m] * f[v];
                        if (dim == 2) {
                            ref_flux(c->eq, c->gamma, c->adv, &si[sidx(M, np, e, m * nd + p, 0)], f, g);
                            for (int v = 0; v < M; ++v) dgy[v] += r.D[q * nd + m] * g[v];
                        }
                    }
                    for (int v = 0; v < M; ++v)
                        li[sidx(M, np, e, q * nd + p, v)] = dfx[v] / dx + (dim == 2 ? dgy[v] / dy : 0.0);
                }
    }
    /* final stage: u^{n+1} = u^n - dt sum_i b_i D_FR f(u^(i)) */
    for (size_t z = 0; z < tot; ++z) u_out[z] = 0.0;
    double* res = (double*)calloc(tot, sizeof(double));
    for (int i = 0; i < S; ++i) {
        const double* si = st + (size_t)i * tot;
        for (size_t z = 0; z < tot; ++z) res[z] += tb[i] * loc[(size_t)i * tot + z];
        for (int d = 0; d < dim; ++d) {
            const int nlines = d == 0 ? nq : nd;
            const double h = d == 0 ? dx : dy;
            for (int e = 0; e < ne; ++e) {
                const int ex = e % nx, ey = e / nx;
                const int en = d == 0 ? ey * nx + (ex + 1) % nx : ((ey + 1) % ny) * nx + ex;   /* high-side neighbour */
                for (int t = 0; t < nlines; ++t) {
                    /* face between e (left/bottom) and en: traces, nodal-flux extrapolations */
                    double um[MM] = {0}, up[MM] = {0}, fhm[MM] = {0}, fhp[MM] = {0}, f[MM], g[MM], fm[MM], fp[MM];
                    for (int m = 0; m < nd; ++m) {
                        const int km = d == 0 ? t * nd + m : m * nd + t;
                        ref_flux(c->eq, c->gamma, c->adv, &si[sidx(M, np, e, km, 0)], f, g);
                        for (int v = 0; v < M; ++v) {
                            um[v] += r.l1[m] * si[sidx(M, np, e, km, v)];
                            fhm[v] += r.l1[m] * (d == 0 ? f[v] : g[v]);
                        }
                        ref_flux(c->eq, c->gamma, c->adv, &si[sidx(M, np, en, km, 0)], f, g);
                        for (int v = 0; v < M; ++v) {
                            up[v] += r.l0[m] * si[sidx(M, np, en, km, v)];
                            fhp[v] += r.l0[m] * (d == 0 ? f[v] : g[v]);
                        }
                    }
                    phys_flux(c, d, um, fm);
                    phys_flux(c, d, up, fp);
                    const int kA = d == 0 ? t * nd + N : N * nd + t, kB = d == 0 ? t * nd : t;
                    const double lam = fmax(sigma_trace(c, d, um, &un[sidx(M, np, e, kA, 0)]),
                                            sigma_trace(c, d, up, &un[sidx(M, np, en, kB, 0)]));
                    double Fs[MM];
                    for (int v = 0; v < M; ++v) Fs[v] = 0.5 * (fm[v] + fp[v]) - 0.5 * lam * (up[v] - um[v]);
                    /* correction of e at its high face and of en at its low face */
                    for (int m = 0; m < nd; ++m) {
                        const int km = d == 0 ? t * nd + m : m * nd + t;
                        for (int v = 0; v < M; ++v) {
                            res[sidx(M, np, e, km, v)] += tb[i] * (Fs[v] - fhm[v]) * (r.l1[m] / r.w[m]) / h;
                            res[sidx(M, np, en, km, v)] -= tb[i] * (Fs[v] - fhp[v]) * (r.l0[m] / r.w[m]) / h;
                        }
                    }
                }
            }
        }
    }
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < np; ++k)
            for (int v = 0; v < M; ++v)
                u_out[((size_t)v * ne + e) * np + k] = un[sidx(M, np, e, k, v)] - dt * res[sidx(M, np, e, k, v)];
    free(st); free(loc); free(un); free(res);
}

void ref_means(const ref_config* c, const double* u, double* ubar)
{
    refel r;
    refel_init(&r, c->N, c->points);
    int M = ref_nvar(c->eq), nd = r.nd, dim = eq_dim(c->eq);
    int nq = dim == 2 ? nd : 1, np = nd * nq, ne = c->nx * c->ny;
    for (int v = 0; v < M; ++v)
        for (int e = 0; e < ne; ++e) {
            double s = 0.0;
            for (int q = 0; q < nq; ++q)
                for (int p = 0; p < nd; ++p)
                    s += r.w[p] * (dim == 2 ? r.w[q] : 1.0) * u[(size_t)v * ne * np + (size_t)e * np + q * nd + p];
            ubar[(size_t)v * ne + e] = s;
        }
}

double ref_compute_dt(const ref_config* c, const double* u)
{
    int M = ref_nvar(c->eq), ne = c->nx * c->ny, dim = eq_dim(c->eq);
    double* ubar = (double*)malloc(sizeof(double) * M * ne);
    ref_means(c, u, ubar);
    double dx = (c->x1 - c->x0) / c->nx, dy = (c->y1 - c->y0) / c->ny;
    double rate = 0.0;
    for (int e = 0; e < ne; ++e) {
        double ub[MM], sx, sy;
        for (int v = 0; v < M; ++v) ub[v] = ubar[(size_t)v * ne + e];
        ref_sigma(c->eq, c->gamma, c->adv, ub, &sx, &sy);
        double re = sx / dx + (dim == 2 ? sy / dy : 0.0);
        if (re > rate) rate = re;
    }
    free(ubar);
    return c->cs * c->cfl / rate;
}

/* ------------------------------------------------------------------ */
/* MUSCL-Hancock on the subcells of one element (Sec. 4.2; details are a
 * reading: minmod slopes on the non-uniform subcell grid, slope scaled
 * to keep face values admissible, Hancock half-step predictor, zero slope
 * when the predicted values are not admissible).                         */
/* ------------------------------------------------------------------ */

typedef struct {
    double xm[NP][MM], xp[NP][MM], ym[NP][MM], yp[NP][MM]; /* predicted face values */
    int slope_limited, fallback;
} mh_out;

static double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

typedef struct {
    const ref_config* c;
    const refel* r;
    const double* u;   /* full state */
    int ne, np, nd, nq, dim, M;
    double dx, dy;
    const double* ghost;   /* far-field ghost states, or NULL */
    double dt;             /* step size (inflow data at the stage times) */
} grid_ctx;

/* far-field ghost state at boundary face point t of the face of element
 * (ex, ey) in direction dir on side (0 low, 1 high); NULL unless far-field */
static const double* ghost_at(const grid_ctx* g, int ex, int ey, int dir, int side, int t)
{
    const ref_config* c = g->c;
    int b = dir * 2 + side;
    if (c->bc[b] != REF_BC_FARFIELD || !g->ghost) return NULL;
    int M = g->M, nq = g->nq, nd = g->nd, nx = c->nx, ny = c->ny;
    size_t xsz = (size_t)ny * nq * M, ysz = (size_t)nx * nd * M;
    if (dir == 0) return g->ghost + side * xsz + ((size_t)ey * nq + t) * M;
    return g->ghost + 2 * xsz + side * ysz + ((size_t)ex * nd + t) * M;
}

/* time-dependent inflow data (Sec. 3.3): g(tau) at a boundary face point,
 * from the polynomial coefficients in the far-field ghost layout */
static int inflow_at(const grid_ctx* g, int ex, int ey, int dir, int side, int t, double tau, double* out)
{
    const ref_config* c = g->c;
    if (c->bc[dir * 2 + side] != REF_BC_INFLOW || !c->inflow) return 0;
    int M = g->M, nq = g->nq, nd = g->nd, nx = c->nx, ny = c->ny;
    size_t xsz = (size_t)ny * nq * M, ysz = (size_t)nx * nd * M;
    size_t gsz = 2 * xsz + (g->dim == 2 ? 2 * ysz : 0);
    size_t off = dir == 0 ? side * xsz + ((size_t)ey * nq + t) * M : 2 * xsz + side * ysz + ((size_t)ex * nd + t) * M;
    double s = tau - c->inflow_tref;
    for (int v = 0; v < M; ++v) {
        double val = 0.0, pw = 1.0;
        for (int k = 0; k < c->inflow_ncoef; ++k) {
            val += c->inflow[(size_t)k * gsz + off + v] * pw;
            pw *= s;
        }
        out[v] = val;
    }
    return 1;
}

/* interface ghost values of an inflow boundary (Sec. 3.3): u^- = g(t^n),
 * U^- = sum_i b_i g(t^n + c_i dt), F^- = sum_i b_i f(g(t^n + c_i dt)) */
static int inflow_ghost(const grid_ctx* g, int ex, int ey, int dir, int side, int t, double* un, double* U,
                        double* F)
{
    const ref_config* c = g->c;
    if (!inflow_at(g, ex, ey, dir, side, t, c->time, un)) return 0;
    double ta[16], tb[4], tc[4];
    ref_tableau(c->stages, ta, tb, tc);
    for (int v = 0; v < g->M; ++v) { U[v] = 0.0; F[v] = 0.0; }
    for (int i = 0; i < c->stages; ++i) {
        double gi[MM], f[MM];
        inflow_at(g, ex, ey, dir, side, t, c->time + tc[i] * g->dt, gi);
        phys_flux(c, dir, gi, f);
        for (int v = 0; v < g->M; ++v) { U[v] += tb[i] * gi[v]; F[v] += tb[i] * f[v]; }
    }
    return 1;
}

/* smallest / largest eigenvalue of the normal flux Jacobian in direction d
 * (for the inflow test: a boundary is fully inflow when every wave enters) */
static double eig_min(const ref_config* c, int d, const double* u)
{
    if (c->eq == REF_LINADV1D) return c->adv;
    if (c->eq == REF_BURGERS1D) return u[0];
    double vn = u[1 + d] / u[0];
    double sx, sy;
    ref_sigma(c->eq, c->gamma, c->adv, u, &sx, &sy);
    return vn - ((d == 0 ? sx : sy) - fabs(vn));
}

static double eig_max(const ref_config* c, int d, const double* u)
{
    if (c->eq == REF_LINADV1D) return c->adv;
    if (c->eq == REF_BURGERS1D) return u[0];
    double vn = u[1 + d] / u[0];
    double sx, sy;
    ref_sigma(c->eq, c->gamma, c->adv, u, &sx, &sy);
    return vn + ((d == 0 ? sx : sy) - fabs(vn));
}

/* solid wall normal to direction d (Sec. 3.3, eq. reflect.time.avg): the
 * ghost state mirrors the interior one, flipping the normal momentum (and,
 * for the ten-moment system, the off-diagonal energy E12); the mirrored
 * normal flux is then -(mirror of F) */
static int wall(const ref_config* c, int dir, int side)
{
    return c->bc[dir * 2 + side] == REF_BC_REFLECT;
}

static double mirror_sign(int eq, int d, int v)
{
    if (v == 1 + d) return -1.0;
    if (is_tenmom(eq) && v == 4) return -1.0;
    return 1.0;
}

static size_t gidx(const grid_ctx* g, int v, int e, int k)
{
    return (size_t)v * g->ne * g->np + (size_t)e * g->np + k;
}

/* neighbour element across a face; -1 for an outflow boundary */
static int nbr_elem(const grid_ctx* g, int ex, int ey, int dir, int side)
{
    const ref_config* c = g->c;
    int nx = c->nx, ny = c->ny;
    if (dir == 0) {
        int t = ex + (side ? 1 : -1);
        if (t < 0) { if (c->bc[0] == REF_BC_PERIODIC) t = nx - 1; else return -1; }
        if (t >= nx) { if (c->bc[1] == REF_BC_PERIODIC) t = 0; else return -1; }
        return ey * nx + t;
    } else {
        int t = ey + (side ? 1 : -1);
        if (t < 0) { if (c->bc[2] == REF_BC_PERIODIC) t = ny - 1; else return -1; }
        if (t >= ny) { if (c->bc[3] == REF_BC_PERIODIC) t = 0; else return -1; }
        return t * nx + ex;
    }
}

static void mh_element(const grid_ctx* g, int ex, int ey, double dt, int blend, mh_out* o)
{
    const ref_config* c = g->c;
    const refel* r = g->r;
    int M = g->M, nd = g->nd, nq = g->nq, dim = g->dim, K = ref_nadm(c->eq), N = r->N;
    int e = ey * c->nx + ex;
    o->slope_limited = 0; o->fallback = 0;
    for (int q = 0; q < nq; ++q)
        for (int p = 0; p < nd; ++p) {
            int k = q * nd + p;
            double u[MM], sx[MM], sy[MM];
            for (int v = 0; v < M; ++v) { u[v] = g->u[gidx(g, v, e, k)]; sx[v] = 0.0; sy[v] = 0.0; }
            double eps[MM];
            for (int kk = 0; kk < K; ++kk) eps[kk] = eps_rel(c) * ref_adm(c->eq, kk, c->gamma, u);
            int u_ok = 1;
            for (int kk = 0; kk < K; ++kk) if (!(eps[kk] > 0.0)) u_ok = 0;
            if (blend == REF_BLEND_MH && u_ok) {
                /* x-neighbours with their reference positions */
                for (int d = 0; d < dim; ++d) {
                    int pos = d == 0 ? p : q;
                    double um[MM], up[MM], xm, xp, x0 = r->xi[pos];
                    if (pos > 0) {
                        int kn = d == 0 ? k - 1 : k - nd;
                        for (int v = 0; v < M; ++v) um[v] = g->u[gidx(g, v, e, kn)];
                        xm = r->xi[pos - 1];
                    } else {
                        int en = nbr_elem(g, ex, ey, d, 0);
                        int kn = d == 0 ? q * nd + N : N * nd + p;
                        double ginb[MM];
                        const double* gh = en < 0 ? ghost_at(g, ex, ey, d, 0, d == 0 ? q : p) : NULL;
                        if (en < 0 && inflow_at(g, ex, ey, d, 0, d == 0 ? q : p, c->time, ginb)) gh = ginb;
                        const int wl = en < 0 && wall(c, d, 0);
                        for (int v = 0; v < M; ++v)
                            um[v] = en >= 0 ? g->u[gidx(g, v, en, kn)]
                                  : (gh ? gh[v] : (wl ? mirror_sign(c->eq, d, v) * u[v] : u[v]));
                        xm = r->xi[N] - 1.0;
                    }
                    if (pos < N) {
                        int kn = d == 0 ? k + 1 : k + nd;
                        for (int v = 0; v < M; ++v) up[v] = g->u[gidx(g, v, e, kn)];
                        xp = r->xi[pos + 1];
                    } else {
                        int en = nbr_elem(g, ex, ey, d, 1);
                        int kn = d == 0 ? q * nd + 0 : 0 * nd + p;
                        double ginb[MM];
                        const double* gh = en < 0 ? ghost_at(g, ex, ey, d, 1, d == 0 ? q : p) : NULL;
                        if (en < 0 && inflow_at(g, ex, ey, d, 1, d == 0 ? q : p, c->time, ginb)) gh = ginb;
                        const int wl = en < 0 && wall(c, d, 1);
                        for (int v = 0; v < M; ++v)
                            up[v] = en >= 0 ? g->u[gidx(g, v, en, kn)]
                                  : (gh ? gh[v] : (wl ? mirror_sign(c->eq, d, v) * u[v] : u[v]));
                        xp = 1.0 + r->xi[0];
                    }
                    for (int v = 0; v < M; ++v) {
                        double s = minmod((u[v] - um[v]) / (x0 - xm), (up[v] - u[v]) / (xp - x0));
                        if (d == 0) sx[v] = s; else sy[v] = s;
                    }
                }
            }
            /* face values of the linear reconstruction (reference units) */
            double hxm = r->sub[p] - r->xi[p], hxp = r->sub[p + 1] - r->xi[p];
            double hym = dim == 2 ? r->sub[q] - r->xi[q] : 0.0;
            double hyp = dim == 2 ? r->sub[q + 1] - r->xi[q] : 0.0;
            double fv[4][MM];
            int nf = dim == 2 ? 4 : 2;
            for (int kk = 0; kk < K && blend == REF_BLEND_MH && u_ok; ++kk) {
                for (int v = 0; v < M; ++v) {
                    fv[0][v] = u[v] + sx[v] * hxm;
                    fv[1][v] = u[v] + sx[v] * hxp;
                    fv[2][v] = u[v] + sy[v] * hym;
                    fv[3][v] = u[v] + sy[v] * hyp;
                }
                double th = 1.0;
                for (int f = 0; f < nf; ++f) {
                    double t = segment_fraction(c, kk, u, fv[f], eps[kk]);
                    if (t < th) th = t;
                }
                if (th < 1.0) {
                    o->slope_limited++;
                    for (int v = 0; v < M; ++v) { sx[v] *= th; sy[v] *= th; }
                }
            }
            for (int v = 0; v < M; ++v) {
                fv[0][v] = u[v] + sx[v] * hxm;
                fv[1][v] = u[v] + sx[v] * hxp;
                fv[2][v] = u[v] + sy[v] * hym;
                fv[3][v] = u[v] + sy[v] * hyp;
            }
            /* Hancock half-step predictor */
            double fm[MM], fp[MM], gm[MM], gp[MM], delta[MM];
            phys_flux(c, 0, fv[0], fm);
            phys_flux(c, 0, fv[1], fp);
            if (dim == 2) { phys_flux(c, 1, fv[2], gm); phys_flux(c, 1, fv[3], gp); }
            for (int v = 0; v < M; ++v) {
                delta[v] = -0.5 * dt * ((fp[v] - fm[v]) / (r->w[p] * g->dx)
                                        + (dim == 2 ? (gp[v] - gm[v]) / (r->w[q] * g->dy) : 0.0));
            }
            double ev[4][MM];
            for (int f = 0; f < nf; ++f)
                for (int v = 0; v < M; ++v) ev[f][v] = fv[f][v] + delta[v];
            int ok = 1;
            for (int f = 0; f < nf && K > 0; ++f)
                if (!admissible_eps(c, ev[f], eps)) ok = 0;
            if (!ok) {
                o->fallback++;
                for (int f = 0; f < nf; ++f)
                    for (int v = 0; v < M; ++v) ev[f][v] = u[v];
            }
            for (int v = 0; v < M; ++v) {
                o->xm[k][v] = ev[0][v];
                o->xp[k][v] = ev[1][v];
                o->ym[k][v] = dim == 2 ? ev[2][v] : u[v];
                o->yp[k][v] = dim == 2 ? ev[3][v] : u[v];
            }
        }
}

/* ------------------------------------------------------------------ */
/* Share of direction d in the low-order update of a face-adjacent subcell
 * (reading for the 2D flux limiter): the update is split as
 * u^L = phi_x u~_x + phi_y u~_y, u~_d = u - dt/(phi_d w h_d) (flux diff.) + dt S,
 * with phi_d proportional to the subcell's own nodal rate sigma_d/(w h_d),
 * so both parts see the Courant number of the whole update.  The subcell
 * has index N in direction d and t in the other one; 1D: 1.              */
/* ------------------------------------------------------------------ */

static double dir_share(const ref_config* c, const refel* r, int d, int t, double dx, double dy,
                        const double* u)
{
    if (eq_dim(c->eq) == 1) return 1.0;
    double sx, sy;
    ref_sigma(c->eq, c->gamma, c->adv, u, &sx, &sy);
    int N = r->N;
    double ax = sx / ((d == 0 ? r->w[N] : r->w[t]) * dx);
    double ay = sy / ((d == 0 ? r->w[t] : r->w[N]) * dy);
    return (d == 0 ? ax : ay) / (ax + ay);
}

/* factor dt / (w_i h_d phi_d) of the flux difference in the low-order update
 * of the face-adjacent subcell with index i (0 or N) along d at line
 * position t, from eq. low.order.update with the direction share above */
static double lo_factor(const ref_config* c, const refel* r, int d, int t, int i, double dx, double dy,
                        const double* u, double dt)
{
    double h = d == 0 ? dx : dy;
    return dt / (r->w[i] * h * dir_share(c, r, d, t, dx, dy, u));
}

double ref_lo_factor(const ref_config* c, int d, int t, int i, const double* u, double dt)
{
    refel r;
    refel_init(&r, c->N, c->points);
    return lo_factor(c, &r, d, t, i, (c->x1 - c->x0) / c->nx, (c->y1 - c->y0) / c->ny, u, dt);
}

/* ------------------------------------------------------------------ */
/* Flux limiter for admissibility in means at one face point (Sec. 4.3;
 * reading).  Side A is the element below the face, B the one above; u
 * their face-adjacent solution points, adj the interior subface flux next
 * to them, S their time-averaged source, k the factors above.  The
 * low-order candidates of the two subcells with face flux G are
 *   A: u_A - kA (G - adj_A) + dt S_A,    B: u_B - kB (adj_B - G) + dt S_B;
 * with G = fLO (the low-order face flux) they are admissible by Theorem 1.
 * For each constraint P_k in order, eps = 0.1 P_k(candidate with fLO), and
 * theta in [0,1] is the fraction of the segment from the fLO candidate to
 * the F candidate keeping P_k >= eps (concavity bound, bisection for a
 * non-concave P_k); F <- theta F + (1 - theta) fLO.  Returns the smallest
 * theta; *bad = 1 when a low-order candidate is itself not admissible
 * (theta = 0 then).                                                      */
/* ------------------------------------------------------------------ */

static double flux_limit_face(const ref_config* c, int hasA, int hasB, const double* uA, const double* uB,
                              const double* adjA, const double* adjB, const double* SA, const double* SB,
                              double kAfac, double kBfac, double dt, const double* fLO, double* F, int* bad)
{
    int M = ref_nvar(c->eq), K = ref_nadm(c->eq);
    double cA[MM], cB[MM], cAlo[MM], cBlo[MM];
    for (int v = 0; v < M; ++v) {
        if (hasA) cAlo[v] = uA[v] - kAfac * (fLO[v] - adjA[v]) + dt * SA[v];
        if (hasB) cBlo[v] = uB[v] - kBfac * (adjB[v] - fLO[v]) + dt * SB[v];
    }
    double theta_face = 1.0;
    *bad = 0;
    for (int k = 0; k < K; ++k) {
        double th = 1.0;
        for (int v = 0; v < M; ++v) {
            if (hasA) cA[v] = uA[v] - kAfac * (F[v] - adjA[v]) + dt * SA[v];
            if (hasB) cB[v] = uB[v] - kBfac * (adjB[v] - F[v]) + dt * SB[v];
        }
        for (int side = 0; side < 2; ++side) {
            if ((side == 0 && !hasA) || (side == 1 && !hasB)) continue;
            const double* lo_c = side == 0 ? cAlo : cBlo;
            const double* hi_c = side == 0 ? cA : cB;
            double Plo = ref_adm(c->eq, k, c->gamma, lo_c);
            if (!(Plo > 0.0)) { *bad = 1; th = 0.0; continue; }
            double eps = eps_rel(c) * Plo;
            double t2 = segment_fraction(c, k, lo_c, hi_c, eps);
            if (t2 < th) th = t2;
        }
        if (th < 1.0)
            for (int v = 0; v < M; ++v) F[v] = th * F[v] + (1.0 - th) * fLO[v];
        if (th < theta_face) theta_face = th;
    }
    return theta_face;
}

double ref_flux_limit_face(const ref_config* c, int hasA, int hasB, const double* uA, const double* uB,
                           const double* adjA, const double* adjB, const double* SA, const double* SB,
                           double kAfac, double kBfac, double dt, const double* fLO, double* F, int* bad)
{
    return flux_limit_face(c, hasA, hasB, uA, uB, adjA, adjB, SA, SB, kAfac, kBfac, dt, fLO, F, bad);
}

/* MUSCL-Hancock predicted face values of every subcell of element (ex, ey)
 * of the state u (the step's own routine; ghost: far-field states or NULL).
 * Outputs [k][v] for the x faces (xm, xp) and y faces (ym, yp); counts[0]
 * subcells with a scaled slope, counts[1] Hancock fallbacks. */
void ref_mh_predict(const ref_config* c, const double* u, int ex, int ey, double dt, const double* ghost,
                    double* xm, double* xp, double* ym, double* yp, int* counts)
{
    refel r;
    refel_init(&r, c->N, c->points);
    int M = ref_nvar(c->eq), nd = r.nd, dim = eq_dim(c->eq);
    int nq = dim == 2 ? nd : 1, np = nd * nq, ne = c->nx * c->ny;
    double dx = (c->x1 - c->x0) / c->nx, dy = (c->y1 - c->y0) / c->ny;
    grid_ctx g = {c, &r, u, ne, np, nd, nq, dim, M, dx, dy, ghost, dt};
    mh_out* o = (mh_out*)malloc(sizeof(mh_out));
    mh_element(&g, ex, ey, dt, c->blend, o);
    for (int k = 0; k < np; ++k)
        for (int v = 0; v < M; ++v) {
            xm[k * M + v] = o->xm[k][v];
            xp[k * M + v] = o->xp[k][v];
            ym[k * M + v] = o->ym[k][v];
            yp[k * M + v] = o->yp[k][v];
        }
    counts[0] = o->slope_limited;
    counts[1] = o->fallback;
    free(o);
}

/* ------------------------------------------------------------------ */
/* Far-field ghost states: boundary traces of a given state             */
/* ------------------------------------------------------------------ */

void ref_boundary_traces(const ref_config* c, const double* u, double* ghost)
{
    refel r;
    refel_init(&r, c->N, c->points);
    int M = ref_nvar(c->eq), nd = r.nd, dim = eq_dim(c->eq);
    int nq = dim == 2 ? nd : 1, np = nd * nq, nx = c->nx, ny = c->ny, ne = nx * ny;
    size_t xsz = (size_t)ny * nq * M, ysz = (size_t)nx * nd * M;
    for (int side = 0; side < 2; ++side)
        for (int ey = 0; ey < ny; ++ey)
            for (int q = 0; q < nq; ++q)
                for (int v = 0; v < M; ++v) {
                    int e = ey * nx + (side ? nx - 1 : 0);
                    double s = 0.0;
                    for (int p = 0; p < nd; ++p)
                        s += (side ? r.l1[p] : r.l0[p]) * u[(size_t)v * ne * np + (size_t)e * np + q * nd + p];
                    ghost[side * xsz + ((size_t)ey * nq + q) * M + v] = s;
                }
    if (dim == 2)
        for (int side = 0; side < 2; ++side)
            for (int ex = 0; ex < nx; ++ex)
                for (int p = 0; p < nd; ++p)
                    for (int v = 0; v < M; ++v) {
                        int e = (side ? ny - 1 : 0) * nx + ex;
                        double s = 0.0;
                        for (int q = 0; q < nd; ++q)
                            s += (side ? r.l1[q] : r.l0[q]) * u[(size_t)v * ne * np + (size_t)e * np + q * nd + p];
                        ghost[2 * xsz + side * ysz + ((size_t)ex * nd + p) * M + v] = s;
                    }
}

/* ------------------------------------------------------------------ */
/* One full step                                                        */
/* ------------------------------------------------------------------ */

int ref_step(const ref_config* c, const double* u_in, double* u_out, double dt,
             const double* alpha_given, double* alpha_out, ref_diag* diag, const double* ghost)
{
    if (c->points == REF_POINTS_GLL && c->blend == REF_BLEND_MH) return -1;
    refel r;
    refel_init(&r, c->N, c->points);
    int M = ref_nvar(c->eq), nd = r.nd, N = c->N, dim = eq_dim(c->eq);
    int nq = dim == 2 ? nd : 1, np = nd * nq, nx = c->nx, ny = c->ny, ne = nx * ny;
    int K = ref_nadm(c->eq);
    double dx = (c->x1 - c->x0) / nx, dy = (c->y1 - c->y0) / ny;
    grid_ctx g = {c, &r, u_in, ne, np, nd, nq, dim, M, dx, dy, ghost, dt};
    int blend = c->blend;
    int limit = c->flux_limiter && blend != REF_BLEND_OFF && K > 0;

    local_out* lo = (local_out*)malloc(sizeof(local_out) * (size_t)ne);
    mh_out* mh = blend != REF_BLEND_OFF ? (mh_out*)malloc(sizeof(mh_out) * (size_t)ne) : NULL;
    double* alpha_raw = (double*)malloc(sizeof(double) * ne);
    double* alpha = (double*)malloc(sizeof(double) * ne);
    /* final face fluxes: x faces [ey][face 0..nx][q][v], y faces [face 0..ny][ex][p][v] */
    double* Fx = (double*)calloc((size_t)ny * (nx + 1) * nq * M, sizeof(double));
    double* Gy = dim == 2 ? (double*)calloc((size_t)(ny + 1) * nx * nd * M, sizeof(double)) : NULL;
    /* interior subface fluxes: x [e][q][p = 0..N-1 for p+1/2][v], y [e][p][q][v] */
    double* fsx = mh ? (double*)calloc((size_t)ne * nq * N * M, sizeof(double)) : NULL;
    double* fsy = mh && dim == 2 ? (double*)calloc((size_t)ne * nd * N * M, sizeof(double)) : NULL;

    ref_diag dg;
    memset(&dg, 0, sizeof(dg));
    dg.min_theta_flux = 1.0; dg.min_theta_scale = 1.0;

    /* 1. local cRK, indicator, subcell predictor, per element */
    long n_sl = 0, n_fb = 0;
#pragma omp parallel for reduction(+ : n_sl, n_fb) schedule(static)
    for (int e = 0; e < ne; ++e) {
        int ex = e % nx, ey = e / nx;
        double ue[MM * NP];
        for (int v = 0; v < M; ++v)
            for (int k = 0; k < np; ++k) ue[v * np + k] = u_in[gidx(&g, v, e, k)];
        local_crk(c, &r, ue, dt, dx, dy, c->x0 + ex * dx, c->y0 + ey * dy, &lo[e]);
        if (c->indicator == REF_IND_PAPER && blend != REF_BLEND_OFF)
            alpha_raw[e] = indicator_raw(c, &r, ue, NULL);
        else if (c->indicator == REF_IND_CONST && blend != REF_BLEND_OFF)
            alpha_raw[e] = c->alpha_const;
        else if (c->indicator == REF_IND_GIVEN && blend != REF_BLEND_OFF)
            alpha_raw[e] = alpha_given[e];
        else if (c->indicator == REF_IND_LEARNED && blend != REF_BLEND_OFF) {
            int fb;
            alpha_raw[e] = learned_alpha(c, &r, ue, &fb);
        } else
            alpha_raw[e] = 0.0;
        if (mh) {
            mh_element(&g, ex, ey, dt, blend, &mh[e]);
            n_sl += mh[e].slope_limited;
            n_fb += mh[e].fallback;
            for (int q = 0; q < nq; ++q)
                for (int p = 0; p < N; ++p)
                    rusanov(c, 0, mh[e].xp[q * nd + p], mh[e].xm[q * nd + p + 1],
                            &fsx[(((size_t)e * nq + q) * N + p) * M]);
            if (dim == 2)
                for (int p = 0; p < nd; ++p)
                    for (int q = 0; q < N; ++q)
                        rusanov(c, 1, mh[e].yp[q * nd + p], mh[e].ym[(q + 1) * nd + p],
                                &fsy[(((size_t)e * nd + p) * N + q) * M]);
        }
    }
    dg.n_slope_limited = n_sl;
    dg.n_hancock_fallback = n_fb;

    /* 2. blending coefficients with neighbour smoothing (reading) */
    for (int e = 0; e < ne; ++e) {
        int ex = e % nx, ey = e / nx;
        double a = alpha_raw[e];
        if ((c->indicator == REF_IND_PAPER || c->indicator == REF_IND_LEARNED) && c->smooth_nbr &&
            blend != REF_BLEND_OFF) {
            for (int d = 0; d < dim; ++d)
                for (int s = 0; s < 2; ++s) {
                    int en = nbr_elem(&g, ex, ey, d, s);
                    if (en >= 0 && 0.5 * alpha_raw[en] > a) a = 0.5 * alpha_raw[en];
                }
        }
        alpha[e] = a;
        if (a > 0.0) dg.n_troubled++;
    }

    /* 3. time-averaged numerical flux at every face, blended and limited */
    long n_lim = 0, n_bad = 0;
    double min_th = 1.0;
    for (int d = 0; d < dim; ++d) {
        int nfaces = d == 0 ? (nx + 1) * ny : (ny + 1) * nx;
#pragma omp parallel for reduction(+ : n_lim, n_bad) reduction(min : min_th) schedule(static)
        for (int fi = 0; fi < nfaces; ++fi) {
            int eL, eR, ex, ey;
            if (d == 0) {
                int i = fi % (nx + 1); ey = fi / (nx + 1);
                ex = i;
                eL = i > 0 ? ey * nx + i - 1 : (c->bc[0] == REF_BC_PERIODIC ? ey * nx + nx - 1 : -1);
                eR = i < nx ? ey * nx + i : (c->bc[1] == REF_BC_PERIODIC ? ey * nx : -1);
            } else {
                int j = fi / nx; ex = fi % nx;
                ey = j;
                eL = j > 0 ? (j - 1) * nx + ex : (c->bc[2] == REF_BC_PERIODIC ? (ny - 1) * nx + ex : -1);
                eR = j < ny ? j * nx + ex : (c->bc[3] == REF_BC_PERIODIC ? ex : -1);
            }
            int npts = d == 0 ? nq : nd;
            for (int t = 0; t < npts; ++t) {
                double Fm[MM], Fp[MM], Um[MM], Up[MM], unm[MM], unp[MM];
                const local_out* A = eL >= 0 ? &lo[eL] : NULL;
                const local_out* B = eR >= 0 ? &lo[eR] : NULL;
                /* central part: EA traces (eq. evaluate) or the extrapolated
                 * averaged flux (eq. extrapolate) */
                const int ae = c->central == REF_CENTRAL_AE;
                for (int v = 0; v < M; ++v) {
                    if (d == 0) {
                        if (A) { Fm[v] = ae ? A->FhR[t][v] : A->FxR[t][v]; Um[v] = A->UxR[t][v]; unm[v] = A->unxR[t][v]; }
                        if (B) { Fp[v] = ae ? B->FhL[t][v] : B->FxL[t][v]; Up[v] = B->UxL[t][v]; unp[v] = B->unxL[t][v]; }
                    } else {
                        if (A) { Fm[v] = ae ? A->GhT[t][v] : A->GyT[t][v]; Um[v] = A->UyT[t][v]; unm[v] = A->unyT[t][v]; }
                        if (B) { Fp[v] = ae ? B->GhB[t][v] : B->GyB[t][v]; Up[v] = B->UyB[t][v]; unp[v] = B->unyB[t][v]; }
                    }
                }
                /* boundary ghost values (Sec. 3.3): outflow copies the interior
                 * side, so F = F^+ (F^-); far-field takes a time-constant state g,
                 * u^- = U^- = g and F^- = f(g); a solid wall mirrors the interior
                 * side (eq. reflect.time.avg) */
                const int wA = !A && wall(c, d, 0), wB = !B && wall(c, d, 1);
                const double* gA = !A ? ghost_at(&g, ex, ey, d, 0, t) : NULL;
                const double* gB = !B ? ghost_at(&g, d == 0 ? ex - 1 : ex, d == 0 ? ey : ey - 1, d, 1, t) : NULL;
                /* time-dependent inflow: u^- = g(t^n) serves as the ghost state,
                 * F^- and U^- are the time averages of the boundary data */
                const int exB = d == 0 ? ex - 1 : ex, eyB = d == 0 ? ey : ey - 1;
                double giA[MM], giB[MM], UiA[MM], UiB[MM], FiA[MM], FiB[MM];
                const int iA = !A && inflow_ghost(&g, ex, ey, d, 0, t, giA, UiA, FiA);
                const int iB = !B && inflow_ghost(&g, exB, eyB, d, 1, t, giB, UiB, FiB);
                if (iA) gA = giA;
                if (iB) gB = giB;
                if (!A) {
                    if (iA) {
                        for (int v = 0; v < M; ++v) { Fm[v] = FiA[v]; Um[v] = UiA[v]; unm[v] = giA[v]; }
                    } else if (gA) {
                        phys_flux(c, d, gA, Fm);
                        for (int v = 0; v < M; ++v) { Um[v] = gA[v]; unm[v] = gA[v]; }
                    } else if (wA) {
                        for (int v = 0; v < M; ++v) {
                            double s = mirror_sign(c->eq, d, v);
                            Fm[v] = -s * Fp[v]; Um[v] = s * Up[v]; unm[v] = s * unp[v];
                        }
                    } else {
                        for (int v = 0; v < M; ++v) { Fm[v] = Fp[v]; Um[v] = Up[v]; unm[v] = unp[v]; }
                    }
                }
                if (!B) {
                    if (iB) {
                        for (int v = 0; v < M; ++v) { Fp[v] = FiB[v]; Up[v] = UiB[v]; unp[v] = giB[v]; }
                    } else if (gB) {
                        phys_flux(c, d, gB, Fp);
                        for (int v = 0; v < M; ++v) { Up[v] = gB[v]; unp[v] = gB[v]; }
                    } else if (wB) {
                        for (int v = 0; v < M; ++v) {
                            double s = mirror_sign(c->eq, d, v);
                            Fp[v] = -s * Fm[v]; Up[v] = s * Um[v]; unp[v] = s * unm[v];
                        }
                    } else {
                        for (int v = 0; v < M; ++v) { Fp[v] = Fm[v]; Up[v] = Um[v]; unp[v] = unm[v]; }
                    }
                }
                /* face-adjacent solution points (ghost: the ghost state) */
                int kA = d == 0 ? t * nd + N : N * nd + t;   /* last subcell of A */
                int kB = d == 0 ? t * nd + 0 : 0 * nd + t;   /* first subcell of B */
                double uA[MM], uB[MM];
                for (int v = 0; v < M; ++v) {
                    if (A) uA[v] = u_in[gidx(&g, v, eL, kA)];
                    if (B) uB[v] = u_in[gidx(&g, v, eR, kB)];
                }
                if (!A) for (int v = 0; v < M; ++v) uA[v] = gA ? gA[v] : (wA ? mirror_sign(c->eq, d, v) : 1.0) * uB[v];
                if (!B) for (int v = 0; v < M; ++v) uB[v] = gB ? gB[v] : (wB ? mirror_sign(c->eq, d, v) : 1.0) * uA[v];
                double lam = fmax(sigma_trace(c, d, unm, uA), sigma_trace(c, d, unp, uB));
                /* dissipative part: D2 (eq. D2), D1 (eq. D1) or D-CSX (eq. dcsx,
                 * one wave speed per stage from that stage's face values) */
                double Dis[MM];
                if (c->dissipation == REF_DISS_DCSX) {
                    double ta[16], tb[4], tc[4];
                    ref_tableau(c->stages, ta, tb, tc);
                    for (int v = 0; v < M; ++v) Dis[v] = 0.0;
                    for (int i = 0; i < c->stages; ++i) {
                        double um[MM], up[MM];
                        for (int v = 0; v < M; ++v) {
                            if (A) um[v] = d == 0 ? A->uixR[i][t][v] : A->uiyT[i][t][v];
                            if (B) up[v] = d == 0 ? B->uixL[i][t][v] : B->uiyB[i][t][v];
                        }
                        if (iA) inflow_at(&g, ex, ey, d, 0, t, c->time + tc[i] * dt, um);
                        else if (!A) for (int v = 0; v < M; ++v) um[v] = gA ? gA[v] : (wA ? mirror_sign(c->eq, d, v) : 1.0) * up[v];
                        if (iB) inflow_at(&g, exB, eyB, d, 1, t, c->time + tc[i] * dt, up);
                        else if (!B) for (int v = 0; v < M; ++v) up[v] = gB ? gB[v] : (wB ? mirror_sign(c->eq, d, v) : 1.0) * um[v];
                        double li = fmax(sigma_trace(c, d, um, uA), sigma_trace(c, d, up, uB));
                        for (int v = 0; v < M; ++v) Dis[v] += tb[i] * 0.5 * li * (up[v] - um[v]);
                    }
                } else if (c->dissipation == REF_DISS_D1) {
                    for (int v = 0; v < M; ++v) Dis[v] = 0.5 * lam * (unp[v] - unm[v]);
                } else {
                    for (int v = 0; v < M; ++v) Dis[v] = 0.5 * lam * (Up[v] - Um[v]);
                }
                double F[MM];
                for (int v = 0; v < M; ++v) F[v] = 0.5 * (Fm[v] + Fp[v]) - Dis[v];
                /* a fully inflow boundary (every wave enters) takes F = F^- */
                const int fiA = iA && eig_min(c, d, giA) > 0.0, fiB = iB && eig_max(c, d, giB) < 0.0;
                if (fiA) for (int v = 0; v < M; ++v) F[v] = Fm[v];
                if (fiB) for (int v = 0; v < M; ++v) F[v] = Fp[v];

                if (blend != REF_BLEND_OFF) {
                    /* predicted values at the face-adjacent subcells */
                    double sA[MM], sB[MM], fLO[MM];
                    for (int v = 0; v < M; ++v) {
                        if (A) sA[v] = d == 0 ? mh[eL].xp[kA][v] : mh[eL].yp[kA][v];
                        if (B) sB[v] = d == 0 ? mh[eR].xm[kB][v] : mh[eR].ym[kB][v];
                    }
                    /* inflow: the boundary data at the half time (the predicted
                     * subcell values are centred there); a fully inflow face
                     * takes its flux */
                    if (iA) inflow_at(&g, ex, ey, d, 0, t, c->time + 0.5 * dt, sA);
                    else if (!A) for (int v = 0; v < M; ++v) sA[v] = gA ? gA[v] : (wA ? mirror_sign(c->eq, d, v) : 1.0) * sB[v];
                    if (iB) inflow_at(&g, exB, eyB, d, 1, t, c->time + 0.5 * dt, sB);
                    else if (!B) for (int v = 0; v < M; ++v) sB[v] = gB ? gB[v] : (wB ? mirror_sign(c->eq, d, v) : 1.0) * sA[v];
                    rusanov(c, d, sA, sB, fLO);   /* eq. mh.at.face (fo.at.face when FO) */
                    if (fiA) phys_flux(c, d, sA, fLO);
                    if (fiB) phys_flux(c, d, sB, fLO);
                    double af = A && B ? 0.5 * (alpha[eL] + alpha[eR]) : alpha[A ? eL : eR];
                    for (int v = 0; v < M; ++v) F[v] = (1.0 - af) * F[v] + af * fLO[v];   /* eq. Fblend */

                    if (limit) {
                        /* candidate low-order updates at the two face-adjacent subcells */
                        double adjA[MM], adjB[MM], SA[MM], SB[MM];
                        double kAfac = 0.0, kBfac = 0.0;
                        if (A) {
                            kAfac = lo_factor(c, &r, d, t, N, dx, dy, uA, dt);
                            for (int v = 0; v < M; ++v) {
                                adjA[v] = d == 0 ? fsx[(((size_t)eL * nq + t) * N + N - 1) * M + v]
                                                 : fsy[(((size_t)eL * nd + t) * N + N - 1) * M + v];
                                SA[v] = lo[eL].S[kA][v];
                            }
                        }
                        if (B) {
                            kBfac = lo_factor(c, &r, d, t, 0, dx, dy, uB, dt);
                            for (int v = 0; v < M; ++v) {
                                adjB[v] = d == 0 ? fsx[(((size_t)eR * nq + t) * N + 0) * M + v]
                                                 : fsy[(((size_t)eR * nd + t) * N + 0) * M + v];
                                SB[v] = lo[eR].S[kB][v];
                            }
                        }
                        int bad = 0;
                        double theta_face = flux_limit_face(c, A != NULL, B != NULL, uA, uB, adjA, adjB, SA, SB,
                                                            kAfac, kBfac, dt, fLO, F, &bad);
                        if (theta_face < 1.0) n_lim++;
                        if (bad) n_bad++;
                        if (theta_face < min_th) min_th = theta_face;
                    }
                }
                double* out = d == 0 ? &Fx[(((size_t)ey * (nx + 1) + ex) * nq + t) * M]
                                     : &Gy[(((size_t)ey * nx + ex) * nd + t) * M];
                for (int v = 0; v < M; ++v) out[v] = F[v];
            }
        }
    }
    dg.n_flux_limited = n_lim;
    dg.n_lo_inadmissible = n_bad;
    dg.min_theta_flux = min_th;

    /* 4. FR update (eq. crkfr.avg / crkfr.source), low-order subcell update
     *    (eq. low.order.update), blend (eq. blended.scheme), scaling */
    long n_sc = 0, n_mb = 0;
    double min_ts = 1.0;
#pragma omp parallel for reduction(+ : n_sc, n_mb) reduction(min : min_ts) schedule(static)
    for (int e = 0; e < ne; ++e) {
        int ex = e % nx, ey = e / nx;
        const local_out* o = &lo[e];
        double unew[MM * NP];
        for (int q = 0; q < nq; ++q)
            for (int p = 0; p < nd; ++p) {
                int k = q * nd + p;
                for (int v = 0; v < M; ++v) {
                    double FL = Fx[(((size_t)ey * (nx + 1) + ex) * nq + q) * M + v];
                    double FR = Fx[(((size_t)ey * (nx + 1) + ex + 1) * nq + q) * M + v];
                    double dfx = 0.0;
                    for (int m = 0; m < nd; ++m) dfx += r.D[p * nd + m] * o->F[q * nd + m][v];
                    double resx = dfx + (FR - o->FhR[q][v]) * r.l1[p] / r.w[p]
                                      - (FL - o->FhL[q][v]) * r.l0[p] / r.w[p];
                    double resy = 0.0;
                    double GB = 0.0, GT = 0.0;
                    if (dim == 2) {
                        GB = Gy[(((size_t)ey * nx + ex) * nd + p) * M + v];
                        GT = Gy[(((size_t)(ey + 1) * nx + ex) * nd + p) * M + v];
                        double dgy = 0.0;
                        for (int m = 0; m < nd; ++m) dgy += r.D[q * nd + m] * o->G[m * nd + p][v];
                        resy = dgy + (GT - o->GhT[p][v]) * r.l1[q] / r.w[q]
                                   - (GB - o->GhB[p][v]) * r.l0[q] / r.w[q];
                    }
                    double un = u_in[gidx(&g, v, e, k)];
                    double uH = un - dt / dx * resx - (dim == 2 ? dt / dy * resy : 0.0) + dt * o->S[k][v];
                    double a = alpha[e];
                    double val = uH;
                    if (blend != REF_BLEND_OFF && a > 0.0) {
                        double fm = p == 0 ? FL : fsx[(((size_t)e * nq + q) * N + p - 1) * M + v];
                        double fp = p == N ? FR : fsx[(((size_t)e * nq + q) * N + p) * M + v];
                        double uL = un - dt / (r.w[p] * dx) * (fp - fm) + dt * o->S[k][v];
                        if (dim == 2) {
                            double gm = q == 0 ? GB : fsy[(((size_t)e * nd + p) * N + q - 1) * M + v];
                            double gp = q == N ? GT : fsy[(((size_t)e * nd + p) * N + q) * M + v];
                            uL -= dt / (r.w[q] * dy) * (gp - gm);
                        }
                        val = (1.0 - a) * uH + a * uL;
                    }
                    unew[v * np + k] = val;
                }
            }
        if (c->scaling && K > 0) {
            int mb = 0;
            double th = scale_element(c, &r, unew, &mb);
            if (mb) n_mb++;
            else if (th < 1.0) n_sc++;
            if (th < min_ts) min_ts = th;
        }
        for (int v = 0; v < M; ++v)
            for (int k = 0; k < np; ++k) u_out[gidx(&g, v, e, k)] = unew[v * np + k];
    }
    dg.n_scaled = n_sc;
    dg.n_mean_inadmissible = n_mb;
    dg.min_theta_scale = min_ts;

    if (alpha_out) for (int e = 0; e < ne; ++e) alpha_out[e] = alpha[e];
    if (diag) *diag = dg;

    free(lo); free(mh); free(alpha_raw); free(alpha);
    free(Fx); free(Gy); free(fsx); free(fsy);
    return n_mb ? -5 : 0;
}

/* ------------------------------------------------------------------ */
/* Small MLP (tanh hidden layers, sigmoid output, mean squared error) for
 * the learned troubled-cell indicator: plain forward and reverse-mode
 * backward, used to check the GPU training kernels.                      */
/* ------------------------------------------------------------------ */

static size_t mlp_nparams(int nl, const int* dims)
{
    size_t n = 0;
    for (int l = 0; l < nl; ++l) n += (size_t)dims[l + 1] * dims[l] + dims[l + 1];
    return n;
}

static size_t mlp_width_sum(int nl, const int* dims)
{
    size_t s = 0;
    for (int l = 0; l <= nl; ++l) s += dims[l];
    return s;
}

/* acts (optional): per row, the activations of every layer concatenated */
void ref_mlp_forward(int nl, const int* dims, const double* params, int nrows,
                     const double* x, double* y, double* acts)
{
    size_t ws = mlp_width_sum(nl, dims);
    double* buf = (double*)malloc(sizeof(double) * ws);
    for (int n = 0; n < nrows; ++n) {
        double* a = buf;
        for (int i = 0; i < dims[0]; ++i) a[i] = x[(size_t)n * dims[0] + i];
        const double* P = params;
        size_t off = 0;
        for (int l = 0; l < nl; ++l) {
            const double* W = P;
            const double* b = P + (size_t)dims[l + 1] * dims[l];
            double* in = buf + off;
            double* out = in + dims[l];
            for (int j = 0; j < dims[l + 1]; ++j) {
                double s = b[j];
                for (int i = 0; i < dims[l]; ++i) s += W[(size_t)j * dims[l] + i] * in[i];
                out[j] = l + 1 < nl ? tanh(s) : 1.0 / (1.0 + exp(-s));
            }
            P = b + dims[l + 1];
            off += dims[l];
        }
        y[n] = buf[ws - 1];
        if (acts) memcpy(acts + (size_t)n * ws, buf, sizeof(double) * ws);
    }
    free(buf);
}

double ref_mlp_loss_grad(int nl, const int* dims, const double* params, int nrows,
                         const double* x, const double* target, double* grad)
{
    size_t ws = mlp_width_sum(nl, dims), npar = mlp_nparams(nl, dims);
    double* acts = (double*)malloc(sizeof(double) * ws * (size_t)nrows);
    double* y = (double*)malloc(sizeof(double) * nrows);
    ref_mlp_forward(nl, dims, params, nrows, x, y, acts);
    if (grad) memset(grad, 0, sizeof(double) * npar);
    double loss = 0.0;
    int maxw = 0;
    for (int l = 0; l <= nl; ++l) if (dims[l] > maxw) maxw = dims[l];
    double* delta = (double*)malloc(sizeof(double) * maxw);
    double* dprev = (double*)malloc(sizeof(double) * maxw);
    /* layer parameter offsets */
    size_t poff[16];
    poff[0] = 0;
    for (int l = 0; l < nl; ++l) poff[l + 1] = poff[l] + (size_t)dims[l + 1] * dims[l] + dims[l + 1];
    size_t aoff[17];
    aoff[0] = 0;
    for (int l = 0; l < nl; ++l) aoff[l + 1] = aoff[l] + dims[l];
    for (int n = 0; n < nrows; ++n) {
        double r = y[n] - target[n];
        loss += r * r;
        if (!grad) continue;
        const double* a = acts + (size_t)n * ws;
        /* output layer: d loss / d pre-activation = 2 r / nrows * y (1 - y) */
        delta[0] = 2.0 * r / nrows * y[n] * (1.0 - y[n]);
        for (int l = nl - 1; l >= 0; --l) {
            const double* in = a + aoff[l];
            const double* W = params + poff[l];
            double* gW = grad + poff[l];
            double* gb = gW + (size_t)dims[l + 1] * dims[l];
            for (int j = 0; j < dims[l + 1]; ++j) {
                gb[j] += delta[j];
                for (int i = 0; i < dims[l]; ++i) gW[(size_t)j * dims[l] + i] += delta[j] * in[i];
            }
            if (l > 0) {
                for (int i = 0; i < dims[l]; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < dims[l + 1]; ++j) s += W[(size_t)j * dims[l] + i] * delta[j];
                    dprev[i] = s * (1.0 - in[i] * in[i]);   /* tanh' */
                }
                for (int i = 0; i < dims[l]; ++i) delta[i] = dprev[i];
            }
        }
    }
    free(acts); free(y); free(delta); free(dprev);
    return loss / nrows;
}
