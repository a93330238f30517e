/* Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * FP64 oracle (tests/test_sanitizers.py compiles it with the oracle source):
 * a few steps of every equation with every boundary kind and the limiter
 * options, plus the element routines the tests call one by one.  Exits 1 on
 * a failed step status; the sanitizers abort on a memory or UB error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/crkfr_oracle.h"

static double gl_x[8], gl_w[8];

static int nvar_of(int eq) { return ref_nvar(eq); }
static int dim_of(int eq) { return eq == REF_EULER2D || eq == REF_TENMOM2D ? 2 : 1; }

/* a smooth admissible state of each equation at reference point (x, y) in [0,1]^2 */
static void state_at(int eq, double x, double y, double* u)
{
    const double r = 1.0 + 0.3 * sin(6.283185307179586 * x) * cos(6.283185307179586 * y);
    const double v1 = 0.2 * cos(6.283185307179586 * x), v2 = 0.1 * sin(6.283185307179586 * y);
    const double p = 0.8 + 0.2 * x * y;
    switch (eq) {
    case REF_LINADV1D:
    case REF_BURGERS1D: u[0] = r - 1.0; break;
    case REF_EULER1D: u[0] = r; u[1] = r * v1; u[2] = p / 0.4 + 0.5 * r * v1 * v1; break;
    case REF_EULER2D:
        u[0] = r; u[1] = r * v1; u[2] = r * v2; u[3] = p / 0.4 + 0.5 * r * (v1 * v1 + v2 * v2); break;
    default: /* ten-moment: rho, rho v, E11, E12, E22 with P = diag(p, 1.1 p) + 0.1 p off-diagonal */
        u[0] = r; u[1] = r * v1; u[2] = r * v2;
        u[3] = 0.5 * p + 0.5 * r * v1 * v1;
        u[4] = 0.5 * 0.1 * p + 0.5 * r * v1 * v2;
        u[5] = 0.5 * 1.1 * p + 0.5 * r * v2 * v2;
        if (eq == REF_TENMOM1D) { u[2] = 0.0; u[4] = 0.05 * p; u[5] = 0.55 * p; }
        break;
    }
}

static double* make_state(int eq, int N, int nx, int ny)
{
    const int M = nvar_of(eq), nd = N + 1, nq = dim_of(eq) == 2 ? nd : 1, np = nd * nq, ne = nx * ny;
    double* u = (double*)malloc(sizeof(double) * (size_t)M * ne * np);
    ref_gl(N, gl_x, gl_w);
    for (int e = 0; e < ne; ++e) {
        const int ex = e % nx, ey = e / nx;
        for (int k = 0; k < np; ++k) {
            double s[6];
            const double x = (ex + gl_x[k % nd]) / nx, y = dim_of(eq) == 2 ? (ey + gl_x[k / nd]) / ny : 0.5;
            /* a jump in the middle of the domain for the limiter chain */
            state_at(eq, x, y, s);
            if (x > 0.5 && eq != REF_LINADV1D && eq != REF_BURGERS1D) { s[0] *= 0.5; for (int v = 1; v < M; ++v) s[v] *= 0.5; }
            for (int v = 0; v < M; ++v) u[((size_t)v * ne + e) * np + k] = s[v];
        }
    }
    return u;
}

static int run(int eq, int N, int nx, int ny, int bc, int blend, int lim, int diss, int central, int source)
{
    ref_config c;
    memset(&c, 0, sizeof(c));
    c.eq = eq; c.N = N; c.nx = nx; c.ny = ny;
    c.stages = N + 1 < 4 ? N + 1 : 4;
    for (int i = 0; i < 4; ++i) c.bc[i] = bc;
    c.blend = blend; c.indicator = REF_IND_PAPER; c.smooth_nbr = 1;
    c.flux_limiter = lim; c.scaling = lim;
    c.source = source && (eq == REF_TENMOM2D || eq == REF_TENMOM1D);
    c.x0 = 0.0; c.x1 = 1.0; c.y0 = 0.0; c.y1 = 1.0;
    c.gamma = 1.4; c.adv = 1.0; c.cfl = 0.05; c.cs = 0.98;
    c.alpha_min = 1e-3; c.alpha_max = 1.0;
    c.src_amp = 2.0; c.src_kappa = 20.0; c.src_xc = 0.5; c.src_yc = 0.5;
    c.dissipation = diss; c.central = central;
    const int M = nvar_of(eq), nd = N + 1, np = dim_of(eq) == 2 ? nd * nd : nd, ne = nx * ny;
    double* u = make_state(eq, N, nx, ny);
    double* out = (double*)malloc(sizeof(double) * (size_t)M * ne * np);
    double* alpha = (double*)calloc((size_t)ne, sizeof(double));
    const size_t gsz = (2 * (size_t)ny * (dim_of(eq) == 2 ? nd : 1) + (dim_of(eq) == 2 ? 2 * (size_t)nx * nd : 0)) * M;
    double* ghost = (double*)malloc(sizeof(double) * gsz);
    ref_boundary_traces(&c, u, ghost);
    const double dt = ref_compute_dt(&c, u);
    int bad = 0;
    for (int s = 0; s < 3; ++s) {
        ref_diag d;
        const int st = ref_step(&c, u, out, dt, alpha, alpha, &d, ghost);
        if (st != 0 && st != -5) bad = 1;
        memcpy(u, out, sizeof(double) * (size_t)M * ne * np);
    }
    double e[8];
    (void)ref_indicator_raw(&c, u, e);
    free(u); free(out); free(alpha); free(ghost);
    return bad;
}

int main(void)
{
    int fails = 0;
    const int eqs[] = {REF_LINADV1D, REF_EULER1D, REF_EULER2D, REF_TENMOM2D, REF_BURGERS1D, REF_TENMOM1D};
    for (int ie = 0; ie < 6; ++ie) {
        const int eq = eqs[ie], d2 = dim_of(eq) == 2;
        const int scalar = eq == REF_LINADV1D || eq == REF_BURGERS1D;
        for (int N = 1; N <= 4; ++N)
            for (int bc = 0; bc <= 3; ++bc) {
                if (bc == REF_BC_REFLECT && scalar) continue;
                const int nx = d2 ? 5 : 9, ny = d2 ? 4 : 1;
                fails += run(eq, N, nx, ny, bc, REF_BLEND_OFF, 0, REF_DISS_D2, REF_CENTRAL_EA, 0);
                fails += run(eq, N, nx, ny, bc, REF_BLEND_MH, !scalar, REF_DISS_D2, REF_CENTRAL_EA, 1);
                fails += run(eq, N, nx, ny, bc, REF_BLEND_FO, !scalar, REF_DISS_DCSX, REF_CENTRAL_AE, 1);
                fails += run(eq, N, nx, ny, bc, REF_BLEND_MH, 0, REF_DISS_D1, REF_CENTRAL_EA, 0);
            }
    }
    printf("sanitized oracle runs done, %d failed statuses\n", fails);
    return fails ? 1 : 0;
}
