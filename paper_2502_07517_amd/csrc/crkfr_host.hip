// Host runtime and C ABI of the cRKFR step (declarations in include/crkfr.h).
//
// The solver owns its device buffers, precomputes the reference-element
// operators in FP64 (Sec. 2: Gauss-Legendre points, Lagrange basis,
// differentiation matrix, boundary values, Radau correction derivatives
// g_R'(xi_p) = l_p(1)/w_p, g_L'(xi_p) = -l_p(0)/w_p, orthonormal Legendre
// values for the indicator) and enqueues one step as
//   k_prep -> k_local -> k_face(x) -> k_face(y) -> k_update
// on its stream.  CFL(N) of eq. time.step.2d comes from the library's own
// Fourier analysis unless the caller gives one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/crkfr.h"
#include "crkfr_internal.hpp"
#include "crkfr_launch.hpp"

using namespace crkfr;

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int crkfr::set_error(int code, const std::string& msg) { return fail(code, msg); }

#define HIP_TRY(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(CRKFR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
    } while (0)

// ----------------------------------------------------------------------------
// reference element (FP64, host)
// ----------------------------------------------------------------------------
struct RefElem {
    int N, points;
    double xi[MAXND], w[MAXND], D[MAXND][MAXND], l0[MAXND], l1[MAXND], sub[MAXND + 1];
    double Pm[MAXND][MAXND];   // Pm[k][p]: orthonormal Legendre coefficient k of the nodal interpolant
};

// Legendre P_n and P_n' on [-1,1] by the Bonnet recurrence
static void legendre_pair(int n, double x, double& P, double& dP)
{
    double pm1 = 1.0, p = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double pn = ((2 * k + 1) * x * p - k * pm1) / (k + 1);
        pm1 = p;
        p = pn;
    }
    P = p;
    dP = n * (pm1 - x * p) / (1.0 - x * x);
}

// Solution points on [0,1] (eq. soln.points): Gauss-Legendre, or
// Gauss-Legendre-Lobatto (the zeros of P_{N+1} - P_{N-1}, which vanishes at
// x = +-1 and is (1 - x^2) P_N' up to a factor; its derivative is
// (2N+1) P_N).  The correction enters as g_R'(xi_p) = l_p(1)/w_p and
// g_L'(xi_p) = -l_p(0)/w_p, the identity of the Radau correction with GL
// points and of g2 with GLL points (eq. fr.equiv).
static void make_ref(int N, int points, RefElem& r)
{
    const int n = N + 1;
    r.N = N;
    r.points = points;
    if (points == CRKFR_POINTS_GLL) {
        for (int i = 0; i < n; ++i) {
            double x = -std::cos(M_PI * i / N);
            if (i > 0 && i < N)
                for (int it = 0; it < 50; ++it) {
                    double Pp, dPp, Pm1, dPm1, PN, dPN;
                    legendre_pair(N + 1, x, Pp, dPp);
                    legendre_pair(N - 1, x, Pm1, dPm1);
                    legendre_pair(N, x, PN, dPN);
                    const double step = (Pp - Pm1) / ((2.0 * N + 1.0) * PN);
                    x -= step;
                    if (std::fabs(step) < 1e-17) break;
                }
            double PN = 1.0, dPN = 0.0;
            if (i > 0 && i < N) legendre_pair(N, x, PN, dPN);
            r.xi[i] = 0.5 + 0.5 * x;
            r.w[i] = 1.0 / (N * (N + 1.0) * PN * PN);   // 2/(N(N+1)P_N^2) halved for [0,1]
        }
        r.xi[0] = 0.0;
        r.xi[N] = 1.0;
    } else {
        // Gauss-Legendre nodes: Newton from the asymptotic guess, then weights
        for (int i = 0; i < n; ++i) {
            double x = std::cos(M_PI * (4.0 * (n - 1 - i) + 3.0) / (4.0 * n + 2.0));
            for (int it = 0; it < 50; ++it) {
                double P, dP;
                legendre_pair(n, x, P, dP);
                double step = P / dP;
                x -= step;
                if (std::fabs(step) < 1e-17) break;
            }
            double P, dP;
            legendre_pair(n, x, P, dP);
            r.xi[i] = 0.5 + 0.5 * x;
            r.w[i] = 1.0 / ((1.0 - x * x) * dP * dP);   // 2/((1-x^2)P'^2) halved for [0,1]
        }
    }
    // barycentric weights, Lagrange values at 0 and 1, differentiation matrix
    double bw[MAXND];
    for (int j = 0; j < n; ++j) {
        double prod = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != j) prod *= (r.xi[j] - r.xi[m]);
        bw[j] = 1.0 / prod;
    }
    for (int side = 0; side < 2; ++side) {
        const double x = side ? 1.0 : 0.0;
        double* l = side ? r.l1 : r.l0;
        bool hit = false;
        for (int j = 0; j < n; ++j)
            if (r.xi[j] == x) hit = true;
        if (hit) {   // a node on the face: the Lagrange values are a unit vector
            for (int j = 0; j < n; ++j) l[j] = r.xi[j] == x ? 1.0 : 0.0;
            continue;
        }
        double den = 0.0, num[MAXND];
        for (int j = 0; j < n; ++j) {
            num[j] = bw[j] / (x - r.xi[j]);
            den += num[j];
        }
        for (int j = 0; j < n; ++j) l[j] = num[j] / den;
    }
    for (int i = 0; i < n; ++i) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            r.D[i][j] = (bw[j] / bw[i]) / (r.xi[i] - r.xi[j]);
            diag -= r.D[i][j];
        }
        r.D[i][i] = diag;
    }
    r.sub[0] = 0.0;
    for (int p = 0; p < n; ++p) r.sub[p + 1] = r.sub[p] + r.w[p];
    r.sub[n] = 1.0;
    // modal projection: V[p][k] = L_k(xi_p) with L_k = sqrt(2k+1) P_k(2 xi - 1);
    // GL: Pm = diag-weighted transpose (the nodal rule is exact to 2N+1);
    // GLL: Pm = V^{-1} by Gauss-Jordan elimination with partial pivoting
    double V[MAXND][MAXND];
    for (int p = 0; p < n; ++p)
        for (int k = 0; k < n; ++k) {
            double P, dP;
            legendre_pair(k, 2.0 * r.xi[p] - 1.0, P, dP);
            V[p][k] = std::sqrt(2.0 * k + 1.0) * P;
        }
    if (points != CRKFR_POINTS_GLL) {
        for (int k = 0; k < n; ++k)
            for (int p = 0; p < n; ++p) r.Pm[k][p] = r.w[p] * V[p][k];
    } else {
        double A[MAXND][2 * MAXND];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < 2 * n; ++j) A[i][j] = j < n ? V[i][j] : (j - n == i ? 1.0 : 0.0);
        for (int col = 0; col < n; ++col) {
            int piv = col;
            for (int i = col + 1; i < n; ++i)
                if (std::fabs(A[i][col]) > std::fabs(A[piv][col])) piv = i;
            for (int j = 0; j < 2 * n; ++j) std::swap(A[col][j], A[piv][j]);
            const double d = A[col][col];
            for (int j = 0; j < 2 * n; ++j) A[col][j] /= d;
            for (int i = 0; i < n; ++i) {
                if (i == col) continue;
                const double f = A[i][col];
                for (int j = 0; j < 2 * n; ++j) A[i][j] -= f * A[col][j];
            }
        }
        // V c = u  =>  c = V^{-1} u: rows of V^{-1} give the coefficients
        for (int k = 0; k < n; ++k)
            for (int p = 0; p < n; ++p) r.Pm[k][p] = A[k][n + p];
    }
}

template <class real>
static void fill_tab(const RefElem& r, int S, RefTab<real>& t)
{
    std::memset(&t, 0, sizeof(t));
    for (int i = 0; i <= r.N; ++i) {
        for (int j = 0; j <= r.N; ++j) {
            t.D[i][j] = (real)r.D[i][j];
            t.Pm[i][j] = (real)r.Pm[i][j];
        }
        t.l0[i] = (real)r.l0[i];
        t.l1[i] = (real)r.l1[i];
        t.bR[i] = (real)(r.l1[i] / r.w[i]);
        t.bL[i] = (real)(r.l0[i] / r.w[i]);
        t.w[i] = (real)r.w[i];
        t.xi[i] = (real)r.xi[i];
    }
    for (int i = 0; i <= r.N + 1; ++i) t.sub[i] = (real)r.sub[i];
    for (int i = 0; i <= r.N; ++i) {
        // (GLL points meet across faces: distance 0, unused since MUSCL-Hancock
        // blending needs GL points)
        const double xm = i > 0 ? r.xi[i - 1] : r.xi[r.N] - 1.0;
        const double xp = i < r.N ? r.xi[i + 1] : 1.0 + r.xi[0];
        t.rdm[i] = r.xi[i] > xm ? (real)(1.0 / (r.xi[i] - xm)) : (real)0;
        t.rdp[i] = xp > r.xi[i] ? (real)(1.0 / (xp - r.xi[i])) : (real)0;
    }
    for (int i = 0; i < S; ++i) {
        t.tb[i] = (real)tab_b(S, i);
        t.ta[i] = i < S - 1 ? (real)tab_a(S, i) : (real)0;
    }
}

// ----------------------------------------------------------------------------
// Fourier analysis of the linear scheme for CFL(N)
//   U = P u, P = sum_i b_i R_i, R_1 = I, R_{i+1} = I - nu_a a_{i+1,i} D R_i
//   D2 flux with dissipation speed lambda, wave speed a = ratio * lambda
//   G = I - (nu_a D + b_R (F_R - nu_a l1^T) - b_L (F_L - nu_a l0^T)) P
//   (D1: the dissipative part of F_R, F_L acts on u instead of U = P u;
//   D-CSX equals D2 for a linear flux)
// spectral radius from the growth of ||G^(2^j)|| under repeated squaring.
// ----------------------------------------------------------------------------
typedef std::complex<double> cplx;

static double spectral_radius(int n, const cplx* G)
{
    cplx A[MAXND * MAXND], B[MAXND * MAXND];
    std::memcpy(A, G, sizeof(cplx) * n * n);
    double logsum = 0.0, scale = 1.0;
    for (int j = 0; j < 48; ++j) {
        double nrm = 0.0;
        for (int i = 0; i < n * n; ++i) nrm += std::norm(A[i]);
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) return 0.0;
        logsum += std::log(nrm) * scale;
        for (int i = 0; i < n * n; ++i) A[i] /= nrm;
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                cplx s = 0.0;
                for (int k = 0; k < n; ++k) s += A[r * n + k] * A[k * n + c];
                B[r * n + c] = s;
            }
        std::memcpy(A, B, sizeof(cplx) * n * n);
        scale *= 0.5;
    }
    return std::exp(logsum);
}

static double max_growth(const RefElem& r, int S, double nu, double ratio, int nk, bool d1)
{
    const int n = r.N + 1;
    const double nua = ratio * nu;
    double P[MAXND][MAXND], R[MAXND][MAXND], T[MAXND][MAXND];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            R[i][j] = i == j ? 1.0 : 0.0;
            P[i][j] = tab_b(S, 0) * R[i][j];
        }
    for (int st = 1; st < S; ++st) {
        const double a = tab_a(S, st - 1);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += r.D[i][k] * R[k][j];
                T[i][j] = (i == j ? 1.0 : 0.0) - nua * a * s;
            }
        std::memcpy(R, T, sizeof(R));
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) P[i][j] += tab_b(S, st) * R[i][j];
    }
    double worst = 0.0;
    for (int ik = 0; ik < nk; ++ik) {
        const double kap = 2.0 * M_PI * ik / (nk - 1);
        const cplx E = std::polar(1.0, kap), Ec = std::conj(E);
        cplx op[MAXND * MAXND], dis[MAXND * MAXND], G[MAXND * MAXND];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cplx FRc = 0.5 * nua * (r.l1[j] + E * r.l0[j]), FRd = -0.5 * nu * (E * r.l0[j] - r.l1[j]);
                cplx FLc = 0.5 * nua * (Ec * r.l1[j] + r.l0[j]), FLd = -0.5 * nu * (r.l0[j] - Ec * r.l1[j]);
                op[i * n + j] = nua * r.D[i][j] + (r.l1[i] / r.w[i]) * (FRc - nua * r.l1[j])
                                - (r.l0[i] / r.w[i]) * (FLc - nua * r.l0[j]);
                dis[i * n + j] = (r.l1[i] / r.w[i]) * FRd - (r.l0[i] / r.w[i]) * FLd;
                if (!d1) op[i * n + j] += dis[i * n + j];
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cplx s = 0.0;
                for (int k = 0; k < n; ++k) s += op[i * n + k] * P[k][j];
                G[i * n + j] = (i == j ? 1.0 : 0.0) - s - (d1 ? dis[i * n + j] : 0.0);
            }
        double rho = spectral_radius(n, G);
        worst = rho > worst ? rho : worst;
    }
    return worst;
}

extern "C" double crkfr_fourier_cfl(int N, int stages, int system, int dissipation, int points, double tol)
{
    if (N < 1 || N > 4 || stages == 1 || stages < 0 || stages > 4 || dissipation < 0 || dissipation > 2 ||
        points < 0 || points > 1)
        return -1.0;
    const bool d1 = dissipation == CRKFR_DISS_D1;
    RefElem r;
    make_ref(N, points, r);
    const int S = stages > 0 ? stages : std::min(N + 1, 4);
    const int nr = system ? 11 : 1, nk = 385;
    auto stable = [&](double nu) {
        for (int ir = 0; ir < nr; ++ir) {
            double ratio = system ? (double)ir / (nr - 1) : 1.0;
            if (max_growth(r, S, nu, ratio, nk, d1) > 1.0 + tol) return false;
        }
        return true;
    };
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 4 && stable(hi); ++it) {
        lo = hi;
        hi *= 2.0;
    }
    for (int it = 0; it < 40; ++it) {
        double mid = 0.5 * (lo + hi);
        if (stable(mid)) lo = mid; else hi = mid;
    }
    return lo;
}

// CFL(N) for (equation kind, stages, D1 or not); the tolerance is 1e-10 except
// for the 4-stage tableau at N = 4 (weak growth below 5e-6 per step)
static double cached_cfl(int eq, int N, int stages, int dissipation, int points)
{
    static std::mutex mu;
    static double cache[2][5][5][2][2] = {};
    const int sys = eq == CRKFR_LINADV1D ? 0 : 1;
    const int d1 = dissipation == CRKFR_DISS_D1 ? 1 : 0;
    std::lock_guard<std::mutex> lk(mu);
    double& v = cache[sys][N][stages][d1][points];
    if (v == 0.0)
        v = crkfr_fourier_cfl(N, stages, sys, dissipation, points, N == 4 && stages == 4 ? 1e-5 : 1e-10);
    return v;
}

// ----------------------------------------------------------------------------
// solver
// ----------------------------------------------------------------------------
struct crkfr_solver {
    crkfr_config cfg;
    crkfr_limiter_opts lim;
    crkfr_source src;
    hipStream_t stream;
    bool own_stream;
    int M, dim, nd, nq, np, ne, C_max;
    int stages, dissipation, central;   // scheme options (crkfr_set_scheme)
    int batch_refs;                     // batches holding this solver's buffers
    double cfl;
    bool mp, has_state;
    int cur;   // which state buffer is current
    RefElem ref;
    void* u[2];
    double* ubar[2];
    void *uHp, *trx, *trY, *Fx, *Gy, *dtS, *ghost;
    double* inflow;          // inflow data: t_ref, number of coefficients, coefficients
    bool has_inflow_data;
    double *alpha_raw, *alpha_out, *alpha_given;
    double* alpha_judge;     // the smoothness indicator's alpha (learned-indicator runs, features)
    float* feat;             // learned-indicator features [e][N]
    const crkfr_mlp* mlp;    // borrowed network of the learned indicator
    double *dt_dev, *t_dev;
    unsigned long long *rate_bits, *diag;
    long long* steps;
    double* stats;           // k_stats partial results [block][STAT_N]
    int stats_blocks;
    double mass0;            // integral of the density when the state was set
    double* bound;           // caller-owned FP64 state bound as u[0] (crkfr_bind_state), or null
    int* edge_list;          // tile-fused step: elements at the tile edges (device), null without a tile shape
    int n_edge;
    int path;                // CRKFR_PATH_*: split, tile-fused (where it serves), faces fused into the update
    bool path_set;           // path chosen by crkfr_set_path or the autotuner (else the default rule)
    int upd_shape;           // CRKFR_UPDATE_*: the update's workgroup shape for elements of 16 points
    bool upd_shape_set;      // chosen by crkfr_set_update_shape or the autotuner (else the default rule)
    bool timing;
    hipEvent_t ev[6];
    float kernel_ms[4];
    hipGraphExec_t graph_exec;
    double graph_t_end;
    int graph_cur;
};

static size_t real_size(const crkfr_solver* s) { return s->mp ? sizeof(float) : sizeof(double); }

static bool is_tenmom(int eq) { return eq == CRKFR_TENMOM2D || eq == CRKFR_TENMOM1D; }

static int eq_nvar(int eq)
{
    switch (eq) {
    case CRKFR_LINADV1D: return 1;
    case CRKFR_EULER1D: return 3;
    case CRKFR_EULER2D: return 4;
    case CRKFR_TENMOM2D: return 6;
    case CRKFR_BURGERS1D: return 1;
    case CRKFR_TENMOM1D: return 6;
    }
    return 0;
}

static Phys make_phys(const crkfr_solver* s)
{
    Phys P;
    P.gamma = s->cfg.gamma;
    P.adv = s->cfg.adv;
    P.source = s->src.enabled && is_tenmom(s->cfg.equation);
    P.amp = s->src.amp;
    P.kappa = s->src.kappa;
    P.xc = s->src.xc;
    P.yc = s->src.yc;
    P.gx = s->src.gx;
    P.gy = s->src.gy;
    return P;
}

template <class real>
static StepArgs<real> step_args(const crkfr_solver* s, int in, int out)
{
    StepArgs<real> a;
    std::memset(&a, 0, sizeof(a));
    a.nx = s->cfg.nx;
    a.ny = s->cfg.ny;
    a.ne = s->ne;
    a.dx = (s->cfg.x1 - s->cfg.x0) / s->cfg.nx;
    a.dy = s->dim == 2 ? (s->cfg.y1 - s->cfg.y0) / s->cfg.ny : 1.0;
    a.x0 = s->cfg.x0;
    a.y0 = s->cfg.y0;
    for (int i = 0; i < 4; ++i) a.bc[i] = s->cfg.bc[i];
    if (s->dim == 1) { a.bc[2] = BC_PERIODIC; a.bc[3] = BC_PERIODIC; }
    a.ubar = s->ubar[in];
    a.u = (const real*)s->u[in];
    a.ubar_out = s->ubar[out];
    a.u_out = (real*)s->u[out];
    a.uHp = (real*)s->uHp;
    a.trx = (real*)s->trx;
    a.trY = (real*)s->trY;
    a.Fx = (real*)s->Fx;
    a.Gy = (real*)s->Gy;
    a.dtS = (s->src.enabled && is_tenmom(s->cfg.equation)) ? (real*)s->dtS : nullptr;
    a.alpha_raw = s->alpha_raw;
    a.alpha_out = s->alpha_out;
    a.alpha_given = s->alpha_given;
    a.ghost = (const real*)s->ghost;
    a.inflow = s->inflow;
    a.tn_dev = s->t_dev + 1;
    a.dt_dev = s->dt_dev;
    a.blend = s->lim.blend;
    a.indicator = s->lim.indicator;
    a.smooth = s->lim.smooth_nbr;
    a.flux_limiter = s->lim.flux_limiter;
    a.scaling = s->lim.scaling;
    a.C = s->C_max;
    a.stages = s->stages;
    a.dissipation = s->dissipation;
    a.central = s->central;
    a.alpha_min = s->lim.alpha_min;
    a.alpha_max = s->lim.alpha_max;
    a.alpha_const = s->lim.alpha_const;
    a.eps_rel = s->lim.eps_rel > 0.0 ? s->lim.eps_rel : 0.1;
    a.eps_abs = s->lim.eps_abs > 0.0 ? s->lim.eps_abs : 1e-13;
    a.phys = make_phys(s);
    fill_tab(s->ref, s->stages, a.R);
    a.idx = 1.0 / a.dx;
    a.idy = 1.0 / a.dy;
    for (int i = 0; i < MAXND; ++i) {
        a.w64[i] = i <= s->cfg.N ? s->ref.w[i] : 0.0;
        a.iwdx[i] = i <= s->cfg.N ? 1.0 / (s->ref.w[i] * a.dx) : 0.0;
        a.iwdy[i] = i <= s->cfg.N ? 1.0 / (s->ref.w[i] * a.dy) : 0.0;
    }
    a.diag = s->diag;
    a.rate_bits = s->rate_bits;
    a.mlp = s->mlp ? mlp_device_params(s->mlp) : nullptr;
    a.mlp_hidden = s->mlp ? mlp_hidden(s->mlp) : 0;
    a.alpha_judge = s->alpha_judge;
    a.feat_out = s->feat;
    a.ind_T = 0.5 * std::pow(10.0, -1.8 * std::pow((double)(s->cfg.N + 1), 0.25));
    a.ind_kT = std::log(9999.0) / a.ind_T;
    return a;
}

template <class real>
static IoArgs<real> io_args(const crkfr_solver* s)
{
    IoArgs<real> a;
    std::memset(&a, 0, sizeof(a));
    a.nx = s->cfg.nx;
    a.ny = s->cfg.ny;
    a.ne = s->ne;
    a.dx = (s->cfg.x1 - s->cfg.x0) / s->cfg.nx;
    a.dy = s->dim == 2 ? (s->cfg.y1 - s->cfg.y0) / s->cfg.ny : 1.0;
    for (int i = 0; i < 4; ++i) a.bc[i] = s->cfg.bc[i];
    a.ubar = s->ubar[s->cur];
    a.u = (real*)s->u[s->cur];
    a.ghost = (real*)s->ghost;
    a.phys = make_phys(s);
    fill_tab(s->ref, s->stages, a.R);
    for (int i = 0; i < MAXND; ++i) {
        a.w64[i] = i <= s->cfg.N ? s->ref.w[i] : 0.0;
        a.l0_64[i] = i <= s->cfg.N ? s->ref.l0[i] : 0.0;
        a.l1_64[i] = i <= s->cfg.N ? s->ref.l1[i] : 0.0;
    }
    a.diag = s->diag;
    a.rate_bits = s->rate_bits;
    a.stats = s->stats;
    return a;
}

static int dispatch_step(const crkfr_solver* s, int phase, int in, int out)
{
    const int N = s->cfg.N;
    const bool lim = s->lim.blend != CRKFR_BLEND_OFF;
    hipStream_t st = s->stream;
    int rc = -1;
    if (s->mp) {
        StepArgs<float> a = step_args<float>(s, in, out);
        if (phase == PH_EDGE_UPDATE) { a.edge_list = s->edge_list; a.n_edge = s->n_edge; }
        switch (s->cfg.equation) {
        case CRKFR_LINADV1D: rc = linadv1d_step_f32(N, lim, phase, a, st); break;
        case CRKFR_BURGERS1D: rc = burgers1d_step_f32(N, lim, phase, a, st); break;
        case CRKFR_TENMOM1D: rc = tenmom1d_step_f32(N, lim, phase, a, st); break;
        case CRKFR_EULER1D: rc = euler1d_step_f32(N, lim, phase, a, st); break;
        case CRKFR_EULER2D: rc = euler2d_step_f32(N, lim, phase, a, st); break;
        case CRKFR_TENMOM2D: rc = tenmom2d_step_f32(N, lim, phase, a, st); break;
        }
    } else {
        StepArgs<double> a = step_args<double>(s, in, out);
        if (phase == PH_EDGE_UPDATE) { a.edge_list = s->edge_list; a.n_edge = s->n_edge; }
        switch (s->cfg.equation) {
        case CRKFR_LINADV1D: rc = linadv1d_step_f64(N, lim, phase, a, st); break;
        case CRKFR_BURGERS1D: rc = burgers1d_step_f64(N, lim, phase, a, st); break;
        case CRKFR_TENMOM1D: rc = tenmom1d_step_f64(N, lim, phase, a, st); break;
        case CRKFR_EULER1D: rc = euler1d_step_f64(N, lim, phase, a, st); break;
        case CRKFR_EULER2D: rc = euler2d_step_f64(N, lim, phase, a, st); break;
        case CRKFR_TENMOM2D: rc = tenmom2d_step_f64(N, lim, phase, a, st); break;
        }
    }
    if (rc) return fail(CRKFR_EINVAL, "no kernel for this configuration");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CRKFR_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return 0;
}

template <class real>
static int dispatch_io_t(const crkfr_solver* s, int phase, IoArgs<real>& a)
{
    const int N = s->cfg.N;
    hipStream_t st = s->stream;
    int rc = -1;
    if constexpr (sizeof(real) == 4) {
        switch (s->cfg.equation) {
        case CRKFR_LINADV1D: rc = linadv1d_io_f32(N, phase, a, st); break;
        case CRKFR_BURGERS1D: rc = burgers1d_io_f32(N, phase, a, st); break;
        case CRKFR_TENMOM1D: rc = tenmom1d_io_f32(N, phase, a, st); break;
        case CRKFR_EULER1D: rc = euler1d_io_f32(N, phase, a, st); break;
        case CRKFR_EULER2D: rc = euler2d_io_f32(N, phase, a, st); break;
        case CRKFR_TENMOM2D: rc = tenmom2d_io_f32(N, phase, a, st); break;
        }
    } else {
        switch (s->cfg.equation) {
        case CRKFR_LINADV1D: rc = linadv1d_io_f64(N, phase, a, st); break;
        case CRKFR_BURGERS1D: rc = burgers1d_io_f64(N, phase, a, st); break;
        case CRKFR_TENMOM1D: rc = tenmom1d_io_f64(N, phase, a, st); break;
        case CRKFR_EULER1D: rc = euler1d_io_f64(N, phase, a, st); break;
        case CRKFR_EULER2D: rc = euler2d_io_f64(N, phase, a, st); break;
        case CRKFR_TENMOM2D: rc = tenmom2d_io_f64(N, phase, a, st); break;
        }
    }
    if (rc) return fail(CRKFR_EINVAL, "no io kernel for this configuration");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CRKFR_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return 0;
}

static int run_io(const crkfr_solver* s, int phase, const double* uin, double* uout, double* means)
{
    if (s->mp) {
        IoArgs<float> a = io_args<float>(s);
        a.uin = uin; a.uout = uout; a.means_out = means;
        return dispatch_io_t<float>(s, phase, a);
    }
    IoArgs<double> a = io_args<double>(s);
    a.uin = uin; a.uout = uout; a.means_out = means;
    return dispatch_io_t<double>(s, phase, a);
}

static void free_all(crkfr_solver* s)
{
    void* ptrs[] = {s->bound ? nullptr : s->u[0], s->u[1], s->stats, s->edge_list, s->ubar[0], s->ubar[1], s->uHp, s->trx, s->trY, s->Fx, s->dtS,
                    s->ghost, s->alpha_raw, s->alpha_out, s->alpha_given, s->alpha_judge, s->feat,
                    s->dt_dev, s->t_dev, s->inflow,
                    s->rate_bits, s->diag, s->steps};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    for (int i = 0; i < 6; ++i)
        if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
}

// values in the far-field ghost layout: x-left, x-right [ny][nq][M], then in 2D
// y-bottom, y-top [nx][nd][M]
static size_t ghost_size(const crkfr_solver* s)
{
    return (2 * (size_t)s->cfg.ny * s->nq + (s->dim == 2 ? 2 * (size_t)s->cfg.nx * s->nd : 0)) * s->M;
}

// CFL(N) when the configuration gives none: the Fourier value of the scheme;
// with GLL points and blending also at most the end subcells' width w_0 =
// 1/(N(N+1)), below which the first-order subcell update (and so the flux
// limiter's guarantee of admissible means) holds
static double default_cfl(const crkfr_solver* s)
{
    double c = cached_cfl(s->cfg.equation, s->cfg.N, s->stages, s->dissipation, s->cfg.points);
    if (s->cfg.points == CRKFR_POINTS_GLL && s->lim.blend != CRKFR_BLEND_OFF) c = std::min(c, s->ref.w[0]);
    return c;
}

// the checks of crkfr_create (no device call)
static int validate_config(const crkfr_config* cfg)
{
    if (cfg->equation < 0 || cfg->equation > 5) return fail(CRKFR_EINVAL, "unknown equation");
    if (cfg->N < 1 || cfg->N > 4) return fail(CRKFR_EINVAL, "N must be in 1..4");
    const int dim = cfg->equation == CRKFR_EULER2D || cfg->equation == CRKFR_TENMOM2D ? 2 : 1;
    if (cfg->nx < 1 || cfg->ny < 1 || (dim == 1 && cfg->ny != 1)) return fail(CRKFR_EINVAL, "bad grid size");
    if (cfg->dtype != CRKFR_FP64 && cfg->dtype != CRKFR_MP32) return fail(CRKFR_EINVAL, "bad dtype");
    if (cfg->points != CRKFR_POINTS_GL && cfg->points != CRKFR_POINTS_GLL)
        return fail(CRKFR_EINVAL, "bad solution points");
    for (int i = 0; i < (dim == 2 ? 4 : 2); ++i)
        if (cfg->bc[i] < 0 || cfg->bc[i] > 4) return fail(CRKFR_EINVAL, "bad boundary kind");
    for (int i = 0; i < (dim == 2 ? 4 : 2); ++i)
        if (cfg->bc[i] == CRKFR_BC_REFLECT && (cfg->equation == CRKFR_LINADV1D || cfg->equation == CRKFR_BURGERS1D))
            return fail(CRKFR_EINVAL, "solid walls are defined for the Euler and ten-moment systems");
    if ((cfg->bc[0] == CRKFR_BC_PERIODIC) != (cfg->bc[1] == CRKFR_BC_PERIODIC) ||
        (dim == 2 && (cfg->bc[2] == CRKFR_BC_PERIODIC) != (cfg->bc[3] == CRKFR_BC_PERIODIC)))
        return fail(CRKFR_EINVAL, "periodic boundaries come in pairs");
    if (!(cfg->x1 > cfg->x0) || (dim == 2 && !(cfg->y1 > cfg->y0))) return fail(CRKFR_EINVAL, "bad domain");
    {   // the kernels index nodes and face points with 32-bit integers
        const long long nd1 = cfg->N + 1, nq1 = dim == 2 ? nd1 : 1, lim = 1ll << 31;
        const long long nodes = (long long)cfg->nx * cfg->ny * nd1 * nq1;
        const long long fxp = (long long)(cfg->nx + 1) * cfg->ny * nq1, fyp = (long long)(cfg->ny + 1) * cfg->nx * nd1;
        if (nodes >= lim || fxp >= lim || fyp >= lim)
            return fail(CRKFR_EINVAL, "grid too large: nodes and face points per direction must stay below 2^31");
    }
    return 0;
}

extern "C" int crkfr_create(const crkfr_config* cfg, void* hip_stream, crkfr_solver** out)
{
    if (!cfg || !out) return fail(CRKFR_EINVAL, "null argument");
    *out = nullptr;
    {
        const int rc = validate_config(cfg);
        if (rc) return rc;
    }
    const int dim = cfg->equation == CRKFR_EULER2D || cfg->equation == CRKFR_TENMOM2D ? 2 : 1;

    crkfr_solver* s = new crkfr_solver();
    std::memset(s, 0, sizeof(*s));
    s->cfg = *cfg;
    s->stream = (hipStream_t)hip_stream;
    if (!s->stream) {
        // graph capture needs a stream of its own (default priority)
        hipError_t e = hipStreamCreate(&s->stream);
        if (e != hipSuccess) {
            delete s;
            return fail(CRKFR_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        s->own_stream = true;
    }
    s->M = eq_nvar(cfg->equation);
    s->dim = dim;
    s->nd = cfg->N + 1;
    s->nq = dim == 2 ? s->nd : 1;
    s->np = s->nd * s->nq;
    s->ne = cfg->nx * cfg->ny;
    s->C_max = 4 * s->M + 1;
    s->stages = std::min(cfg->N + 1, 4);
    s->dissipation = CRKFR_DISS_D2;
    s->central = CRKFR_CENTRAL_EA;
    s->mp = cfg->dtype == CRKFR_MP32;
    if (s->cfg.cs <= 0.0) s->cfg.cs = 0.98;
    s->lim.blend = CRKFR_BLEND_OFF;
    s->lim.alpha_min = 1e-3;
    s->lim.alpha_max = 1.0;
    s->lim.smooth_nbr = 1;
    make_ref(cfg->N, cfg->points, s->ref);
    s->cfl = cfg->cfl > 0.0 ? cfg->cfl : default_cfl(s);

    const size_t rs = real_size(s), M = s->M, ne = s->ne, np = s->np;
    const size_t nstate = M * ne * np;
    auto alloc = [&](void** p, size_t bytes) -> bool {
        if (bytes == 0) return true;
        return hipMalloc(p, bytes) == hipSuccess;
    };
    bool ok = true;
    ok &= alloc(&s->u[0], nstate * rs);
    ok &= alloc(&s->u[1], nstate * rs);
    if (s->mp) {
        ok &= alloc((void**)&s->ubar[0], M * ne * sizeof(double));
        ok &= alloc((void**)&s->ubar[1], M * ne * sizeof(double));
    }
    ok &= alloc(&s->uHp, nstate * rs);
    ok &= alloc(&s->trx, 2 * (size_t)s->C_max * ne * s->nq * rs);
    if (dim == 2) ok &= alloc(&s->trY, 2 * (size_t)s->C_max * ne * s->nd * rs);
    {   // the x and y face fluxes in one allocation (the checkerboard step keeps
        // the colour-1 elements' face fluxes, M ne / 2 4 (N + 1) values, in it)
        const size_t fx = M * (size_t)cfg->ny * (cfg->nx + 1) * s->nq;
        const size_t fy = dim == 2 ? M * (size_t)(cfg->ny + 1) * cfg->nx * s->nd : 0;
        ok &= alloc(&s->Fx, (fx + fy) * rs);
        if (dim == 2 && s->Fx) s->Gy = (char*)s->Fx + fx * rs;
    }
    if (is_tenmom(cfg->equation)) ok &= alloc(&s->dtS, nstate * rs);
    ok &= alloc(&s->ghost, (2 * (size_t)cfg->ny * s->nq + (dim == 2 ? 2 * (size_t)cfg->nx * s->nd : 0)) * M * rs);
    bool any_inflow = false;
    for (int i = 0; i < (dim == 2 ? 4 : 2); ++i) any_inflow |= cfg->bc[i] == CRKFR_BC_INFLOW;
    if (any_inflow) {
        ok &= alloc((void**)&s->inflow, (2 + CRKFR_INFLOW_MAXCOEF * ghost_size(s)) * sizeof(double));
        if (s->inflow) ok &= hipMemset(s->inflow, 0, 2 * sizeof(double)) == hipSuccess;   // no data yet
    }
    ok &= alloc((void**)&s->alpha_raw, ne * sizeof(double));
    ok &= alloc((void**)&s->alpha_out, ne * sizeof(double));
    ok &= alloc((void**)&s->alpha_given, ne * sizeof(double));
    ok &= alloc((void**)&s->alpha_judge, ne * sizeof(double));
    ok &= alloc((void**)&s->feat, ne * (size_t)cfg->N * sizeof(float));
    ok &= alloc((void**)&s->dt_dev, sizeof(double));
    ok &= alloc((void**)&s->t_dev, 2 * sizeof(double));   // t, and t^n of the current step
    ok &= alloc((void**)&s->rate_bits, RATE_SLOTS * sizeof(unsigned long long));
    ok &= alloc((void**)&s->diag, D_NCOUNT * sizeof(unsigned long long));
    ok &= alloc((void**)&s->steps, sizeof(long long));
    {
        int el = 0, eu = 0, nq1 = 0;
        int grc = -1;
        switch (cfg->equation) {
        case CRKFR_LINADV1D: grc = linadv1d_geometry(cfg->N, &el, &eu, &nq1); break;
        case CRKFR_BURGERS1D: grc = burgers1d_geometry(cfg->N, &el, &eu, &nq1); break;
        case CRKFR_TENMOM1D: grc = tenmom1d_geometry(cfg->N, &el, &eu, &nq1); break;
        case CRKFR_EULER1D: grc = euler1d_geometry(cfg->N, &el, &eu, &nq1); break;
        case CRKFR_EULER2D: grc = euler2d_geometry(cfg->N, &el, &eu, &nq1); break;
        case CRKFR_TENMOM2D: grc = tenmom2d_geometry(cfg->N, &el, &eu, &nq1); break;
        }
        s->stats_blocks = grc == 0 ? (s->ne + eu - 1) / eu : 0;
        ok &= grc == 0 && alloc((void**)&s->stats, (size_t)s->stats_blocks * STAT_N * sizeof(double));
    }
    s->path = CRKFR_PATH_FACE_UPDATE;
    {   // tile-fused step: the elements at the tile edges, in tile order
        int tx = 0, ty = 0;
        if (ok && cfg->equation == CRKFR_EULER2D && euler2d_tile_shape(cfg->N, cfg->dtype == CRKFR_MP32, &tx, &ty) == 0) {
            std::vector<int> list;
            const int nx = cfg->nx, ny = cfg->ny;
            for (int gy0 = 0; gy0 < ny; gy0 += ty)
                for (int gx0 = 0; gx0 < nx; gx0 += tx)
                    for (int iy = 0; iy < ty && gy0 + iy < ny; ++iy)
                        for (int ix = 0; ix < tx && gx0 + ix < nx; ++ix) {
                            const int gx = gx0 + ix, gy = gy0 + iy;
                            const bool inner = ix > 0 && ix < tx - 1 && iy > 0 && iy < ty - 1 && gx + 1 < nx &&
                                               gy + 1 < ny;
                            if (!inner) list.push_back(gy * nx + gx);
                        }
            s->n_edge = (int)list.size();
            ok &= alloc((void**)&s->edge_list, list.size() * sizeof(int));
            if (ok && !list.empty())
                ok &= hipMemcpy(s->edge_list, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice) ==
                      hipSuccess;
        }
    }
    if (!ok) {
        free_all(s);
        delete s;
        return fail(CRKFR_ENOMEM, "device allocation failed");
    }
    (void)hipMemsetAsync(s->alpha_raw, 0, ne * sizeof(double), s->stream);
    (void)hipMemsetAsync(s->alpha_out, 0, ne * sizeof(double), s->stream);
    (void)hipMemsetAsync(s->alpha_given, 0, ne * sizeof(double), s->stream);
    (void)hipMemsetAsync(s->alpha_judge, 0, ne * sizeof(double), s->stream);
    (void)hipMemsetAsync(s->diag, 0, D_NCOUNT * sizeof(unsigned long long), s->stream);
    if (hipStreamSynchronize(s->stream) != hipSuccess) {
        free_all(s);
        delete s;
        return fail(CRKFR_EHIP, "stream synchronize failed");
    }
    *out = s;
    return 0;
}

extern "C" void crkfr_destroy(crkfr_solver* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    free_all(s);
    delete s;
}

static void invalidate_graph(crkfr_solver* s)
{
    if (s->graph_exec) {
        (void)hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
    }
}

extern "C" int crkfr_set_limiter(crkfr_solver* s, const crkfr_limiter_opts* o)
{
    if (!s || !o) return fail(CRKFR_EINVAL, "null argument");
    if (o->blend < 0 || o->blend > 2 || o->indicator < 0 || o->indicator > 3)
        return fail(CRKFR_EINVAL, "bad limiter option");
    if (o->flux_limiter && o->blend == CRKFR_BLEND_OFF)
        return fail(CRKFR_EINVAL, "the flux limiter needs a low-order blend (FO or MH)");
    if (o->blend == CRKFR_BLEND_MH && s->cfg.points == CRKFR_POINTS_GLL)
        return fail(CRKFR_EINVAL, "MUSCL-Hancock blending needs Gauss-Legendre points");
    s->lim = *o;
    if (s->cfg.cfl <= 0.0) s->cfl = default_cfl(s);
    invalidate_graph(s);
    return 0;
}

extern "C" int crkfr_set_inflow(crkfr_solver* s, const double* coeffs, int ncoef, double t_ref, int on_device)
{
    if (!s || !coeffs) return fail(CRKFR_EINVAL, "null argument");
    if (!s->inflow) return fail(CRKFR_EINVAL, "the configuration has no inflow boundary");
    if (ncoef < 1 || ncoef > CRKFR_INFLOW_MAXCOEF) return fail(CRKFR_EINVAL, "ncoef must be in 1..5");
    const size_t n = ghost_size(s) * ncoef;
    const double head[2] = {t_ref, (double)ncoef};
    // the step kernels read the buffer on the solver's stream: ordered after this copy
    HIP_TRY(hipMemcpyAsync(s->inflow, head, sizeof(head), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->inflow + 2, coeffs, n * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
    if (!on_device) HIP_TRY(hipStreamSynchronize(s->stream));   // the caller may reuse its host buffer
    s->has_inflow_data = true;
    return 0;
}

extern "C" int crkfr_set_source(crkfr_solver* s, const crkfr_source* src)
{
    if (!s || !src) return fail(CRKFR_EINVAL, "null argument");
    if (src->enabled && !is_tenmom(s->cfg.equation))
        return fail(CRKFR_EINVAL, "sources are implemented for the ten-moment system");
    s->src = *src;
    invalidate_graph(s);
    return 0;
}

extern "C" int crkfr_set_scheme(crkfr_solver* s, const crkfr_scheme* o)
{
    if (!s || !o) return fail(CRKFR_EINVAL, "null argument");
    if (s->batch_refs > 0) return fail(CRKFR_ESTATE, "solver is a batch member: destroy the batch first");
    const int S = o->stages > 0 ? o->stages : std::min(s->cfg.N + 1, 4);
    if (S < 2 || S > 4) return fail(CRKFR_EINVAL, "stages must be 0 (N+1 up to 4) or 2..4");
    if (o->dissipation < 0 || o->dissipation > 2 || o->central < 0 || o->central > 1)
        return fail(CRKFR_EINVAL, "bad dissipation or central option");
    const int need = 4 * s->M + 1 + (o->dissipation == CRKFR_DISS_DCSX ? S * s->M : 0);
    if (need > s->C_max) {
        // the D-CSX dissipation keeps every stage's face values: larger trace buffers
        const size_t rs = real_size(s), ne = s->ne;
        void *trx = nullptr, *trY = nullptr;
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (hipMalloc(&trx, 2 * (size_t)need * ne * s->nq * rs) != hipSuccess)
            return fail(CRKFR_ENOMEM, "device allocation failed");
        if (s->dim == 2 && hipMalloc(&trY, 2 * (size_t)need * ne * s->nd * rs) != hipSuccess) {
            (void)hipFree(trx);
            return fail(CRKFR_ENOMEM, "device allocation failed");
        }
        (void)hipFree(s->trx);
        if (s->trY) (void)hipFree(s->trY);
        s->trx = trx;
        s->trY = trY;
        s->C_max = need;
    }
    s->stages = S;
    s->dissipation = o->dissipation;
    s->central = o->central;
    if (s->cfg.cfl <= 0.0) s->cfl = default_cfl(s);
    invalidate_graph(s);
    return 0;
}

// statistics of the current state (k_stats), reduced over the blocks in a fixed order
struct StateStats {
    double min_rho, min_p1, min_p2, mass;
    long long nonfinite;
};

static int state_stats(crkfr_solver* s, StateStats* out)
{
    int rc = run_io(s, PH_STATS, nullptr, nullptr, nullptr);
    if (rc) return rc;
    std::vector<double> h((size_t)s->stats_blocks * STAT_N);
    HIP_TRY(hipMemcpyAsync(h.data(), s->stats, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const double big = 1.79769313486231570e308;
    StateStats r = {big, big, big, 0.0, 0};
    for (int b = 0; b < s->stats_blocks; ++b) {
        const double* x = &h[(size_t)b * STAT_N];
        r.min_rho = std::min(r.min_rho, x[STAT_MINRHO]);
        r.min_p1 = std::min(r.min_p1, x[STAT_MINP1]);
        r.min_p2 = std::min(r.min_p2, x[STAT_MINP2]);
        r.nonfinite += (long long)x[STAT_NONFINITE];
        r.mass += x[STAT_MASS];
    }
    const int K = s->cfg.equation == CRKFR_EULER1D || s->cfg.equation == CRKFR_EULER2D ? 2
                : (is_tenmom(s->cfg.equation) ? 3 : 0);
    if (K < 2) r.min_p1 = 0.0;
    if (K < 3) r.min_p2 = 0.0;
    *out = r;
    return 0;
}

static int load_state(crkfr_solver* s, const double* src, double* tmp);

extern "C" int crkfr_set_state(crkfr_solver* s, const double* u, int on_device)
{
    if (!s || !u) return fail(CRKFR_EINVAL, "null argument");
    if (s->batch_refs > 0 && s->bound) return fail(CRKFR_ESTATE, "solver is a batch member: destroy the batch first");
    const size_t n = (size_t)s->M * s->ne * s->np;
    if (s->bound) {
        // the bound buffer goes back to the caller: a buffer of the library's own again
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (hipMalloc(&s->u[0], n * real_size(s)) != hipSuccess) {
            s->u[0] = s->bound;
            return fail(CRKFR_ENOMEM, "device allocation failed");
        }
        s->bound = nullptr;
    }
    const double* src = u;
    double* tmp = nullptr;
    if (!on_device) {
        HIP_TRY(hipMalloc((void**)&tmp, n * sizeof(double)));
        HIP_TRY(hipMemcpyAsync(tmp, u, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
        src = tmp;
    }
    return load_state(s, src, tmp);
}

extern "C" int crkfr_bind_state(crkfr_solver* s, double* u_dev)
{
    if (!s || !u_dev) return fail(CRKFR_EINVAL, "null argument");
    if (s->mp) return fail(CRKFR_EINVAL, "an MP32 state is FP64 means plus FP32 deviations: use crkfr_set_state");
    if (s->batch_refs > 0) return fail(CRKFR_ESTATE, "solver is a batch member: destroy the batch first");
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (!s->bound && s->u[0]) (void)hipFree(s->u[0]);
    s->bound = u_dev;
    s->u[0] = u_dev;
    return load_state(s, u_dev, nullptr);
}

extern "C" int crkfr_state_ptr(crkfr_solver* s, double** u_dev)
{
    if (!s || !u_dev) return fail(CRKFR_EINVAL, "null argument");
    if (s->mp) return fail(CRKFR_EINVAL, "an MP32 state has no FP64 nodal buffer");
    if (!s->has_state) return fail(CRKFR_ESTATE, "no state set");
    *u_dev = (double*)s->u[s->cur];
    return 0;
}

// import src (device) as the state in buffer 0: admissibility, means, rate,
// ghosts, the mass for the drift diagnostic; tmp (if any) is freed
static int load_state(crkfr_solver* s, const double* src, double* tmp)
{
    s->cur = 0;
    const double zero = 0.0;
    HIP_TRY(hipMemcpyAsync(s->t_dev, &zero, sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemsetAsync(s->rate_bits, 0, RATE_SLOTS * sizeof(unsigned long long), s->stream));
    HIP_TRY(hipMemsetAsync(s->diag, 0, D_NCOUNT * sizeof(unsigned long long), s->stream));
    HIP_TRY(hipMemsetAsync(s->steps, 0, sizeof(long long), s->stream));
    int rc = run_io(s, PH_IMPORT, src, nullptr, nullptr);
    if (!rc) rc = run_io(s, PH_GHOST, nullptr, nullptr, nullptr);
    unsigned long long bad = 0;
    if (!rc) {
        HIP_TRY(hipMemcpyAsync(&bad, s->diag + D_MEANBAD, sizeof(bad), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    if (tmp) (void)hipFree(tmp);
    HIP_TRY(hipMemsetAsync(s->diag, 0, D_NCOUNT * sizeof(unsigned long long), s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (rc) return rc;
    StateStats st;
    rc = state_stats(s, &st);
    if (rc) return rc;
    s->mass0 = st.mass;
    s->has_state = true;
    invalidate_graph(s);
    if (bad) return fail(CRKFR_EINADMISSIBLE_INPUT, std::to_string(bad) + " nodes violate the admissibility constraints");
    return 0;
}

extern "C" int crkfr_set_alpha(crkfr_solver* s, const double* alpha, int on_device)
{
    if (!s || !alpha) return fail(CRKFR_EINVAL, "null argument");
    HIP_TRY(hipMemcpyAsync(s->alpha_given, alpha, s->ne * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return 0;
}

extern "C" int crkfr_set_mlp(crkfr_solver* s, const crkfr_mlp* m)
{
    if (!s) return fail(CRKFR_EINVAL, "null argument");
    if (m && mlp_inputs(m) != s->cfg.N) return fail(CRKFR_EINVAL, "the network's inputs must equal N");
    s->mlp = m;
    invalidate_graph(s);
    return 0;
}

extern "C" int crkfr_features(crkfr_solver* s, float* feat, double* alpha_ind, int on_device)
{
    if (!s) return fail(CRKFR_EINVAL, "null argument");
    if (!s->has_state) return fail(CRKFR_ESTATE, "no state set");
    int rc = dispatch_step(s, PH_FEATURES, s->cur, 1 - s->cur);
    if (rc) return rc;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (feat) HIP_TRY(hipMemcpyAsync(feat, s->feat, (size_t)s->ne * s->cfg.N * sizeof(float), kind, s->stream));
    if (alpha_ind) HIP_TRY(hipMemcpyAsync(alpha_ind, s->alpha_judge, s->ne * sizeof(double), kind, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return 0;
}

extern "C" int crkfr_compute_dt(crkfr_solver* s, double* dt)
{
    if (!s || !dt) return fail(CRKFR_EINVAL, "null argument");
    if (!s->has_state) return fail(CRKFR_ESTATE, "no state set");
    unsigned long long bits[RATE_SLOTS];
    HIP_TRY(hipMemcpyAsync(bits, s->rate_bits, sizeof(bits), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    double rate = 0.0;
    for (int i = 0; i < RATE_SLOTS; ++i) {
        double r;
        std::memcpy(&r, &bits[i], sizeof(r));
        rate = r > rate ? r : rate;
    }
    *dt = s->cfg.cs * s->cfl / rate;
    return 0;
}

// the learned indicator needs a network whose inputs match the degree
static int check_learned(const crkfr_solver* s)
{
    if (s->lim.blend == CRKFR_BLEND_OFF || s->lim.indicator != CRKFR_IND_LEARNED) return 0;
    if (!s->mlp) return fail(CRKFR_ESTATE, "the learned indicator needs a network (crkfr_set_mlp)");
    if (mlp_inputs(s->mlp) != s->cfg.N) return fail(CRKFR_EINVAL, "the network's inputs must equal N");
    return 0;
}

// the tile-fused step serves 2D Euler with elements of 4 or 16 points, the
// limiter chain off and the D2 dissipation; elsewhere that path takes the
// update with the faces fused in
// the checkerboard step serves 2D grids with every boundary periodic, even
// sides, the limiter chain off, D2 and no source
static bool checker_serves(const crkfr_solver* s)
{
    bool ok = s->dim == 2 && s->lim.blend == CRKFR_BLEND_OFF && s->dissipation == CRKFR_DISS_D2 &&
              s->cfg.nx % 2 == 0 && s->cfg.ny % 2 == 0 && !(s->src.enabled && is_tenmom(s->cfg.equation));
    for (int i = 0; i < 4; ++i) ok = ok && s->cfg.bc[i] == CRKFR_BC_PERIODIC;
    return ok;
}

static int path_in_use(const crkfr_solver* s)
{
    // unless the caller chose one: without the limiter chain the checkerboard
    // step where it serves, else the faces fused into the update; the split
    // step with the limiter chain (the limited face flux, done once per face
    // there, would be computed by both neighbours)
    const int p = s->path_set ? s->path
                              : (s->lim.blend != CRKFR_BLEND_OFF ? CRKFR_PATH_SPLIT
                                                                  : (checker_serves(s) ? CRKFR_PATH_CHECKER
                                                                                       : CRKFR_PATH_FACE_UPDATE));
    if (p == CRKFR_PATH_TILE)
        return s->edge_list && s->lim.blend == CRKFR_BLEND_OFF && s->dissipation == CRKFR_DISS_D2
                   ? CRKFR_PATH_TILE : CRKFR_PATH_FACE_UPDATE;
    if (p == CRKFR_PATH_CHECKER) return checker_serves(s) ? CRKFR_PATH_CHECKER : CRKFR_PATH_FACE_UPDATE;
    return p;
}

extern "C" int crkfr_set_path(crkfr_solver* s, int path)
{
    if (!s) return fail(CRKFR_EINVAL, "null argument");
    if (path < CRKFR_PATH_SPLIT || path > CRKFR_PATH_CHECKER) return fail(CRKFR_EINVAL, "bad step path");
    if (s->batch_refs > 0) return fail(CRKFR_ESTATE, "solver is a batch member: destroy the batch first");
    s->path = path;
    s->path_set = true;
    invalidate_graph(s);
    return 0;
}

extern "C" int crkfr_path_in_use(const crkfr_solver* s) { return s ? path_in_use(s) : -1; }

// the update's workgroup shape (elements of 16 points): one wavefront for the
// FP64 checkerboard's colour-0 update and the limited FP64 split update,
// which were faster so, 256 lanes elsewhere, unless the caller or the
// autotuner chose
static int update_shape_in_use(const crkfr_solver* s)
{
    if (s->np != 16) return CRKFR_UPDATE_BLOCK;
    if (s->upd_shape_set) return s->upd_shape;
    const int path = path_in_use(s);
    const bool lim = s->lim.blend != CRKFR_BLEND_OFF;
    return !s->mp && (path == CRKFR_PATH_CHECKER || (path == CRKFR_PATH_SPLIT && lim)) ? CRKFR_UPDATE_WAVE
                                                                                        : CRKFR_UPDATE_BLOCK;
}

extern "C" int crkfr_set_update_shape(crkfr_solver* s, int shape)
{
    if (!s) return fail(CRKFR_EINVAL, "null argument");
    if (shape < -1 || shape > CRKFR_UPDATE_WAVE) return fail(CRKFR_EINVAL, "bad update shape");
    if (s->batch_refs > 0) return fail(CRKFR_ESTATE, "solver is a batch member: destroy the batch first");
    s->upd_shape = shape < 0 ? CRKFR_UPDATE_BLOCK : shape;
    s->upd_shape_set = shape >= 0;
    invalidate_graph(s);
    return 0;
}

extern "C" int crkfr_update_shape_in_use(const crkfr_solver* s) { return s ? update_shape_in_use(s) : -1; }

static int enqueue_step(crkfr_solver* s, double dt_fixed, double t_end);

// ----------------------------------------------------------------------------
// path autotuning: time each kernel path that serves the configuration over a
// few steps from the current state, keep the fastest, and remember it in a
// JSON-lines cache file keyed by what selects the kernels
// ----------------------------------------------------------------------------
static std::string tune_key(const crkfr_solver* s)
{
    char buf[320];
    std::snprintf(buf, sizeof(buf),
                  "eq=%d M=%d N=%d dtype=%s nx=%d ny=%d points=%d stages=%d diss=%d central=%d blend=%d "
                  "ind=%d flux=%d scale=%d src=%d",
                  s->cfg.equation, s->M, s->cfg.N, s->mp ? "mp32" : "fp64", s->cfg.nx, s->cfg.ny, s->cfg.points,
                  s->stages, s->dissipation, s->central, s->lim.blend, s->lim.indicator, s->lim.flux_limiter,
                  s->lim.scaling, (int)(s->src.enabled != 0));
    return buf;
}

static const char* const PATH_NAMES[4] = {"split", "tile", "face_update", "checker"};

static const char* const SHAPE_NAMES[2] = {"block", "wave"};

// the path stored for key, or -1; *shape: the update shape stored with it, or -1
static int tune_cache_lookup(const char* path, const std::string& key, int* shape)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    const std::string want = "\"key\": \"" + key + "\"";
    char line[1024];
    int found = -1;
    *shape = -1;
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strstr(line, want.c_str())) continue;
        const char* p = std::strstr(line, "\"path\": \"");
        if (!p) continue;
        p += std::strlen("\"path\": \"");
        int fp = -1, fs = -1;
        for (int i = 0; i < 4; ++i) {
            const size_t n = std::strlen(PATH_NAMES[i]);
            if (std::strncmp(p, PATH_NAMES[i], n) == 0 && p[n] == '"') fp = i;
        }
        const char* q = std::strstr(line, "\"update_shape\": \"");
        if (q) {
            q += std::strlen("\"update_shape\": \"");
            for (int i = 0; i < 2; ++i) {
                const size_t n = std::strlen(SHAPE_NAMES[i]);
                if (std::strncmp(q, SHAPE_NAMES[i], n) == 0 && q[n] == '"') fs = i;
            }
        }
        if (fp >= 0) {   // the last entry wins
            found = fp;
            *shape = fs;
        }
    }
    std::fclose(f);
    return found;
}

extern "C" int crkfr_autotune(crkfr_solver* s, int steps, const char* cache_path, crkfr_tune_result* out)
{
    if (!s || !out) return fail(CRKFR_EINVAL, "null argument");
    if (steps < 1) return fail(CRKFR_EINVAL, "steps must be >= 1");
    if (!s->has_state) return fail(CRKFR_ESTATE, "no state set");
    if (s->batch_refs > 0) return fail(CRKFR_ESTATE, "solver is a batch member: destroy the batch first");
    std::memset(out, 0, sizeof(*out));
    const std::string key = tune_key(s);
    if (cache_path && *cache_path) {
        int shape = -1;
        const int p = tune_cache_lookup(cache_path, key, &shape);
        if (p >= 0) {
            s->path = p;
            s->path_set = true;
            s->upd_shape = shape < 0 ? CRKFR_UPDATE_BLOCK : shape;
            s->upd_shape_set = shape >= 0;
            invalidate_graph(s);
            out->path = path_in_use(s);
            out->update_shape = update_shape_in_use(s);
            out->from_cache = 1;
            return 0;
        }
    }
    // the trials advance the state, the clock, the time-step slots and the
    // counters: keep them and put them back after each path
    const size_t n = (size_t)s->M * s->ne * s->np;
    const int cur0 = s->cur;
    struct Small {
        unsigned long long rate[RATE_SLOTS], diag[D_NCOUNT];
        double t[2], dt;
        long long steps;
    } small;
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpy(small.rate, s->rate_bits, sizeof(small.rate), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(small.diag, s->diag, sizeof(small.diag), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(small.t, s->t_dev, sizeof(small.t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&small.dt, s->dt_dev, sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&small.steps, s->steps, sizeof(long long), hipMemcpyDeviceToHost));
    void* keep_u = nullptr;
    double* keep_ubar = nullptr;
    HIP_TRY(hipMalloc(&keep_u, n * real_size(s)));
    if (s->mp && hipMalloc((void**)&keep_ubar, (size_t)s->M * s->ne * sizeof(double)) != hipSuccess) {
        (void)hipFree(keep_u);
        return fail(CRKFR_ENOMEM, "device allocation failed");
    }
    int rc = 0;
    auto restore = [&]() -> int {
        s->cur = cur0;
        HIP_TRY(hipMemcpy(s->u[cur0], keep_u, n * real_size(s), hipMemcpyDeviceToDevice));
        if (keep_ubar) HIP_TRY(hipMemcpy(s->ubar[cur0], keep_ubar, (size_t)s->M * s->ne * sizeof(double),
                                         hipMemcpyDeviceToDevice));
        HIP_TRY(hipMemcpy(s->rate_bits, small.rate, sizeof(small.rate), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->diag, small.diag, sizeof(small.diag), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->t_dev, small.t, sizeof(small.t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->dt_dev, &small.dt, sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->steps, &small.steps, sizeof(long long), hipMemcpyHostToDevice));
        return 0;
    };
    if (hipMemcpy(keep_u, s->u[cur0], n * real_size(s), hipMemcpyDeviceToDevice) != hipSuccess ||
        (keep_ubar && hipMemcpy(keep_ubar, s->ubar[cur0], (size_t)s->M * s->ne * sizeof(double),
                                hipMemcpyDeviceToDevice) != hipSuccess))
        rc = fail(CRKFR_EHIP, "state copy failed");
    const int path0 = s->path, shape0 = s->upd_shape;
    const bool set0 = s->path_set, shape_set0 = s->upd_shape_set;
    const bool tm = s->timing;
    s->timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(CRKFR_EHIP, "hipEventCreate failed");
    int best = -1, best_shape = CRKFR_UPDATE_BLOCK;
    float best_ms = 0.f;
    const int nshape = s->np == 16 ? 2 : 1;      // the update shapes differ for elements of 16 points
    for (int p = 0; p < 4 && !rc; ++p) {
        s->path = p;
        s->path_set = true;
        if (path_in_use(s) != p) continue;       // the path does not serve this configuration
        for (int sh = 0; sh < nshape && !rc; ++sh) {
            s->upd_shape = sh;
            s->upd_shape_set = true;
            rc = enqueue_step(s, 0.0, 0.0);     // warm-up
            if (!rc && hipEventRecord(e0, s->stream) != hipSuccess) rc = fail(CRKFR_EHIP, "hipEventRecord failed");
            for (int i = 0; i < steps && !rc; ++i) rc = enqueue_step(s, 0.0, 0.0);
            if (!rc && (hipEventRecord(e1, s->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = fail(CRKFR_EHIP, "timing events failed");
            float ms = 0.f;
            if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = fail(CRKFR_EHIP, "hipEventElapsedTime failed");
            if (!rc) {
                const float per = ms / steps;
                if (out->ms[p] <= 0.f || per < out->ms[p]) out->ms[p] = per;
                if (best < 0 || per < best_ms) {
                    best = p;
                    best_shape = sh;
                    best_ms = per;
                }
            }
            const int rrc = restore();
            if (!rc) rc = rrc;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(keep_u);
    if (keep_ubar) (void)hipFree(keep_ubar);
    s->timing = tm;
    s->path = rc || best < 0 ? path0 : best;
    s->path_set = rc || best < 0 ? set0 : true;
    s->upd_shape = rc || best < 0 ? shape0 : best_shape;
    s->upd_shape_set = rc || best < 0 ? shape_set0 : nshape > 1;
    invalidate_graph(s);
    if (rc) return rc;
    out->path = path_in_use(s);
    out->update_shape = update_shape_in_use(s);
    if (cache_path && *cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(CRKFR_EINVAL, std::string("cannot append to the autotune cache ") + cache_path);
        std::fprintf(f, "{\"key\": \"%s\", \"path\": \"%s\", \"update_shape\": \"%s\", \"ms_per_step\": {",
                     key.c_str(), PATH_NAMES[best], SHAPE_NAMES[out->update_shape]);
        bool first = true;
        for (int p = 0; p < 4; ++p) {
            if (out->ms[p] <= 0.f) continue;
            std::fprintf(f, "%s\"%s\": %.6g", first ? "" : ", ", PATH_NAMES[p], (double)out->ms[p]);
            first = false;
        }
        std::fprintf(f, "}}\n");
        std::fclose(f);
    }
    return 0;
}

static int enqueue_step(crkfr_solver* s, double dt_fixed, double t_end)
{
    int lrc = check_learned(s);
    if (lrc) return lrc;
    if (s->inflow && !s->has_inflow_data) return fail(CRKFR_ESTATE, "inflow boundaries need data (crkfr_set_inflow)");
    PrepArgs pa;
    pa.dt_dev = s->dt_dev;
    pa.t_dev = s->t_dev;
    pa.t_end = t_end;
    pa.dt_fixed = dt_fixed;
    pa.cfl_cs = s->cfg.cs * s->cfl;
    pa.rate_bits = s->rate_bits;
    pa.diag = s->diag;
    pa.steps = s->steps;
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(RATE_SLOTS), 0, s->stream, pa);
    const int in = s->cur, out = 1 - s->cur;
    const bool tm = s->timing;
    const int path = path_in_use(s);
    const bool tile = path == CRKFR_PATH_TILE, fu = path == CRKFR_PATH_FACE_UPDATE;
    if (path == CRKFR_PATH_CHECKER) {
        // colour 0 local; colour 1 local, faces and update; colour 0 update
        if (tm) (void)hipEventRecord(s->ev[0], s->stream);
        int rc = dispatch_step(s, PH_CB_LOCAL, in, out);
        if (tm) (void)hipEventRecord(s->ev[1], s->stream);
        if (!rc) rc = dispatch_step(s, PH_CB_WHITE, in, out);
        if (tm) (void)hipEventRecord(s->ev[2], s->stream);
        if (tm) (void)hipEventRecord(s->ev[3], s->stream);
        if (!rc) rc = dispatch_step(s, update_shape_in_use(s) == CRKFR_UPDATE_WAVE ? PH_CB_UPDATE_W : PH_CB_UPDATE,
                                    in, out);
        if (tm) (void)hipEventRecord(s->ev[4], s->stream);
        s->cur = out;
        return rc;
    }
    if (tm) (void)hipEventRecord(s->ev[0], s->stream);
    int rc = dispatch_step(s, tile ? PH_TILE : PH_LOCAL, in, out);
    if (tm) (void)hipEventRecord(s->ev[1], s->stream);
    if (!rc && !fu) rc = dispatch_step(s, tile ? PH_TILE_FACE_X : PH_FACE_X, in, out);
    if (tm) (void)hipEventRecord(s->ev[2], s->stream);
    if (!rc && !fu && s->dim == 2) rc = dispatch_step(s, tile ? PH_TILE_FACE_Y : PH_FACE_Y, in, out);
    if (tm) (void)hipEventRecord(s->ev[3], s->stream);
    const bool wu = update_shape_in_use(s) == CRKFR_UPDATE_WAVE;
    if (!rc && (!tile || s->n_edge > 0))
        rc = dispatch_step(s, tile ? PH_EDGE_UPDATE : (fu ? (wu ? PH_UPDATE_FU_W : PH_UPDATE_FU)
                                                          : (wu ? PH_UPDATE_W : PH_UPDATE)), in, out);
    if (tm) (void)hipEventRecord(s->ev[4], s->stream);
    s->cur = out;
    return rc;
}

extern "C" int crkfr_step(crkfr_solver* s, double dt)
{
    if (!s) return fail(CRKFR_EINVAL, "null argument");
    if (!s->has_state) return fail(CRKFR_ESTATE, "no state set");
    return enqueue_step(s, dt > 0.0 ? dt : 0.0, 0.0);
}

// two steps (ping-pong of the state buffers) captured once as a HIP graph
static int build_graph(crkfr_solver* s, double t_end)
{
    invalidate_graph(s);
    const bool tm = s->timing;
    s->timing = false;
    hipGraph_t g;
    const int cur0 = s->cur;
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        s->timing = tm;
        return fail(CRKFR_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    int rc = enqueue_step(s, 0.0, t_end);
    if (!rc) rc = enqueue_step(s, 0.0, t_end);
    e = hipStreamEndCapture(s->stream, &g);
    s->timing = tm;
    s->cur = cur0;
    if (rc) {
        if (e == hipSuccess) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(CRKFR_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(CRKFR_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    s->graph_t_end = t_end;
    s->graph_cur = cur0;
    return 0;
}

extern "C" int crkfr_advance(crkfr_solver* s, double t_end, int max_steps)
{
    if (!s) return fail(CRKFR_EINVAL, "null argument");
    if (!s->has_state) return fail(CRKFR_ESTATE, "no state set");
    if (max_steps < 0) return fail(CRKFR_EINVAL, "max_steps < 0");
    if (!s->graph_exec || s->graph_t_end != t_end || s->graph_cur != s->cur) {
        int rc = build_graph(s, t_end);
        if (rc) return rc;
    }
    int done = 0;
    while (done < max_steps) {
        if (max_steps - done >= 2) {
            HIP_TRY(hipGraphLaunch(s->graph_exec, s->stream));
            done += 2;
        } else {
            int rc = enqueue_step(s, 0.0, t_end);
            if (rc) return rc;
            done += 1;
            continue;
        }
        if (done % 64 == 0 && t_end > 0.0) {
            double t = 0.0;
            HIP_TRY(hipMemcpyAsync(&t, s->t_dev, sizeof(double), hipMemcpyDeviceToHost, s->stream));
            HIP_TRY(hipStreamSynchronize(s->stream));
            if (t >= t_end) break;
        }
    }
    return 0;
}

extern "C" int crkfr_get_state(crkfr_solver* s, double* out, int on_device)
{
    if (!s || !out) return fail(CRKFR_EINVAL, "null argument");
    if (!s->has_state) return fail(CRKFR_ESTATE, "no state set");
    const size_t n = (size_t)s->M * s->ne * s->np;
    double* dst = out;
    double* tmp = nullptr;
    if (!on_device) {
        HIP_TRY(hipMalloc((void**)&tmp, n * sizeof(double)));
        dst = tmp;
    }
    int rc = run_io(s, PH_EXPORT, nullptr, dst, nullptr);
    if (!rc && tmp) HIP_TRY(hipMemcpyAsync(out, tmp, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (tmp) (void)hipFree(tmp);
    return rc;
}

extern "C" int crkfr_get_means(crkfr_solver* s, double* out)
{
    if (!s || !out) return fail(CRKFR_EINVAL, "null argument");
    if (!s->has_state) return fail(CRKFR_ESTATE, "no state set");
    const size_t n = (size_t)s->M * s->ne;
    double* tmp = nullptr;
    HIP_TRY(hipMalloc((void**)&tmp, n * sizeof(double)));
    int rc = run_io(s, PH_EXPORT, nullptr, nullptr, tmp);
    if (!rc) HIP_TRY(hipMemcpyAsync(out, tmp, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    (void)hipFree(tmp);
    return rc;
}

extern "C" int crkfr_get_alpha(crkfr_solver* s, double* out)
{
    if (!s || !out) return fail(CRKFR_EINVAL, "null argument");
    HIP_TRY(hipMemcpyAsync(out, s->alpha_out, s->ne * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return 0;
}

extern "C" int crkfr_get_diag(crkfr_solver* s, crkfr_diag* out)
{
    if (!s || !out) return fail(CRKFR_EINVAL, "null argument");
    unsigned long long d[D_NCOUNT];
    double t = 0.0, dt = 0.0;
    long long steps = 0;
    HIP_TRY(hipMemcpyAsync(d, s->diag, sizeof(d), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(&t, s->t_dev, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(&dt, s->dt_dev, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(&steps, s->steps, sizeof(long long), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    out->n_troubled = (long long)d[D_TROUBLED];
    out->n_flux_limited = (long long)d[D_FLUXLIM];
    out->n_lo_inadmissible = (long long)d[D_LOBAD];
    out->n_slope_limited = (long long)d[D_SLOPELIM];
    out->n_hancock_fallback = (long long)d[D_FALLBACK];
    out->n_scaled = (long long)d[D_SCALED];
    out->n_mean_inadmissible = (long long)d[D_MEANBAD];
    std::memcpy(&out->min_theta_flux, &d[D_THFLUX], sizeof(double));
    std::memcpy(&out->min_theta_scale, &d[D_THSCALE], sizeof(double));
    out->t = t;
    out->dt = dt;
    out->steps = steps;
    out->n_learned_fallback = (long long)d[D_LFALLBACK];
    out->n_learned_disagree = 0;
    out->max_alpha_dev = 0.0;
    if (s->lim.indicator == CRKFR_IND_LEARNED && s->lim.blend != CRKFR_BLEND_OFF) {
        // judge: the learned alpha against the smoothness indicator's, per element
        std::vector<double> al(s->ne), ai(s->ne);
        HIP_TRY(hipMemcpyAsync(al.data(), s->alpha_raw, s->ne * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipMemcpyAsync(ai.data(), s->alpha_judge, s->ne * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        for (int e = 0; e < s->ne; ++e) {
            if ((al[e] > 0.0) != (ai[e] > 0.0)) ++out->n_learned_disagree;
            double dv = std::fabs(al[e] - ai[e]);
            if (dv > out->max_alpha_dev) out->max_alpha_dev = dv;
        }
    }
    StateStats st = {0.0, 0.0, 0.0, 0.0, 0};
    if (s->has_state) {
        int rc = state_stats(s, &st);
        if (rc) return rc;
    }
    out->min_rho = st.min_rho;
    out->min_p = st.min_p1;
    out->min_p2 = st.min_p2;
    out->n_nonfinite = st.nonfinite;
    out->mass = st.mass;
    out->mass_drift = (st.mass - s->mass0) / (s->mass0 != 0.0 ? std::fabs(s->mass0) : 1.0);
    if (out->n_mean_inadmissible > 0)
        return fail(CRKFR_EINADMISSIBLE_MEAN, "an element mean left the admissible set");
    return 0;
}

extern "C" int crkfr_nvar(const crkfr_solver* s) { return s ? s->M : 0; }
extern "C" int crkfr_nodes_per_element(const crkfr_solver* s) { return s ? s->np : 0; }
extern "C" double crkfr_cfl_in_use(const crkfr_solver* s) { return s ? s->cfl : 0.0; }

extern "C" int crkfr_set_timing(crkfr_solver* s, int on)
{
    if (!s) return fail(CRKFR_EINVAL, "null argument");
    if (on && !s->ev[0])
        for (int i = 0; i < 6; ++i) HIP_TRY(hipEventCreate(&s->ev[i]));
    s->timing = on != 0;
    return 0;
}

extern "C" int crkfr_get_kernel_times(crkfr_solver* s, float* ms4)
{
    if (!s || !ms4) return fail(CRKFR_EINVAL, "null argument");
    if (!s->ev[0]) return fail(CRKFR_ESTATE, "timing not enabled");
    HIP_TRY(hipEventSynchronize(s->ev[4]));
    for (int i = 0; i < 4; ++i) HIP_TRY(hipEventElapsedTime(&ms4[i], s->ev[i], s->ev[i + 1]));
    return 0;
}

extern "C" const char* crkfr_last_error(void) { return g_last_error.c_str(); }

// ----------------------------------------------------------------------------
// one step without device allocation: the step's intermediate buffers live in
// a file-scope device array (each device holds its own copy); host code uses
// its device address from hipGetSymbolAddress, taken once per device
// ----------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[CRKFR_STATIC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static unsigned char* g_scratch[MAX_DEVICES];
static std::mutex g_scratch_mutex;

static int scratch_on_device(unsigned char** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(CRKFR_EINVAL, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CRKFR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = (unsigned char*)p;
    }
    *out = g_scratch[dev];
    return 0;
}

// zero n 64-bit words (a kernel rather than hipMemsetAsync, which graph
// capture would record as a memset node)
static __global__ void k_zero_u64(unsigned long long* p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

extern "C" int crkfr_step_static(const crkfr_config* cfg, const crkfr_limiter_opts* lim, const double* u_in,
                                 double* u_out, double dt, void* hip_stream)
{
    if (!cfg || !u_in || !u_out) return fail(CRKFR_EINVAL, "null argument");
    if (u_in == u_out) return fail(CRKFR_EINVAL, "input and output must be distinct buffers");
    {
        const int rc = validate_config(cfg);
        if (rc) return rc;
    }
    if (cfg->dtype != CRKFR_FP64) return fail(CRKFR_EINVAL, "the static step is FP64 only");
    if (!(dt > 0.0)) return fail(CRKFR_EINVAL, "the static step needs dt > 0");
    const int dim = cfg->equation == CRKFR_EULER2D || cfg->equation == CRKFR_TENMOM2D ? 2 : 1;
    for (int i = 0; i < (dim == 2 ? 4 : 2); ++i)
        if (cfg->bc[i] == CRKFR_BC_INFLOW) return fail(CRKFR_EINVAL, "inflow boundaries need a solver (crkfr_set_inflow)");
    if (lim) {
        if (lim->blend < 0 || lim->blend > 2 || (lim->indicator != CRKFR_IND_PAPER && lim->indicator != CRKFR_IND_CONST))
            return fail(CRKFR_EINVAL, "the static step takes the smoothness indicator or a constant alpha");
        if (lim->flux_limiter && lim->blend == CRKFR_BLEND_OFF)
            return fail(CRKFR_EINVAL, "the flux limiter needs a low-order blend (FO or MH)");
        if (lim->blend == CRKFR_BLEND_MH && cfg->points == CRKFR_POINTS_GLL)
            return fail(CRKFR_EINVAL, "MUSCL-Hancock blending needs Gauss-Legendre points");
    }
    unsigned char* base = nullptr;
    {
        const int rc = scratch_on_device(&base);
        if (rc) return rc;
    }
    // a solver on the stack whose buffers are the caller's state and the scratch
    crkfr_solver s;
    std::memset(&s, 0, sizeof(s));
    s.cfg = *cfg;
    if (s.cfg.cs <= 0.0) s.cfg.cs = 0.98;
    s.stream = (hipStream_t)hip_stream;
    s.M = eq_nvar(cfg->equation);
    s.dim = dim;
    s.nd = cfg->N + 1;
    s.nq = dim == 2 ? s.nd : 1;
    s.np = s.nd * s.nq;
    s.ne = cfg->nx * cfg->ny;
    s.C_max = 4 * s.M + 1;
    s.stages = std::min(cfg->N + 1, 4);
    s.dissipation = CRKFR_DISS_D2;
    s.central = CRKFR_CENTRAL_EA;
    s.path = CRKFR_PATH_FACE_UPDATE;   // no face flux arrays in the scratch layout
    s.path_set = true;
    s.cfl = 1.0;   // dt is given
    if (lim) s.lim = *lim;
    else s.lim.blend = CRKFR_BLEND_OFF;
    if (s.lim.alpha_max <= 0.0) s.lim.alpha_max = 1.0;
    make_ref(cfg->N, cfg->points, s.ref);
    // layout: the words k_prep and the counters use, then the step's buffers
    const size_t M = s.M, ne = s.ne, np = s.np;
    const size_t head_words = 4 + RATE_SLOTS + D_NCOUNT;
    size_t off = 0;
    auto take = [&](size_t bytes) { unsigned char* p = base + off; off += (bytes + 255) & ~(size_t)255; return p; };
    unsigned long long* head = (unsigned long long*)take(head_words * 8);
    s.dt_dev = (double*)head;
    s.t_dev = (double*)(head + 1);         // t, t^n
    s.steps = (long long*)(head + 3);
    s.rate_bits = head + 4;
    s.diag = head + 4 + RATE_SLOTS;
    s.uHp = take(M * ne * np * 8);
    s.trx = take(2 * (size_t)s.C_max * ne * s.nq * 8);
    if (dim == 2) s.trY = take(2 * (size_t)s.C_max * ne * s.nd * 8);
    if (s.lim.blend != CRKFR_BLEND_OFF) {
        s.alpha_raw = (double*)take(ne * 8);
        s.alpha_out = (double*)take(ne * 8);
    }
    bool farfield = false;
    for (int i = 0; i < (dim == 2 ? 4 : 2); ++i) farfield |= cfg->bc[i] == CRKFR_BC_FARFIELD;
    if (farfield) s.ghost = take(ghost_size(&s) * 8);
    if (off > CRKFR_STATIC_SCRATCH_BYTES)
        return fail(CRKFR_EINVAL, "grid too large for the static scratch (" + std::to_string(off) + " bytes needed, " +
                                      std::to_string((size_t)CRKFR_STATIC_SCRATCH_BYTES) + " held)");
    s.u[0] = (void*)u_in;
    s.u[1] = u_out;
    s.cur = 0;
    s.has_state = true;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s.stream, head, (int)head_words);
    int rc = 0;
    if (farfield) rc = run_io(&s, PH_GHOST, nullptr, nullptr, nullptr);
    if (!rc) rc = enqueue_step(&s, dt, 0.0);
    if (!rc) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(CRKFR_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return rc;
}

// ----------------------------------------------------------------------------
// batches: many instances advanced together, one launch per phase and degree
// group (persistent workgroups over a table of work items), the steps
// captured as one HIP graph
// ----------------------------------------------------------------------------
struct BatchGroup {
    int eq, N, lim;
    bool fu;                  // faces fused into the update (every member on that path)
    bool mp;
    std::vector<int> members;
    void* d_args[2];          // StepArgs<real>[members] for state parity 0 / 1
    int2* d_work[4];
    int nwork[4];
    int grid[4];              // persistent workgroups per phase (0: one per work item)
};

struct crkfr_batch {
    std::vector<crkfr_solver*> s;
    std::vector<int> cur0;
    hipStream_t stream;
    bool own_stream;
    std::vector<BatchGroup> groups;
    PrepArgs* d_prep;
    int parity;
    hipGraphExec_t graph;
    int graph_parity;
    hipEvent_t ev0, ev1;
    bool timing;              // per-phase events, steps not replayed from the graph
    hipEvent_t pev[5];
    float phase_ms[4];
};

static int eq_geometry(int eq, int N, int* el, int* eu, int* nq)
{
    switch (eq) {
    case CRKFR_LINADV1D: return linadv1d_geometry(N, el, eu, nq);
    case CRKFR_BURGERS1D: return burgers1d_geometry(N, el, eu, nq);
    case CRKFR_TENMOM1D: return tenmom1d_geometry(N, el, eu, nq);
    case CRKFR_EULER1D: return euler1d_geometry(N, el, eu, nq);
    case CRKFR_EULER2D: return euler2d_geometry(N, el, eu, nq);
    case CRKFR_TENMOM2D: return tenmom2d_geometry(N, el, eu, nq);
    }
    return -1;
}

static int launch_group_phase(const crkfr_batch* b, const BatchGroup& g, int wphase, int grid)
{
    if (g.nwork[wphase] == 0) return 0;
    if (g.fu && (wphase == BPH_FACE_X || wphase == BPH_FACE_Y)) return 0;   // inside the update
    int rc = -1;
    const int2* w = g.d_work[wphase];
    const int nw = g.nwork[wphase];
    const int phase = g.fu && wphase == BPH_UPDATE ? BPH_UPDATE_FU : wphase;
    if (g.mp) {
        const StepArgs<float>* args = (const StepArgs<float>*)g.d_args[b->parity];
        switch (g.eq) {
        case CRKFR_LINADV1D: rc = linadv1d_batch_f32(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_BURGERS1D: rc = burgers1d_batch_f32(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_TENMOM1D: rc = tenmom1d_batch_f32(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_EULER1D: rc = euler1d_batch_f32(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_EULER2D: rc = euler2d_batch_f32(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_TENMOM2D: rc = tenmom2d_batch_f32(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        }
    } else {
        const StepArgs<double>* args = (const StepArgs<double>*)g.d_args[b->parity];
        switch (g.eq) {
        case CRKFR_LINADV1D: rc = linadv1d_batch_f64(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_BURGERS1D: rc = burgers1d_batch_f64(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_TENMOM1D: rc = tenmom1d_batch_f64(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_EULER1D: rc = euler1d_batch_f64(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_EULER2D: rc = euler2d_batch_f64(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        case CRKFR_TENMOM2D: rc = tenmom2d_batch_f64(g.N, g.lim, phase, args, w, nw, grid, b->stream); break;
        }
    }
    if (rc) return fail(CRKFR_EINVAL, "no batched kernel for this group");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CRKFR_EHIP, std::string("batched launch: ") + hipGetErrorString(e));
    return 0;
}

static int enqueue_batch_step(crkfr_batch* b)
{
    hipLaunchKernelGGL(k_prep_batch, dim3((unsigned)b->s.size()), dim3(RATE_SLOTS), 0, b->stream, b->d_prep);
    if (b->timing) (void)hipEventRecord(b->pev[0], b->stream);
    for (int ph = 0; ph < 4; ++ph) {
        for (const BatchGroup& g : b->groups) {
            int rc = launch_group_phase(b, g, ph, g.grid[ph]);
            if (rc) return rc;
        }
        if (b->timing) (void)hipEventRecord(b->pev[ph + 1], b->stream);
    }
    b->parity ^= 1;
    for (size_t i = 0; i < b->s.size(); ++i) b->s[i]->cur = b->parity ? 1 - b->cur0[i] : b->cur0[i];
    return 0;
}

static void free_batch(crkfr_batch* b)
{
    for (BatchGroup& g : b->groups) {
        for (int i = 0; i < 2; ++i)
            if (g.d_args[i]) (void)hipFree(g.d_args[i]);
        for (int i = 0; i < 4; ++i)
            if (g.d_work[i]) (void)hipFree(g.d_work[i]);
    }
    if (b->d_prep) (void)hipFree(b->d_prep);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    for (int i = 0; i < 5; ++i)
        if (b->pev[i]) (void)hipEventDestroy(b->pev[i]);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

template <class real>
static int upload_group_args(crkfr_batch* b, BatchGroup& g)
{
    for (int par = 0; par < 2; ++par) {
        std::vector<StepArgs<real>> h;
        for (int m : g.members) {
            crkfr_solver* s = b->s[m];
            const int in = par ? 1 - b->cur0[m] : b->cur0[m];
            h.push_back(step_args<real>(s, in, 1 - in));
        }
        HIP_TRY(hipMalloc(&g.d_args[par], h.size() * sizeof(StepArgs<real>)));
        HIP_TRY(hipMemcpy(g.d_args[par], h.data(), h.size() * sizeof(StepArgs<real>), hipMemcpyHostToDevice));
    }
    return 0;
}

extern "C" int crkfr_batch_create(crkfr_solver* const* solvers, int count, void* hip_stream, crkfr_batch** out)
{
    if (!solvers || count < 1 || !out) return fail(CRKFR_EINVAL, "null argument or empty batch");
    *out = nullptr;
    crkfr_batch* b = new crkfr_batch();
    b->stream = (hipStream_t)hip_stream;
    if (!b->stream) {
        hipError_t e = hipStreamCreate(&b->stream);
        if (e != hipSuccess) {
            delete b;
            return fail(CRKFR_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        b->own_stream = true;
    }
    for (int i = 0; i < count; ++i) {
        crkfr_solver* s = solvers[i];
        if (!s || !s->has_state) {
            free_batch(b);
            delete b;
            return fail(CRKFR_ESTATE, "every batch member needs a state");
        }
        int lrc = check_learned(s);
        if (!lrc && s->inflow && !s->has_inflow_data)
            lrc = fail(CRKFR_ESTATE, "inflow boundaries need data (crkfr_set_inflow)");
        if (lrc) {
            free_batch(b);
            delete b;
            return lrc;
        }
        (void)hipStreamSynchronize(s->stream);
        b->s.push_back(s);
        b->cur0.push_back(s->cur);
    }
    // group members by equation, degree, arithmetic and limiting
    for (int i = 0; i < count; ++i) {
        crkfr_solver* s = b->s[i];
        const int lim = s->lim.blend != CRKFR_BLEND_OFF;
        BatchGroup* g = nullptr;
        for (BatchGroup& gg : b->groups)
            if (gg.eq == s->cfg.equation && gg.N == s->cfg.N && gg.mp == s->mp && gg.lim == lim) g = &gg;
        const bool mfu = path_in_use(s) == CRKFR_PATH_FACE_UPDATE || path_in_use(s) == CRKFR_PATH_CHECKER;
        if (g && g->fu != mfu) g->fu = false;
        if (!g) {
            BatchGroup ng;
            std::memset(ng.d_args, 0, sizeof(ng.d_args));
            std::memset(ng.d_work, 0, sizeof(ng.d_work));
            std::memset(ng.nwork, 0, sizeof(ng.nwork));
            std::memset(ng.grid, 0, sizeof(ng.grid));
            ng.eq = s->cfg.equation;
            ng.N = s->cfg.N;
            ng.mp = s->mp;
            ng.lim = lim;
            ng.fu = mfu;
            b->groups.push_back(ng);
            g = &b->groups.back();
        }
        g->members.push_back(i);
    }
    for (BatchGroup& g : b->groups) {
        int rc = g.mp ? upload_group_args<float>(b, g) : upload_group_args<double>(b, g);
        if (rc) { free_batch(b); delete b; return rc; }
        int el = 0, eu = 0, nq = 0;
        eq_geometry(g.eq, g.N, &el, &eu, &nq);
        std::vector<int2> work[4];
        for (size_t j = 0; j < g.members.size(); ++j) {
            crkfr_solver* s = b->s[g.members[j]];
            const int nx = s->cfg.nx, ny = s->cfg.ny, nd = s->nd;
            const long long cnt[4] = {
                (s->ne + el - 1) / el,
                ((long long)ny * (nx + 1) * nq + 255) / 256,
                s->dim == 2 ? ((long long)(ny + 1) * nx * nd + 255) / 256 : 0,
                (s->ne + eu - 1) / eu};
            for (int ph = 0; ph < 4; ++ph)
                for (long long w = 0; w < cnt[ph]; ++w) work[ph].push_back(make_int2((int)j, (int)w));
        }
        for (int ph = 0; ph < 4; ++ph) {
            g.nwork[ph] = (int)work[ph].size();
            if (g.nwork[ph] == 0) continue;
            if (hipMalloc((void**)&g.d_work[ph], work[ph].size() * sizeof(int2)) != hipSuccess ||
                hipMemcpy(g.d_work[ph], work[ph].data(), work[ph].size() * sizeof(int2), hipMemcpyHostToDevice)
                    != hipSuccess) {
                free_batch(b);
                delete b;
                return fail(CRKFR_ENOMEM, "batch work tables");
            }
        }
    }
    std::vector<PrepArgs> prep;
    for (crkfr_solver* s : b->s) {
        PrepArgs pa;
        pa.dt_dev = s->dt_dev;
        pa.t_dev = s->t_dev;
        pa.t_end = 0.0;
        pa.dt_fixed = 0.0;
        pa.cfl_cs = s->cfg.cs * s->cfl;
        pa.rate_bits = s->rate_bits;
        pa.diag = s->diag;
        pa.steps = s->steps;
        prep.push_back(pa);
    }
    if (hipMalloc((void**)&b->d_prep, prep.size() * sizeof(PrepArgs)) != hipSuccess ||
        hipMemcpy(b->d_prep, prep.data(), prep.size() * sizeof(PrepArgs), hipMemcpyHostToDevice) != hipSuccess) {
        free_batch(b);
        delete b;
        return fail(CRKFR_ENOMEM, "batch time-step table");
    }
    (void)hipEventCreate(&b->ev0);
    (void)hipEventCreate(&b->ev1);
    for (crkfr_solver* s : b->s) ++s->batch_refs;
    *out = b;
    return 0;
}

extern "C" void crkfr_batch_destroy(crkfr_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (crkfr_solver* s : b->s) --s->batch_refs;
    free_batch(b);
    delete b;
}

extern "C" int crkfr_batch_step(crkfr_batch* b)
{
    if (!b) return fail(CRKFR_EINVAL, "null argument");
    return enqueue_batch_step(b);
}

extern "C" int crkfr_batch_advance(crkfr_batch* b, int steps)
{
    if (!b || steps < 0) return fail(CRKFR_EINVAL, "bad argument");
    if (b->timing) {
        for (int k = 0; k < steps; ++k) {
            int rc = enqueue_batch_step(b);
            if (rc) return rc;
        }
        return 0;
    }
    if (!b->graph || b->graph_parity != b->parity) {
        if (b->graph) {
            (void)hipGraphExecDestroy(b->graph);
            b->graph = nullptr;
        }
        hipGraph_t g;
        const int par0 = b->parity;
        hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(CRKFR_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        int rc = enqueue_batch_step(b);
        if (!rc) rc = enqueue_batch_step(b);
        e = hipStreamEndCapture(b->stream, &g);
        b->parity = par0;
        for (size_t i = 0; i < b->s.size(); ++i) b->s[i]->cur = b->parity ? 1 - b->cur0[i] : b->cur0[i];
        if (rc) {
            if (e == hipSuccess) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(CRKFR_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(CRKFR_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        b->graph_parity = par0;
    }
    int done = 0;
    for (; done + 2 <= steps; done += 2) HIP_TRY(hipGraphLaunch(b->graph, b->stream));
    if (done < steps) return enqueue_batch_step(b);
    return 0;
}

extern "C" int crkfr_batch_sync(crkfr_batch* b)
{
    if (!b) return fail(CRKFR_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(b->stream));
    return 0;
}

extern "C" int crkfr_batch_set_t_end(crkfr_batch* b, double t_end)
{
    if (!b) return fail(CRKFR_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(b->stream));
    std::vector<PrepArgs> prep(b->s.size());
    HIP_TRY(hipMemcpy(prep.data(), b->d_prep, prep.size() * sizeof(PrepArgs), hipMemcpyDeviceToHost));
    for (PrepArgs& p : prep) p.t_end = t_end > 0.0 ? t_end : 0.0;
    HIP_TRY(hipMemcpy(b->d_prep, prep.data(), prep.size() * sizeof(PrepArgs), hipMemcpyHostToDevice));
    return 0;
}

extern "C" int crkfr_batch_set_timing(crkfr_batch* b, int on)
{
    if (!b) return fail(CRKFR_EINVAL, "null argument");
    if (on && !b->pev[0])
        for (int i = 0; i < 5; ++i) HIP_TRY(hipEventCreate(&b->pev[i]));
    b->timing = on != 0;
    return 0;
}

extern "C" int crkfr_batch_phase_times(crkfr_batch* b, float* ms4)
{
    if (!b || !ms4) return fail(CRKFR_EINVAL, "null argument");
    if (!b->pev[0]) return fail(CRKFR_ESTATE, "timing is off");
    HIP_TRY(hipEventSynchronize(b->pev[4]));
    for (int i = 0; i < 4; ++i) HIP_TRY(hipEventElapsedTime(&ms4[i], b->pev[i], b->pev[i + 1]));
    return 0;
}

extern "C" int crkfr_batch_num_groups(const crkfr_batch* b) { return b ? (int)b->groups.size() : 0; }

extern "C" int crkfr_batch_grid(crkfr_batch* b, int group, int phase, int set_to)
{
    if (!b || group < 0 || group >= (int)b->groups.size() || phase < 0 || phase > 3)
        return fail(CRKFR_EINVAL, "bad group or phase");
    if (set_to >= 0) {
        b->groups[group].grid[phase] = set_to;
        if (b->graph) {
            (void)hipGraphExecDestroy(b->graph);
            b->graph = nullptr;
        }
    }
    return b->groups[group].grid[phase];
}

// time each phase of each group for a set of persistent grid sizes and keep
// the fastest; phases are re-run on the current state (their outputs are
// recomputed by the next step), so the state is not advanced
extern "C" int crkfr_batch_autotune(crkfr_batch* b, int reps)
{
    if (!b || reps < 1) return fail(CRKFR_EINVAL, "bad argument");
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    // the trial runs touch each member's time-step slots, clock and counters:
    // keep them and put them back afterwards
    struct Saved {
        unsigned long long rate[RATE_SLOTS], diag[D_NCOUNT];
        double t, dt;
        long long steps;
    };
    std::vector<Saved> saved(b->s.size());
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < b->s.size(); ++i) {
        crkfr_solver* s = b->s[i];
        HIP_TRY(hipMemcpy(saved[i].rate, s->rate_bits, sizeof(saved[i].rate), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(saved[i].diag, s->diag, sizeof(saved[i].diag), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&saved[i].t, s->t_dev, sizeof(double), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&saved[i].dt, s->dt_dev, sizeof(double), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&saved[i].steps, s->steps, sizeof(long long), hipMemcpyDeviceToHost));
    }
    // the step's inputs must exist: one k_prep so every dt is set
    hipLaunchKernelGGL(k_prep_batch, dim3((unsigned)b->s.size()), dim3(RATE_SLOTS), 0, b->stream, b->d_prep);
    for (BatchGroup& g : b->groups)
        for (int ph = 0; ph < 4; ++ph) {
            if (g.nwork[ph] == 0 || (g.fu && (ph == BPH_FACE_X || ph == BPH_FACE_Y))) continue;
            const int cands[] = {0, ncu, 2 * ncu, 4 * ncu, 8 * ncu, 16 * ncu};
            float best = 1e30f;
            int best_grid = 0;
            for (int c : cands) {
                if (c >= g.nwork[ph]) continue;
                int rc = launch_group_phase(b, g, ph, c);   // warm-up
                if (rc) return rc;
                HIP_TRY(hipEventRecord(b->ev0, b->stream));
                for (int r = 0; r < reps; ++r) {
                    rc = launch_group_phase(b, g, ph, c);
                    if (rc) return rc;
                }
                HIP_TRY(hipEventRecord(b->ev1, b->stream));
                HIP_TRY(hipEventSynchronize(b->ev1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
                if (ms < best) { best = ms; best_grid = c; }
            }
            g.grid[ph] = best_grid;
        }
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < b->s.size(); ++i) {
        crkfr_solver* s = b->s[i];
        HIP_TRY(hipMemcpy(s->rate_bits, saved[i].rate, sizeof(saved[i].rate), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->diag, saved[i].diag, sizeof(saved[i].diag), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->t_dev, &saved[i].t, sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->dt_dev, &saved[i].dt, sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->steps, &saved[i].steps, sizeof(long long), hipMemcpyHostToDevice));
    }
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return 0;
}
