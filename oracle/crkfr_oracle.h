/*
 * crkfr_oracle.h -- plain FP64 CPU oracle for one compact Runge-Kutta Flux
 * Reconstruction (cRKFR) time step (Babbar & Chen, arXiv 2502.07517).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * Layout of nodal arrays (both 1D and 2D):
 *     u[var][ey][ex][q][p]      p = x-node (fastest), q = y-node
 * In 1D, ny = 1 and q takes the single value 0.
 */
#ifndef CRKFR_ORACLE_H
#define CRKFR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define REF_MAXN 4
#define REF_MAXND (REF_MAXN + 1)
#define REF_MAXNP (REF_MAXND * REF_MAXND)
#define REF_MAXM 6

enum { REF_LINADV1D = 0, REF_EULER1D = 1, REF_EULER2D = 2, REF_TENMOM2D = 3, REF_BURGERS1D = 4,
       REF_TENMOM1D = 5 };
/* dissipative part of the numerical flux (Sec. 3.1.1): eqs. D2, D1, dcsx */
enum { REF_DISS_D2 = 0, REF_DISS_D1 = 1, REF_DISS_DCSX = 2 };
/* central part (Sec. 3.1.2): eq. evaluate (EA) or eq. extrapolate (AE) */
enum { REF_CENTRAL_EA = 0, REF_CENTRAL_AE = 1 };
enum { REF_BC_PERIODIC = 0, REF_BC_OUTFLOW = 1, REF_BC_FARFIELD = 2, REF_BC_REFLECT = 3, REF_BC_INFLOW = 4 };
enum { REF_BLEND_OFF = 0, REF_BLEND_FO = 1, REF_BLEND_MH = 2 };
enum { REF_IND_PAPER = 0, REF_IND_CONST = 1, REF_IND_GIVEN = 2, REF_IND_LEARNED = 3 };
/* solution points (Sec. 2, eq. soln.points): Gauss-Legendre with the Radau
 * correction, or Gauss-Legendre-Lobatto with the g2 correction */
enum { REF_POINTS_GL = 0, REF_POINTS_GLL = 1 };

typedef struct {
    int eq, N, nx, ny, stages;
    int bc[4];            /* x-left, x-right, y-bottom, y-top */
    int blend, indicator, smooth_nbr, flux_limiter, scaling, source;
    double x0, x1, y0, y1;
    double gamma, adv, cfl, cs;
    double alpha_min, alpha_max, alpha_const;
    double src_amp, src_kappa, src_xc, src_yc;   /* W = A exp(-kappa r^2) + gx x + gy y */
    double src_gx, src_gy;
    /* learned indicator (indicator == REF_IND_LEARNED): an MLP with layer
     * sizes mlp_dims[0..mlp_nl] (mlp_dims[0] = N inputs, one output), tanh
     * hidden layers and a sigmoid output, parameters per layer W[out][in]
     * then b[out]; feature box [mlp_lo, mlp_hi] per input */
    int mlp_nl;
    const int* mlp_dims;
    const double* mlp_params;
    const double* mlp_lo;
    const double* mlp_hi;
    int dissipation;      /* REF_DISS_* */
    int central;          /* REF_CENTRAL_* */
    int points;           /* REF_POINTS_*; MUSCL-Hancock blending needs GL points */
    /* time-dependent inflow boundaries (REF_BC_INFLOW, Sec. 3.3): boundary
     * data g(tau) = sum_k inflow[k][...] (tau - inflow_tref)^k, k <
     * inflow_ncoef, with [...] the layout of the far-field ghost states;
     * time = t^n of the step */
    const double* inflow;
    int inflow_ncoef;
    double inflow_tref;
    double time;
    /* admissibility margins of the limiter chain (<= 0: the defaults): the
     * flux limiter and the subcell reconstruction keep P_k >= eps_rel times
     * P_k of their reference state (0.1); the scaling limiter keeps P_k >=
     * min(eps_abs, P_k(mean)) (1e-13) */
    double eps_rel, eps_abs;
} ref_config;

typedef struct {
    long n_troubled;          /* elements with alpha_e > 0 */
    long n_flux_limited;      /* face points where theta < 1 */
    long n_lo_inadmissible;   /* face points whose low-order candidate failed */
    long n_slope_limited;     /* subcells whose MH slope was scaled */
    long n_hancock_fallback;  /* subcells that fell back to zero slope */
    long n_scaled;            /* elements where the scaling limiter acted */
    long n_mean_inadmissible; /* elements whose mean left the admissible set */
    double min_theta_flux, min_theta_scale;
} ref_diag;

/* reference element on [0,1] */
void ref_gl(int N, double* xi, double* w);
void ref_gll(int N, double* xi, double* w);   /* N >= 1; exact to degree 2N-1 */
void ref_lagrange_at(int N, const double* xi, double x, double* l);
void ref_diff_matrix(int N, const double* xi, double* D);
void ref_legendre_orthonormal(int N, const double* xi, double* L); /* L[k*(N+1)+p] = L_k(xi_p) */
void ref_tableau(int s, double* a /*4x4*/, double* b /*4*/, double* c /*4*/);

/* physics (exposed for pins) */
int ref_nvar(int eq);
int ref_nadm(int eq);
void ref_flux(int eq, double gamma, double adv, const double* u, double* f, double* g);
void ref_sigma(int eq, double gamma, double adv, const double* u, double* sx, double* sy);
double ref_adm(int eq, int k, double gamma, const double* u);

/* local cRK on one element: time averages at the nodes (eq. disc.avg.flux,
 * time.avg.sol and the source averages of the source-term appendix). */
void ref_local_crk(const ref_config* c, const double* ue /*[var][q][p]*/, double dt,
                   double xe0, double ye0, double* F, double* G, double* U, double* S);

/* smoothness indicator of one element (raw, before neighbour smoothing) */
double ref_indicator_raw(const ref_config* c, const double* ue, double* energy_out);

/* features of the learned indicator for one element, feat[k-1], k = 1..N:
 * log10(max(r_k, 1e-12)) / 6 + 1, at least -1, with r_k the share of the
 * degree-k shell in the energy of the shells 0..k (0 when that energy is 0) */
void ref_indicator_features(const ref_config* c, const double* ue, double* feat);

/* learned blending coefficient of one element (before neighbour smoothing);
 * *fallback = 1 when a feature left the box and the indicator was used */
double ref_learned_alpha(const ref_config* c, const double* ue, int* fallback);

/* Zhang-Shu scaling of one element in place; returns theta (min over constraints) */
double ref_scale_element(const ref_config* c, double* ue, int* mean_bad);

/* time step from the element means, eq. time.step.2d */
double ref_compute_dt(const ref_config* c, const double* u);

/* boundary traces of u at every boundary face point, the ghost states of
 * far-field boundaries: x-left [ny][N+1][M], x-right [ny][N+1][M],
 * y-bottom [nx][N+1][M], y-top [nx][N+1][M], concatenated (1D: one point per side) */
void ref_boundary_traces(const ref_config* c, const double* u, double* ghost);

/* factor dt / (w_i h_d phi_d) of the flux difference in the low-order update
 * of the face-adjacent subcell with index i (0 or N) along direction d at
 * line position t (the state u of that subcell gives phi_d; 1D: phi = 1) */
double ref_lo_factor(const ref_config* c, int d, int t, int i, const double* u, double dt);

/* flux limiter at one face point (the routine ref_step uses): F (in/out)
 * moves towards fLO so that the low-order candidates of both face-adjacent
 * subcells keep P_k >= 0.1 P_k(candidate with fLO); returns the smallest
 * theta, *bad = 1 when a candidate with fLO is not admissible */
double ref_flux_limit_face(const ref_config* c, int hasA, int hasB, const double* uA, const double* uB,
                           const double* adjA, const double* adjB, const double* SA, const double* SB,
                           double kAfac, double kBfac, double dt, const double* fLO, double* F, int* bad);

/* MUSCL-Hancock predicted face values [k][v] of the subcells of element
 * (ex, ey) (the routine ref_step uses); counts: slope scalings, fallbacks */
void ref_mh_predict(const ref_config* c, const double* u, int ex, int ey, double dt, const double* ghost,
                    double* xm, double* xp, double* ym, double* yp, int* counts);

/* one full step; alpha_given used when indicator == GIVEN; alpha_out (optional)
 * receives the final blending coefficient per element; ghost (far-field
 * boundaries only) as written by ref_boundary_traces. */
/* status: 0, -5 (a mean left the admissible set), -1 (unsupported options:
 * MUSCL-Hancock blending with GLL points) */
int ref_step(const ref_config* c, const double* u_in, double* u_out, double dt,
             const double* alpha_given, double* alpha_out, ref_diag* diag, const double* ghost);

/* one step of the scheme in its stage form (eq. crkfr): every stage's flux
 * goes through the FR derivative with its own Rusanov numerical flux at the
 * faces, and the update combines the stages with the weights b_i; periodic
 * boundaries, no limiter, no source.  Independent of ref_step; with the
 * D-CSX dissipation and EA central part ref_step computes the same update. */
void ref_step_crkfr_form(const ref_config* c, const double* u_in, double* u_out, double dt);

/* element means [var][ey][ex] */
void ref_means(const ref_config* c, const double* u, double* ubar);

/* small MLP for the learned indicator: layers 0..nl-1, sizes dims[0..nl] */
void ref_mlp_forward(int nl, const int* dims, const double* params, int nrows,
                     const double* x, double* y, double* acts);
double ref_mlp_loss_grad(int nl, const int* dims, const double* params, int nrows,
                         const double* x, const double* target, double* grad);

#ifdef __cplusplus
}
#endif
#endif
