/*
 * crkfr.h -- C ABI of the MI355X (gfx950) compact Runge-Kutta Flux
 * Reconstruction step (Babbar & Chen, arXiv 2502.07517).
 *
 * One call of crkfr_step advances the nodal solution by one time step of the
 * time-averaged cRKFR scheme, eq. (crkfr.avg), optionally with the source
 * average of App. B, eq. (crkfr.source), and with the limiter chain of Sec. 4:
 * subcell blending, eq. (blended.scheme), with MUSCL-Hancock or first-order
 * subcells, the flux limiter for admissibility in means (Sec. 4.3), and the
 * Zhang-Shu scaling limiter (Sec. 3.2).
 *
 * Conventions
 *   - Return codes: 0 = success; negative = error (CRKFR_E*).  After an
 *     error crkfr_last_error() returns a message (thread-local).
 *   - Nodal layout everywhere: u[var][ey][ex][q][p], p the x node, q the y
 *     node, doubles; 1D: u[var][ex][p].  Nodes are the Gauss-Legendre points
 *     of [0,1] mapped to each element (Sec. 2, eq. soln.points).
 *   - Host buffers passed in stay owned by the caller and are only read or
 *     written during the call.  Device buffers the library allocates are
 *     owned by the solver and freed by crkfr_destroy.
 *   - Every call is ordered on the stream given to crkfr_create.  Calls that
 *     return data to the host synchronise that stream; crkfr_step and
 *     crkfr_advance only enqueue work.
 *   - No exceptions cross the ABI.  The solver object is not thread-safe.
 */
#ifndef CRKFR_H
#define CRKFR_H

#ifdef __cplusplus
extern "C" {
#endif

#define CRKFR_OK 0
#define CRKFR_EINVAL (-1)              /* bad argument or unsupported option */
#define CRKFR_ENOMEM (-2)              /* device allocation failed */
#define CRKFR_EHIP (-3)                /* HIP runtime error, text in crkfr_last_error */
#define CRKFR_EINADMISSIBLE_INPUT (-4) /* set_state: a node violates P_k > 0 */
#define CRKFR_EINADMISSIBLE_MEAN (-5)  /* last step left an element mean outside U_ad */
#define CRKFR_ESTATE (-6)              /* call order (e.g. step before set_state) */

/* equations: scalar linear advection u_t + a u_x = 0 (Sec. 5.1.1), 1D Euler
 * (eq. 1deuler), 2D Euler (eq. 2deuler), ten-moment system (eq. tmp),
 * Burgers' equation u_t + (u^2/2)_x = 0 (Sec. 5.1.3), and the ten-moment
 * system in one dimension (the same six variables with x dependence only,
 * as in the two-rarefaction test of Sec. 5.4.2) */
enum { CRKFR_LINADV1D = 0, CRKFR_EULER1D = 1, CRKFR_EULER2D = 2, CRKFR_TENMOM2D = 3, CRKFR_BURGERS1D = 4,
       CRKFR_TENMOM1D = 5 };

/* dissipative part of the time-averaged numerical flux (Sec. 3.1.1): D2
 * lambda/2 (U+ - U-) (eq. D2, the default), D1 lambda/2 (u+ - u-) with the
 * current solution (eq. D1), D-CSX sum_i b_i lambda_i/2 (u(i)+ - u(i)-) with a
 * wave speed per stage (eq. dcsx); central part (Sec. 3.1.2): EA traces
 * sum_i b_i f(u(i)+-) (eq. evaluate, the default) or the extrapolated
 * time-averaged flux (eq. extrapolate) */
enum { CRKFR_DISS_D2 = 0, CRKFR_DISS_D1 = 1, CRKFR_DISS_DCSX = 2 };

/* solution points (Sec. 2, eq. soln.points) and their correction function:
 * Gauss-Legendre with the Radau correction, or Gauss-Legendre-Lobatto with
 * g2; both enter through g_R'(xi_p) = l_p(1)/w_p (eq. fr.equiv).  The state
 * holds nodal values at the chosen points; MUSCL-Hancock blending needs GL
 * points (first-order blending works with both). */
enum { CRKFR_POINTS_GL = 0, CRKFR_POINTS_GLL = 1 };
enum { CRKFR_CENTRAL_EA = 0, CRKFR_CENTRAL_AE = 1 };

/* boundary kinds (Sec. 3.3): periodic; outflow (ghost values copy the
 * interior side, so the boundary flux is the interior time-averaged flux, the
 * paper's rule for fully outflow boundaries); far-field (ghost state fixed to
 * the boundary traces of the state given to crkfr_set_state, used through the
 * D2 numerical flux, the paper's inflow rule with a time-constant state);
 * solid wall (eq. reflect.time.avg: the ghost traces mirror the interior
 * ones — normal momentum, and the ten-moment E12, change sign in u and U,
 * the other components in F — and the subcell ghosts mirror the boundary
 * subcell; Euler and ten-moment only); time-dependent inflow (the boundary
 * data g(x_b, t) of crkfr_set_inflow: u^- = g(t^n), U^- = sum_i b_i
 * g(t^n + c_i dt), F^- = sum_i b_i f(g(t^n + c_i dt)); F = F^- where every
 * wave of the normal flux Jacobian at g(t^n) enters the domain, otherwise
 * the D2 flux with these ghost values; the subcell ghost is g(t^n), its
 * predicted value g(t^n + dt/2)) */
enum { CRKFR_BC_PERIODIC = 0, CRKFR_BC_OUTFLOW = 1, CRKFR_BC_FARFIELD = 2, CRKFR_BC_REFLECT = 3,
       CRKFR_BC_INFLOW = 4 };
#define CRKFR_INFLOW_MAXCOEF 5

/* arithmetic: FP64 throughout, or FP32 bulk with FP64 element means and
 * FP64 admissibility roots (the state is held as FP64 means plus FP32
 * nodal deviations) */
enum { CRKFR_FP64 = 0, CRKFR_MP32 = 1 };

enum { CRKFR_BLEND_OFF = 0, CRKFR_BLEND_FO = 1, CRKFR_BLEND_MH = 2 };

/* blending coefficient source: the smoothness indicator (Sec. 4), a
 * constant, a caller-given per-element field, or the learned MLP */
enum { CRKFR_IND_PAPER = 0, CRKFR_IND_CONST = 1, CRKFR_IND_GIVEN = 2, CRKFR_IND_LEARNED = 3 };

typedef struct {
    int equation;       /* CRKFR_LINADV1D .. CRKFR_TENMOM1D */
    int N;              /* polynomial degree, 1..4; the cRK tableau has min(N+1, 4) stages */
    int nx, ny;         /* elements per direction (ny = 1 in 1D) */
    int bc[4];          /* x-left, x-right, y-bottom, y-top */
    int dtype;          /* CRKFR_FP64 or CRKFR_MP32 */
    double x0, x1, y0, y1;
    double gamma;       /* Euler: ratio of specific heats */
    double adv;         /* linear advection speed */
    double cfl;         /* CFL(N) of eq. time.step.2d; <= 0: the library's Fourier analysis */
    double cs;          /* safety factor C_s of eq. time.step.2d (paper: 0.98) */
    int points;         /* CRKFR_POINTS_GL (default, Radau correction) or CRKFR_POINTS_GLL (g2) */
} crkfr_config;

typedef struct {
    int blend;          /* CRKFR_BLEND_* */
    int indicator;      /* CRKFR_IND_* */
    int smooth_nbr;     /* alpha_e <- max(alpha_e, max over face neighbours alpha / 2) */
    int flux_limiter;   /* 1: flux limiter for admissibility in means (needs blend != OFF) */
    int scaling;        /* 1: Zhang-Shu scaling limiter */
    double alpha_min, alpha_max, alpha_const;
    /* admissibility margins (<= 0: the defaults).  eps_rel (0.1): the flux
     * limiter keeps P_k of each face-adjacent low-order candidate at least
     * eps_rel P_k(candidate with the low-order face flux) (Sec. 4.3), and the
     * MUSCL-Hancock reconstruction keeps its face and predicted values at
     * eps_rel P_k(subcell value) (Sec. 4.2); eps_abs (1e-13): the scaling
     * limiter (Sec. 3.2) keeps every node at P_k >= min(eps_abs, P_k(mean)). */
    double eps_rel, eps_abs;
} crkfr_limiter_opts;

/* ten-moment source (eq. tenmom.source) with the potential
 * W(x, y) = amp exp(-kappa ((x-xc)^2 + (y-yc)^2)) + gx x + gy y */
typedef struct {
    int enabled;
    double amp, kappa, xc, yc, gx, gy;
} crkfr_source;

typedef struct {
    long long n_troubled;          /* elements with alpha_e > 0 */
    long long n_flux_limited;      /* face points where the flux limiter acted */
    long long n_lo_inadmissible;   /* face points whose low-order candidate was not admissible */
    long long n_slope_limited;     /* subcells whose MUSCL-Hancock slope was scaled */
    long long n_hancock_fallback;  /* subcells that fell back to a zero slope */
    long long n_scaled;            /* elements changed by the scaling limiter */
    long long n_mean_inadmissible; /* elements whose mean left the admissible set */
    double min_theta_flux, min_theta_scale;
    double t, dt;                  /* time reached and last step size */
    long long steps;               /* steps taken with dt > 0 */
    /* learned indicator, judged by the smoothness indicator on the same state: */
    long long n_learned_fallback;  /* elements whose features left the network's box (indicator used) */
    long long n_learned_disagree;  /* elements troubled (alpha > 0) by one indicator but not the other */
    double max_alpha_dev;          /* max over elements of |alpha_learned - alpha_indicator| (raw) */
    /* the current state, reduced on the device when crkfr_get_diag is called
     * (the constraints P_k of eq. uad.form at the nodes, in FP64): */
    double min_rho;                /* min over nodes of the density (linear advection, Burgers: of u) */
    double min_p;                  /* min over nodes of P_1: Euler pressure, ten-moment P11 (0 if none) */
    double min_p2;                 /* min over nodes of P_2: ten-moment det P (0 if none) */
    long long n_nonfinite;         /* nodes with a non-finite variable */
    double mass;                   /* integral of the density (of u) over the domain */
    double mass_drift;             /* (mass - mass at set_state) / |mass at set_state| (absolute if 0) */
} crkfr_diag;

typedef struct crkfr_solver crkfr_solver;
typedef struct crkfr_mlp crkfr_mlp;

/* Create a solver on the current HIP device, ordered on hip_stream (a
 * hipStream_t; NULL: the solver creates a stream of its own, default
 * priority, destroyed with it).  Allocates every device buffer the step
 * needs.  Errors: EINVAL (N outside 1..4, sizes < 1, 2^31 or more nodes or
 * face points in one direction, bad enums), ENOMEM, EHIP. */
int crkfr_create(const crkfr_config* cfg, void* hip_stream, crkfr_solver** out);
void crkfr_destroy(crkfr_solver* s);

/* Scheme options: number of cRK stages (0: min(N+1, 4), the paper's pairing;
 * 2, 3, 4: cRK22, cRK33, cRK44 of eqs. crk22-crk44), dissipation and central
 * part of the numerical flux.  When the configuration's cfl is <= 0 the CFL
 * number is recomputed for the new options by the library's Fourier
 * analysis.  Errors: EINVAL (bad option), ENOMEM (D-CSX keeps every stage's
 * face values and may enlarge the trace buffers), ESTATE (the solver is a
 * member of a live batch, which holds its buffers and options). */
typedef struct {
    int stages;
    int dissipation;    /* CRKFR_DISS_* */
    int central;        /* CRKFR_CENTRAL_* */
} crkfr_scheme;
int crkfr_set_scheme(crkfr_solver* s, const crkfr_scheme* opts);

/* Limiter options (Sec. 4).  Default: blending off, no limiters. */
int crkfr_set_limiter(crkfr_solver* s, const crkfr_limiter_opts* opts);

/* Source term (App. B; ten-moment only).  Default: none. */
int crkfr_set_source(crkfr_solver* s, const crkfr_source* src);

/* Boundary data of the inflow boundaries (Sec. 3.3) as a polynomial in time:
 * g(x_b, t) = sum_{k < ncoef} coeffs[k][...] (t - t_ref)^k, 1 <= ncoef <= 5.
 * coeffs[k] holds one state per boundary face point in the layout x-left
 * [ny][nq][nvar], x-right [ny][nq][nvar], then in 2D y-bottom [nx][nd][nvar],
 * y-top [nx][nd][nvar] (nq = N+1 in 2D, 1 in 1D; nd = N+1); entries of
 * boundaries that are not inflow are ignored.  Host (on_device = 0, copied
 * before return) or device memory (copied in stream order).  The data stays
 * until the next call: callers with data that a polynomial of degree 4 does
 * not represent re-anchor it (e.g. the Taylor expansion at t^n before each
 * step).  Steps fail with ESTATE until it is set.  Errors: EINVAL (no inflow
 * boundary, bad ncoef). */
int crkfr_set_inflow(crkfr_solver* s, const double* coeffs, int ncoef, double t_ref, int on_device);

/* Set the nodal state (layout above, nvar*ny*nx*(N+1)^d doubles).  u points
 * to host memory, or to device memory when on_device = 1.  Also sets t = 0,
 * computes the element means, the wave-speed rate for eq. time.step.2d and the
 * far-field ghost states.  Errors: EINADMISSIBLE_INPUT if a node has P_k <= 0. */
int crkfr_set_state(crkfr_solver* s, const double* u, int on_device);

/* Bind a caller-owned FP64 device buffer (nvar*ny*nx*(N+1)^d doubles, the
 * nodal layout above) as the solver's state, without a copy (eq. crkfr.avg
 * advances it in place of a library buffer).  The buffer becomes one of the
 * two buffers the steps alternate between: the state is in it now and after
 * every even number of steps since this call (crkfr_advance and
 * crkfr_batch_advance keep step pairs), in a library buffer after odd
 * numbers; crkfr_state_ptr says where it is.  The caller keeps ownership and
 * must keep the buffer alive until crkfr_destroy or the next set_state or
 * bind_state.  Otherwise like crkfr_set_state with a device pointer (t = 0,
 * means, time-step rate, far-field ghosts; the data is only read here).
 * Errors: EINVAL (MP32 solver: its state is FP64 means plus FP32 deviations,
 * use set_state; null pointer), EINADMISSIBLE_INPUT, ESTATE (batch member). */
int crkfr_bind_state(crkfr_solver* s, double* u_dev);
/* Device pointer of the current FP64 nodal state (the bound buffer or a
 * library buffer); EINVAL for MP32 solvers. */
int crkfr_state_ptr(crkfr_solver* s, double** u_dev);

/* Per-element blending coefficients for CRKFR_IND_GIVEN, [ey][ex] doubles. */
int crkfr_set_alpha(crkfr_solver* s, const double* alpha, int on_device);

/* Network of the learned indicator (CRKFR_IND_LEARNED), borrowed: it must
 * have N inputs and outlive its use by this solver; NULL detaches it.  Steps
 * with the learned indicator and no network fail with ESTATE. */
int crkfr_set_mlp(crkfr_solver* s, const crkfr_mlp* m);

/* Features of the learned indicator for the current state, [e][N] floats
 * (see crkfr_mlp_create), and the smoothness indicator's alpha before
 * neighbour smoothing, [e] doubles: the training pairs of the network.
 * Either output may be NULL; on_device = 1: device pointers.  Synchronises. */
int crkfr_features(crkfr_solver* s, float* feat, double* alpha_ind, int on_device);

/* Time step of eq. time.step.2d from the current element means (synchronises). */
int crkfr_compute_dt(crkfr_solver* s, double* dt);

/* One step.  dt > 0: that step size; dt <= 0: the step size of eq.
 * time.step.2d computed on the device from the current means (no host sync). */
int crkfr_step(crkfr_solver* s, double dt);

/* Steps with device-computed dt until t_end (last step clipped) or
 * max_steps; runs the steps as one captured HIP graph per step pair. */
int crkfr_advance(crkfr_solver* s, double t_end, int max_steps);

/* Read back (synchronise).  get_state writes the nodal state in the layout
 * above (for MP32 the FP64 sum of mean and deviation); get_means writes
 * [var][ey][ex]; get_alpha the blending coefficients of the last step. */
int crkfr_get_state(crkfr_solver* s, double* out, int on_device);
int crkfr_get_means(crkfr_solver* s, double* out);
int crkfr_get_alpha(crkfr_solver* s, double* out);
/* Diagnostics of the last step (counters) and of the current state (min_rho,
 * min_p, min_p2, n_nonfinite, mass, mass_drift: a device reduction, so the
 * call synchronises and launches one kernel); returns EINADMISSIBLE_MEAN if
 * the last step left an element mean outside U_ad. */
int crkfr_get_diag(crkfr_solver* s, crkfr_diag* out);

/* Number of variables, nodes per element and the CFL number in use. */
int crkfr_nvar(const crkfr_solver* s);
int crkfr_nodes_per_element(const crkfr_solver* s);
double crkfr_cfl_in_use(const crkfr_solver* s);

/* CFL(N) by the library's Fourier analysis of the linear scheme (host only):
 * the largest lambda dt/dx with spectral radius <= 1 + tol for all wave
 * numbers; system = 0: wave speed equal to the dissipation speed (scalar
 * linear flux), system = 1: every ratio of wave to dissipation speed in [0,1];
 * stages 0 = min(N+1, 4); dissipation CRKFR_DISS_* (D-CSX equals D2 for a
 * linear flux); points CRKFR_POINTS_*.  Returns -1 for bad arguments. */
double crkfr_fourier_cfl(int N, int stages, int system, int dissipation, int points, double tol);

/* Kernel path of a step (the results agree up to rounding order):
 *  CRKFR_PATH_SPLIT: the local cRK procedure, the x faces, the y faces, the
 *    update, one kernel each (face fluxes through HBM);
 *  CRKFR_PATH_FACE_UPDATE: the local procedure, then one
 *    kernel in which each element's lanes compute its 4 (N+1) face fluxes
 *    (every face computed by both neighbours, in the same arithmetic) and
 *    update it;
 *  CRKFR_PATH_TILE: for 2D Euler with N = 1 or 3, the limiter chain off and
 *    the D2 dissipation, one workgroup per tile of elements (N = 3: 8 x 4 in
 *    FP64, 8 x 8 in FP32 bulk; N = 1: 16 x 8, 16 x 16) runs the local
 *    procedure, the faces inside the tile and the whole update of the
 *    elements whose four neighbours lie in the tile out of LDS, then the
 *    faces on tile edges and the update of the tile-edge elements follow;
 *    other configurations take CRKFR_PATH_FACE_UPDATE;
 *  CRKFR_PATH_CHECKER: for 2D grids with every boundary periodic, even nx
 *    and ny, the limiter chain off, D2 and no source, the elements split
 *    like a checkerboard (colour 0: ex + ey even): the local procedure of
 *    colour 0 (its traces to HBM); the local procedure of colour 1, whose
 *    four neighbours are all colour 0, with each of its face fluxes computed
 *    once from its own traces and its neighbour's and stored, and its
 *    update, without partial update or traces of its own in HBM; the update
 *    of colour 0 from the stored face fluxes.  Other configurations take
 *    CRKFR_PATH_FACE_UPDATE.
 * Until crkfr_set_path or crkfr_autotune chooses one, a solver takes, with
 * the limiter chain off, the checkerboard step where it serves and the
 * face-update path elsewhere, and with the limiter chain on the split path
 * (the limited face flux would be computed by both neighbours).
 * crkfr_path_in_use returns the path the next step takes.  Errors: EINVAL,
 * ESTATE (the solver is a member of a live batch; batches take the face-update
 * path for groups whose members all have it, the split path otherwise). */
enum { CRKFR_PATH_SPLIT = 0, CRKFR_PATH_TILE = 1, CRKFR_PATH_FACE_UPDATE = 2, CRKFR_PATH_CHECKER = 3 };
int crkfr_set_path(crkfr_solver* s, int path);
int crkfr_path_in_use(const crkfr_solver* s);

/* Workgroup shape of the update kernels (the update of the split and
 * face-update paths, the colour-0 update of the checkerboard step) for
 * elements of 16 points (2D, N = 3): CRKFR_UPDATE_BLOCK, 16 elements in 256
 * lanes; CRKFR_UPDATE_WAVE, 4 elements in one wavefront.  Both give the
 * same results bit for bit; which is faster depends on the path, the
 * arithmetic and the limiter chain.  shape = -1 returns to the default rule:
 * one wavefront for the FP64 checkerboard step and for the FP64 step with
 * the limiter chain on the split path, 256 lanes otherwise.  Elements of other sizes keep their
 * workgroups (crkfr_update_shape_in_use returns CRKFR_UPDATE_BLOCK).
 * Errors: EINVAL (bad shape), ESTATE (the solver is a member of a live
 * batch; batches keep the 256-lane shape). */
enum { CRKFR_UPDATE_BLOCK = 0, CRKFR_UPDATE_WAVE = 1 };
int crkfr_set_update_shape(crkfr_solver* s, int shape);
int crkfr_update_shape_in_use(const crkfr_solver* s);

/* Kernel-path autotuner.  Times each path that serves the solver's
 * configuration (the tile-fused path only where it applies), for elements of
 * 16 points with both update workgroup shapes, over `steps` eagerly enqueued
 * steps from the current state after one warm-up step, keeps the fastest
 * (crkfr_set_path, crkfr_set_update_shape), and puts the state, the clock,
 * the time-step slots and the counters back as they were.  cache_path (may
 * be NULL) names a JSON-lines file: one object per tuned configuration,
 *   {"key": "eq=2 M=4 N=3 dtype=fp64 nx=512 ny=512 points=0 stages=4 diss=1
 *    central=0 blend=0 ind=0 flux=0 scale=0 src=0", "path": "face_update",
 *    "update_shape": "block", "ms_per_step": {"split": 0.37, "tile": 0.43,
 *    "face_update": 0.33}}
 * (the key holds N, M, the arithmetic, the grid and every option that selects
 * kernels); a configuration found there takes its stored path without timing
 * (from_cache = 1, ms all 0), a new one is timed and appended (the last entry
 * of a key wins).  Needs a state; allocates one state-sized device buffer
 * while it runs and synchronises the solver's stream.  Errors: EINVAL (bad
 * argument, cache file not writable), ESTATE (no state, batch member), EHIP. */
typedef struct {
    int path;          /* the path the next step takes (CRKFR_PATH_*) */
    int from_cache;    /* 1: read from the cache file, nothing timed */
    float ms[4];       /* ms per step of split, tile-fused, face-update, checkerboard (the faster
                          update shape); 0: not timed */
    int update_shape;  /* the update workgroup shape the next step takes (CRKFR_UPDATE_*) */
} crkfr_tune_result;
int crkfr_autotune(crkfr_solver* s, int steps, const char* cache_path, crkfr_tune_result* out);

/* Device time per kernel of the last step measured with HIP events (ms):
 * [0] local cRK, [1] x faces, [2] y faces, [3] update; with the tile-fused
 * step: [0] the tile kernel, [1], [2] the faces on tile edges, [3] the update
 * of the tile-edge elements; with the face-update path [1] and [2] are 0;
 * with the checkerboard step [0] the colour-0 local procedure, [1] the
 * colour-1 kernel (local procedure, faces, update), [2] 0, [3] the colour-0
 * update.
 * Needs timing = 1. */
int crkfr_set_timing(crkfr_solver* s, int on);
int crkfr_get_kernel_times(crkfr_solver* s, float* ms4);

/* ---- batches --------------------------------------------------------------
 * Many solvers advanced together: each step is one batched time-step kernel
 * (one workgroup per instance) and, per phase of the step and per group of
 * members with equal equation, degree, arithmetic and limiting, one launch of
 * persistent workgroups walking a table of (instance, block) work items.  The
 * solvers stay owned by the caller, must have a state, and must not be used
 * on their own while the batch runs; call crkfr_batch_sync before reading
 * their state.  Batches run the face-update path for groups whose members
 * all have it and the split path otherwise (no tile-fused path).  Members must outlive the batch; the batch keeps the options
 * each member had at creation.  Each member keeps its own time step (eq.
 * time.step.2d). */
typedef struct crkfr_batch crkfr_batch;
int crkfr_batch_create(crkfr_solver* const* solvers, int count, void* hip_stream, crkfr_batch** out);
void crkfr_batch_destroy(crkfr_batch* b);
/* one step of every member (enqueue only) */
int crkfr_batch_step(crkfr_batch* b);
/* steps, replaying a captured two-step HIP graph */
int crkfr_batch_advance(crkfr_batch* b, int steps);
int crkfr_batch_sync(crkfr_batch* b);
/* end time of every member: each member's last step is clipped to reach
 * t_end and later steps have dt = 0 (t_end <= 0: no end time, the default) */
int crkfr_batch_set_t_end(crkfr_batch* b, double t_end);
/* per-phase device times (ms) of the last batched step, all groups of a phase
 * together: [0] local, [1] x faces, [2] y faces, [3] update.  With timing on,
 * crkfr_batch_advance enqueues the steps one by one instead of the graph. */
int crkfr_batch_set_timing(crkfr_batch* b, int on);
int crkfr_batch_phase_times(crkfr_batch* b, float* ms4);
int crkfr_batch_num_groups(const crkfr_batch* b);
/* persistent workgroups of (group, phase 0..3: local, x faces, y faces,
 * update); set_to >= 0 sets it (0: one workgroup per work item); returns it */
int crkfr_batch_grid(crkfr_batch* b, int group, int phase, int set_to);
/* time each phase of each group for persistent grids of 0, 1, 2, 4, 8, 16
 * workgroups per compute unit and keep the fastest (state not advanced) */
int crkfr_batch_autotune(crkfr_batch* b, int reps);

/* ---- learned troubled-cell indicator ---------------------------------------
 * A network n_inputs -> hidden -> hidden -> 1 with tanh hidden layers and a
 * sigmoid output maps an element's features to its blending coefficient.
 * Features (n_inputs = N): with e_s the energy of the orthonormal Legendre
 * modes of the indicator quantity (rho p; ten-moment: rho (p11 + p22) / 2)
 * whose highest degree is s -- the energies the smoothness indicator of
 * Sec. 4 compares -- and r_s = e_s / (e_0 + ... + e_s) (0 if that sum is 0),
 * feature s - 1 = max(log10(max(r_s, 1e-12)) / 6 + 1, -1), in [-1, 1], s = 1..N.
 * In a step the output y gives alpha = 0 if y < alpha_min, else
 * min(y, alpha_max), followed by the same neighbour smoothing; an element
 * whose features leave the network's box [lo, hi] takes the smoothness
 * indicator's alpha instead (a fallback, counted in the diagnostics).
 * The network is trained on pairs (features, indicator alpha) that the
 * method produces (crkfr_features) by minimising the mean squared error with
 * Adam; training runs on the GPU.  Parameters, per layer: W[out][in]
 * row-major then b[out] (floats).  Calls are ordered on the network's stream
 * (NULL: a stream of its own); the data pointers x (rows x n_inputs floats),
 * t and y (rows floats) are device pointers owned by the caller. */
int crkfr_mlp_create(int n_inputs, int hidden, unsigned long long seed, void* hip_stream, crkfr_mlp** out);
void crkfr_mlp_destroy(crkfr_mlp* m);
/* number of network parameters (hidden 8, 16 or 32; n_inputs 1..4) */
int crkfr_mlp_num_params(const crkfr_mlp* m);
/* set / read the parameters (host or device buffer); setting resets Adam's moments */
int crkfr_mlp_set_params(crkfr_mlp* m, const float* params, int on_device);
int crkfr_mlp_get_params(crkfr_mlp* m, float* params, int on_device);
/* feature box (host arrays of n_inputs); default [-1, 1], i.e. no fallback */
int crkfr_mlp_set_box(crkfr_mlp* m, const float* lo, const float* hi);
int crkfr_mlp_get_box(crkfr_mlp* m, float* lo, float* hi);
/* box = [min - margin, max + margin] of the rows of x, per feature (synchronises) */
int crkfr_mlp_fit_box(crkfr_mlp* m, const float* x, int n, float margin);
/* y[r] = network(x[r]) for n rows (enqueue only) */
int crkfr_mlp_forward(crkfr_mlp* m, const float* x, int n, float* y);
/* mean squared error over n rows and its gradient w.r.t. the parameters
 * (host arrays; grad may be NULL); synchronises */
int crkfr_mlp_loss_grad(crkfr_mlp* m, const float* x, const float* t, int n, double* loss, float* grad);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) over consecutive minibatches of
 * `batch` rows (shuffle the rows beforehand), `epochs` passes; writes the
 * mean loss seen in each epoch to loss_per_epoch (host, may be NULL) */
int crkfr_mlp_train(crkfr_mlp* m, const float* x, const float* t, int n, int epochs, int batch, float lr,
                    float* loss_per_epoch);

/* ---- one step without device allocation ----------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  One FP64
 * step of size dt > 0 (the face-update path, D2 dissipation, EA central part,
 * min(N+1, 4) stages) from u_in to u_out, both caller-owned device buffers of
 * nvar*ny*nx*(N+1)^d doubles in the nodal layout above (distinct, u_in only
 * read).  lim may be NULL (limiter off); its indicator must be
 * CRKFR_IND_PAPER or CRKFR_IND_CONST.  Far-field ghost states are the
 * boundary traces of u_in; inflow boundaries are refused.  The step's
 * intermediate buffers (partial update, face traces, blending coefficients,
 * ghost states, counters) live in a device array of
 * CRKFR_STATIC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends; grids whose buffers exceed it are refused with EINVAL
 * (2D Euler N = 3 needs about 2.7 KB per element: some 24,000 elements).
 * No device memory is allocated or freed.  Enqueued on hip_stream (NULL: the
 * null stream), no synchronisation.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race. */
#define CRKFR_STATIC_SCRATCH_BYTES (64u << 20)
int crkfr_step_static(const crkfr_config* cfg, const crkfr_limiter_opts* lim, const double* u_in, double* u_out,
                      double dt, void* hip_stream);

const char* crkfr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
