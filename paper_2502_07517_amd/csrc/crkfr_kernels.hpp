// gfx950 kernels of one cRKFR step (Babbar & Chen, arXiv 2502.07517).
//
//   k_local   per element, one lane per solution point: the local cRK
//             procedure (eqs. crkfr, crk22/33/44, disc.avg.flux, time.avg.sol,
//             App. B source averages), EA face traces (eq. evaluate), the
//             volume part of the FR update with the extrapolated averaged flux
//             folded in (eq. crkfr.avg), and, with limiting, the smoothness
//             indicator and the MUSCL-Hancock subcell predictor (Sec. 4).
//   k_face    per face point: D2 time-averaged numerical flux (eqs.
//             numflux.general, D2), boundary ghosts (Sec. 3.3), blend with the
//             low-order face flux (eq. Fblend) and the flux limiter for
//             admissibility in means (Sec. 4.3), admissibility roots in FP64.
//   k_update  per element: correction-function part of the FR update, the
//             low-order subcell update (eq. low.order.update), the blend (eq.
//             blended.scheme), FP64 element means (eq. upmean), Zhang-Shu
//             scaling in FP64 and the wave-speed rate for the next time step
//             (eq. time.step.2d).
//
// Layouts (e = ey*nx + ex, k = q*(N+1) + p):
//   state      u[var][e][k]                        (MP32: FP64 means ubar[var][e] + FP32 deviations)
//   uHp        [var][e][k]   u^n + volume part of the FR update
//   traces x   trx[side][comp][e][q], side 0 = left face, 1 = right face
//   traces y   trY[side][comp][e][p], side 0 = bottom, 1 = top
//              comps: F_EA (M), U (M), sigma of u^n trace (1)
//                     + limiting: predicted subcell face value (M), adjacent interior subface flux (M)
//   face flux  Fx[var][ey][i = 0..nx][q], Gy[var][j = 0..ny][ex][p]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "crkfr_physics.hpp"

namespace crkfr {

constexpr int MAXND = 5;
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_FARFIELD = 2, BC_REFLECT = 3, BC_INFLOW = 4 };
enum { BLEND_OFF = 0, BLEND_FO = 1, BLEND_MH = 2 };
enum { IND_PAPER = 0, IND_CONST = 1, IND_GIVEN = 2, IND_LEARNED = 3 };
enum { DISS_D2 = 0, DISS_D1 = 1, DISS_DCSX = 2 };
enum { CENTRAL_EA = 0, CENTRAL_AE = 1 };
enum { D_TROUBLED = 0, D_FLUXLIM, D_LOBAD, D_SLOPELIM, D_FALLBACK, D_SCALED, D_MEANBAD, D_LFALLBACK,
       D_THFLUX, D_THSCALE, D_NCOUNT };

// learned indicator: network N -> H -> H -> 1 (tanh, tanh, sigmoid), H <= MLP_HMAX;
// width MLP_HFAST has an unrolled evaluation with one hidden unit per lane
constexpr int MLP_HMAX = 32;
constexpr int MLP_HFAST = 16;
__host__ __device__ constexpr int mlp_nparams(int nin, int H) { return H * nin + H + H * H + H + H + 1; }
// the wave-speed rate of eq. time.step.2d is max-reduced into RATE_SLOTS
// addresses (slot = workgroup index mod RATE_SLOTS) to spread the atomics
constexpr int RATE_SLOTS = 256;

template <class real>
struct RefTab {
    real D[MAXND][MAXND];
    real l0[MAXND], l1[MAXND], bR[MAXND], bL[MAXND], w[MAXND], xi[MAXND];
    real sub[MAXND + 1];
    real Pm[MAXND][MAXND];  // Pm[k][p]: orthonormal Legendre coefficient k of the nodal interpolant
    real rdm[MAXND], rdp[MAXND];   // 1 / distance to the previous / next solution point (across faces too)
    real ta[4], tb[4];      // cRK tableau: a_{i+1,i}, b_i
};

template <class real>
struct StepArgs {
    int nx, ny, ne;
    double dx, dy, x0, y0;
    int bc[4];
    const double* ubar;    // MP32 element means of the input state
    const real* u;         // FP64 nodal state / MP32 deviations
    double* ubar_out;
    real* u_out;
    real* uHp;
    real* trx;
    real* trY;
    real* Fx;
    real* Gy;
    real* dtS;             // dt * time-averaged source [var][e][k] (source runs)
    double* alpha_raw;     // per element, before neighbour smoothing
    double* alpha_out;     // per element, final
    const double* alpha_given;
    const real* ghost;     // far-field ghost states, xL [ny][nq][M] | xR | yB [nx][nd][M] | yT
    // time-dependent inflow data: [0] t_ref, [1] number of coefficients, then
    // coefficient k at 2 + k * (ghost size) in the far-field ghost layout
    const double* inflow;
    const double* tn_dev;  // t^n of the current step (written by the time-step kernel)
    const double* dt_dev;
    int blend, indicator, smooth, flux_limiter, scaling, C;
    double alpha_min, alpha_max, alpha_const;
    // admissibility margins: relative (flux limiter, subcell reconstruction)
    // and absolute (scaling limiter floor)
    double eps_rel, eps_abs;
    Phys phys;
    RefTab<real> R;
    double w64[MAXND];
    double iwdx[MAXND], iwdy[MAXND];   // 1 / (w_i dx), 1 / (w_i dy)
    double idx, idy;                   // 1 / dx, 1 / dy (correctly rounded, as on the device)
    unsigned long long* diag;
    unsigned long long* rate_bits;
    const float* mlp;      // learned indicator: parameters, then the feature box lo[N], hi[N]
    int mlp_hidden;
    double* alpha_judge;   // learned indicator: the smoothness indicator's alpha per element
    float* feat_out;       // k_features: learned-indicator features [e][N]
    double ind_T, ind_kT;  // indicator threshold T(N) = 0.5 10^(-1.8 (N+1)^(1/4)) and ln(9999) / T
    int stages;            // cRK stages (tableau in R.ta, R.tb)
    int dissipation;       // DISS_*: D2 (eq. D2), D1 (eq. D1), D-CSX (eq. dcsx)
    int central;           // CENTRAL_*: EA traces (eq. evaluate) or extrapolation (eq. extrapolate)
    // tile-fused step: the elements at the edges of the tiles (updated by the
    // update phase), null for the split step
    const int* edge_list;
    int n_edge;
};

// trace components per face point: F (M), U (M; u^n for D1), sigma (1),
// limiting: predicted subcell value (M), adjacent subface flux (M),
// D-CSX: the stage values u^(i) (stages x M) from TRACE_STAGES on
template <int M>
__host__ __device__ constexpr int trace_stage_offset() { return 4 * M + 1; }

template <int DIM, int N>
struct Geo {
    static constexpr int nd = N + 1, nq = DIM == 2 ? N + 1 : 1, np = nd * nq;
    // elements per workgroup: 256 lanes, except one wavefront for elements of
    // 3, 5 or 9 points (their sums go through LDS; a one-wavefront workgroup
    // makes the barriers local to the wavefront)
    static constexpr int EB = (np <= 16 && np != 2 && np != 4 && np != 16 ? 64 : (np == 25 ? 128 : 256)) / np;
    static constexpr int BLOCK = EB * np;
};

// k_local: one-wavefront workgroups while an element has at most 16 points
// (barriers then order a single wavefront), 256 lanes otherwise
template <int DIM, int N>
struct LGeo {
    static constexpr int nd = N + 1, nq = DIM == 2 ? N + 1 : 1, np = nd * nq;
    // (25-point elements: two wavefronts, five elements; fewer wavefronts
    // meet at each barrier than with 256 lanes: 4 % off the limited FP32
    // local phase)
    static constexpr int TPB = np <= 16 ? 64 : (np == 25 ? 128 : 256);
    static constexpr int EB = TPB / np;
    static constexpr int BLOCK = EB * np;
};

// the update's workgroup shape: WB = 0 the Geo workgroups, WB = 1 one
// wavefront per workgroup for elements of 16 points (which shape is faster
// depends on the path and the limiter chain; the autotuner times both)
template <int DIM, int N>
struct GeoW1 {
    static constexpr int nd = N + 1, nq = DIM == 2 ? N + 1 : 1, np = nd * nq;
    static constexpr int EB = np == 16 ? 4 : Geo<DIM, N>::EB;
    static constexpr int BLOCK = EB * np;
};
template <int DIM, int N, int WB>
using UGeo = std::conditional_t<WB == 1, GeoW1<DIM, N>, Geo<DIM, N>>;

// the np lanes of an element lie in one wavefront at a power-of-two offset
template <int np>
__device__ __forceinline__ constexpr bool elem_in_wave()
{
    return np == 2 || np == 4 || np == 8 || np == 16 || np == 32 || np == 64;
}

// lane exchange within DPP rows (16 lanes) or quads, as VALU moves: row_ror:n
// for 16-lane elements, quad permutations swapping lanes 1 and 2 apart for 2-
// and 4-lane elements
template <int CTRL>
__device__ __forceinline__ double dpp_double(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_float(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_ROW_ROR = 0x120;   // + n for row_ror:n
// the value of lane (i + S) mod 4 of lane i's quad (quad_perm [S, S+1, S+2, S+3] mod 4)
constexpr int dpp_quad_rot_ctrl(int S)
{
    return ((S + 0) & 3) | (((S + 1) & 3) << 2) | (((S + 2) & 3) << 4) | (((S + 3) & 3) << 6);
}
template <int S, class real>
__device__ __forceinline__ real dpp_quad_rot(real x)
{
    if constexpr (sizeof(real) == 8) return dpp_double<dpp_quad_rot_ctrl(S)>(x);
    else return dpp_float<dpp_quad_rot_ctrl(S)>(x);
}
// the value of lane (i - S) mod 16 of lane i's row (row_ror:S)
template <int S, class real>
__device__ __forceinline__ real dpp_row_ror(real x)
{
    if constexpr (sizeof(real) == 8) return dpp_double<DPP_ROW_ROR + S>(x);
    else return dpp_float<DPP_ROW_ROR + S>(x);
}

template <int np>
__device__ __forceinline__ constexpr bool elem_in_dpp() { return np == 2 || np == 4 || np == 16; }

// ordering of an element's LDS exchanges: when the element's lanes share one
// wavefront, a wavefront-scope fence (the wavefront's LDS accesses complete in
// issue order) instead of a workgroup barrier, so wavefronts without a
// troubled element do not wait for the others
template <int np>
__device__ __forceinline__ void elem_sync()
{
    if constexpr (elem_in_wave<np>()) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}
// whether any lane of the workgroup (elements across wavefronts) or of the
// wavefront (elements within one) has pred
template <int np>
__device__ __forceinline__ bool elem_any(bool pred)
{
    if constexpr (elem_in_wave<np>()) return __any(pred);
    else return __syncthreads_or(pred);
}

// sum, minimum or maximum over the element's lanes, every lane gets the same
// bits; np in {2, 4, 16}
enum { RED_SUM = 0, RED_MIN = 1, RED_MAX = 2 };
template <int np, int OP, class T>
__device__ __forceinline__ T dpp_elem_reduce(T x)
{
    auto op = [](T a, T b) { return OP == RED_MIN ? (b < a ? b : a) : (OP == RED_MAX ? (b > a ? b : a) : a + b); };
    auto mv = [](T y, auto ctrl) {
        if constexpr (sizeof(T) == 8) return dpp_double<decltype(ctrl)::value>(y);
        else return dpp_float<decltype(ctrl)::value>(y);
    };
    if constexpr (np == 16) {
        x = op(x, mv(x, std::integral_constant<int, DPP_ROW_ROR + 8>{}));
        x = op(x, mv(x, std::integral_constant<int, DPP_ROW_ROR + 4>{}));
        x = op(x, mv(x, std::integral_constant<int, DPP_ROW_ROR + 2>{}));
        x = op(x, mv(x, std::integral_constant<int, DPP_ROW_ROR + 1>{}));
    } else {
        x = op(x, mv(x, std::integral_constant<int, DPP_QUAD_XOR1>{}));
        if constexpr (np == 4) x = op(x, mv(x, std::integral_constant<int, DPP_QUAD_XOR2>{}));
    }
    return x;
}

// v_mfma_f64_4x4x4 computes four 4x4x4 products per wavefront: block b takes
// A[i][kk] from lane 16 kk + 4 b + i, B[kk][j] from lane 16 kk + 4 b + j and
// leaves D[i][j] = sum_kk A[i][kk] B[kk][j] + C[i][j] on lane 16 i + 4 b + j.
// A 16-node element (N = 3 in 2D) laid out as one block, node (p, q) on lane
// 16 q + 4 b + p, takes its y derivatives as one product with the derivative
// matrix (the contraction runs over q, the lane's 16-lane row), and its x
// derivatives as a product with the identity, which moves node (q, p)'s value
// to node (p, q)'s lane, then one with the derivative matrix.
__device__ __forceinline__ double mfma4(double a, double b, double c)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}
// element (within the workgroup) and node index of a lane in that layout
__device__ __forceinline__ void mfma_lane(int tid, int& le, int& k)
{
    const int l = tid & 63;
    le = 4 * (tid >> 6) + ((l >> 2) & 3);
    k = ((l >> 4) << 2) | (l & 3);
}
// sum or minimum over an element's lanes in that layout, pairing the nodes
// as dpp_elem_reduce<16> does (8 apart, 4 apart, 2 apart, 1 apart), so that
// both give the same bits
template <int OP>
__device__ __forceinline__ double mfma_elem_reduce(double x)
{
    auto op = [](double a, double b) { return OP == RED_MIN ? (b < a ? b : a) : (OP == RED_MAX ? (b > a ? b : a) : a + b); };
    x = op(x, __shfl_xor(x, 32, 64));
    x = op(x, __shfl_xor(x, 16, 64));
    x = op(x, dpp_double<DPP_QUAD_XOR2>(x));
    x = op(x, dpp_double<DPP_QUAD_XOR1>(x));
    return x;
}

// cRK tableaux of eqs. crk22, crk33, crk44: sub-diagonal a_{i+1,i} and weights b_i
__host__ __device__ constexpr double tab_a(int S, int i)
{
    return S == 2 ? 0.5 : (S == 3 ? (i == 0 ? 1.0 / 3.0 : 2.0 / 3.0) : (i == 2 ? 1.0 : 0.5));
}
__host__ __device__ constexpr double tab_b(int S, int i)
{
    return S == 2 ? (i == 0 ? 0.0 : 1.0)
         : S == 3 ? (i == 0 ? 0.25 : (i == 1 ? 0.0 : 0.75))
                  : ((i == 0 || i == 3) ? 1.0 / 6.0 : 1.0 / 3.0);
}

template <class real>
__device__ __forceinline__ constexpr bool is_mp() { return sizeof(real) == 4; }

// LDS layouts of an element's nodal values: node-major (value v of node k at
// k M + v), or split into 16-byte planes (value v of node k at
// ((v / W) np + k) W + v % W, W values per 16 bytes).  With planes a wide
// access reads one plane of one node, and the np <= 16 nodes of an element
// sit in distinct 16-byte bank groups: writes of every node, derivative
// reads along a row or a column and trace reads are free of bank conflicts.
template <int M, int np>
struct NodeMajor {
    static constexpr int SIZE = np * M;
    __host__ __device__ static constexpr int at(int k, int v) { return k * M + v; }
};
template <class real, int M, int np>
struct Planes {
    static constexpr int W = 16 / (int)sizeof(real), NPL = (M + W - 1) / W, SIZE = NPL * np * W;
    __host__ __device__ static constexpr int at(int k, int v) { return ((v / W) * np + k) * W + v % W; }
};

// ----------------------------------------------------------------------------
// state access
// ----------------------------------------------------------------------------
template <class Eq, class real>
__device__ __forceinline__ void load_node(const StepArgs<real>& a, int np, int e, int k, real* u)
{
    // one 64-bit address per array; the variables lie whole planes apart
    const real* const un = a.u + (size_t)e * np + k;
    const size_t vs = (size_t)a.ne * np;
#pragma unroll
    for (int v = 0; v < Eq::M; ++v) {
        if constexpr (is_mp<real>())
            u[v] = (real)(a.ubar[(size_t)v * a.ne + e] + (double)un[v * vs]);
        else
            u[v] = un[v * vs];
    }
}

// neighbour element across a face (dir 0: x, 1: y; side 0: low, 1: high), -1 at a non-periodic boundary
template <class real>
__device__ __forceinline__ int nbr(const StepArgs<real>& a, int ex, int ey, int dir, int side)
{
    if (dir == 0) {
        int t = ex + (side ? 1 : -1);
        if (t < 0) { if (a.bc[0] != BC_PERIODIC) return -1; t = a.nx - 1; }
        if (t >= a.nx) { if (a.bc[1] != BC_PERIODIC) return -1; t = 0; }
        return ey * a.nx + t;
    }
    int t = ey + (side ? 1 : -1);
    if (t < 0) { if (a.bc[2] != BC_PERIODIC) return -1; t = a.ny - 1; }
    if (t >= a.ny) { if (a.bc[3] != BC_PERIODIC) return -1; t = 0; }
    return t * a.nx + ex;
}

// far-field ghost state at point t of the boundary face of element (ex, ey); null otherwise
template <class real>
__device__ __forceinline__ const real* ghost_at(const StepArgs<real>& a, int M, int nd, int nq,
                                                int ex, int ey, int dir, int side, int t)
{
    if (a.bc[dir * 2 + side] != BC_FARFIELD) return nullptr;
    size_t xsz = (size_t)a.ny * nq * M, ysz = (size_t)a.nx * nd * M;
    if (dir == 0) return a.ghost + side * xsz + ((size_t)ey * nq + t) * M;
    return a.ghost + 2 * xsz + side * ysz + ((size_t)ex * nd + t) * M;
}

// time-dependent inflow (Sec. 3.3): the boundary data g(tau) at a boundary
// face point, from its polynomial in tau - t_ref (Horner's rule in FP64)
template <class real>
__device__ __forceinline__ bool inflow_at(const StepArgs<real>& a, int M, int nd, int nq, int dim, int ex, int ey,
                                          int dir, int side, int t, double tau, real* out)
{
    if (a.bc[dir * 2 + side] != BC_INFLOW) return false;
    const size_t xsz = (size_t)a.ny * nq * M, ysz = (size_t)a.nx * nd * M;
    const size_t gsz = 2 * xsz + (dim == 2 ? 2 * ysz : 0);
    const size_t off = dir == 0 ? side * xsz + ((size_t)ey * nq + t) * M
                                : 2 * xsz + side * ysz + ((size_t)ex * nd + t) * M;
    const double s = tau - a.inflow[0];
    const double ncd = a.inflow[1];
    const int nc = ncd >= 1.0 && ncd <= 5.0 ? (int)ncd : 0;   // at most the coefficients the buffer holds
    const double* cf = a.inflow + 2 + off;
    for (int v = 0; v < M; ++v) {
        double val = 0.0;
        for (int k = nc - 1; k >= 0; --k) val = val * s + cf[(size_t)k * gsz + v];
        out[v] = (real)val;
    }
    return true;
}

// smallest / largest eigenvalue of the normal flux Jacobian (fully inflow
// faces: every wave enters the domain)
template <class Eq, class real>
__device__ __forceinline__ real eig_extreme(int d, const real* u, bool largest, const Phys& P)
{
    if constexpr (Eq::ID == 0) return (real)P.adv;
    else if constexpr (Eq::ID == 4) return u[0];
    else {
        const real vn = u[1 + d] / u[0];
        const real c = (d == 0 ? Eq::sx(u, P) : Eq::sy(u, P)) - fabs(vn);
        return largest ? vn + c : vn - c;
    }
}

// solid wall normal to direction dir (Sec. 3.3, eq. reflect.time.avg): the
// ghost mirrors the interior state, flipping the normal momentum (and the
// ten-moment E12); the mirrored normal flux is -(mirror of the flux)
template <class real>
__device__ __forceinline__ bool is_wall(const StepArgs<real>& a, int dir, int side)
{
    return a.bc[dir * 2 + side] == BC_REFLECT;
}

template <class Eq>
__device__ __forceinline__ constexpr bool mirror_flips(int dir, int v)
{
    return v == 1 + dir || (Eq::K == 3 && v == 4);   // ten-moment: E12 flips too
}

// ----------------------------------------------------------------------------
// admissibility helpers (FP64)
// ----------------------------------------------------------------------------
template <class Eq>
__device__ double bisect_root(int k, const double* a, const double* b, double eps, const Phys& P)
{
    double lo = 0.0, hi = 1.0, z[Eq::M];
    for (int it = 0; it < 60; ++it) {
        double mid = 0.5 * (lo + hi);
#pragma unroll
        for (int v = 0; v < Eq::M; ++v) z[v] = a[v] + mid * (b[v] - a[v]);
        if (Eq::adm(k, z, P) >= eps) lo = mid; else hi = mid;
    }
    return lo;
}

// fraction of the segment a -> b keeping P_k >= eps, given Pa = P_k(a):
// concavity bound, else bisection
template <class Eq>
__device__ double segment_fraction(int k, const double* a, double Pa, const double* b, double eps, const Phys& P)
{
    if (Eq::adm_ge(k, b, eps, P)) return 1.0;
    const double Pb = Eq::adm(k, b, P);
    if (Pb >= eps) return 1.0;
    if (Eq::concave(k)) {
        double t = (Pa - eps) / (Pa - Pb);
        return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    }
    return bisect_root<Eq>(k, a, b, eps, P);
}

template <class Eq>
__device__ bool admissible_eps(const double* u, const double* eps, const Phys& P)
{
#pragma unroll
    for (int k = 0; k < Eq::K; ++k)
        if (!Eq::adm_ge(k, u, eps[k], P)) return false;
    return true;
}

template <class Eq, class real>
__device__ __forceinline__ void flux_dir(int d, const real* u, real* f, const Phys& P)
{
    if (d == 0) Eq::fx(u, f, P); else Eq::gy(u, f, P);
}

template <class Eq, class real>
__device__ __forceinline__ void rusanov(int d, const real* a, const real* b, real* out, const Phys& P)
{
    real fa[Eq::M], fb[Eq::M];
    flux_dir<Eq>(d, a, fa, P);
    flux_dir<Eq>(d, b, fb, P);
    real la = d == 0 ? Eq::sx(a, P) : Eq::sy(a, P);
    real lb = d == 0 ? Eq::sx(b, P) : Eq::sy(b, P);
    real lam = fmax(la, lb);
#pragma unroll
    for (int v = 0; v < Eq::M; ++v) out[v] = (real)0.5 * (fa[v] + fb[v]) - (real)0.5 * lam * (b[v] - a[v]);
}

// Rusanov flux normal to a direction that may differ between the lanes of a
// wavefront: branch-free where the system provides fn / sn, else rusanov()
template <class Eq, class = void>
struct has_normal_flux : std::false_type {};
template <class Eq>
struct has_normal_flux<Eq, std::void_t<decltype(&Eq::fn)>> : std::true_type {};

template <class Eq, class real>
__device__ __forceinline__ void rusanov_n(int d, const real* a, const real* b, real* out, const Phys& P)
{
    if constexpr (has_normal_flux<Eq>::value) {
        real fa[Eq::M], fb[Eq::M];
        Eq::fn(d, a, fa, P);
        Eq::fn(d, b, fb, P);
        real lam = fmax(Eq::sn(d, a, P), Eq::sn(d, b, P));
#pragma unroll
        for (int v = 0; v < Eq::M; ++v) out[v] = (real)0.5 * (fa[v] + fb[v]) - (real)0.5 * lam * (b[v] - a[v]);
    } else {
        rusanov<Eq>(d, a, b, out, P);
    }
}

__device__ __forceinline__ void atomic_min_pos(unsigned long long* p, double v)
{
    atomicMin(p, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ void atomic_max_pos(unsigned long long* p, double v)
{
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// ----------------------------------------------------------------------------
// MUSCL-Hancock predictor of one subcell (Sec. 4.2; reading: minmod slopes
// on the non-uniform subcell grid, slope scaled to keep the reconstructed
// face values admissible, Hancock half step, zero slope when the predicted
// values are not admissible).  The element's nodal values are in sh[k][v].
// Outputs the predicted values at the x faces (xm, xp) and y faces (ym, yp).
// ----------------------------------------------------------------------------
template <class Eq, int N, class L, class real>
__device__ void mh_subcell(const StepArgs<real>& a, int ex, int ey, int p, int q,
                           const real* u, const real* sh, double dt,
                           real* xm, real* xp, real* ym, real* yp, int& nlim, int& nfb)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int M = Eq::M, nd = G::nd, nq = G::nq, np = G::np, K = Eq::K;
    const Phys& P = a.phys;
    const int k = q * nd + p;
    real sx[M], sy[M];
#pragma unroll
    for (int v = 0; v < M; ++v) { sx[v] = 0; sy[v] = 0; }
    double ud[M], eps[K > 0 ? K : 1], Pu[K > 0 ? K : 1];
#pragma unroll
    for (int v = 0; v < M; ++v) ud[v] = (double)u[v];
    bool u_ok = true;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
        Pu[kk] = Eq::adm(kk, ud, P);
        eps[kk] = a.eps_rel * Pu[kk];
        if (!(eps[kk] > 0.0)) u_ok = false;
    }
    const bool mh = a.blend == BLEND_MH && u_ok;
    if (mh) {
#pragma unroll
        for (int d = 0; d < Eq::DIM; ++d) {
            const int pos = d == 0 ? p : q;
            real um[M], up[M];
            if (pos > 0) {
                const int kn = d == 0 ? k - 1 : k - nd;
#pragma unroll
                for (int v = 0; v < M; ++v) um[v] = sh[L::at(kn, v)];
            } else {
                int en = nbr(a, ex, ey, d, 0);
                if (en >= 0) {
                    load_node<Eq>(a, np, en, d == 0 ? q * nd + N : N * nd + p, um);
                } else {
                    const real* g = ghost_at(a, M, nd, nq, ex, ey, d, 0, d == 0 ? q : p);
                    if (g) {
#pragma unroll
                        for (int v = 0; v < M; ++v) um[v] = g[v];
                    } else if (inflow_at(a, M, nd, nq, Eq::DIM, ex, ey, d, 0, d == 0 ? q : p, *a.tn_dev, um)) {
                    } else if (is_wall(a, d, 0)) {
#pragma unroll
                        for (int v = 0; v < M; ++v) um[v] = mirror_flips<Eq>(d, v) ? -u[v] : u[v];
                    } else {
#pragma unroll
                        for (int v = 0; v < M; ++v) um[v] = u[v];
                    }
                }
            }
            if (pos < N) {
                const int kn = d == 0 ? k + 1 : k + nd;
#pragma unroll
                for (int v = 0; v < M; ++v) up[v] = sh[L::at(kn, v)];
            } else {
                int en = nbr(a, ex, ey, d, 1);
                if (en >= 0) {
                    load_node<Eq>(a, np, en, d == 0 ? q * nd + 0 : 0 * nd + p, up);
                } else {
                    const real* g = ghost_at(a, M, nd, nq, ex, ey, d, 1, d == 0 ? q : p);
                    if (g) {
#pragma unroll
                        for (int v = 0; v < M; ++v) up[v] = g[v];
                    } else if (inflow_at(a, M, nd, nq, Eq::DIM, ex, ey, d, 1, d == 0 ? q : p, *a.tn_dev, up)) {
                    } else if (is_wall(a, d, 1)) {
#pragma unroll
                        for (int v = 0; v < M; ++v) up[v] = mirror_flips<Eq>(d, v) ? -u[v] : u[v];
                    } else {
#pragma unroll
                        for (int v = 0; v < M; ++v) up[v] = u[v];
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < M; ++v) {
                real s1 = (u[v] - um[v]) * a.R.rdm[pos], s2 = (up[v] - u[v]) * a.R.rdp[pos];
                real s = s1 * s2 <= 0 ? (real)0 : (fabs(s1) < fabs(s2) ? s1 : s2);
                if (d == 0) sx[v] = s; else sy[v] = s;
            }
        }
    }
    const real hxm = a.R.sub[p] - a.R.xi[p], hxp = a.R.sub[p + 1] - a.R.xi[p];
    const real hym = Eq::DIM == 2 ? a.R.sub[q] - a.R.xi[q] : (real)0;
    const real hyp = Eq::DIM == 2 ? a.R.sub[q + 1] - a.R.xi[q] : (real)0;
    constexpr int NF = Eq::DIM == 2 ? 4 : 2;
    if (mh) {
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
            double th = 1.0;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                double fv[M];
#pragma unroll
                for (int v = 0; v < M; ++v) {
                    real s = f < 2 ? sx[v] : sy[v];
                    real h = f == 0 ? hxm : (f == 1 ? hxp : (f == 2 ? hym : hyp));
                    fv[v] = (double)(u[v] + s * h);
                }
                double t = segment_fraction<Eq>(kk, ud, Pu[kk], fv, eps[kk], P);
                th = t < th ? t : th;
            }
            if (th < 1.0) {
                ++nlim;
#pragma unroll
                for (int v = 0; v < M; ++v) { sx[v] = (real)(th * (double)sx[v]); sy[v] = (real)(th * (double)sy[v]); }
            }
        }
    }
    real fv0[M], fv1[M], fv2[M], fv3[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
        fv0[v] = u[v] + sx[v] * hxm;
        fv1[v] = u[v] + sx[v] * hxp;
        fv2[v] = u[v] + sy[v] * hym;
        fv3[v] = u[v] + sy[v] * hyp;
    }
    // Hancock half-step predictor
    real fa[M], fb[M], delta[M];
    Eq::fx(fv0, fa, P);
    Eq::fx(fv1, fb, P);
    const real hdt = (real)(0.5 * dt);
    const real cx = hdt / (a.R.w[p] * (real)a.dx);
#pragma unroll
    for (int v = 0; v < M; ++v) delta[v] = -cx * (fb[v] - fa[v]);
    if constexpr (Eq::DIM == 2) {
        Eq::gy(fv2, fa, P);
        Eq::gy(fv3, fb, P);
        const real cy = hdt / (a.R.w[q] * (real)a.dy);
#pragma unroll
        for (int v = 0; v < M; ++v) delta[v] -= cy * (fb[v] - fa[v]);
    }
#pragma unroll
    for (int v = 0; v < M; ++v) {
        xm[v] = fv0[v] + delta[v];
        xp[v] = fv1[v] + delta[v];
        ym[v] = Eq::DIM == 2 ? fv2[v] + delta[v] : u[v];
        yp[v] = Eq::DIM == 2 ? fv3[v] + delta[v] : u[v];
    }
    bool ok = true;
    if constexpr (K > 0) {
        double ev[M];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int v = 0; v < M; ++v)
                ev[v] = (double)(f == 0 ? xm[v] : (f == 1 ? xp[v] : (f == 2 ? ym[v] : yp[v])));
            if (!admissible_eps<Eq>(ev, eps, P)) ok = false;
        }
    }
    if (!ok) {
        ++nfb;
#pragma unroll
        for (int v = 0; v < M; ++v) { xm[v] = u[v]; xp[v] = u[v]; ym[v] = u[v]; yp[v] = u[v]; }
    }
}

// ----------------------------------------------------------------------------
// smoothness indicator (reading of the Hennemann indicator, Sec. 4) and the
// learned indicator's features
// ----------------------------------------------------------------------------
// orthonormal Legendre coefficient (p, q) of the interpolant of the element's
// indicator quantity eps[k * stride] (projection table Pm: GL quadrature for
// GL points, the inverse Vandermonde matrix for GLL points)
template <int DIM, int N, class real>
__device__ __forceinline__ real modal_coeff(const RefTab<real>& R, int p, int q, const real* eps, int stride,
                                            int rstride)
{
    constexpr int nd = N + 1;
    real m = 0;
    if constexpr (DIM == 2) {
#pragma unroll
        for (int s2 = 0; s2 < nd; ++s2)
#pragma unroll
            for (int r = 0; r < nd; ++r)
                m += R.Pm[p][r] * R.Pm[q][s2] * eps[s2 * rstride + r * stride];
    } else {
#pragma unroll
        for (int r = 0; r < nd; ++r) m += R.Pm[p][r] * eps[r * stride];
    }
    return m;
}

// shell energies en[s] = sum of squared coefficients whose highest degree is s
// (the indicator's arithmetic runs in the step's precision)
template <int DIM, int N, class real>
__device__ __forceinline__ void shell_energies(const real* m2, int stride, int rstride, real* en)
{
    constexpr int nd = N + 1, np = DIM == 2 ? nd * nd : nd;
#pragma unroll
    for (int s2 = 0; s2 < nd; ++s2) en[s2] = 0;
#pragma unroll
    for (int kk = 0; kk < np; ++kk) {
        int pp = kk % nd, qq = kk / nd;
        en[pp > qq ? pp : qq] += m2[qq * rstride + pp * stride];
    }
}

// alpha of the smoothness indicator: logistic of the energy ratio E around
// the threshold T(N) with slope kT = ln(9999) / T, clipped to
// [alpha_min, alpha_max] (0 below alpha_min)
template <int N, class real>
__device__ __forceinline__ double indicator_alpha(const real* en, double amin, double amax, double T, double kT)
{
    real totN = 0, totNm1 = 0;
#pragma unroll
    for (int s2 = 0; s2 <= N; ++s2) totN += en[s2];
#pragma unroll
    for (int s2 = 0; s2 < N; ++s2) totNm1 += en[s2];
    const real E1 = totN > 0 ? en[N] / totN : (real)0;
    const real E2 = totNm1 > 0 ? en[N - 1] / totNm1 : (real)0;
    const real E = E1 > E2 ? E1 : E2;
    double al = (double)((real)1 / ((real)1 + exp(-(real)kT * (E - (real)T))));
    if (al < amin) al = 0.0;
    if (al > amax) al = amax;
    return al;
}

// features of the learned indicator: for shells s = 1..N the share r_s of
// shell s in the energy of shells 0..s, as log10(max(r_s, 1e-12)) / 6 + 1
// (at least -1)
// feature of shell s from its energy and the cumulative energy of shells 0..s
template <class real>
__device__ __forceinline__ real learned_feature(real es, real cum)
{
    const real r = cum > 0 ? es / cum : (real)0;
    // floor exactly -1, so a box edge at -1 is decided the same everywhere
    return r > (real)1e-12 ? fmax(log10(r) / (real)6 + (real)1, (real)-1) : (real)-1;
}
template <int N, class real>
__device__ __forceinline__ void learned_features(const real* en, real* ft)
{
    real cum = en[0];
#pragma unroll
    for (int s2 = 1; s2 <= N; ++s2) {
        cum += en[s2];
        ft[s2 - 1] = learned_feature(en[s2], cum);
    }
}

// activations of the learned indicator's network: the library functions in
// FP64 steps; in FP32-bulk steps tanh x = 1 - 2 / (1 + e^(2x)) and the
// logistic function from the hardware exponential and reciprocal (exact limits
// at +-infinity, absolute error about 1e-7)
template <class real>
__device__ __forceinline__ real act_tanh(real x)
{
    if constexpr (sizeof(real) == 4) return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * x));
    else return tanh(x);
}
template <class real>
__device__ __forceinline__ real act_sigmoid(real x)
{
    if constexpr (sizeof(real) == 4) return __builtin_amdgcn_rcpf(1.0f + __expf(-x));
    else return (real)1 / ((real)1 + exp(-x));
}

// ----------------------------------------------------------------------------
// k_local
// ----------------------------------------------------------------------------
// LDS reals per element in the tile-fused step: the stage arrays u, f, g in
// 16-byte planes, then the 4 (N+1) face points x (2M + 1) trace components
template <class Eq, int N, class real>
__host__ __device__ constexpr int elem_region()
{
    constexpr int nd = N + 1, np = Eq::DIM == 2 ? nd * nd : nd;
    using L = Planes<real, Eq::M, np>;
    constexpr int stage = 2 * L::SIZE + (Eq::DIM == 2 ? L::SIZE : np);
    constexpr int traces = (Eq::DIM == 2 ? 4 * nd : 2) * (2 * Eq::M + 1);
    return stage > traces ? stage : traces;
}
// component c of the face traces of element e at position t of side sd
// (0 left, 1 right, 2 bottom, 3 top): the x faces' array for sides 0, 1, the
// y faces' for 2, 3; components of one array lie trace_stride apart
// (x and y faces of a 2D element carry N + 1 points each; 1D: one x point)
template <class Eq, int N, class real>
__device__ __forceinline__ size_t trace_stride(const StepArgs<real>& a)
{
    return (size_t)a.ne * (Eq::DIM == 2 ? N + 1 : 1);
}
template <class Eq, int N, class real>
__device__ __forceinline__ real* trace_at(const StepArgs<real>& a, int sd, int c, int e, int t)
{
    constexpr int npt = Eq::DIM == 2 ? N + 1 : 1;
    return (sd < 2 ? a.trx : a.trY) + (size_t)c * trace_stride<Eq, N>(a) + (size_t)e * npt + t;
}
// checkerboard step: element of index i among those of colour c (0: ex + ey
// even, 1: odd) of a grid with an even number of columns (row-major, nx / 2
// elements of each colour per row)
__device__ __forceinline__ int cb_element(int i, int c, int nx)
{
    const int h = nx >> 1;
    const int ey = (int)((unsigned)i / (unsigned)h), j = i - ey * h;
    return ey * nx + 2 * j + ((ey + c) & 1);
}
// and the index of element (ex, ey) among those of its colour
__device__ __forceinline__ int cb_index(int ex, int ey, int nx) { return ey * (nx >> 1) + (ex >> 1); }

template <class Eq, int N, class real, int EB, bool MFL = false>
__device__ __forceinline__ void update_finish(const StepArgs<real>& a, int e, int le, int k, bool act,
                                              const real* unew, const real* FL, const real* FR, const real* GB,
                                              const real* GT, const real* dts, int vblock);

// TG = void: the split step (LGeo blocks of elements; uHp and the face traces
// to HBM).  TG = a tile geometry: one tile of TX x TY elements per workgroup
// (the tile-fused step); the element's stage arrays lie in tile_buf, uHp goes
// to uhp_out (registers), the face traces to the element's part of tile_buf
// and, for faces on the tile's edge, to HBM as well.
// CB (checkerboard step, periodic 2D grids of even sides, limiter off, D2):
// 1 the elements of colour 0 (ex + ey even), as the split step; 2 the
// elements of colour 1, whose four neighbours all have colour 0 and have
// written their traces: each lane computes the flux of its face point from
// its own traces (registers) and the neighbour's (HBM), stores it for the
// colour-0 update, and the element is updated in place (no uHp, no traces
// of its own in HBM).
template <class Eq, int N, class real, bool LIM, class TG = void, int CB = 0>
__device__ void local_body(const StepArgs<real>& a, int vblock, real* tile_buf = nullptr, real* uhp_out = nullptr)
{
    constexpr bool TILE = !std::is_void<TG>::value;
    static_assert(!(TILE && LIM), "the tile-fused step has no limiter chain");
    static_assert(!(CB && (LIM || TILE || Eq::DIM != 2)), "the checkerboard step: 2D, limiter off");
    using G = std::conditional_t<TILE, TG, LGeo<Eq::DIM, N>>;
    constexpr int M = Eq::M, DIM = Eq::DIM, nd = G::nd, nq = G::nq, np = G::np, EB = G::EB;
    const int S = a.stages;
    constexpr int MY = DIM == 2 ? M : 1;
    // element arrays in 16-byte planes (L::at(node, v)); the y fluxes (2D)
    // likewise, one value per node in 1D
    using L = Planes<real, M, np>;
    constexpr int PW = L::W;
    constexpr int GS = DIM == 2 ? PW : 1;     // node stride of value 0 in sh_g
    // one region of SB reals per element: the stage arrays u, f, g (in the
    // tile-fused step then the element's face traces)
    constexpr int SB = TILE ? elem_region<Eq, N, real>() : 2 * L::SIZE + (DIM == 2 ? L::SIZE : np);
    // face values of the final part; before it, the predicted yp of the subcells
    constexpr int HW = 4 * nd > np ? 4 * nd : np;
    __shared__ real sh_h[EB][M][HW];

    const Phys& P = a.phys;
    // 16-point FP64 elements take their derivatives on the matrix cores, their
    // nodes laid out as the blocks of v_mfma_f64_4x4x4 (mfma4)
    constexpr bool MFD = DIM == 2 && np == 16 && sizeof(real) == 8 && !TILE;
    int le, k;
    if constexpr (MFD) {
        mfma_lane(threadIdx.x, le, k);
    } else {
        le = threadIdx.x / np;
        k = threadIdx.x - le * np;
    }
    const int p = k % nd, q = k / nd;
    auto at = [](int kk, int v) { return L::at(kk, v); };
    real* su;
    if constexpr (TILE) {
        su = tile_buf + le * SB;
    } else {
        __shared__ real sh_buf[EB][SB];
        su = &sh_buf[le][0];
    }
    real* const sf = su + L::SIZE;
    real* const sg = su + 2 * L::SIZE;
    int ex, ey, e, tix = 0, tiy = 0;
    bool act;
    if constexpr (TILE) {
        const int ntx = (a.nx + G::TX - 1) / G::TX;
        tix = le % G::TX;
        tiy = le / G::TX;
        const int gx = (vblock % ntx) * G::TX + tix, gy = (vblock / ntx) * G::TY + tiy;
        act = gx < a.nx && gy < a.ny;
        ex = gx < a.nx ? gx : a.nx - 1;
        ey = gy < a.ny ? gy : a.ny - 1;
        e = ey * a.nx + ex;
    } else if constexpr (CB != 0) {
        const int i = vblock * EB + le, nc = a.ne >> 1;
        act = i < nc;
        e = cb_element(act ? i : nc - 1, CB - 1, a.nx);
        ey = (int)((unsigned)e / (unsigned)a.nx);
        ex = e - ey * a.nx;
    } else {
        const int e0 = vblock * EB + le;
        act = e0 < a.ne;
        e = act ? e0 : a.ne - 1;
        ey = (int)((unsigned)e / (unsigned)a.nx);
        ex = e - ey * a.nx;
    }
    const double dt = *a.dt_dev;
    const real rdt = (real)dt, idx = (real)a.idx, idy = (real)a.idy;
    const real xn = (real)(a.x0 + ((double)ex + (double)a.R.xi[p]) * a.dx);
    const real yn = DIM == 2 ? (real)(a.y0 + ((double)ey + (double)a.R.xi[q]) * a.dy) : (real)0;
    const bool src = Eq::K == 3 && P.source;          // ten-moment systems carry the source
    const int C = a.C;
    const size_t nes = (size_t)a.ne;

    real un[M];
    load_node<Eq>(a, np, e, k, un);

    if constexpr (LIM) {
        // ---- smoothness indicator (reading of the Hennemann indicator) or
        //      the learned indicator over the same modal energies ----
        __shared__ real sh_m[EB][2][MLP_HMAX];
#pragma unroll
        for (int v = 0; v < M; ++v) su[at(k, v)] = un[v];
        const bool modal = a.indicator == IND_PAPER || a.indicator == IND_LEARNED;
        if (modal) sf[at(k, 0)] = Eq::ind(un, P);
        elem_sync<np>();
        if (modal) {
            real m = modal_coeff<DIM, N>(a.R, p, q, sf, PW, nd * PW);
            sg[k * GS] = m * m;
        }
        elem_sync<np>();
        double al_ind = 0.0;
        bool inbox = true;
        if (modal) {
            // every lane sums the shell energies in the same order (same bits);
            // lane 0 forms the indicator's alpha, lanes 1..N the learned
            // indicator's features (feature s on lane s)
            real en[nd];
            shell_energies<DIM, N>(sg, GS, nd * GS, en);
            if (k == 0 && act) {
                al_ind = indicator_alpha<N>(en, a.alpha_min, a.alpha_max, a.ind_T, a.ind_kT);
                if (a.indicator == IND_PAPER) a.alpha_raw[e] = al_ind;
                else a.alpha_judge[e] = al_ind;
            }
            if (a.indicator == IND_LEARNED && k >= 1 && k <= N) {
                real cum = en[0], es = 0, cs = 0;
#pragma unroll
                for (int s2 = 1; s2 <= N; ++s2) {
                    cum += en[s2];
                    if (s2 == k) { es = en[s2]; cs = cum; }
                }
                sf[at(k - 1, 0)] = learned_feature(es, cs);
            }
        } else if (k == 0 && act) {
            if (a.indicator == IND_CONST) a.alpha_raw[e] = a.alpha_const;
            else if (a.indicator == IND_GIVEN) a.alpha_raw[e] = a.alpha_given[e];
        }
        if (a.indicator == IND_LEARNED) {
            // the network: hidden units spread over the element's lanes
            elem_sync<np>();
            if (k == 0) {
                // the features inside the training box, else the indicator decides
                const float* box = a.mlp + mlp_nparams(N, a.mlp_hidden);
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const real ft = sf[at(j, 0)];
                    if (!(ft >= (double)box[j] && ft <= (double)box[N + j])) inbox = false;
                }
                if (act && !inbox) atomicAdd(&a.diag[D_LFALLBACK], 1ull);
            }
            const int H = a.mlp_hidden;
            const float* W1 = a.mlp;
            const float* b1 = W1 + H * N;
            const float* W2 = b1 + H;
            const float* b2 = W2 + H * H;
            const float* w3 = b2 + H;
            real out = 0;                     // output layer's sum, valid on lane 0
            if (np >= MLP_HFAST && H == MLP_HFAST) {
                // one unit per lane; the unit's rows of W2 as 16-byte loads
                // (W2 starts H (N + 1) floats into a 256-byte aligned buffer)
                const int j = k < H ? k : H - 1;
                const float4* row = reinterpret_cast<const float4*>(W2 + j * MLP_HFAST);
                float4 w2r[MLP_HFAST / 4];
#pragma unroll
                for (int c = 0; c < MLP_HFAST / 4; ++c) w2r[c] = row[c];
                real s = (real)b1[j];
#pragma unroll
                for (int i = 0; i < N; ++i) s += (real)W1[j * N + i] * sf[at(i, 0)];
                if (k < H) sh_m[le][0][k] = act_tanh(s);
                elem_sync<np>();
                real s2 = (real)b2[j];
#pragma unroll
                for (int c = 0; c < MLP_HFAST / 4; ++c) {
                    s2 += (real)w2r[c].x * sh_m[le][0][4 * c];
                    s2 += (real)w2r[c].y * sh_m[le][0][4 * c + 1];
                    s2 += (real)w2r[c].z * sh_m[le][0][4 * c + 2];
                    s2 += (real)w2r[c].w * sh_m[le][0][4 * c + 3];
                }
                const real h2 = k < H ? act_tanh(s2) : (real)0;
                if constexpr (np == MLP_HFAST && elem_in_dpp<np>() && is_mp<real>()) {
                    // FP32 bulk: sum of w3_j h2_j over the element's lanes
                    // (FP64 steps keep the sequential order of the general path)
                    out = dpp_elem_reduce<np, RED_SUM>((real)w3[j] * h2) + (real)w3[H];
                } else {
                    if (k < H) sh_m[le][1][k] = h2;
                    elem_sync<np>();
                    if (k == 0) {
                        out = (real)w3[H];
#pragma unroll
                        for (int i = 0; i < MLP_HFAST; ++i) out += (real)w3[i] * sh_m[le][1][i];
                    }
                }
            } else {
                for (int j = k; j < H; j += np) {
                    real s = (real)b1[j];
#pragma unroll
                    for (int i = 0; i < N; ++i) s += (real)W1[j * N + i] * sf[at(i, 0)];
                    sh_m[le][0][j] = act_tanh(s);
                }
                elem_sync<np>();
                for (int j = k; j < H; j += np) {
                    real s = (real)b2[j];
                    for (int i = 0; i < H; ++i) s += (real)W2[j * H + i] * sh_m[le][0][i];
                    sh_m[le][1][j] = act_tanh(s);
                }
                elem_sync<np>();
                if (k == 0) {
                    out = (real)w3[H];
                    for (int j = 0; j < H; ++j) out += (real)w3[j] * sh_m[le][1][j];
                }
            }
            if (k == 0 && act) {
                double y = (double)act_sigmoid(out);
                if (y < a.alpha_min) y = 0.0;
                if (y > a.alpha_max) y = a.alpha_max;
                a.alpha_raw[e] = inbox ? y : al_ind;
            }
        }
        // ---- MUSCL-Hancock predictor; the face-adjacent subcells' predicted
        //      values and the subface fluxes next to them, spread over the
        //      lanes like the face points (one subface flux per face point) ----
        real xm[M], xp[M], ym[M], yp[M];
        int nlim = 0, nfb = 0;
        mh_subcell<Eq, N, L>(a, ex, ey, p, q, un, su, dt, xm, xp, ym, yp, nlim, nfb);
        elem_sync<np>();
        // xm, xp, ym, yp in sf, su (the nodal values are no longer needed), sg, sh_h
        real* sh_yp = &sh_h[le][0][0];
#pragma unroll
        for (int v = 0; v < M; ++v) {
            sf[at(k, v)] = xm[v];
            su[at(k, v)] = xp[v];
            if constexpr (DIM == 2) {
                sg[at(k, v)] = ym[v];
                sh_yp[k * M + v] = yp[v];
            }
        }
        elem_sync<np>();
        if (act) {
            constexpr int NFP = DIM == 2 ? 4 * nd : 2;
#pragma unroll
            for (int j = 0; j < (NFP + np - 1) / np; ++j) {
                const int fp = k + j * np;
                if (fp >= NFP) break;
                const int sd = DIM == 2 ? fp / nd : fp, t = DIM == 2 ? fp % nd : 0, side = sd & 1;
                const int d = sd >> 1;
                // subcells i0 | i0 + 1 along d at line position t; the face's own subcell
                const int i0 = side ? N - 1 : 0;
                const int kl = d == 0 ? t * nd + i0 : i0 * nd + t, kr = kl + (d == 0 ? 1 : nd);
                const int kf = side ? kr : kl;
                real lft[M], rgt[M], own[M], fs[M];
#pragma unroll
                for (int v = 0; v < M; ++v) {
                    if constexpr (DIM == 2) {
                        lft[v] = d == 0 ? su[at(kl, v)] : sh_yp[kl * M + v];
                        rgt[v] = d == 0 ? sf[at(kr, v)] : sg[at(kr, v)];
                        own[v] = side ? (d == 0 ? su[at(kf, v)] : sh_yp[kf * M + v])
                                      : (d == 0 ? sf[at(kf, v)] : sg[at(kf, v)]);
                    } else {
                        lft[v] = su[at(kl, v)];
                        rgt[v] = sf[at(kr, v)];
                        own[v] = side ? su[at(kf, v)] : sf[at(kf, v)];
                    }
                }
                real* const lb = trace_at<Eq, N>(a, sd, side * C + 2 * M + 1, e, t);
                const size_t cs = trace_stride<Eq, N>(a);
                rusanov_n<Eq>(d, lft, rgt, fs, P);
#pragma unroll
                for (int v = 0; v < M; ++v) {
                    lb[v * cs] = own[v];
                    lb[(M + v) * cs] = fs[v];
                }
            }
            if (nlim) atomicAdd(&a.diag[D_SLOPELIM], (unsigned long long)nlim);
            if (nfb) atomicAdd(&a.diag[D_FALLBACK], (unsigned long long)nfb);
        }
        elem_sync<np>();
    }

    // ---- local cRK procedure ----
    // Face points are spread over the lanes: point fp = k + j*np (j < FPL)
    // lies on side s (0 left, 1 right, 2 bottom, 3 top) at line position t.
    constexpr int NFP = DIM == 2 ? 4 * nd : 2;
    constexpr int FPL = (NFP + np - 1) / np;
    real ui[M], F[M], Gs[M], U[M], Sa[M], tr[FPL][M], sig[FPL];
#pragma unroll
    for (int v = 0; v < M; ++v) { ui[v] = un[v]; F[v] = 0; Gs[v] = 0; U[v] = 0; Sa[v] = 0; }
#pragma unroll
    for (int j = 0; j < FPL; ++j) {
        sig[j] = 0;
#pragma unroll
        for (int v = 0; v < M; ++v) tr[j][v] = 0;
    }
    // node index of position r on the line of face point fp, and its side
    auto fside = [&](int fp) { return DIM == 2 ? fp / nd : fp; };
    auto fpos = [&](int fp) { return DIM == 2 ? fp % nd : 0; };
    auto fnode = [&](int fp, int r) {
        const int sd = fside(fp), t = fpos(fp);
        return sd < 2 ? t * nd + r : r * nd + t;
    };
    // this lane's face lines: offsets of the line's nodes (value 0), counted
    // from the face.  The solution points are symmetric about the element's
    // centre, so the value at the upper face is the sum of l_0(xi_r) times
    // the node r places from that face: one set of weights (wavefront-uniform,
    // in scalar registers) serves both sides of every face.
    int fkn[FPL][nd];
#pragma unroll
    for (int j = 0; j < FPL; ++j) {
        const int fp = k + j * np < NFP ? k + j * np : NFP - 1;
        const bool hi = fside(fp) & 1;
#pragma unroll
        for (int r = 0; r < nd; ++r) fkn[j][r] = at(fnode(fp, hi ? N - r : r), 0);
    }
    const real* fw0 = a.R.l0;
    // rows of the derivative matrix scaled by the inverse element widths: the
    // divergence d f / dx + d g / dy is then one chain of products.
    // 16-point elements (N = 3 in 2D) fill a DPP row of 16 lanes with their
    // x lines in quads: the line values come from the neighbouring lanes by
    // quad rotations (x) and row rotations by 4, 8, 12 (y) instead of through
    // LDS, and the coefficients are taken in the rotated order
    // (not for the limited FP64 kernel: its registers would exceed the 168
    // that keep three wavefronts per SIMD)
    constexpr bool DPPD = MFD || (DIM == 2 && np == 16 && !(LIM && sizeof(real) == 8));
    // (FP64: the products' operands instead, see mfma4: the y product's A and
    // the x product's B both hold D[p][q] on node (p, q)'s lane, scaled by the
    // inverse widths; the identity)
    const real cAy = MFD ? a.R.D[p][q] * idy : (real)0, cBx = MFD ? a.R.D[p][q] * idx : (real)0;
    const real cI = p == q ? (real)1 : (real)0;
    real Dx[nd], Dy[nd];
#pragma unroll
    for (int r = 0; r < nd; ++r) {
        if constexpr (DPPD) {
            Dx[r] = a.R.D[p][(p + r) & 3] * idx;     // lane (p + r) mod 4 of the quad
            Dy[r] = a.R.D[q][(q - r) & 3] * idy;     // lane 4 ((q - r) mod 4) + p of the row
        } else {
            Dx[r] = a.R.D[p][r] * idx;
            Dy[r] = DIM == 2 ? a.R.D[q][r] * idy : (real)0;
        }
    }
    // d f / dx + d g / dy at this lane's node: from registers (fv, gv: this
    // lane's values) across the lanes, or from the arrays in LDS
    auto divergence = [&](const real* fv, const real* gv, int v) {
        if constexpr (MFD) {
            const real ft = mfma4(fv[v], cI, 0.0);     // node (q, p)'s f on node (p, q)'s lane
            return (real)mfma4(ft, cBx, mfma4(cAy, gv[v], 0.0));
        } else if constexpr (DPPD) {
            real d = Dx[0] * fv[v];
            d += Dx[1] * dpp_quad_rot<1>(fv[v]);
            d += Dx[2] * dpp_quad_rot<2>(fv[v]);
            d += Dx[3] * dpp_quad_rot<3>(fv[v]);
            d += Dy[0] * gv[v];
            d += Dy[1] * dpp_row_ror<4>(gv[v]);
            d += Dy[2] * dpp_row_ror<8>(gv[v]);
            d += Dy[3] * dpp_row_ror<12>(gv[v]);
            return d;
        } else {
            real d = Dx[0] * sf[at(q * nd, v)];
#pragma unroll
            for (int r = 1; r < nd; ++r) d += Dx[r] * sf[at(q * nd + r, v)];
            if constexpr (DIM == 2) {
#pragma unroll
                for (int r = 0; r < nd; ++r) d += Dy[r] * sg[at(r * nd + p, v)];
            }
            return d;
        }
    };

#pragma unroll 1
    for (int i = 0; i < S; ++i) {
        real f[M], g[M], s[M];
        Eq::fxy(ui, f, g, P);
        if (src) Eq::src(ui, xn, yn, s, P);
        else {
#pragma unroll
            for (int v = 0; v < M; ++v) s[v] = 0;
        }
        const real bi = a.R.tb[i];
#pragma unroll
        for (int v = 0; v < M; ++v) {
            F[v] += bi * f[v];
            if constexpr (DIM == 2) Gs[v] += bi * g[v];
            U[v] += bi * ui[v];
            if (src) Sa[v] += bi * s[v];
            su[at(k, v)] = ui[v];
            if constexpr (!DPPD) {
                sf[at(k, v)] = f[v];
                if constexpr (DIM == 2) sg[at(k, v)] = g[v];
            }
        }
        elem_sync<np>();
        // EA traces: normal flux of the interpolated stage value at the face points
#pragma unroll
        for (int j = 0; j < FPL; ++j) {
            const int fp = k + j * np;
            if (j == FPL - 1 && fp >= NFP) break;
            const int sd = fside(fp);
            real uf[M], ff[M], gf[M];
#pragma unroll
            for (int v = 0; v < M; ++v) uf[v] = 0;
#pragma unroll
            for (int r = 0; r < nd; ++r) {
                const int kn = fkn[j][r];
#pragma unroll
                for (int v = 0; v < M; ++v) uf[v] += fw0[r] * su[kn + at(0, v)];
            }
            if constexpr (has_normal_flux<Eq>::value) {
                Eq::fn(sd < 2 ? 0 : 1, uf, ff, P);
#pragma unroll
                for (int v = 0; v < M; ++v) tr[j][v] += bi * ff[v];
            } else {
                Eq::fxy(uf, ff, gf, P);
#pragma unroll
                for (int v = 0; v < M; ++v) tr[j][v] += bi * (sd < 2 ? ff[v] : gf[v]);
            }
            if (!TILE && act && (a.dissipation == DISS_DCSX || (i == 0 && a.dissipation == DISS_D1))) {
                // stage values at the face (D-CSX), or u^n in place of U (D1)
                real* base = sd < 2 ? a.trx : a.trY;
                const int npt = sd < 2 ? nq : nd, side = sd & 1, t = fpos(fp);
                const int c0 = a.dissipation == DISS_DCSX ? trace_stage_offset<M>() + i * M : M;
#pragma unroll
                for (int v = 0; v < M; ++v) base[((size_t)(side * C + c0 + v) * nes + e) * npt + t] = uf[v];
            }
            if (i == 0) {
                real nodev[M];
                const int kadj = fkn[j][0];
#pragma unroll
                for (int v = 0; v < M; ++v) nodev[v] = su[kadj + at(0, v)];
                sig[j] = Eq::sig_trace(sd < 2 ? 0 : 1, uf, nodev, P);
            }
        }
        if (i < S - 1) {
            const real ai = a.R.ta[i];
#pragma unroll
            for (int v = 0; v < M; ++v) ui[v] = un[v] - rdt * ai * (divergence(f, g, v) - s[v]);
        }
        elem_sync<np>();
    }

    // (colour 1 of the checkerboard step: the neighbours' traces on the facing
    // sides are loaded here, so that they arrive while the volume part runs;
    // every boundary is periodic)
    real nbF[FPL][M], nbU[FPL][M], nbS[FPL];
    if constexpr (CB == 2) {
        const size_t cs = trace_stride<Eq, N>(a);
#pragma unroll
        for (int j = 0; j < FPL; ++j) {
            const int fp = k + j * np < NFP ? k + j * np : NFP - 1;
            const int sd = fside(fp), t = fpos(fp), side = sd & 1;
            const bool xd = sd < 2;
            const int nxe = xd ? (side ? (ex + 1 == a.nx ? 0 : ex + 1) : (ex == 0 ? a.nx - 1 : ex - 1)) : ex;
            const int nye = xd ? ey : (side ? (ey + 1 == a.ny ? 0 : ey + 1) : (ey == 0 ? a.ny - 1 : ey - 1));
            const real* nb = trace_at<Eq, N>(a, sd ^ 1, (1 - side) * C, cb_index(nxe, nye, a.nx), t);
#pragma unroll
            for (int v = 0; v < M; ++v) {
                nbF[j][v] = nb[v * cs];
                nbU[j][v] = nb[(M + v) * cs];
            }
            nbS[j] = nb[2 * M * cs];
        }
    }

    // ---- volume part of the FR update, traces of U, extrapolated averaged flux ----
#pragma unroll
    for (int v = 0; v < M; ++v) {
        su[at(k, v)] = U[v];
        sf[at(k, v)] = F[v];
        if constexpr (DIM == 2) sg[at(k, v)] = Gs[v];
    }
    elem_sync<np>();
    real vol[M], Ut[FPL][M];
#pragma unroll
    for (int v = 0; v < M; ++v) vol[v] = divergence(F, Gs, v);
#pragma unroll
    for (int j = 0; j < FPL; ++j) {
        const int fp = k + j * np;
        if (j == FPL - 1 && fp >= NFP) break;
        const int sd = fside(fp), t = fpos(fp);
        real hf[M];
#pragma unroll
        for (int v = 0; v < M; ++v) { Ut[j][v] = 0; hf[v] = 0; }
#pragma unroll
        for (int r = 0; r < nd; ++r) {
            const int kn = fkn[j][r];
#pragma unroll
            for (int v = 0; v < M; ++v) {
                Ut[j][v] += fw0[r] * su[kn + at(0, v)];
                hf[v] += fw0[r] * (sd < 2 ? sf[kn + at(0, v)] : sg[DIM == 2 ? kn + at(0, v) : 0]);
            }
        }
#pragma unroll
        for (int v = 0; v < M; ++v) {
            sh_h[le][v][sd * nd + t] = hf[v];
            if (a.central == CENTRAL_AE) tr[j][v] = hf[v];   // extrapolated averaged flux as the central part
        }
    }
    elem_sync<np>();
    if constexpr (TILE) {
        // uHp to registers; the face traces to the element's region (its
        // stage arrays are read no more); faces on the tile's edge to HBM too
        constexpr int TC = 2 * M + 1;
        const size_t gi = (size_t)e * np + k;
#pragma unroll
        for (int v = 0; v < M; ++v) {
            real corr = (sh_h[le][v][nd + q] * a.R.bR[p] - sh_h[le][v][q] * a.R.bL[p]) * idx;
            if constexpr (DIM == 2)
                corr += (sh_h[le][v][3 * nd + p] * a.R.bR[q] - sh_h[le][v][2 * nd + p] * a.R.bL[q]) * idy;
            uhp_out[v] = un[v] - rdt * (vol[v] - Sa[v]) + rdt * corr;
            if (act && src && a.dtS) a.dtS[(size_t)v * nes * np + gi] = rdt * Sa[v];
        }
#pragma unroll
        for (int j = 0; j < FPL; ++j) {
            const int fp = k + j * np;
            if (j == FPL - 1 && fp >= NFP) break;
            const int sd = fside(fp), t = fpos(fp), side = sd & 1;
#pragma unroll
            for (int v = 0; v < M; ++v) {
                su[fp * TC + v] = tr[j][v];
                su[fp * TC + M + v] = Ut[j][v];
            }
            su[fp * TC + 2 * M] = sig[j];
            const bool edge_face = sd == 0 ? tix == 0 : sd == 1 ? (tix == G::TX - 1 || ex + 1 >= a.nx)
                                 : sd == 2 ? tiy == 0 : (tiy == G::TY - 1 || ey + 1 >= a.ny);
            if (act && edge_face) {
                real* const lb = trace_at<Eq, N>(a, sd, side * C, e, t);
                const size_t cs = trace_stride<Eq, N>(a);
#pragma unroll
                for (int v = 0; v < M; ++v) {
                    lb[v * cs] = tr[j][v];
                    lb[(M + v) * cs] = Ut[j][v];
                }
                lb[2 * M * cs] = sig[j];
            }
        }
        return;
    }
    if constexpr (CB == 2) {
        // the partial update in registers, then the element's face fluxes
        __shared__ real sh_Fc[EB][NFP][M];
        real uhp[M];
#pragma unroll
        for (int v = 0; v < M; ++v) {
            real corr = (sh_h[le][v][nd + q] * a.R.bR[p] - sh_h[le][v][q] * a.R.bL[p]) * idx;
            corr += (sh_h[le][v][3 * nd + p] * a.R.bR[q] - sh_h[le][v][2 * nd + p] * a.R.bL[q]) * idy;
            uhp[v] = un[v] - rdt * (vol[v] - Sa[v]) + rdt * corr;
        }
        const size_t nwf = (size_t)(a.ne >> 1) * NFP;   // stride of one variable's colour-1 face fluxes
#pragma unroll
        for (int j = 0; j < FPL; ++j) {
            const int fp = k + j * np;
            if (j == FPL - 1 && fp >= NFP) break;
            const int side = fside(fp) & 1;
            real Fm[M], Fp[M], Um[M], Up[M], sm, sp;
#pragma unroll
            for (int v = 0; v < M; ++v) {
                const real Fn = nbF[j][v], Un = nbU[j][v];
                Fm[v] = side ? tr[j][v] : Fn;
                Fp[v] = side ? Fn : tr[j][v];
                Um[v] = side ? Ut[j][v] : Un;
                Up[v] = side ? Un : Ut[j][v];
            }
            {
                const real sn = nbS[j];
                sm = side ? sig[j] : sn;
                sp = side ? sn : sig[j];
            }
            const real lam = fmax(sm, sp);
            real F[M];
#pragma unroll
            for (int v = 0; v < M; ++v) {
                F[v] = (real)0.5 * (Fm[v] + Fp[v]) - (real)0.5 * lam * (Up[v] - Um[v]);
                sh_Fc[le][fp][v] = F[v];
            }
            if (act) {
                // the element's face fluxes for the colour-0 update, by colour
                // index and face point (whole cache lines)
                real* const out = a.Fx + (size_t)cb_index(ex, ey, a.nx) * NFP + fp;
#pragma unroll
                for (int v = 0; v < M; ++v) out[v * nwf] = F[v];
            }
        }
        elem_sync<np>();
        real FLv[M], FRv[M], GBv[M], GTv[M], unew[M], dts[M];
#pragma unroll
        for (int v = 0; v < M; ++v) {
            FLv[v] = sh_Fc[le][q][v];
            FRv[v] = sh_Fc[le][nd + q][v];
            real val = uhp[v] - rdt * idx * (FRv[v] * a.R.bR[p] - FLv[v] * a.R.bL[p]);
            GBv[v] = sh_Fc[le][2 * nd + p][v];
            GTv[v] = sh_Fc[le][3 * nd + p][v];
            val -= rdt * idy * (GTv[v] * a.R.bR[q] - GBv[v] * a.R.bL[q]);
            unew[v] = val;
            dts[v] = 0;
        }
        update_finish<Eq, N, real, EB, MFD>(a, e, le, k, act, unew, FLv, FRv, GBv, GTv, dts, vblock);
        return;
    }
    if (!act) return;
    // one 64-bit address per lane and array; the variables and trace
    // components lie whole planes apart (wavefront-uniform strides)
    const size_t gi = (size_t)e * np + k, vs = nes * np;
    // (the checkerboard's colour 0 stores its partial update by colour index)
    real* const uhp = a.uHp + (CB ? (size_t)cb_index(ex, ey, a.nx) * np + k : gi);
#pragma unroll
    for (int v = 0; v < M; ++v) {
        real corr = (sh_h[le][v][nd + q] * a.R.bR[p] - sh_h[le][v][q] * a.R.bL[p]) * idx;
        if constexpr (DIM == 2)
            corr += (sh_h[le][v][3 * nd + p] * a.R.bR[q] - sh_h[le][v][2 * nd + p] * a.R.bL[q]) * idy;
        uhp[v * vs] = un[v] - rdt * (vol[v] - Sa[v]) + rdt * corr;
        if (src && a.dtS) a.dtS[gi + v * vs] = rdt * Sa[v];
    }
#pragma unroll
    for (int j = 0; j < FPL; ++j) {
        const int fp = k + j * np;
        if (j == FPL - 1 && fp >= NFP) break;
        const int sd = fside(fp), t = fpos(fp), side = sd & 1;
        // the checkerboard's colour 0 stores its traces by colour index, so
        // that they fill whole cache lines
        real* const lb = trace_at<Eq, N>(a, sd, side * C, CB ? cb_index(ex, ey, a.nx) : e, t);
        const size_t cs = trace_stride<Eq, N>(a);
        const bool write_U = a.dissipation != DISS_D1;
#pragma unroll
        for (int v = 0; v < M; ++v) {
            lb[v * cs] = tr[j][v];
            if (write_U) lb[(M + v) * cs] = Ut[j][v];
        }
        lb[2 * M * cs] = sig[j];
    }
}

// smoothed blending coefficient alpha_e <- max(alpha_e, max_nbr alpha / 2)
template <class real>
__device__ __forceinline__ double alpha_smoothed(const StepArgs<real>& a, int e, int ex, int ey, int dim)
{
    double al = a.alpha_raw[e];
    if ((a.indicator == IND_PAPER || a.indicator == IND_LEARNED) && a.smooth) {
        for (int d = 0; d < dim; ++d)
            for (int s = 0; s < 2; ++s) {
                int en = nbr(a, ex, ey, d, s);
                if (en >= 0) {
                    double h = 0.5 * a.alpha_raw[en];
                    al = h > al ? h : al;
                }
            }
    }
    return al;
}

// dt / (w h phi_d): the factor of the flux difference in direction d's part
// of the low-order update of a face-adjacent subcell, whose share phi_d is
// proportional to the subcell's own nodal rate sigma_d / (w h_d).  With
// a_x = sigma_x / (w_x dx), a_y = sigma_y / (w_y dy) and d = 0 it is
// dt (a_x + a_y) / sigma_x = dt (1/(w_x dx) + (sigma_y/sigma_x) / (w_y dy)).
// i: index of the subcell along d (0 or N; the weights are symmetric).
template <class Eq, int N, class real>
__device__ __forceinline__ double lo_factor(const StepArgs<real>& a, int d, int t, int i, const real* u, double dt)
{
    if constexpr (Eq::DIM == 1) return dt * a.iwdx[i];
    const double sx = (double)Eq::sx(u, a.phys), sy = (double)Eq::sy(u, a.phys);
    return dt * (d == 0 ? a.iwdx[i] + (sy / sx) * a.iwdy[t] : a.iwdy[i] + (sx / sy) * a.iwdx[t]);
}

// ----------------------------------------------------------------------------
// k_face: one lane per face point of direction D
// ----------------------------------------------------------------------------
// FUSED: called by the element on either side of the face (the update with
// the faces fused in): both smoothed alphas are computed here, the flux goes
// to Fret, and the limiter counters are kept only where count is set (one
// side per face)
template <class Eq, int N, class real, bool LIM, int D, bool INTERIOR, bool FUSED = false>
__device__ __forceinline__ void face_point(const StepArgs<real>& a, int t, int eL, int eR, int exL, int eyL, int exR,
                                           int eyR, size_t outi, bool owner, real* Fret = nullptr,
                                           bool count = true);

template <class Eq, int N, class real, bool LIM, int D>
__device__ void face_body(const StepArgs<real>& a, int vblock)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int nd = G::nd, nq = G::nq;
    constexpr int npt = D == 0 ? nq : nd;
    // 32-bit indices: face points per direction stay below 2^31 (checked when
    // the solver is created)
    const unsigned total = D == 0 ? (unsigned)a.ny * (unsigned)(a.nx + 1) * nq : (unsigned)(a.ny + 1) * (unsigned)a.nx * nd;
    const unsigned tid = (unsigned)vblock * blockDim.x + threadIdx.x;
    if (tid >= total) return;
    const int t = (int)(tid % npt);
    const unsigned line = tid / npt;
    int eL, eR, exL, eyL, exR, eyR;
    size_t outi;
    bool owner = false;     // this lane stores the smoothed alpha of element eR
    if (D == 0) {
        const int i = (int)(line % (unsigned)(a.nx + 1));
        const int ey = (int)(line / (unsigned)(a.nx + 1));
        eL = i > 0 ? ey * a.nx + i - 1 : (a.bc[0] == BC_PERIODIC ? ey * a.nx + a.nx - 1 : -1);
        eR = i < a.nx ? ey * a.nx + i : (a.bc[1] == BC_PERIODIC ? ey * a.nx : -1);
        exL = i > 0 ? i - 1 : a.nx - 1; eyL = ey;
        exR = i < a.nx ? i : 0; eyR = ey;
        outi = ((size_t)ey * (a.nx + 1) + i) * nq + t;
        owner = t == 0 && i < a.nx;
    } else {
        const int ex = (int)(line % (unsigned)a.nx);
        const int j = (int)(line / (unsigned)a.nx);
        eL = j > 0 ? (j - 1) * a.nx + ex : (a.bc[2] == BC_PERIODIC ? (a.ny - 1) * a.nx + ex : -1);
        eR = j < a.ny ? j * a.nx + ex : (a.bc[3] == BC_PERIODIC ? ex : -1);
        exL = ex; eyL = j > 0 ? j - 1 : a.ny - 1;
        exR = ex; eyR = j < a.ny ? j : 0;
        outi = ((size_t)j * a.nx + ex) * nd + t;
    }
    // interior faces (both elements present: every face of a periodic grid)
    // take a path without the boundary cases
    if (eL >= 0 && eR >= 0) face_point<Eq, N, real, LIM, D, true>(a, t, eL, eR, exL, eyL, exR, eyR, outi, owner);
    else face_point<Eq, N, real, LIM, D, false>(a, t, eL, eR, exL, eyL, exR, eyR, outi, owner);
}

template <class Eq, int N, class real, bool LIM, int D, bool INTERIOR, bool FUSED>
__device__ __forceinline__ void face_point(const StepArgs<real>& a, int t, int eL, int eR, int exL, int eyL, int exR,
                                           int eyR, size_t outi, bool owner, real* Fret, bool count)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int M = Eq::M, nd = G::nd, nq = G::nq, np = G::np, K = Eq::K;
    const Phys& P = a.phys;
    const int npt = D == 0 ? nq : nd;
    const real* trb = D == 0 ? a.trx : a.trY;
    const size_t nes = (size_t)a.ne;
    const int C = a.C;
    const bool hA = INTERIOR || eL >= 0, hB = INTERIOR || eR >= 0;
    // ghost states (far-field) for a missing side
    const real* gA = hA ? nullptr : ghost_at(a, M, nd, nq, exR, eyR, D, 0, t);
    const real* gB = hB ? nullptr : ghost_at(a, M, nd, nq, exL, eyL, D, 1, t);
    const int kA = D == 0 ? t * nd + N : N * nd + t;
    const int kB = D == 0 ? t * nd : t;
    const size_t pA = hA ? (size_t)eL * npt + t : 0, pB = hB ? (size_t)eR * npt + t : 0;
#define TRA(c) trb[(size_t)(1 * C + (c)) * nes * npt + pA]
#define TRB(c) trb[(size_t)(0 * C + (c)) * nes * npt + pB]
    real Fm[M], Fp[M], Um[M], Up[M], uA[M], uB[M];
    real sm = 0, sp = 0;
    // the face-adjacent solution points enter the flux limiter, the ghosts of
    // a missing side and the D-CSX wave speeds only
    const bool need_u = LIM || !INTERIOR || a.dissipation == DISS_DCSX;
    if (hA) {
#pragma unroll
        for (int v = 0; v < M; ++v) { Fm[v] = TRA(v); Um[v] = TRA(M + v); }
        sm = TRA(2 * M);
        if (need_u) load_node<Eq>(a, np, eL, kA, uA);
    }
    if (hB) {
#pragma unroll
        for (int v = 0; v < M; ++v) { Fp[v] = TRB(v); Up[v] = TRB(M + v); }
        sp = TRB(2 * M);
        if (need_u) load_node<Eq>(a, np, eR, kB, uB);
    }
    const bool wA = !hA && is_wall(a, D, 0), wB = !hB && is_wall(a, D, 1);
    // time-dependent inflow: u^- = g(t^n), U^- = sum b_i g(t^n + c_i dt),
    // F^- = sum b_i f(g(t^n + c_i dt)) (c_i = a_{i,i-1} for these tableaux)
    const bool iA = !hA && a.bc[D * 2 + 0] == BC_INFLOW, iB = !hB && a.bc[D * 2 + 1] == BC_INFLOW;
    const double tn = (iA || iB) ? *a.tn_dev : 0.0, dtn = (iA || iB) ? *a.dt_dev : 0.0;
    // the ghost of a missing side belongs to the boundary element on the other side
    const int gex = iA ? exR : exL, gey = iA ? eyR : eyL, gside = iA ? 0 : 1;
    real gn[M];
    if (iA || iB) {
        real gU[M], gF[M];
        inflow_at(a, M, nd, nq, Eq::DIM, gex, gey, D, gside, t, tn, gn);
#pragma unroll
        for (int v = 0; v < M; ++v) { gU[v] = 0; gF[v] = 0; }
        for (int i = 0; i < a.stages; ++i) {
            real gi[M], fi[M];
            const double ci = i > 0 ? (double)a.R.ta[i - 1] : 0.0;
            inflow_at(a, M, nd, nq, Eq::DIM, gex, gey, D, gside, t, tn + ci * dtn, gi);
            flux_dir<Eq>(D, gi, fi, P);
            const real bi = a.R.tb[i];
#pragma unroll
            for (int v = 0; v < M; ++v) { gU[v] += bi * gi[v]; gF[v] += bi * fi[v]; }
        }
        const real sg = Eq::sig_trace(D, gn, gn, P);
        const bool d1 = a.dissipation == DISS_D1;
#pragma unroll
        for (int v = 0; v < M; ++v) {
            if (iA) { Fm[v] = gF[v]; Um[v] = d1 ? gn[v] : gU[v]; uA[v] = gn[v]; }
            else { Fp[v] = gF[v]; Up[v] = d1 ? gn[v] : gU[v]; uB[v] = gn[v]; }
        }
        if (iA) sm = sg; else sp = sg;
    }
    if (!hA && !iA) {
        if (gA) {
            flux_dir<Eq>(D, gA, Fm, P);
#pragma unroll
            for (int v = 0; v < M; ++v) { Um[v] = gA[v]; uA[v] = gA[v]; }
            sm = Eq::sig_trace(D, gA, gA, P);
        } else if (wA) {
#pragma unroll
            for (int v = 0; v < M; ++v) {
                const bool fl = mirror_flips<Eq>(D, v);
                Fm[v] = fl ? Fp[v] : -Fp[v];
                Um[v] = fl ? -Up[v] : Up[v];
                uA[v] = fl ? -uB[v] : uB[v];
            }
            sm = sp;
        } else {
#pragma unroll
            for (int v = 0; v < M; ++v) { Fm[v] = Fp[v]; Um[v] = Up[v]; uA[v] = uB[v]; }
            sm = sp;
        }
    }
    if (!hB && !iB) {
        if (gB) {
            flux_dir<Eq>(D, gB, Fp, P);
#pragma unroll
            for (int v = 0; v < M; ++v) { Up[v] = gB[v]; uB[v] = gB[v]; }
            sp = Eq::sig_trace(D, gB, gB, P);
        } else if (wB) {
#pragma unroll
            for (int v = 0; v < M; ++v) {
                const bool fl = mirror_flips<Eq>(D, v);
                Fp[v] = fl ? Fm[v] : -Fm[v];
                Up[v] = fl ? -Um[v] : Um[v];
                uB[v] = fl ? -uA[v] : uA[v];
            }
            sp = sm;
        } else {
#pragma unroll
            for (int v = 0; v < M; ++v) { Fp[v] = Fm[v]; Up[v] = Um[v]; uB[v] = uA[v]; }
            sp = sm;
        }
    }
    const real lam = fmax(sm, sp);
    real F[M];
#pragma unroll
    for (int v = 0; v < M; ++v) F[v] = (real)0.5 * (Fm[v] + Fp[v]) - (real)0.5 * lam * (Up[v] - Um[v]);
    if (a.dissipation == DISS_DCSX) {
        // eq. dcsx: one wave speed per stage from that stage's face values
#pragma unroll
        for (int v = 0; v < M; ++v) F[v] = (real)0.5 * (Fm[v] + Fp[v]);
        for (int i = 0; i < a.stages; ++i) {
            real sm_[M], sp_[M];
            const int c0 = trace_stage_offset<M>() + i * M;
            if (hA) {
#pragma unroll
                for (int v = 0; v < M; ++v) sm_[v] = TRA(c0 + v);
            }
            if (hB) {
#pragma unroll
                for (int v = 0; v < M; ++v) sp_[v] = TRB(c0 + v);
            }
            if (iA || iB) {
                const double ci = i > 0 ? (double)a.R.ta[i - 1] : 0.0;
                inflow_at(a, M, nd, nq, Eq::DIM, gex, gey, D, gside, t, tn + ci * dtn, iA ? sm_ : sp_);
            }
            if (!hA && !iA) {
#pragma unroll
                for (int v = 0; v < M; ++v)
                    sm_[v] = gA ? gA[v] : (wA && mirror_flips<Eq>(D, v) ? -sp_[v] : sp_[v]);
            }
            if (!hB && !iB) {
#pragma unroll
                for (int v = 0; v < M; ++v)
                    sp_[v] = gB ? gB[v] : (wB && mirror_flips<Eq>(D, v) ? -sm_[v] : sm_[v]);
            }
            const real li = fmax(Eq::sig_trace(D, sm_, uA, P), Eq::sig_trace(D, sp_, uB, P));
            const real bi = a.R.tb[i];
#pragma unroll
            for (int v = 0; v < M; ++v) F[v] -= bi * (real)0.5 * li * (sp_[v] - sm_[v]);
        }
    }
    // a fully inflow boundary (every wave enters) takes F = F^-
    const bool fi = (iA && eig_extreme<Eq>(D, gn, false, P) > 0) || (iB && eig_extreme<Eq>(D, gn, true, P) < 0);
    if (fi) {
#pragma unroll
        for (int v = 0; v < M; ++v) F[v] = iA ? Fm[v] : Fp[v];
    }

    if constexpr (LIM) {
        real sA[M], sB[M], fLO[M];
        if (hA) {
#pragma unroll
            for (int v = 0; v < M; ++v) sA[v] = TRA(2 * M + 1 + v);
        }
        if (hB) {
#pragma unroll
            for (int v = 0; v < M; ++v) sB[v] = TRB(2 * M + 1 + v);
        }
        // inflow: the boundary data at the half time, where the predicted
        // subcell values are centred; a fully inflow face takes its flux
        if (iA || iB) inflow_at(a, M, nd, nq, Eq::DIM, gex, gey, D, gside, t, tn + 0.5 * dtn, iA ? sA : sB);
        if (!hA && !iA) {
#pragma unroll
            for (int v = 0; v < M; ++v) sA[v] = gA ? gA[v] : (wA && mirror_flips<Eq>(D, v) ? -sB[v] : sB[v]);
        }
        if (!hB && !iB) {
#pragma unroll
            for (int v = 0; v < M; ++v) sB[v] = gB ? gB[v] : (wB && mirror_flips<Eq>(D, v) ? -sA[v] : sA[v]);
        }
        rusanov<Eq>(D, sA, sB, fLO, P);
        if (fi) flux_dir<Eq>(D, iA ? sA : sB, fLO, P);
        // smoothed alphas: the x faces compute them, the lane at position 0
        // of the face to the left of each element stores that element's;
        // the y faces and the update read them
        double aA, aB;
        if constexpr (D == 0 || FUSED) {
            aA = hA ? alpha_smoothed(a, eL, exL, eyL, Eq::DIM) : 0.0;
            aB = hB ? alpha_smoothed(a, eR, exR, eyR, Eq::DIM) : 0.0;
            if (!FUSED && owner) a.alpha_out[eR] = aB;
        } else {
            aA = hA ? a.alpha_out[eL] : 0.0;
            aB = hB ? a.alpha_out[eR] : 0.0;
        }
        const real af = (real)(hA && hB ? 0.5 * (aA + aB) : (hA ? aA : aB));
#pragma unroll
        for (int v = 0; v < M; ++v) F[v] = (1 - af) * F[v] + af * fLO[v];

        if constexpr (K > 0) {
            if (a.flux_limiter) {
                const double dt = *a.dt_dev;
                double kA2 = 0.0, kB2 = 0.0;
                double adjA[M], adjB[M], SA[M], SB[M], cAlo[M], cBlo[M], uAd[M], uBd[M];
                if (hA) {
                    kA2 = lo_factor<Eq, N>(a, D, t, N, uA, dt);
#pragma unroll
                    for (int v = 0; v < M; ++v) {
                        adjA[v] = (double)TRA(3 * M + 1 + v);
                        SA[v] = a.dtS ? (double)a.dtS[((size_t)v * nes + eL) * np + kA] : 0.0;
                        uAd[v] = (double)uA[v];
                        cAlo[v] = uAd[v] - kA2 * ((double)fLO[v] - adjA[v]) + SA[v];
                    }
                }
                if (hB) {
                    kB2 = lo_factor<Eq, N>(a, D, t, 0, uB, dt);
#pragma unroll
                    for (int v = 0; v < M; ++v) {
                        adjB[v] = (double)TRB(3 * M + 1 + v);
                        SB[v] = a.dtS ? (double)a.dtS[((size_t)v * nes + eR) * np + kB] : 0.0;
                        uBd[v] = (double)uB[v];
                        cBlo[v] = uBd[v] - kB2 * (adjB[v] - (double)fLO[v]) + SB[v];
                    }
                }
                double Fd[M];
#pragma unroll
                for (int v = 0; v < M; ++v) Fd[v] = (double)F[v];
                double theta_face = 1.0;
                bool bad = false;
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    double th = 1.0;
#pragma unroll
                    for (int side = 0; side < 2; ++side) {
                        if ((side == 0 && !hA) || (side == 1 && !hB)) continue;
                        double cF[M];
#pragma unroll
                        for (int v = 0; v < M; ++v)
                            cF[v] = side == 0 ? uAd[v] - kA2 * (Fd[v] - adjA[v]) + SA[v]
                                              : uBd[v] - kB2 * (adjB[v] - Fd[v]) + SB[v];
                        const double* lo = side == 0 ? cAlo : cBlo;
                        double Plo = Eq::adm(kk, lo, P);
                        if (!(Plo > 0.0)) { bad = true; th = 0.0; continue; }
                        double t2 = segment_fraction<Eq>(kk, lo, Plo, cF, a.eps_rel * Plo, P);
                        th = t2 < th ? t2 : th;
                    }
                    if (th < 1.0) {
#pragma unroll
                        for (int v = 0; v < M; ++v) Fd[v] = th * Fd[v] + (1.0 - th) * (double)fLO[v];
                    }
                    theta_face = th < theta_face ? th : theta_face;
                }
#pragma unroll
                for (int v = 0; v < M; ++v) F[v] = (real)Fd[v];
                if (theta_face < 1.0 && count) {
                    atomicAdd(&a.diag[D_FLUXLIM], 1ull);
                    atomic_min_pos(&a.diag[D_THFLUX], theta_face);
                }
                if (bad && count) atomicAdd(&a.diag[D_LOBAD], 1ull);
            }
        }
    }
#undef TRA
#undef TRB
    if constexpr (FUSED) {
#pragma unroll
        for (int v = 0; v < M; ++v) Fret[v] = F[v];
    } else {
        real* out = D == 0 ? a.Fx : a.Gy;
        const size_t nf = D == 0 ? (size_t)a.ny * (a.nx + 1) * nq : (size_t)(a.ny + 1) * a.nx * nd;
#pragma unroll
        for (int v = 0; v < M; ++v) out[(size_t)v * nf + outi] = F[v];
    }
}

// the time-averaged numerical flux at face point fp of element (ex, ey) of
// the update with the faces fused in (fp = side (nd) + t: sides left, right,
// bottom, top); the element on the upper side of a face keeps its limiter
// counters (and the element below a boundary face without an upper side)
template <class Eq, int N, class real, bool LIM>
__device__ __forceinline__ void elem_face_flux(const StepArgs<real>& a, int ex, int ey, int fp, real* F)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int M = Eq::M, nd = G::nd, nq = G::nq;
    const int sd = Eq::DIM == 2 ? fp / nd : fp, t = Eq::DIM == 2 ? fp % nd : 0, side = sd & 1;
    if constexpr (!LIM) {
        // an interior face without limiter or D-CSX: the Rusanov-type flux of
        // the time-averaged traces, with the direction a run-time operand, so
        // that the lanes of the x and the y faces of a wavefront run one
        // instruction stream
        const bool xd = sd < 2;
        const int i = xd ? ex + side : ey + side;
        const int n = xd ? a.nx : a.ny;
        const int b = i == 0 ? (xd ? a.bc[0] : a.bc[2]) : i == n ? (xd ? a.bc[1] : a.bc[3]) : BC_PERIODIC;
        if (a.dissipation != DISS_DCSX && b == BC_PERIODIC) {
            const int iL = i > 0 ? i - 1 : n - 1, iR = i < n ? i : 0;
            const int eL = xd ? ey * a.nx + iL : iL * a.nx + ex, eR = xd ? ey * a.nx + iR : iR * a.nx + ex;
            const int npt = xd ? nq : nd;
            const real* trb = xd ? a.trx : a.trY;
            const size_t st = (size_t)a.ne * npt;
            const real* A = trb + (size_t)a.C * st + (size_t)eL * npt + t;   // traces of eL on its upper side
            const real* B = trb + (size_t)eR * npt + t;                      // traces of eR on its lower side
            const real lam = fmax(A[2 * M * st], B[2 * M * st]);
#pragma unroll
            for (int v = 0; v < M; ++v)
                F[v] = (real)0.5 * (A[v * st] + B[v * st]) - (real)0.5 * lam * (B[(M + v) * st] - A[(M + v) * st]);
            return;
        }
    }
    if (sd < 2) {
        const int i = ex + side;   // x face i of row ey
        const int eL = i > 0 ? ey * a.nx + i - 1 : (a.bc[0] == BC_PERIODIC ? ey * a.nx + a.nx - 1 : -1);
        const int eR = i < a.nx ? ey * a.nx + i : (a.bc[1] == BC_PERIODIC ? ey * a.nx : -1);
        const int exL = i > 0 ? i - 1 : a.nx - 1, exR = i < a.nx ? i : 0;
        const bool count = side == 0 || eR < 0;
        if (eL >= 0 && eR >= 0)
            face_point<Eq, N, real, LIM, 0, true, true>(a, t, eL, eR, exL, ey, exR, ey, 0, false, F, count);
        else
            face_point<Eq, N, real, LIM, 0, false, true>(a, t, eL, eR, exL, ey, exR, ey, 0, false, F, count);
    } else if constexpr (Eq::DIM == 2) {
        const int j = ey + side;   // y face j of column ex
        const int eL = j > 0 ? (j - 1) * a.nx + ex : (a.bc[2] == BC_PERIODIC ? (a.ny - 1) * a.nx + ex : -1);
        const int eR = j < a.ny ? j * a.nx + ex : (a.bc[3] == BC_PERIODIC ? ex : -1);
        const int eyL = j > 0 ? j - 1 : a.ny - 1, eyR = j < a.ny ? j : 0;
        const bool count = side == 0 || eR < 0;
        if (eL >= 0 && eR >= 0)
            face_point<Eq, N, real, LIM, 1, true, true>(a, t, eL, eR, ex, eyL, ex, eyR, 0, false, F, count);
        else
            face_point<Eq, N, real, LIM, 1, false, true>(a, t, eL, eR, ex, eyL, ex, eyR, 0, false, F, count);
    }
}

// ----------------------------------------------------------------------------
// Sums over the np lanes of one element (lanes of an element are contiguous).
// When np divides the wavefront the sum is a butterfly of wavefront shuffles;
// otherwise the M sums go through LDS with two barriers.  Every lane gets
// every total.
// ----------------------------------------------------------------------------
template <int M, int np, int EB>
__device__ __forceinline__ void elem_sums(const double* in, double* out, double (*sh)[M][np], double (*shm)[M],
                                          int le, int k)
{
    if constexpr (elem_in_dpp<np>()) {
#pragma unroll
        for (int v = 0; v < M; ++v) out[v] = dpp_elem_reduce<np, RED_SUM>(in[v]);
    } else if constexpr (elem_in_wave<np>()) {
#pragma unroll
        for (int v = 0; v < M; ++v) {
            double x = in[v];
#pragma unroll
            for (int m = 1; m < np; m <<= 1) x += __shfl_xor(x, m, np);
            out[v] = x;
        }
    } else {
#pragma unroll
        for (int v = 0; v < M; ++v) sh[le][v][k] = in[v];
        __syncthreads();
        for (int v = k; v < M; v += np) {
            double x = 0.0;
#pragma unroll
            for (int kk = 0; kk < np; ++kk) x += sh[le][v][kk];
            shm[le][v] = x;
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < M; ++v) out[v] = shm[le][v];
    }
}

// minimum over the lanes of one element, one barrier pair when through LDS
template <int np>
__device__ __forceinline__ double elem_min(double x, double (*sh)[np], int le, int k)
{
    if constexpr (elem_in_dpp<np>()) {
        return dpp_elem_reduce<np, RED_MIN>(x);
    } else if constexpr (elem_in_wave<np>()) {
#pragma unroll
        for (int m = 1; m < np; m <<= 1) {
            double y = __shfl_xor(x, m, np);
            x = y < x ? y : x;
        }
        return x;
    } else {
        sh[le][k] = x;
        __syncthreads();
        double r = 1.0;
#pragma unroll
        for (int kk = 0; kk < np; ++kk) r = sh[le][kk] < r ? sh[le][kk] : r;
        __syncthreads();
        return r;
    }
}

// workgroup max of the per-element rates (one value per element, lane k = 0
// of each element holds it), one atomic per workgroup into slot
// blockIdx % RATE_SLOTS; every lane must call it (it has a barrier)
template <int EB>
__device__ __forceinline__ void block_rate_max(double rate, int le, int k, int vblock, unsigned long long* slots)
{
    __shared__ double sh_w[EB];
    if (k == 0) sh_w[le] = rate;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
#pragma unroll
        for (int l = 0; l < EB; ++l) r = sh_w[l] > r ? sh_w[l] : r;
        atomic_max_pos(&slots[vblock % RATE_SLOTS], r);
    }
}

// wavefront max of the per-element rates (lane k = 0 of each element holds
// its rate, the other lanes 0), one atomic per wavefront into slot (wavefront
// index mod RATE_SLOTS), no workgroup barrier: a wavefront that is done
// leaves without waiting for the workgroup's other wavefronts.  Every lane of
// the wavefront calls it (DPP rows and shuffles read all 64 lanes).
__device__ __forceinline__ void wave_rate_max(double rate, int vblock, unsigned long long* slots)
{
    double r = dpp_elem_reduce<16, RED_MAX>(rate);          // each 16-lane row
    double y = __shfl_xor(r, 16, 64);
    r = y > r ? y : r;
    y = __shfl_xor(r, 32, 64);
    r = y > r ? y : r;
    if ((threadIdx.x & 63) == 0)
        atomic_max_pos(&slots[(vblock * (blockDim.x / 64) + threadIdx.x / 64) % RATE_SLOTS], r);
}

// ----------------------------------------------------------------------------
// k_update
// ----------------------------------------------------------------------------
template <class Eq, int N, class real, int EB, bool MFL>
__device__ __forceinline__ void update_finish(const StepArgs<real>& a, int e, int le, int k, bool act,
                                              const real* unew, const real* FL, const real* FR, const real* GB,
                                              const real* GT, const real* dts, int vblock);

// k_update: one lane per node; elements from 0 in order, or (tile-fused step)
// the list of elements at the edges of the tiles.  FU: the faces fused in --
// the element's lanes first compute its 4 (N+1) face fluxes (each face is
// computed by the elements on both sides, in the same arithmetic) and its
// smoothed alpha; without FU the face phases have stored them.
template <class Eq, int N, class real, bool LIM, bool FU = false, int CB = 0, int WB = 0>
__device__ void update_body(const StepArgs<real>& a, int vblock)
{
    using G = UGeo<Eq::DIM, N, WB>;
    constexpr int M = Eq::M, DIM = Eq::DIM, nd = G::nd, nq = G::nq, np = G::np, EB = G::EB;
    __shared__ real sh_u[EB][np][M];
    __shared__ real sh_f[EB][np][M];
    __shared__ real sh_g[EB][np][DIM == 2 ? M : 1];
    constexpr int NFP = DIM == 2 ? 4 * nd : 2;
    // the element's face fluxes in LDS: computed here (FU) or, on the
    // checkerboard's colour 0, gathered from the colour-1 neighbours
    constexpr bool SHF = FU || (CB != 0 && DIM == 2);
    __shared__ real sh_F[SHF ? EB : 1][NFP][M];

    const Phys& P = a.phys;
    const int le = threadIdx.x / np, k = threadIdx.x - le * np;
    const int p = k % nd, q = k / nd;
    const int e0 = vblock * EB + le;
    // CB = 1: the colour-0 elements of the checkerboard step
    const int nel = a.edge_list ? a.n_edge : (CB ? a.ne >> 1 : a.ne);
    const bool act = e0 < nel;
    const int e = a.edge_list ? a.edge_list[act ? e0 : nel - 1]
                              : (CB ? cb_element(act ? e0 : nel - 1, 0, a.nx) : (act ? e0 : a.ne - 1));
    const int ey = (int)((unsigned)e / (unsigned)a.nx), ex = e - ey * a.nx;
    const double dt = *a.dt_dev;
    const real rdt = (real)dt, idx = (real)a.idx, idy = (real)a.idy;
    const size_t nes = (size_t)a.ne, gi = (size_t)e * np + k;
    const size_t nfx = (size_t)a.ny * (a.nx + 1) * nq, nfy = (size_t)(a.ny + 1) * a.nx * nd;
    const size_t iL = ((size_t)ey * (a.nx + 1) + ex) * nq + q, iR = iL + nq;
    const size_t iB = ((size_t)ey * a.nx + ex) * nd + p, iT = iB + (size_t)a.nx * nd;

    if constexpr (FU) {
        // the element's face fluxes into LDS, face point fp = side (nd) + t
#pragma unroll
        for (int j = 0; j < (NFP + np - 1) / np; ++j) {
            const int fp = k + j * np;
            if (fp < NFP) elem_face_flux<Eq, N, real, LIM>(a, ex, ey, fp, sh_F[le][fp]);
        }
        elem_sync<np>();
    }
    // CB: the colour-0 element's face fluxes, stored by its colour-1
    // neighbours (every boundary periodic): left face = the left neighbour's
    // right face, and so on; one face point per lane, each value loaded once
    if constexpr (CB != 0 && DIM == 2) {
        constexpr int NF = 4 * nd;
        const size_t nwf = (size_t)(a.ne >> 1) * NF;
        const int exl = ex == 0 ? a.nx - 1 : ex - 1, exr = ex + 1 == a.nx ? 0 : ex + 1;
        const int eyb = ey == 0 ? a.ny - 1 : ey - 1, eyt = ey + 1 == a.ny ? 0 : ey + 1;
#pragma unroll
        for (int j = 0; j < (NFP + np - 1) / np; ++j) {
            const int fp = k + j * np;
            if (fp < NFP) {
                const int sd = fp / nd, t = fp - sd * nd;
                const size_t c = sd == 0 ? (size_t)cb_index(exl, ey, a.nx) * NF + nd + t
                               : sd == 1 ? (size_t)cb_index(exr, ey, a.nx) * NF + t
                               : sd == 2 ? (size_t)cb_index(ex, eyb, a.nx) * NF + 3 * nd + t
                                         : (size_t)cb_index(ex, eyt, a.nx) * NF + 2 * nd + t;
#pragma unroll
                for (int v = 0; v < M; ++v) sh_F[le][fp][v] = a.Fx[v * nwf + c];
            }
        }
        elem_sync<np>();
    }
    real uH[M], FLv[M], FRv[M], GBv[M], GTv[M], dts[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
        FLv[v] = SHF ? sh_F[SHF ? le : 0][DIM == 2 ? q : 0][v] : a.Fx[v * nfx + iL];
        FRv[v] = SHF ? sh_F[SHF ? le : 0][DIM == 2 ? nd + q : 1][v] : a.Fx[v * nfx + iR];
        real val = a.uHp[v * nes * np + (CB ? (size_t)cb_index(ex, ey, a.nx) * np + k : gi)] -
                   rdt * idx * (FRv[v] * a.R.bR[p] - FLv[v] * a.R.bL[p]);
        if constexpr (DIM == 2) {
            GBv[v] = SHF ? sh_F[SHF ? le : 0][2 * nd + p][v] : a.Gy[v * nfy + iB];
            GTv[v] = SHF ? sh_F[SHF ? le : 0][3 * nd + p][v] : a.Gy[v * nfy + iT];
            val -= rdt * idy * (GTv[v] * a.R.bR[q] - GBv[v] * a.R.bL[q]);
        } else {
            GBv[v] = 0;
            GTv[v] = 0;
        }
        uH[v] = val;
        dts[v] = a.dtS ? a.dtS[(size_t)v * nes * np + gi] : (real)0;
    }
    real unew[M];
#pragma unroll
    for (int v = 0; v < M; ++v) unew[v] = uH[v];

    if constexpr (LIM) {
        // smoothed by the x-face phase, or here with the faces fused in
        double al;
        if constexpr (FU) {
            al = alpha_smoothed(a, e, ex, ey, DIM);
            if (k == 0 && act) a.alpha_out[e] = al;
        } else {
            al = a.alpha_out[e];
        }
        if (k == 0 && act && al > 0.0) atomicAdd(&a.diag[D_TROUBLED], 1ull);
        const bool any = elem_any<np>(act && al > 0.0);
        if (any) {
            // recompute the subcell predictor and the low-order update (eq. low.order.update)
            real un[M];
            load_node<Eq>(a, np, e, k, un);
#pragma unroll
            for (int v = 0; v < M; ++v) sh_u[le][k][v] = un[v];
            elem_sync<np>();
            real xm[M], xp[M], ym[M], yp[M];
            int nlim = 0, nfb = 0;
            if (al > 0.0)
                mh_subcell<Eq, N, NodeMajor<M, np>>(a, ex, ey, p, q, un, &sh_u[le][0][0], dt, xm, xp, ym, yp, nlim,
                                                    nfb);
            elem_sync<np>();
#pragma unroll
            for (int v = 0; v < M; ++v) {
                sh_f[le][k][v] = xm[v];
                if constexpr (DIM == 2) sh_g[le][k][v] = ym[v];
            }
            elem_sync<np>();
            real fxp[M], gyp[M];
#pragma unroll
            for (int v = 0; v < M; ++v) { fxp[v] = 0; gyp[v] = 0; }
            if (al > 0.0) {
                if (p < N) {
                    real nb[M];
#pragma unroll
                    for (int v = 0; v < M; ++v) nb[v] = sh_f[le][k + 1][v];
                    rusanov<Eq>(0, xp, nb, fxp, P);
                }
                if constexpr (DIM == 2) {
                    if (q < N) {
                        real nb[M];
#pragma unroll
                        for (int v = 0; v < M; ++v) nb[v] = sh_g[le][k + nd][v];
                        rusanov<Eq>(1, yp, nb, gyp, P);
                    }
                }
            }
            elem_sync<np>();
#pragma unroll
            for (int v = 0; v < M; ++v) {
                sh_f[le][k][v] = fxp[v];
                if constexpr (DIM == 2) sh_g[le][k][v] = gyp[v];
            }
            elem_sync<np>();
            if (al > 0.0) {
                const real ralpha = (real)al;
#pragma unroll
                for (int v = 0; v < M; ++v) {
                    real fm = p == 0 ? FLv[v] : sh_f[le][k - 1][v];
                    real fp = p == N ? FRv[v] : fxp[v];
                    real uL = un[v] - rdt / (a.R.w[p] * (real)a.dx) * (fp - fm);
                    if constexpr (DIM == 2) {
                        real gm = q == 0 ? GBv[v] : sh_g[le][k - nd][v];
                        real gp = q == N ? GTv[v] : gyp[v];
                        uL -= rdt / (a.R.w[q] * (real)a.dy) * (gp - gm);
                    }
                    if (a.dtS) uL += a.dtS[(size_t)v * nes * np + gi];
                    unew[v] = (1 - ralpha) * uH[v] + ralpha * uL;
                }
            }
        }
    }

    update_finish<Eq, N, real, EB>(a, e, le, k, act, unew, FLv, FRv, GBv, GTv, dts, vblock);
}

// the update after the nodal values unew of eq. crkfr.avg (blended, eq.
// blended.scheme): FP64 element means (MP32: the FP64 mean update of eq.
// upmean from this lane's face fluxes FL, FR (row q) and GB, GT (column p),
// with the source average dts = dt S of App. B), Zhang-Shu scaling, the store
// of u^{n+1} and the wave-speed rate of the next step.  Every lane of the
// workgroup calls it (element reductions, rate reduction); lanes with act
// false store nothing and report no rate.
template <class Eq, int N, class real, int EB, bool MFL>
__device__ __forceinline__ void update_finish(const StepArgs<real>& a, int e, int le, int k, bool act,
                                              const real* unew, const real* FL, const real* FR, const real* GB,
                                              const real* GT, const real* dts, int vblock)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int M = Eq::M, DIM = Eq::DIM, nd = G::nd, np = G::np, K = Eq::K;
    constexpr bool MP = is_mp<real>();
    static_assert(!MFL || (!MP && np == 16), "the matrix-core layout: 16-node FP64 elements");
    constexpr bool DPP = elem_in_dpp<np>();
    __shared__ double sh_d[DPP ? 1 : EB][np];
    __shared__ double sh_r[elem_in_wave<np>() ? 1 : EB][M][np];
    __shared__ double sh_m[elem_in_wave<np>() ? 1 : EB][M];
    __shared__ double sh_r2[elem_in_wave<np>() || !MP ? 1 : EB][2 * M][np];
    __shared__ double sh_m2[elem_in_wave<np>() || !MP ? 1 : EB][2 * M];
    const Phys& P = a.phys;
    const int p = k % nd, q = k / nd;
    const double dt = *a.dt_dev;
    const size_t nes = (size_t)a.ne, gi = (size_t)e * np + k;

    // ---- FP64 element means (MP32: FP64 mean update from the face fluxes,
    //      eq. upmean with the source average of App. B) ----
    const double wk = a.w64[p] * (DIM == 2 ? a.w64[q] : 1.0);
    double part[2 * M], sums[2 * M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
        part[v] = wk * (double)unew[v];
        double c = 0.0;
        if constexpr (MP) {
            if (p == 0) c -= dt * a.idx * (DIM == 2 ? a.w64[q] : 1.0) * ((double)FR[v] - (double)FL[v]);
            if constexpr (DIM == 2) {
                if (q == 0) c -= dt * a.idy * a.w64[p] * ((double)GT[v] - (double)GB[v]);
            }
            if (a.dtS) c += wk * (double)dts[v];
        }
        part[M + v] = c;
    }
    double ubar[M], um[M];
    if constexpr (MP) {
        elem_sums<2 * M, np, EB>(part, sums, sh_r2, sh_m2, le, k);
#pragma unroll
        for (int v = 0; v < M; ++v) {
            ubar[v] = sums[v];
            um[v] = a.ubar[(size_t)v * nes + e] + sums[M + v];
        }
    } else {
        // (MFL: the element's lanes laid out as the blocks of v_mfma_f64_4x4x4)
        if constexpr (MFL) {
#pragma unroll
            for (int v = 0; v < M; ++v) sums[v] = mfma_elem_reduce<RED_SUM>(part[v]);
        } else {
            elem_sums<M, np, EB>(part, sums, sh_r, sh_m, le, k);
        }
#pragma unroll
        for (int v = 0; v < M; ++v) { ubar[v] = sums[v]; um[v] = sums[v]; }
    }
    // nodal values in FP64 relative to the mean the state keeps
    double ud[M];
#pragma unroll
    for (int v = 0; v < M; ++v) ud[v] = MP ? um[v] + ((double)unew[v] - ubar[v]) : (double)unew[v];

    // ---- Zhang-Shu scaling (reading: eps_k = min(eps_abs, P_k(mean)); linear
    //      root for density, 60-step bisection otherwise); every lane runs
    //      every barrier, the per-element early exit is a flag ----
    if constexpr (K > 0) {
        if (a.scaling) {
            bool mean_bad = false;
            double th_all = 1.0;
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                double Pbar = Eq::adm(kk, um, P);
                if (!(Pbar > 0.0)) mean_bad = true;
                double t = 1.0;
                if (!mean_bad) {
                    double eps = Pbar < a.eps_abs ? Pbar : a.eps_abs;
                    if (!Eq::adm_ge(kk, ud, eps, P)) {
                        if (kk == 0) t = (um[0] - eps) / (um[0] - ud[0]);
                        else t = bisect_root<Eq>(kk, um, ud, eps, P);
                    }
                }
                // (an element's lanes in one wavefront: no exchange when no lane scales)
                double th;
                if constexpr (MFL) th = __all(t >= 1.0) ? 1.0 : mfma_elem_reduce<RED_MIN>(t);
                else if constexpr (elem_in_wave<np>()) th = __all(t >= 1.0) ? 1.0 : elem_min<np>(t, sh_d, le, k);
                else th = elem_min<np>(t, sh_d, le, k);
                if (!mean_bad) {
                    if (th < 1.0) {
#pragma unroll
                        for (int v = 0; v < M; ++v) ud[v] = um[v] + th * (ud[v] - um[v]);
                    }
                    th_all = th < th_all ? th : th_all;
                }
            }
            if (mean_bad) th_all = 0.0;
            if (k == 0 && act) {
                if (mean_bad) atomicAdd(&a.diag[D_MEANBAD], 1ull);
                else if (th_all < 1.0) atomicAdd(&a.diag[D_SCALED], 1ull);
                if (th_all < 1.0) atomic_min_pos(&a.diag[D_THSCALE], th_all);
            }
        } else if (k == 0 && act) {
            bool bad = false;
#pragma unroll
            for (int kk = 0; kk < K; ++kk)
                if (!bad && !(Eq::adm(kk, um, P) > 0.0)) bad = true;
            if (bad) atomicAdd(&a.diag[D_MEANBAD], 1ull);
        }
    }

    // ---- store, next-step rate ----
    if (act) {
        real* const uo = a.u_out + gi;
#pragma unroll
        for (int v = 0; v < M; ++v) {
            if constexpr (MP) uo[v * nes * np] = (real)(ud[v] - um[v]);
            else uo[v * nes * np] = (real)ud[v];
        }
        if constexpr (MP) {
            if (k == 0) {
#pragma unroll
                for (int v = 0; v < M; ++v) a.ubar_out[(size_t)v * nes + e] = um[v];
            }
        }
    }
    double rate = 0.0;
    if (k == 0 && act) {
        real ur[M];
#pragma unroll
        for (int v = 0; v < M; ++v) ur[v] = (real)um[v];
        rate = (double)Eq::sx(ur, P) / a.dx + (DIM == 2 ? (double)Eq::sy(ur, P) / a.dy : 0.0);
        if (!(rate == rate)) rate = 1e300;
    }
    if constexpr (elem_in_dpp<np>() && Geo<DIM, N>::BLOCK % 64 == 0) wave_rate_max(rate, vblock, a.rate_bits);
    else block_rate_max<EB>(rate, le, k, vblock, a.rate_bits);
}

// ----------------------------------------------------------------------------
// single-instance kernels
// ----------------------------------------------------------------------------
// Workgroups are dispatched to the 8 XCDs in turn (workgroup b to XCD b mod 8),
// each with its own L2.  The local phase maps them so that each XCD works on
// one contiguous range of blocks: an element's neighbours, whose boundary
// nodes and means the MUSCL-Hancock stencil reads, then mostly sit in the
// same L2 (11-13 % off the limited FP32 local phase).  The other phases keep
// the plain order: contiguous ranges would put a cluster of troubled
// elements, whose update is several times dearer, on one XCD.
__device__ __forceinline__ int xcd_block(int b, int n)
{
    constexpr int X = 8;
    const int per = n / X, rem = n % X, x = b % X, i = b / X;
    return x * per + (x < rem ? x : rem) + i;
}

// The FP32-bulk local phase of 2D Euler with 25-point elements, and the FP64
// one with 16-point elements (derivatives on the matrix cores) with the
// limiter chain, need a few registers more than the 128 that keep four
// wavefronts per SIMD; held to 128 they keep four, without spills.
template <class Eq, int N, class real, bool LIM = false>
constexpr int local_min_waves()
{
    return Eq::M == 4 && Eq::DIM == 2 && ((sizeof(real) == 4 && N == 4) || (sizeof(real) == 8 && N == 3)) ? 4 : 1;
}

template <class Eq, int N, class real, bool LIM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(local_min_waves<Eq, N, real, LIM>())))
k_local(const StepArgs<real> a)
{
    local_body<Eq, N, real, LIM>(a, xcd_block(blockIdx.x, gridDim.x));
}

template <class Eq, int N, class real, bool LIM, int D>
__global__ void __launch_bounds__(256) k_face(const StepArgs<real> a) { face_body<Eq, N, real, LIM, D>(a, blockIdx.x); }

// the checkerboard step: colour 0 local, colour 1 local + faces + update,
// colour 0 update from the stored face fluxes
template <class Eq, int N, class real>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(local_min_waves<Eq, N, real>())))
k_cb_local(const StepArgs<real> a)
{
    if constexpr (Eq::DIM == 2) local_body<Eq, N, real, false, void, 1>(a, xcd_block(blockIdx.x, gridDim.x));
}
// the colour-1 kernel of 16-point FP64 elements (derivatives on the matrix
// cores) fits the 128 registers of four wavefronts per SIMD without spills
template <class Eq, int N, class real>
constexpr int white_min_waves()
{
    return sizeof(real) == 8 && Eq::M == 4 && Eq::DIM == 2 && N == 3 ? 4 : 1;
}
template <class Eq, int N, class real>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(white_min_waves<Eq, N, real>())))
k_cb_white(const StepArgs<real> a)
{
    if constexpr (Eq::DIM == 2) local_body<Eq, N, real, false, void, 2>(a, xcd_block(blockIdx.x, gridDim.x));
}
template <class Eq, int N, class real, int WB = 0>
__global__ void __launch_bounds__(256) k_cb_update(const StepArgs<real> a)
{
    update_body<Eq, N, real, false, false, 1, WB>(a, blockIdx.x);
}

template <class Eq, int N, class real, bool LIM, bool FU = false, int WB = 0>
__global__ void __launch_bounds__(256) k_update(const StepArgs<real> a)
{
    // with the faces fused in and no limiter, the blocks of an XCD take one
    // contiguous range of elements, so that the traces an element shares with
    // its neighbours are fetched into one L2
    update_body<Eq, N, real, LIM, FU, 0, WB>(a, FU && !LIM ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x);
}

// ----------------------------------------------------------------------------
// tile-fused step (limiter off): one workgroup per tile of TX x TY elements,
// one lane per node.  The local cRK procedure of every element, the fluxes of
// the faces inside the tile and the whole update of the tile's inner elements
// (all four neighbours in the tile) stay in LDS and registers; only u^n is
// read and u^{n+1} written for them.  The elements at the tile's edge write
// uHp, their traces on the tile's edge faces and the fluxes of their faces
// inside the tile; the faces on tile edges (k_tile_face, the boundary
// conditions included) and the update of the edge elements (k_update over
// their list) follow.  Elements of 4 or 16 points (N = 1, 3 in 2D): an
// element's lanes share a wavefront, so its exchanges need no workgroup
// barrier.  Tiles of 512 lanes for FP64 (the local procedure holds some 190
// VGPRs: two wavefronts per SIMD), 1024 lanes for FP32 bulk.
// ----------------------------------------------------------------------------
template <int DIM, int N, int RB>
struct TGeo {
    static constexpr int nd = N + 1, nq = DIM == 2 ? N + 1 : 1, np = nd * nq;
    static constexpr bool OK = DIM == 2 && (np == 4 || np == 16);
    static constexpr int TX = np == 4 ? 16 : 8, TY = np == 4 ? (RB == 8 ? 8 : 16) : (RB == 8 ? 4 : 8);
    static constexpr int EB = TX * TY, BLOCK = EB * np;
};
template <class Eq, int N, class real>
constexpr int tile_block_v = TGeo<Eq::DIM, N, (int)sizeof(real)>::BLOCK;

// an element of the tile at (ix, iy) is inner when its four neighbours lie in
// the tile (and in the grid)
__device__ __forceinline__ bool tile_inner(int ix, int iy, int TX, int TY, int gx, int gy, int nx, int ny)
{
    return ix > 0 && ix < TX - 1 && iy > 0 && iy < TY - 1 && gx + 1 < nx && gy + 1 < ny;
}

template <class Eq, int N, class real>
__global__ void __launch_bounds__((tile_block_v<Eq, N, real>)) k_tile(const StepArgs<real> a)
{
    using TG = TGeo<Eq::DIM, N, (int)sizeof(real)>;
    constexpr int M = Eq::M, nd = TG::nd, nq = TG::nq, np = TG::np, TX = TG::TX, TY = TG::TY, EB = TG::EB;
    constexpr int SB = elem_region<Eq, N, real>(), TC = 2 * M + 1;
    __shared__ real tile_buf[EB * SB];
    __shared__ real sh_fx[TY][TX + 1][nq][M];   // x face i of tile row iy (left of element i)
    __shared__ real sh_gy[TY + 1][TX][nd][M];   // y face j of tile column ix (below element j)
    const int vblock = blockIdx.x;
    real uhp[M];
    local_body<Eq, N, real, false, TG>(a, vblock, tile_buf, uhp);
    __syncthreads();

    const int ntx = (a.nx + TX - 1) / TX;
    const int gx0 = (vblock % ntx) * TX, gy0 = (vblock / ntx) * TY;
    const size_t nfx = (size_t)a.ny * (a.nx + 1) * nq, nfy = (size_t)(a.ny + 1) * a.nx * nd;
    // ---- the faces inside the tile: time-averaged numerical flux, eqs.
    //      numflux.general with D2 (D1: the U slots hold u^n traces) ----
    constexpr int NXF = TY * (TX - 1) * nq, NYF = (TY - 1) * TX * nd;
    for (int f = threadIdx.x; f < NXF + NYF; f += blockDim.x) {
        int ixA, iyA, ixB, iyB, t, fpA, fpB;
        if (f < NXF) {
            t = f % nq;
            const int r = f / nq;
            ixA = r % (TX - 1); iyA = r / (TX - 1); ixB = ixA + 1; iyB = iyA;
            fpA = nd + t; fpB = t;                  // right face of A, left face of B
        } else {
            const int f2 = f - NXF;
            t = f2 % nd;
            const int r = f2 / nd;
            ixA = r % TX; iyA = r / TX; ixB = ixA; iyB = iyA + 1;
            fpA = 3 * nd + t; fpB = 2 * nd + t;     // top face of A, bottom face of B
        }
        if (gx0 + ixB >= a.nx || gy0 + iyB >= a.ny) continue;   // B outside the grid (A is inside)
        const real* tA = tile_buf + (iyA * TX + ixA) * SB + fpA * TC;
        const real* tB = tile_buf + (iyB * TX + ixB) * SB + fpB * TC;
        const real lam = fmax(tA[2 * M], tB[2 * M]);
        const bool to_hbm = !tile_inner(ixA, iyA, TX, TY, gx0 + ixA, gy0 + iyA, a.nx, a.ny) ||
                            !tile_inner(ixB, iyB, TX, TY, gx0 + ixB, gy0 + iyB, a.nx, a.ny);
#pragma unroll
        for (int v = 0; v < M; ++v) {
            const real F = (real)0.5 * (tA[v] + tB[v]) - (real)0.5 * lam * (tB[M + v] - tA[M + v]);
            if (f < NXF) {
                sh_fx[iyA][ixB][t][v] = F;
                if (to_hbm) a.Fx[v * nfx + ((size_t)(gy0 + iyA) * (a.nx + 1) + gx0 + ixB) * nq + t] = F;
            } else {
                sh_gy[iyB][ixA][t][v] = F;
                if (to_hbm) a.Gy[v * nfy + ((size_t)(gy0 + iyB) * a.nx + gx0 + ixA) * nd + t] = F;
            }
        }
    }
    __syncthreads();

    // ---- inner elements: the correction-function part of the FR update (eq.
    //      crkfr.avg) from the LDS face fluxes, then the rest of the update;
    //      edge elements: uHp to HBM for the update phase ----
    const int le = threadIdx.x / np, k = threadIdx.x - le * np;
    const int p = k % nd, q = k / nd, ix = le % TX, iy = le / TX;
    const int gx = gx0 + ix, gy = gy0 + iy;
    const bool act = gx < a.nx && gy < a.ny;
    const bool in = act && tile_inner(ix, iy, TX, TY, gx, gy, a.nx, a.ny);
    const int e = (gy < a.ny ? gy : a.ny - 1) * a.nx + (gx < a.nx ? gx : a.nx - 1);
    const size_t nes = (size_t)a.ne, gi = (size_t)e * np + k;
    if (act && !in) {
#pragma unroll
        for (int v = 0; v < M; ++v) a.uHp[(size_t)v * nes * np + gi] = uhp[v];
    }
    if (__any(in)) {   // whole wavefronts: the update reduces over each element's lanes
        const real rdt = (real)*a.dt_dev, idx = (real)a.idx, idy = (real)a.idy;
        real unew[M], FL[M], FR[M], GB[M], GT[M], dts[M];
#pragma unroll
        for (int v = 0; v < M; ++v) {
            FL[v] = sh_fx[iy][ix][q][v];
            FR[v] = sh_fx[iy][ix + 1][q][v];
            GB[v] = sh_gy[iy][ix][p][v];
            GT[v] = sh_gy[iy + 1][ix][p][v];
            unew[v] = uhp[v] - rdt * idx * (FR[v] * a.R.bR[p] - FL[v] * a.R.bL[p])
                    - rdt * idy * (GT[v] * a.R.bR[q] - GB[v] * a.R.bL[q]);
            dts[v] = a.dtS ? a.dtS[(size_t)v * nes * np + gi] : (real)0;
        }
        update_finish<Eq, N, real, EB>(a, e, le, k, in, unew, FL, FR, GB, GT, dts, vblock);
    }
}

// faces on tile edges (x: face lines i = 0, TX, 2 TX, ... and nx of every
// row; y: j = 0, TY, ... and ny of every column), one lane per face point,
// with the boundary conditions of k_face
template <class Eq, int N, class real, int D>
__global__ void __launch_bounds__(256) k_tile_face(const StepArgs<real> a)
{
    using TG = TGeo<Eq::DIM, N, (int)sizeof(real)>;
    constexpr int nd = TG::nd, nq = TG::nq;
    const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
    int eL, eR, exL, eyL, exR, eyR, t;
    size_t outi;
    if (D == 0) {
        const int nlx = (a.nx + TG::TX - 1) / TG::TX + 1;
        if (tid >= (unsigned)a.ny * (unsigned)nlx * nq) return;
        t = (int)(tid % nq);
        const unsigned line = tid / nq;
        const int li = (int)(line % (unsigned)nlx), ey = (int)(line / (unsigned)nlx);
        const int i = li * TG::TX < a.nx ? li * TG::TX : a.nx;
        eL = i > 0 ? ey * a.nx + i - 1 : (a.bc[0] == BC_PERIODIC ? ey * a.nx + a.nx - 1 : -1);
        eR = i < a.nx ? ey * a.nx + i : (a.bc[1] == BC_PERIODIC ? ey * a.nx : -1);
        exL = i > 0 ? i - 1 : a.nx - 1; eyL = ey;
        exR = i < a.nx ? i : 0; eyR = ey;
        outi = ((size_t)ey * (a.nx + 1) + i) * nq + t;
    } else {
        const int nly = (a.ny + TG::TY - 1) / TG::TY + 1;
        if (tid >= (unsigned)nly * (unsigned)a.nx * nd) return;
        t = (int)(tid % nd);
        const unsigned line = tid / nd;
        const int ex = (int)(line % (unsigned)a.nx), lj = (int)(line / (unsigned)a.nx);
        const int j = lj * TG::TY < a.ny ? lj * TG::TY : a.ny;
        eL = j > 0 ? (j - 1) * a.nx + ex : (a.bc[2] == BC_PERIODIC ? (a.ny - 1) * a.nx + ex : -1);
        eR = j < a.ny ? j * a.nx + ex : (a.bc[3] == BC_PERIODIC ? ex : -1);
        exL = ex; eyL = j > 0 ? j - 1 : a.ny - 1;
        exR = ex; eyR = j < a.ny ? j : 0;
        outi = ((size_t)j * a.nx + ex) * nd + t;
    }
    if (eL >= 0 && eR >= 0) face_point<Eq, N, real, false, D, true>(a, t, eL, eR, exL, eyL, exR, eyR, outi, false);
    else face_point<Eq, N, real, false, D, false>(a, t, eL, eR, exL, eyL, exR, eyR, outi, false);
}

// ----------------------------------------------------------------------------
// batched kernels: persistent workgroups walk a table of (instance, block)
// work items of one phase over every instance of one degree; each instance's
// arguments are read from device memory (block-uniform, scalar loads)
// ----------------------------------------------------------------------------
enum { BPH_LOCAL = 0, BPH_FACE_X = 1, BPH_FACE_Y = 2, BPH_UPDATE = 3, BPH_UPDATE_FU = 4 };

template <class Eq, int N, class real, bool LIM, int PH>
__device__ __forceinline__ void batch_item(const StepArgs<real>& a, int block)
{
    if constexpr (PH == BPH_LOCAL) local_body<Eq, N, real, LIM>(a, block);
    else if constexpr (PH == BPH_FACE_X) face_body<Eq, N, real, LIM, 0>(a, block);
    else if constexpr (PH == BPH_FACE_Y) face_body<Eq, N, real, LIM, 1>(a, block);
    else if constexpr (PH == BPH_UPDATE_FU) update_body<Eq, N, real, LIM, true>(a, block);
    else update_body<Eq, N, real, LIM>(a, block);
}

// an instance's arguments in the table.  The local and face phases read them
// through the constant address space (the table does not change during a
// launch): the pointers loaded from there are known to address global memory,
// so their accesses compile to global, not flat, memory instructions (flat
// loads also count against the LDS wait counter; 13 % off the limited FP32
// local phase).  The update phase keeps the generic reads: compiled with
// global accesses it held 104 instead of 90 VGPRs (four instead of five
// wavefronts per SIMD) and ran 10 % slower when no element is troubled.
template <class real, int PH>
__device__ __forceinline__ const StepArgs<real>& table_args(const StepArgs<real>* args, int i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (PH != BPH_UPDATE && PH != BPH_UPDATE_FU) {
        using CArgs = const __attribute__((address_space(4))) StepArgs<real>;
        return ((CArgs*)args)[i];
    }
#endif
    return args[i];
}

// one workgroup per (instance, block) work item.  The limited FP32 update of
// 16-point 2D Euler elements is held to six wavefronts per SIMD (80 VGPRs, a
// few registers spilled in the troubled-element path): 10 % faster when few
// elements are troubled, 6 % slower when most are.  The other phases and
// configurations keep the compiler's choice (the six-variable ten-moment
// update would spill some 80 registers).
template <class Eq, int N, class real, bool LIM, int PH>
constexpr int batch_min_waves()
{
    if constexpr (PH == BPH_LOCAL) return local_min_waves<Eq, N, real, LIM>();
    return PH == BPH_UPDATE && LIM && sizeof(real) == 4 && Eq::M == 4 && Geo<Eq::DIM, N>::np == 16 ? 6 : 1;
}

template <class Eq, int N, class real, bool LIM, int PH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(batch_min_waves<Eq, N, real, LIM, PH>())))
k_batch(const StepArgs<real>* __restrict__ args, const int2* __restrict__ work, int nwork)
{
    if ((int)blockIdx.x >= nwork) return;
    const int2 it = work[PH == BPH_LOCAL || PH == BPH_UPDATE_FU ? xcd_block(blockIdx.x, nwork) : (int)blockIdx.x];
    batch_item<Eq, N, real, LIM, PH>(table_args<real, PH>(args, it.x), it.y);
}

// persistent workgroups walking the work table (the loop keeps more values
// live than one item per workgroup does, so the autotuner weighs both)
template <class Eq, int N, class real, bool LIM, int PH>
__global__ void __launch_bounds__(256) k_batch_persistent(const StepArgs<real>* __restrict__ args,
                                                           const int2* __restrict__ work, int nwork)
{
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 it = work[PH == BPH_LOCAL || PH == BPH_UPDATE_FU ? xcd_block(w, nwork) : w];
        batch_item<Eq, N, real, LIM, PH>(table_args<real, PH>(args, it.x), it.y);
        __syncthreads();   // LDS of this work item is reused by the next
    }
}

// ----------------------------------------------------------------------------
// small kernels
// ----------------------------------------------------------------------------
struct PrepArgs {
    double* dt_dev;
    double* t_dev;
    double t_end;
    double dt_fixed;
    double cfl_cs;
    unsigned long long* rate_bits;
    unsigned long long* diag;
    long long* steps;
};

// time step of eq. time.step.2d from the rate of the current means, last
// step clipped; one workgroup of RATE_SLOTS lanes reduces and clears the slots
__device__ __forceinline__ void prep_body(const PrepArgs& a)
{
    __shared__ double sh[RATE_SLOTS / 64];
    const int t = threadIdx.x;
    double r = __longlong_as_double((long long)a.rate_bits[t]);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        double y = __shfl_xor(r, m, 64);
        r = y > r ? y : r;
    }
    if ((t & 63) == 0) sh[t / 64] = r;
    __syncthreads();
    a.rate_bits[t] = 0ull;
    if (t != 0) return;
    double rate = 0.0;
    for (int w = 0; w < RATE_SLOTS / 64; ++w) rate = sh[w] > rate ? sh[w] : rate;
    double dt = a.dt_fixed > 0.0 ? a.dt_fixed : a.cfl_cs / rate;
    double tt = *a.t_dev;
    if (a.t_end > 0.0 && tt + dt > a.t_end) dt = a.t_end - tt;
    if (dt < 0.0) dt = 0.0;
    *a.dt_dev = dt;
    a.t_dev[1] = tt;   // t^n of this step (inflow data)
    *a.t_dev = tt + dt;
    for (int i = 0; i < D_THFLUX; ++i) a.diag[i] = 0ull;
    a.diag[D_THFLUX] = (unsigned long long)__double_as_longlong(1.0);
    a.diag[D_THSCALE] = (unsigned long long)__double_as_longlong(1.0);
    if (dt > 0.0) *a.steps += 1;   // steps past the end time (dt = 0) do not count
}

[[maybe_unused]] static __global__ void __launch_bounds__(RATE_SLOTS) k_prep(PrepArgs a) { prep_body(a); }

// one workgroup per instance of a batch
[[maybe_unused]] static __global__ void __launch_bounds__(RATE_SLOTS) k_prep_batch(const PrepArgs* __restrict__ arr)
{
    prep_body(arr[blockIdx.x]);
}

// ----------------------------------------------------------------------------
// state import / export, ghost states
// ----------------------------------------------------------------------------
template <class real>
struct IoArgs {
    int nx, ny, ne;
    double dx, dy;
    int bc[4];
    const double* uin;     // FP64 nodal input  [var][e][k]
    double* uout;          // FP64 nodal output [var][e][k]
    double* means_out;     // FP64 means [var][e]
    double* ubar;          // MP32 means of the state
    real* u;               // FP64 nodal state / MP32 deviations
    real* ghost;
    Phys phys;
    RefTab<real> R;
    double w64[MAXND];
    double l0_64[MAXND], l1_64[MAXND];
    unsigned long long* diag;
    unsigned long long* rate_bits;
    double* stats;         // k_stats: per-block partial results [block][STAT_N]
};

// per-block partial results of k_stats: minima of the density (u for scalar
// equations) and of P_1, P_2 over the nodes, the number of nodes with a
// non-finite variable, and the block's share of the integral of the density
enum { STAT_MINRHO = 0, STAT_MINP1, STAT_MINP2, STAT_NONFINITE, STAT_MASS, STAT_N };

// import an FP64 nodal state: admissibility check, MP32 split into FP64
// means + FP32 deviations, rate of eq. time.step.2d; one lane per node
template <class Eq, int N, class real>
__global__ void __launch_bounds__(256) k_import(const IoArgs<real> a)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int M = Eq::M, DIM = Eq::DIM, nd = G::nd, np = G::np, EB = G::EB;
    __shared__ double sh[EB][np];
    __shared__ double shm[EB][M];
    const int le = threadIdx.x / np, k = threadIdx.x - le * np;
    const int p = k % nd, q = k / nd;
    const int e0 = blockIdx.x * EB + le;
    const bool act = e0 < a.ne;
    const int e = act ? e0 : a.ne - 1;
    const size_t nes = (size_t)a.ne, gi = (size_t)e * np + k;
    double u[M];
#pragma unroll
    for (int v = 0; v < M; ++v) u[v] = a.uin[(size_t)v * nes * np + gi];
    bool bad = false;
#pragma unroll
    for (int kk = 0; kk < Eq::K; ++kk)
        if (!bad && !(Eq::adm(kk, u, a.phys) > 0.0)) bad = true;
    if (bad && act) atomicAdd(&a.diag[D_MEANBAD], 1ull);
    const double wk = a.w64[p] * (DIM == 2 ? a.w64[q] : 1.0);
    double m[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
        sh[le][k] = wk * u[v];
        __syncthreads();
        if (k == 0) {
            double s = 0.0;
            for (int kk = 0; kk < np; ++kk) s += sh[le][kk];
            shm[le][v] = s;
        }
        __syncthreads();
        m[v] = shm[le][v];
    }
    if (act) {
#pragma unroll
        for (int v = 0; v < M; ++v) {
            if constexpr (is_mp<real>()) a.u[(size_t)v * nes * np + gi] = (real)(u[v] - m[v]);
            else if ((const void*)a.uin != (const void*)a.u) a.u[(size_t)v * nes * np + gi] = (real)u[v];
        }
        if (k == 0) {
            if constexpr (is_mp<real>()) {
#pragma unroll
                for (int v = 0; v < M; ++v) a.ubar[(size_t)v * nes + e] = m[v];
            }
            real ur[M];
#pragma unroll
            for (int v = 0; v < M; ++v) ur[v] = (real)m[v];
            double rate = (double)Eq::sx(ur, a.phys) / a.dx + (DIM == 2 ? (double)Eq::sy(ur, a.phys) / a.dy : 0.0);
            if (!(rate == rate)) rate = 1e300;
            atomic_max_pos(&a.rate_bits[e % RATE_SLOTS], rate);
        }
    }
}

// export the nodal state in FP64 and the FP64 element means
template <class Eq, int N, class real>
__global__ void __launch_bounds__(256) k_export(const IoArgs<real> a)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int M = Eq::M, DIM = Eq::DIM, nd = G::nd, np = G::np, EB = G::EB;
    __shared__ double sh[EB][np];
    const int le = threadIdx.x / np, k = threadIdx.x - le * np;
    const int p = k % nd, q = k / nd;
    const int e0 = blockIdx.x * EB + le;
    const bool act = e0 < a.ne;
    const int e = act ? e0 : a.ne - 1;
    const size_t nes = (size_t)a.ne, gi = (size_t)e * np + k;
    const double wk = a.w64[p] * (DIM == 2 ? a.w64[q] : 1.0);
#pragma unroll
    for (int v = 0; v < M; ++v) {
        double val = (double)a.u[(size_t)v * nes * np + gi];
        if constexpr (is_mp<real>()) val += a.ubar[(size_t)v * nes + e];
        if (act && a.uout) a.uout[(size_t)v * nes * np + gi] = val;
        if (a.means_out) {
            if constexpr (is_mp<real>()) {
                // MP32 state: the FP64 mean is held exactly, deviations have zero mean
                if (k == 0 && act) a.means_out[(size_t)v * nes + e] = a.ubar[(size_t)v * nes + e];
            } else {
                sh[le][k] = wk * val;
                __syncthreads();
                if (k == 0 && act) {
                    double s = 0.0;
                    for (int kk = 0; kk < np; ++kk) s += sh[le][kk];
                    a.means_out[(size_t)v * nes + e] = s;
                }
                __syncthreads();
            }
        }
    }
}

// statistics of the current state for the diagnostics (eq. uad.form at the
// nodes, the integral of the density), one lane per node; each block writes
// its partial results (tree reductions in a fixed order: deterministic)
template <class Eq, int N, class real>
__global__ void __launch_bounds__(256) k_stats(const IoArgs<real> a)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int M = Eq::M, DIM = Eq::DIM, nd = G::nd, np = G::np, EB = G::EB, BL = G::BLOCK, K = Eq::K;
    __shared__ double sh[STAT_N][BL];
    const int le = threadIdx.x / np, k = threadIdx.x - le * np;
    const int p = k % nd, q = k / nd;
    const int e0 = blockIdx.x * EB + le;
    const bool act = e0 < a.ne;
    const int e = act ? e0 : a.ne - 1;
    const size_t nes = (size_t)a.ne, gi = (size_t)e * np + k;
    double u[M];
    bool fin = true;
#pragma unroll
    for (int v = 0; v < M; ++v) {
        double val = (double)a.u[(size_t)v * nes * np + gi];
        if constexpr (is_mp<real>()) val += a.ubar[(size_t)v * nes + e];
        u[v] = val;
        fin = fin && isfinite(val);
    }
    const double big = 1.79769313486231570e308;
    const double area = a.dx * (DIM == 2 ? a.dy : 1.0);
    double mass;
    if constexpr (is_mp<real>()) mass = k == 0 ? a.ubar[e] * area : 0.0;   // the FP64 mean is held exactly
    else mass = a.w64[p] * (DIM == 2 ? a.w64[q] : 1.0) * u[0] * area;
    sh[STAT_MINRHO][threadIdx.x] = act ? u[0] : big;
    sh[STAT_MINP1][threadIdx.x] = act && K > 1 ? Eq::adm(1 < K ? 1 : 0, u, a.phys) : big;
    sh[STAT_MINP2][threadIdx.x] = act && K > 2 ? Eq::adm(2 < K ? 2 : 0, u, a.phys) : big;
    sh[STAT_NONFINITE][threadIdx.x] = act && !fin ? 1.0 : 0.0;
    sh[STAT_MASS][threadIdx.x] = act ? mass : 0.0;
    __syncthreads();
    for (int w = 1; w < BL; w <<= 1) {
        if ((threadIdx.x & (2 * w - 1)) == 0 && threadIdx.x + w < BL) {
#pragma unroll
            for (int j = 0; j < STAT_N; ++j) {
                const double x = sh[j][threadIdx.x], y = sh[j][threadIdx.x + w];
                sh[j][threadIdx.x] = j < STAT_NONFINITE ? (y < x ? y : x) : x + y;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < STAT_N; ++j) a.stats[(size_t)blockIdx.x * STAT_N + j] = sh[j][0];
    }
}

// far-field ghost states: traces of the state at every boundary face point
template <class Eq, int N, class real>
__global__ void k_ghost(const IoArgs<real> a)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int M = Eq::M, nd = G::nd, nq = G::nq, np = G::np;
    const int nx_pts = a.ny * nq, ny_pts = Eq::DIM == 2 ? a.nx * nd : 1;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 2 * nx_pts + (Eq::DIM == 2 ? 2 * ny_pts : 0)) return;
    const size_t nes = (size_t)a.ne;
    int e, dir, side, t;
    if (tid < 2 * nx_pts) {
        dir = 0; side = tid / nx_pts;
        int r = tid % nx_pts, ey = r / nq;
        t = r % nq;
        e = ey * a.nx + (side ? a.nx - 1 : 0);
    } else {
        int r0 = tid - 2 * nx_pts;
        dir = 1; side = r0 / ny_pts;
        int r = r0 % ny_pts, ex = r / nd;
        t = r % nd;
        e = (side ? a.ny - 1 : 0) * a.nx + ex;
    }
    const double* lw = side ? a.l1_64 : a.l0_64;
#pragma unroll
    for (int v = 0; v < M; ++v) {
        double s = 0.0;
        for (int j = 0; j < nd; ++j) {
            int k = dir == 0 ? t * nd + j : j * nd + t;
            double val = (double)a.u[((size_t)v * nes + e) * np + k];
            if constexpr (is_mp<real>()) val += a.ubar[(size_t)v * nes + e];
            s += lw[j] * val;
        }
        a.ghost[(size_t)tid * M + v] = (real)s;
    }
}

// features of the learned indicator and the smoothness indicator's alpha
// for the current state (the quantities the next step's indicator uses);
// one lane per node: feat_out[e][N] and alpha_judge[e]
template <class Eq, int N, class real>
__global__ void __launch_bounds__(256) k_features(const StepArgs<real> a)
{
    using G = Geo<Eq::DIM, N>;
    constexpr int DIM = Eq::DIM, nd = G::nd, np = G::np, EB = G::EB;
    __shared__ real sh_e[EB][np];
    __shared__ real sh_m2[EB][np];
    const int le = threadIdx.x / np, k = threadIdx.x - le * np;
    const int p = k % nd, q = k / nd;
    const int e0 = blockIdx.x * EB + le;
    const bool act = e0 < a.ne;
    const int e = act ? e0 : a.ne - 1;
    real un[Eq::M];
    load_node<Eq>(a, np, e, k, un);
    sh_e[le][k] = Eq::ind(un, a.phys);
    __syncthreads();
    real m = modal_coeff<DIM, N>(a.R, p, q, &sh_e[le][0], 1, nd);
    sh_m2[le][k] = m * m;
    __syncthreads();
    if (k == 0 && act) {
        real en[nd], ft[N];
        shell_energies<DIM, N>(&sh_m2[le][0], 1, nd, en);
        a.alpha_judge[e] = indicator_alpha<N>(en, a.alpha_min, a.alpha_max, a.ind_T, a.ind_kT);
        learned_features<N>(en, ft);
#pragma unroll
        for (int j = 0; j < N; ++j) a.feat_out[(size_t)e * N + j] = (float)ft[j];
    }
}

}  // namespace crkfr
