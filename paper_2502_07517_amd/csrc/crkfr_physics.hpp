// Physics of the cRKFR step for gfx950: fluxes, spectral radii, admissibility
// functions, indicator quantity and the ten-moment source.
//   linear advection            f = a u                         (Sec. 5.1.1)
//   1D / 2D Euler               eqs. 1deuler, state, 2deuler, 2dstate
//   ten-moment system           eq. tmp, source eq. tenmom.source (2D and 1D)
//   Burgers                     f = u^2 / 2                     (Sec. 5.1.3)
// Bulk arithmetic is in `real` (double or float); admissibility functions
// P_k (eq. uad.form) are always evaluated in double.
#pragma once
#include <hip/hip_runtime.h>

namespace crkfr {

struct Phys {
    double gamma, adv;
    int source;
    double amp, kappa, xc, yc, gx, gy;   // W = amp exp(-kappa r^2) + gx x + gy y
};

// reciprocal of the density: v_rcp_f32 (1 ulp for normal numbers) in the FP32
// bulk arithmetic; in FP64 the hardware estimate refined by two Newton-Raphson
// steps r <- r + r (1 - x r) (each squares the relative error), within about
// one ulp of 1/x for normal x instead of the correctly rounded division
// sequence (the density is positive and normal wherever the flux is used)
template <class real>
__device__ __forceinline__ real recip(real x)
{
    if constexpr (sizeof(real) == 4) {
        return __builtin_amdgcn_rcpf(x);
    } else {
        double r = __builtin_amdgcn_rcp(x);
        r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
        return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    }
}

// trace value, or the face-adjacent node where the trace density is not positive
// (value selection keeps both arrays in registers)
template <int M, class real>
__device__ __forceinline__ void pick_trace(const real* tr, const real* node, real* u)
{
    const bool t = tr[0] > 0;
#pragma unroll
    for (int v = 0; v < M; ++v) u[v] = t ? tr[v] : node[v];
}

// ---------------------------------------------------------------- linear advection
template <class real>
struct LinAdv1D {
    static constexpr int M = 1, DIM = 1, K = 0, ID = 0;
    __device__ static inline void fx(const real* u, real* f, const Phys& P) { f[0] = (real)P.adv * u[0]; }
    __device__ static inline void gy(const real*, real* g, const Phys&) { g[0] = 0; }
    __device__ static inline real sx(const real*, const Phys& P) { return fabs((real)P.adv); }
    __device__ static inline real sy(const real*, const Phys&) { return 0; }
    __device__ static inline double adm(int, const double*, const Phys&) { return 1.0; }
    __device__ static inline bool adm_ge(int, const double*, double eps, const Phys&) { return 1.0 >= eps; }
    __device__ static inline bool concave(int) { return true; }
    __device__ static inline real ind(const real* u, const Phys&) { return u[0]; }
    __device__ static inline real sig_trace(int, const real*, const real*, const Phys& P) { return fabs((real)P.adv); }
    __device__ static inline void src(const real*, real, real, real* s, const Phys&) { s[0] = 0; }
    __device__ static inline void fxy(const real* u, real* f, real* g, const Phys& P) { fx(u, f, P); g[0] = 0; }
};

// ---------------------------------------------------------------- Burgers
template <class real>
struct Burgers1D {
    static constexpr int M = 1, DIM = 1, K = 0, ID = 4;
    __device__ static inline void fx(const real* u, real* f, const Phys&) { f[0] = (real)0.5 * u[0] * u[0]; }
    __device__ static inline void gy(const real*, real* g, const Phys&) { g[0] = 0; }
    __device__ static inline real sx(const real* u, const Phys&) { return fabs(u[0]); }
    __device__ static inline real sy(const real*, const Phys&) { return 0; }
    __device__ static inline double adm(int, const double*, const Phys&) { return 1.0; }
    __device__ static inline bool adm_ge(int, const double*, double eps, const Phys&) { return 1.0 >= eps; }
    __device__ static inline bool concave(int) { return true; }
    __device__ static inline real ind(const real* u, const Phys&) { return u[0]; }
    __device__ static inline real sig_trace(int, const real* tr, const real*, const Phys&) { return fabs(tr[0]); }
    __device__ static inline void src(const real*, real, real, real* s, const Phys&) { s[0] = 0; }
    __device__ static inline void fxy(const real* u, real* f, real* g, const Phys& P) { fx(u, f, P); g[0] = 0; }
};

// ---------------------------------------------------------------- Euler 1D
template <class real>
struct Euler1D {
    static constexpr int M = 3, DIM = 1, K = 2, ID = 1;
    __device__ static inline real pres(const real* u, const Phys& P)
    {
        return ((real)P.gamma - 1) * (u[2] - (real)0.5 * u[1] * u[1] * recip(u[0]));
    }
    __device__ static inline void fx(const real* u, real* f, const Phys& P)
    {
        real v = u[1] * recip(u[0]);
        real p = ((real)P.gamma - 1) * (u[2] - (real)0.5 * u[1] * v);
        f[0] = u[1];
        f[1] = u[1] * v + p;
        f[2] = (u[2] + p) * v;
    }
    __device__ static inline void gy(const real*, real* g, const Phys&) { g[0] = g[1] = g[2] = 0; }
    __device__ static inline real sx(const real* u, const Phys& P)
    {
        real ir = recip(u[0]), v = u[1] * ir;
        real p = ((real)P.gamma - 1) * (u[2] - (real)0.5 * u[1] * v);
        return fabs(v) + sqrt((real)P.gamma * p * ir);
    }
    __device__ static inline real sy(const real*, const Phys&) { return 0; }
    __device__ static inline double adm(int k, const double* u, const Phys& P)
    {
        if (k == 0) return u[0];
        return (P.gamma - 1.0) * (u[2] - 0.5 * u[1] * u[1] / u[0]);
    }
    // adm(k, u) >= eps, for positive density without the division (times rho)
    __device__ static inline bool adm_ge(int k, const double* u, double eps, const Phys& P)
    {
        if (k == 0) return u[0] >= eps;
        if (!(u[0] > 0.0)) return adm(k, u, P) >= eps;
        return (P.gamma - 1.0) * (u[2] * u[0] - 0.5 * u[1] * u[1]) >= eps * u[0];
    }
    __device__ static inline bool concave(int) { return true; }
    // rho p = (gamma - 1) (rho E - m^2 / 2): no division
    __device__ static inline real ind(const real* u, const Phys& P)
    {
        return ((real)P.gamma - 1) * (u[0] * u[2] - (real)0.5 * u[1] * u[1]);
    }
    // trace wave speed: pressure clipped at zero; non-positive density -> node
    __device__ static inline real sig_trace(int, const real* tr, const real* node, const Phys& P)
    {
        real u[M];
        pick_trace<M>(tr, node, u);
        real ir = recip(u[0]), v = u[1] * ir;
        real p = ((real)P.gamma - 1) * (u[2] - (real)0.5 * u[1] * v);
        return fabs(v) + sqrt((real)P.gamma * fmax(p, (real)0) * ir);
    }
    __device__ static inline void src(const real*, real, real, real* s, const Phys&) { s[0] = s[1] = s[2] = 0; }
    __device__ static inline void fxy(const real* u, real* f, real* g, const Phys& P)
    {
        real ir = recip(u[0]), v = u[1] * ir;
        real p = ((real)P.gamma - 1) * (u[2] - (real)0.5 * u[1] * v);
        f[0] = u[1];
        f[1] = u[1] * v + p;
        f[2] = (u[2] + p) * v;
        g[0] = g[1] = g[2] = 0;
    }
};

// ---------------------------------------------------------------- Euler 2D
template <class real>
struct Euler2D {
    static constexpr int M = 4, DIM = 2, K = 2, ID = 2;
    __device__ static inline real pres(const real* u, const Phys& P)
    {
        return ((real)P.gamma - 1) * (u[3] - (real)0.5 * (u[1] * u[1] + u[2] * u[2]) * recip(u[0]));
    }
    // pressure and velocities with one reciprocal of the density
    __device__ static inline real pvv(const real* u, real& v1, real& v2, real& ir, const Phys& P)
    {
        ir = recip(u[0]);
        v1 = u[1] * ir;
        v2 = u[2] * ir;
        return ((real)P.gamma - 1) * (u[3] - (real)0.5 * (u[1] * v1 + u[2] * v2));
    }
    __device__ static inline void fx(const real* u, real* f, const Phys& P)
    {
        real v1, v2, ir, p = pvv(u, v1, v2, ir, P);
        f[0] = u[1];
        f[1] = u[1] * v1 + p;
        f[2] = u[2] * v1;
        f[3] = (u[3] + p) * v1;
    }
    __device__ static inline void gy(const real* u, real* g, const Phys& P)
    {
        real v1, v2, ir, p = pvv(u, v1, v2, ir, P);
        g[0] = u[2];
        g[1] = u[1] * v2;
        g[2] = u[2] * v2 + p;
        g[3] = (u[3] + p) * v2;
    }
    __device__ static inline real sx(const real* u, const Phys& P)
    {
        real v1, v2, ir, p = pvv(u, v1, v2, ir, P);
        return fabs(v1) + sqrt((real)P.gamma * p * ir);
    }
    __device__ static inline real sy(const real* u, const Phys& P)
    {
        real v1, v2, ir, p = pvv(u, v1, v2, ir, P);
        return fabs(v2) + sqrt((real)P.gamma * p * ir);
    }
    // flux and wave speed normal to direction d (0: x, 1: y) without a branch
    // on d (lanes of one wavefront may differ in d): the arithmetic of fx / gy
    // and sx / sy (a product plus zero is the product)
    __device__ static inline void fn(int d, const real* u, real* f, const Phys& P)
    {
        real v1, v2, ir, p = pvv(u, v1, v2, ir, P);
        const bool y = d != 0;
        const real vn = y ? v2 : v1;
        f[0] = y ? u[2] : u[1];
        f[1] = u[1] * vn + (y ? (real)0 : p);
        f[2] = u[2] * vn + (y ? p : (real)0);
        f[3] = (u[3] + p) * vn;
    }
    __device__ static inline real sn(int d, const real* u, const Phys& P)
    {
        real v1, v2, ir, p = pvv(u, v1, v2, ir, P);
        return fabs(d != 0 ? v2 : v1) + sqrt((real)P.gamma * p * ir);
    }
    __device__ static inline double adm(int k, const double* u, const Phys& P)
    {
        if (k == 0) return u[0];
        return (P.gamma - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
    }
    // adm(k, u) >= eps, for positive density without the division (times rho)
    __device__ static inline bool adm_ge(int k, const double* u, double eps, const Phys& P)
    {
        if (k == 0) return u[0] >= eps;
        if (!(u[0] > 0.0)) return adm(k, u, P) >= eps;
        return (P.gamma - 1.0) * (u[3] * u[0] - 0.5 * (u[1] * u[1] + u[2] * u[2])) >= eps * u[0];
    }
    __device__ static inline bool concave(int) { return true; }
    // rho p = (gamma - 1) (rho E - |m|^2 / 2): no division
    __device__ static inline real ind(const real* u, const Phys& P)
    {
        return ((real)P.gamma - 1) * (u[0] * u[3] - (real)0.5 * (u[1] * u[1] + u[2] * u[2]));
    }
    __device__ static inline real sig_trace(int d, const real* tr, const real* node, const Phys& P)
    {
        real u[M];
        pick_trace<M>(tr, node, u);
        real v1, v2, ir, p = pvv(u, v1, v2, ir, P);
        real c = sqrt((real)P.gamma * fmax(p, (real)0) * ir);
        return fabs(d == 0 ? v1 : v2) + c;
    }
    __device__ static inline void src(const real*, real, real, real* s, const Phys&) { s[0] = s[1] = s[2] = s[3] = 0; }
    // both fluxes with one reciprocal of the density
    __device__ static inline void fxy(const real* u, real* f, real* g, const Phys& P)
    {
        real v1, v2, ir, p = pvv(u, v1, v2, ir, P);
        real ep = u[3] + p;
        f[0] = u[1];
        f[1] = u[1] * v1 + p;
        f[2] = u[2] * v1;
        f[3] = ep * v1;
        g[0] = u[2];
        g[1] = u[1] * v2;
        g[2] = u[2] * v2 + p;
        g[3] = ep * v2;
    }
};

// ---------------------------------------------------------------- ten-moment 2D
template <class real>
struct TenMom2D {
    static constexpr int M = 6, DIM = 2, K = 3, ID = 3;
    __device__ static inline void fx(const real* u, real* f, const Phys&)
    {
        real ir = recip(u[0]), v1 = u[1] * ir, v2 = u[2] * ir;
        real P11 = 2 * u[3] - u[1] * v1, P12 = 2 * u[4] - u[1] * v2;
        f[0] = u[1];
        f[1] = P11 + u[1] * v1;
        f[2] = P12 + u[1] * v2;
        f[3] = (u[3] + P11) * v1;
        f[4] = u[4] * v1 + (real)0.5 * (P11 * v2 + P12 * v1);
        f[5] = u[5] * v1 + P12 * v2;
    }
    __device__ static inline void gy(const real* u, real* g, const Phys&)
    {
        real ir = recip(u[0]), v1 = u[1] * ir, v2 = u[2] * ir;
        real P12 = 2 * u[4] - u[1] * v2, P22 = 2 * u[5] - u[2] * v2;
        g[0] = u[2];
        g[1] = P12 + u[1] * v2;
        g[2] = P22 + u[2] * v2;
        g[3] = u[3] * v2 + P12 * v1;
        g[4] = u[4] * v2 + (real)0.5 * (P12 * v2 + P22 * v1);
        g[5] = (u[5] + P22) * v2;
    }
    __device__ static inline real sx(const real* u, const Phys&)
    {
        real ir = recip(u[0]), v1 = u[1] * ir;
        return fabs(v1) + sqrt(3 * (2 * u[3] - u[1] * v1) * ir);
    }
    __device__ static inline real sy(const real* u, const Phys&)
    {
        real ir = recip(u[0]), v2 = u[2] * ir;
        return fabs(v2) + sqrt(3 * (2 * u[5] - u[2] * v2) * ir);
    }
    __device__ static inline double adm(int k, const double* u, const Phys&)
    {
        if (k == 0) return u[0];
        double r = u[0], v1 = u[1] / r, v2 = u[2] / r;
        double P11 = 2.0 * u[3] - r * v1 * v1;
        if (k == 1) return P11;
        double P12 = 2.0 * u[4] - r * v1 * v2, P22 = 2.0 * u[5] - r * v2 * v2;
        return P11 * P22 - P12 * P12;
    }
    // adm(k, u) >= eps, for positive density without the divisions (times rho, rho^2)
    __device__ static inline bool adm_ge(int k, const double* u, double eps, const Phys& P)
    {
        if (k == 0) return u[0] >= eps;
        const double r = u[0];
        if (!(r > 0.0)) return adm(k, u, P) >= eps;
        const double a11 = 2.0 * u[3] * r - u[1] * u[1];   // rho P11
        if (k == 1) return a11 >= eps * r;
        const double a12 = 2.0 * u[4] * r - u[1] * u[2], a22 = 2.0 * u[5] * r - u[2] * u[2];
        return a11 * a22 - a12 * a12 >= eps * r * r;
    }
    __device__ static inline bool concave(int k) { return k != 2; }   // det P is not concave
    __device__ static inline real ind(const real* u, const Phys&)
    {
        // rho (P11 + P22) / 2 = rho (E11 + E22) - |rho v|^2 / 2: no division
        return u[0] * (u[3] + u[5]) - (real)0.5 * (u[1] * u[1] + u[2] * u[2]);
    }
    __device__ static inline real sig_trace(int d, const real* tr, const real* node, const Phys&)
    {
        real u[M];
        pick_trace<M>(tr, node, u);
        const real ir = recip(u[0]);
        const real m = d == 0 ? u[1] : u[2], en = d == 0 ? u[3] : u[5];
        const real vn = m * ir;
        return fabs(vn) + sqrt(3 * fmax(2 * en - m * vn, (real)0) * ir);
    }
    __device__ static inline void fxy(const real* u, real* f, real* g, const Phys&)
    {
        real ir = recip(u[0]), v1 = u[1] * ir, v2 = u[2] * ir;
        real P11 = 2 * u[3] - u[1] * v1, P12 = 2 * u[4] - u[1] * v2, P22 = 2 * u[5] - u[2] * v2;
        f[0] = u[1];
        f[1] = P11 + u[1] * v1;
        f[2] = P12 + u[1] * v2;
        f[3] = (u[3] + P11) * v1;
        f[4] = u[4] * v1 + (real)0.5 * (P11 * v2 + P12 * v1);
        f[5] = u[5] * v1 + P12 * v2;
        g[0] = u[2];
        g[1] = f[2];
        g[2] = P22 + u[2] * v2;
        g[3] = u[3] * v2 + P12 * v1;
        g[4] = u[4] * v2 + (real)0.5 * (P12 * v2 + P22 * v1);
        g[5] = (u[5] + P22) * v2;
    }
    // s = s^x + s^y with grad W of W = amp exp(-kappa r^2) + gx x + gy y
    __device__ static inline void src(const real* u, real x, real y, real* s, const Phys& P)
    {
        real dx = x - (real)P.xc, dy = y - (real)P.yc;
        real W = (real)P.amp * exp(-(real)P.kappa * (dx * dx + dy * dy));
        real Wx = -2 * (real)P.kappa * dx * W + (real)P.gx;
        real Wy = -2 * (real)P.kappa * dy * W + (real)P.gy;
        // rho v = the momentum: no division
        s[0] = 0;
        s[1] = (real)-0.5 * u[0] * Wx;
        s[2] = (real)-0.5 * u[0] * Wy;
        s[3] = (real)-0.5 * u[1] * Wx;
        s[4] = (real)-0.25 * u[2] * Wx - (real)0.25 * u[1] * Wy;
        s[5] = (real)-0.5 * u[2] * Wy;
    }
};

// ---------------------------------------------------------------- ten-moment 1D
// The six-variable ten-moment system with x dependence only (eq. tmp with
// g = 0): x flux, x wave speed and the source with W = W(x) (the potential's
// y offset is dropped; the linear y term gy still acts on rho v2, E12, E22).
template <class real>
struct TenMom1D {
    using T2 = TenMom2D<real>;
    static constexpr int M = 6, DIM = 1, K = 3, ID = 5;
    __device__ static inline void fx(const real* u, real* f, const Phys& P) { T2::fx(u, f, P); }
    __device__ static inline void gy(const real*, real* g, const Phys&)
    {
#pragma unroll
        for (int v = 0; v < M; ++v) g[v] = 0;
    }
    __device__ static inline real sx(const real* u, const Phys& P) { return T2::sx(u, P); }
    __device__ static inline real sy(const real*, const Phys&) { return 0; }
    __device__ static inline double adm(int k, const double* u, const Phys& P) { return T2::adm(k, u, P); }
    __device__ static inline bool adm_ge(int k, const double* u, double eps, const Phys& P)
    {
        return T2::adm_ge(k, u, eps, P);
    }
    __device__ static inline bool concave(int k) { return T2::concave(k); }
    __device__ static inline real ind(const real* u, const Phys& P) { return T2::ind(u, P); }
    __device__ static inline real sig_trace(int, const real* tr, const real* node, const Phys& P)
    {
        return T2::sig_trace(0, tr, node, P);
    }
    __device__ static inline void fxy(const real* u, real* f, real* g, const Phys& P)
    {
        T2::fx(u, f, P);
        gy(u, g, P);
    }
    __device__ static inline void src(const real* u, real x, real, real* s, const Phys& P)
    {
        T2::src(u, x, (real)P.yc, s, P);
    }
};

}  // namespace crkfr
