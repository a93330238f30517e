"""ctypes marshalling for the FP64 CPU oracle (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

LINADV1D, EULER1D, EULER2D, TENMOM2D, BURGERS1D, TENMOM1D = 0, 1, 2, 3, 4, 5
DISS_D2, DISS_D1, DISS_DCSX = 0, 1, 2
CENTRAL_EA, CENTRAL_AE = 0, 1
POINTS_GL, POINTS_GLL = 0, 1
PERIODIC, OUTFLOW, FARFIELD, REFLECT, INFLOW = 0, 1, 2, 3, 4
BLEND_OFF, BLEND_FO, BLEND_MH = 0, 1, 2
IND_PAPER, IND_CONST, IND_GIVEN, IND_LEARNED = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crkfr_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")


def build(force=True):
    """Compile the oracle with gcc: -O3, OpenMP, no fast-math."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
               "-Wall", "-Wno-unused-function", "-o", _SO, _SRC, "-lm"]
        subprocess.check_call(cmd)
    return _SO


class RefConfig(ctypes.Structure):
    _fields_ = [
        ("eq", ctypes.c_int), ("N", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("stages", ctypes.c_int), ("bc", ctypes.c_int * 4),
        ("blend", ctypes.c_int), ("indicator", ctypes.c_int), ("smooth_nbr", ctypes.c_int),
        ("flux_limiter", ctypes.c_int), ("scaling", ctypes.c_int), ("source", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("adv", ctypes.c_double), ("cfl", ctypes.c_double), ("cs", ctypes.c_double),
        ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double), ("alpha_const", ctypes.c_double),
        ("src_amp", ctypes.c_double), ("src_kappa", ctypes.c_double),
        ("src_xc", ctypes.c_double), ("src_yc", ctypes.c_double),
        ("src_gx", ctypes.c_double), ("src_gy", ctypes.c_double),
        ("mlp_nl", ctypes.c_int), ("mlp_dims", ctypes.POINTER(ctypes.c_int)),
        ("mlp_params", ctypes.POINTER(ctypes.c_double)),
        ("mlp_lo", ctypes.POINTER(ctypes.c_double)), ("mlp_hi", ctypes.POINTER(ctypes.c_double)),
        ("dissipation", ctypes.c_int), ("central", ctypes.c_int), ("points", ctypes.c_int),
        ("inflow", ctypes.POINTER(ctypes.c_double)), ("inflow_ncoef", ctypes.c_int),
        ("inflow_tref", ctypes.c_double), ("time", ctypes.c_double),
        ("eps_rel", ctypes.c_double), ("eps_abs", ctypes.c_double),
    ]

    @staticmethod
    def make(eq, N, nx, ny=1, *, stages=None, bc=(PERIODIC,) * 4, blend=BLEND_OFF,
             indicator=IND_PAPER, smooth_nbr=1, flux_limiter=0, scaling=0, source=0,
             domain=(0.0, 1.0, 0.0, 1.0), gamma=1.4, adv=1.0, cfl=0.0, cs=0.98,
             alpha_min=1e-3, alpha_max=1.0, alpha_const=0.0,
             src=(0.0, 0.0, 0.0, 0.0), src_lin=(0.0, 0.0), mlp=None, dissipation=DISS_D2,
             central=CENTRAL_EA, points=POINTS_GL, eps_rel=0.0, eps_abs=0.0):
        """mlp: (dims, params, lo, hi) of the learned indicator (dims[0] = N)."""
        c = RefConfig()
        c.eq, c.N, c.nx, c.ny = eq, N, nx, ny
        c.stages = stages if stages is not None else min(N + 1, 4)
        for i in range(4):
            c.bc[i] = bc[i]
        c.blend, c.indicator, c.smooth_nbr = blend, indicator, smooth_nbr
        c.flux_limiter, c.scaling, c.source = flux_limiter, scaling, source
        c.x0, c.x1, c.y0, c.y1 = domain
        c.gamma, c.adv, c.cfl, c.cs = gamma, adv, cfl, cs
        c.alpha_min, c.alpha_max, c.alpha_const = alpha_min, alpha_max, alpha_const
        c.src_amp, c.src_kappa, c.src_xc, c.src_yc = src
        c.src_gx, c.src_gy = src_lin
        c.dissipation, c.central, c.points = dissipation, central, points
        c.eps_rel, c.eps_abs = eps_rel, eps_abs
        if mlp is not None:
            c.set_mlp(*mlp)
        return c

    def set_inflow(self, coeffs, t_ref):
        """Inflow boundary data g(tau) = sum_k coeffs[k] (tau - t_ref)^k, each
        coeffs[k] in the layout of the far-field ghost states."""
        keep = _f64(coeffs)
        self._inflow_keep = keep   # the C side only borrows the array
        self.inflow = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.inflow_ncoef = keep.shape[0]
        self.inflow_tref = float(t_ref)

    def set_mlp(self, dims, params, lo, hi):
        keep = (np.ascontiguousarray(dims, dtype=np.int32), _f64(params), _f64(lo), _f64(hi))
        assert keep[0][0] == self.N and keep[2].size == self.N and keep[3].size == self.N
        self._mlp_keep = keep   # the C side only borrows these arrays
        self.mlp_nl = keep[0].size - 1
        self.mlp_dims = keep[0].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        self.mlp_params = keep[1].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.mlp_lo = keep[2].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.mlp_hi = keep[3].ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class RefDiag(ctypes.Structure):
    _fields_ = [
        ("n_troubled", ctypes.c_long), ("n_flux_limited", ctypes.c_long),
        ("n_lo_inadmissible", ctypes.c_long), ("n_slope_limited", ctypes.c_long),
        ("n_hancock_fallback", ctypes.c_long), ("n_scaled", ctypes.c_long),
        ("n_mean_inadmissible", ctypes.c_long),
        ("min_theta_flux", ctypes.c_double), ("min_theta_scale", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(RefConfig)
        L.ref_gl.argtypes = [ctypes.c_int, dp, dp]
        L.ref_gll.argtypes = [ctypes.c_int, dp, dp]
        L.ref_lagrange_at.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp]
        L.ref_diff_matrix.argtypes = [ctypes.c_int, dp, dp]
        L.ref_legendre_orthonormal.argtypes = [ctypes.c_int, dp, dp]
        L.ref_tableau.argtypes = [ctypes.c_int, dp, dp, dp]
        L.ref_nvar.argtypes = [ctypes.c_int]
        L.ref_nadm.argtypes = [ctypes.c_int]
        L.ref_flux.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.ref_sigma.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.ref_adm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        L.ref_adm.restype = ctypes.c_double
        L.ref_local_crk.argtypes = [cp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
        L.ref_indicator_raw.argtypes = [cp, dp, dp]
        L.ref_indicator_raw.restype = ctypes.c_double
        L.ref_scale_element.argtypes = [cp, dp, ctypes.POINTER(ctypes.c_int)]
        L.ref_scale_element.restype = ctypes.c_double
        L.ref_compute_dt.argtypes = [cp, dp]
        L.ref_compute_dt.restype = ctypes.c_double
        L.ref_step.argtypes = [cp, dp, dp, ctypes.c_double, dp, dp, ctypes.POINTER(RefDiag), dp]
        L.ref_boundary_traces.argtypes = [cp, dp, dp]
        L.ref_means.argtypes = [cp, dp, dp]
        L.ref_step_crkfr_form.argtypes = [cp, dp, dp, ctypes.c_double]
        L.ref_lo_factor.argtypes = [cp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double]
        L.ref_lo_factor.restype = ctypes.c_double
        L.ref_flux_limit_face.argtypes = [cp, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp,
                                          ctypes.POINTER(ctypes.c_int)]
        L.ref_flux_limit_face.restype = ctypes.c_double
        L.ref_mh_predict.argtypes = [cp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, dp, dp, dp,
                                     ctypes.POINTER(ctypes.c_int)]
        ip = ctypes.POINTER(ctypes.c_int)
        L.ref_indicator_features.argtypes = [cp, dp, dp]
        L.ref_learned_alpha.argtypes = [cp, dp, ctypes.POINTER(ctypes.c_int)]
        L.ref_learned_alpha.restype = ctypes.c_double
        L.ref_mlp_forward.argtypes = [ctypes.c_int, ip, dp, ctypes.c_int, dp, dp, dp]
        L.ref_mlp_loss_grad.argtypes = [ctypes.c_int, ip, dp, ctypes.c_int, dp, dp, dp]
        L.ref_mlp_loss_grad.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def gl(N):
    xi, w = np.zeros(N + 1), np.zeros(N + 1)
    lib().ref_gl(N, _p(xi), _p(w))
    return xi, w


def gll(N):
    xi, w = np.zeros(N + 1), np.zeros(N + 1)
    lib().ref_gll(N, _p(xi), _p(w))
    return xi, w


def nodes(N, points=0):
    """Solution points and weights on [0, 1]: GL (points = POINTS_GL) or GLL."""
    return gll(N) if points == POINTS_GLL else gl(N)


def lagrange_at(N, xi, x):
    l = np.zeros(N + 1)
    lib().ref_lagrange_at(N, _p(_f64(xi)), float(x), _p(l))
    return l


def diff_matrix(N, xi):
    D = np.zeros((N + 1, N + 1))
    lib().ref_diff_matrix(N, _p(_f64(xi)), _p(D))
    return D


def legendre_orthonormal(N, xi):
    L = np.zeros((N + 1, N + 1))
    lib().ref_legendre_orthonormal(N, _p(_f64(xi)), _p(L))
    return L


def tableau(s):
    a, b, c = np.zeros((4, 4)), np.zeros(4), np.zeros(4)
    lib().ref_tableau(s, _p(a), _p(b), _p(c))
    return a[:s, :s].copy(), b[:s].copy(), c[:s].copy()


def nvar(eq):
    return lib().ref_nvar(eq)


def nadm(eq):
    return lib().ref_nadm(eq)


def flux(eq, u, gamma=1.4, adv=1.0):
    u = _f64(u)
    f, g = np.zeros(6), np.zeros(6)
    lib().ref_flux(eq, gamma, adv, _p(u), _p(f), _p(g))
    M = nvar(eq)
    return f[:M], g[:M]


def sigma(eq, u, gamma=1.4, adv=1.0):
    sx, sy = ctypes.c_double(), ctypes.c_double()
    lib().ref_sigma(eq, gamma, adv, _p(_f64(u)), ctypes.byref(sx), ctypes.byref(sy))
    return sx.value, sy.value


def adm(eq, k, u, gamma=1.4):
    return lib().ref_adm(eq, k, gamma, _p(_f64(u)))


def _is2d(eq):
    return eq in (EULER2D, TENMOM2D)


def _np(cfg):
    nd = cfg.N + 1
    return nd * nd if _is2d(cfg.eq) else nd


def local_crk(cfg, ue, dt, xe0=0.0, ye0=0.0):
    M, npn = nvar(cfg.eq), _np(cfg)
    ue = _f64(ue).reshape(M, npn)
    F, G, U, S = (np.zeros((M, npn)) for _ in range(4))
    lib().ref_local_crk(ctypes.byref(cfg), _p(ue), dt, xe0, ye0, _p(F), _p(G), _p(U), _p(S))
    return F, G, U, S


def indicator_raw(cfg, ue):
    e = np.zeros(cfg.N + 1)
    a = lib().ref_indicator_raw(ctypes.byref(cfg), _p(_f64(ue)), _p(e))
    return a, e


def indicator_features(cfg, ue):
    """Features of the learned indicator of one element (N values)."""
    ue = _f64(ue)
    f = np.zeros(cfg.N)
    lib().ref_indicator_features(ctypes.byref(cfg), _p(ue), _p(f))
    return f


def learned_alpha(cfg, ue):
    """(alpha, fallback) of the learned indicator for one element."""
    ue = _f64(ue)
    fb = ctypes.c_int(0)
    a = lib().ref_learned_alpha(ctypes.byref(cfg), _p(ue), ctypes.byref(fb))
    return a, bool(fb.value)


def lo_factor(cfg, d, t, i, u, dt):
    """dt / (w_i h_d phi_d) of the low-order update of a face-adjacent subcell."""
    return lib().ref_lo_factor(ctypes.byref(cfg), d, t, i, _p(_f64(u)), float(dt))


def flux_limit_face(cfg, F, fLO, dt, A=None, B=None):
    """Flux limiter at one face point.  A, B: (u, adj, S, k) of the subcell
    below / above the face, or None for a missing side.  Returns (F limited,
    theta, bad)."""
    M = nvar(cfg.eq)
    z = np.zeros(M)
    ua, adja, sa, ka = A if A is not None else (z, z, z, 0.0)
    ub, adjb, sb, kb = B if B is not None else (z, z, z, 0.0)
    Fo = _f64(F).copy()
    bad = ctypes.c_int(0)
    th = lib().ref_flux_limit_face(ctypes.byref(cfg), int(A is not None), int(B is not None),
                                   _p(_f64(ua)), _p(_f64(ub)), _p(_f64(adja)), _p(_f64(adjb)),
                                   _p(_f64(sa)), _p(_f64(sb)), float(ka), float(kb), float(dt),
                                   _p(_f64(fLO)), _p(Fo), ctypes.byref(bad))
    return Fo, th, bool(bad.value)


def mh_predict(cfg, u, ex, ey, dt, ghost=None):
    """MUSCL-Hancock predicted face values of element (ex, ey): (xm, xp, ym,
    yp) as [node][var] arrays, and (slope scalings, fallbacks)."""
    M, npn = nvar(cfg.eq), _np(cfg)
    outs = [np.zeros((npn, M)) for _ in range(4)]
    cnt = (ctypes.c_int * 2)()
    gp = _p(_f64(ghost)) if ghost is not None else None
    lib().ref_mh_predict(ctypes.byref(cfg), _p(_f64(u)), ex, ey, float(dt), gp, *[_p(o) for o in outs], cnt)
    return outs, (cnt[0], cnt[1])


def scale_element(cfg, ue):
    ue = _f64(ue).copy()
    bad = ctypes.c_int()
    th = lib().ref_scale_element(ctypes.byref(cfg), _p(ue), ctypes.byref(bad))
    return ue, th, bool(bad.value)


def compute_dt(cfg, u):
    return lib().ref_compute_dt(ctypes.byref(cfg), _p(_f64(u)))


def means(cfg, u):
    M = nvar(cfg.eq)
    ub = np.zeros((M, cfg.ny, cfg.nx))
    lib().ref_means(ctypes.byref(cfg), _p(_f64(u)), _p(ub))
    return ub


def boundary_traces(cfg, u):
    """Ghost states of far-field boundaries: the boundary traces of u."""
    M, nd = nvar(cfg.eq), cfg.N + 1
    nq = nd if _is2d(cfg.eq) else 1
    n = 2 * cfg.ny * nq * M + (2 * cfg.nx * nd * M if _is2d(cfg.eq) else 0)
    g = np.zeros(n)
    lib().ref_boundary_traces(ctypes.byref(cfg), _p(_f64(u)), _p(g))
    return g


def has_farfield(cfg):
    return any(cfg.bc[i] == FARFIELD for i in range(4))


def step(cfg, u, dt, alpha_given=None, ghost=None, t=None):
    """One cRKFR step; returns (u_new, alpha, diag dict, status).  t: the
    time t^n of the step (inflow boundaries)."""
    if t is not None:
        cfg.time = float(t)
    u = _f64(u)
    out = np.empty_like(u)
    ne = cfg.nx * cfg.ny
    alpha = np.zeros(ne)
    ag = _f64(alpha_given).reshape(ne) if alpha_given is not None else np.zeros(ne)
    if has_farfield(cfg) and ghost is None:
        raise ValueError("far-field boundaries need the ghost states (boundary_traces of the initial state)")
    gp = _p(_f64(ghost)) if ghost is not None else None
    d = RefDiag()
    st = lib().ref_step(ctypes.byref(cfg), _p(u), _p(out), float(dt), _p(ag), _p(alpha), ctypes.byref(d), gp)
    return out, alpha, d.as_dict(), st


def step_crkfr_form(cfg, u, dt):
    """One step of the stage form (eq. crkfr); periodic, no limiter."""
    u = _f64(u)
    out = np.empty_like(u)
    lib().ref_step_crkfr_form(ctypes.byref(cfg), _p(u), _p(out), float(dt))
    return out


def mlp_forward(dims, params, x):
    dims_c = (ctypes.c_int * len(dims))(*dims)
    x = _f64(x)
    n = x.shape[0]
    y = np.zeros(n)
    lib().ref_mlp_forward(len(dims) - 1, dims_c, _p(_f64(params)), n, _p(x), _p(y), None)
    return y


def mlp_loss_grad(dims, params, x, target):
    dims_c = (ctypes.c_int * len(dims))(*dims)
    params = _f64(params)
    x = _f64(x)
    g = np.zeros_like(params)
    loss = lib().ref_mlp_loss_grad(len(dims) - 1, dims_c, _p(params), x.shape[0], _p(x),
                                   _p(_f64(target)), _p(g))
    return loss, g
