"""Thin ctypes binding of libcrkfr.so (include/crkfr.h): argument marshalling
only; every step of the scheme runs in the library's HIP kernels.

Arrays may be numpy (host) or torch CUDA tensors (device pointers are passed
through); torch is used only for device memory and streams.
"""
import ctypes
import os

import numpy as np

LINADV1D, EULER1D, EULER2D, TENMOM2D, BURGERS1D, TENMOM1D = 0, 1, 2, 3, 4, 5
DISS_D2, DISS_D1, DISS_DCSX = 0, 1, 2
POINTS_GL, POINTS_GLL = 0, 1
CENTRAL_EA, CENTRAL_AE = 0, 1
PERIODIC, OUTFLOW, FARFIELD, REFLECT, INFLOW = 0, 1, 2, 3, 4
FP64, MP32 = 0, 1
BLEND_OFF, BLEND_FO, BLEND_MH = 0, 1, 2
PATH_SPLIT, PATH_TILE, PATH_FACE_UPDATE, PATH_CHECKER = 0, 1, 2, 3
UPDATE_BLOCK, UPDATE_WAVE = 0, 1
IND_PAPER, IND_CONST, IND_GIVEN, IND_LEARNED = 0, 1, 2, 3
NVAR = {LINADV1D: 1, EULER1D: 3, EULER2D: 4, TENMOM2D: 6, BURGERS1D: 1, TENMOM1D: 6}
EINADMISSIBLE_MEAN = -5

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrkfr.so")


class Config(ctypes.Structure):
    _fields_ = [("equation", ctypes.c_int), ("N", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("bc", ctypes.c_int * 4), ("dtype", ctypes.c_int),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("gamma", ctypes.c_double), ("adv", ctypes.c_double), ("cfl", ctypes.c_double), ("cs", ctypes.c_double),
                ("points", ctypes.c_int)]


class LimiterOpts(ctypes.Structure):
    _fields_ = [("blend", ctypes.c_int), ("indicator", ctypes.c_int), ("smooth_nbr", ctypes.c_int),
                ("flux_limiter", ctypes.c_int), ("scaling", ctypes.c_int),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double), ("alpha_const", ctypes.c_double),
                ("eps_rel", ctypes.c_double), ("eps_abs", ctypes.c_double)]


class Scheme(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int), ("dissipation", ctypes.c_int), ("central", ctypes.c_int)]


class Source(ctypes.Structure):
    _fields_ = [("enabled", ctypes.c_int), ("amp", ctypes.c_double), ("kappa", ctypes.c_double),
                ("xc", ctypes.c_double), ("yc", ctypes.c_double), ("gx", ctypes.c_double), ("gy", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int), ("from_cache", ctypes.c_int), ("ms", ctypes.c_float * 4),
                ("update_shape", ctypes.c_int)]


class Diag(ctypes.Structure):
    _fields_ = [("n_troubled", ctypes.c_longlong), ("n_flux_limited", ctypes.c_longlong),
                ("n_lo_inadmissible", ctypes.c_longlong), ("n_slope_limited", ctypes.c_longlong),
                ("n_hancock_fallback", ctypes.c_longlong), ("n_scaled", ctypes.c_longlong),
                ("n_mean_inadmissible", ctypes.c_longlong),
                ("min_theta_flux", ctypes.c_double), ("min_theta_scale", ctypes.c_double),
                ("t", ctypes.c_double), ("dt", ctypes.c_double), ("steps", ctypes.c_longlong),
                ("n_learned_fallback", ctypes.c_longlong), ("n_learned_disagree", ctypes.c_longlong),
                ("max_alpha_dev", ctypes.c_double), ("min_rho", ctypes.c_double), ("min_p", ctypes.c_double),
                ("min_p2", ctypes.c_double), ("n_nonfinite", ctypes.c_longlong), ("mass", ctypes.c_double),
                ("mass_drift", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SYMBOLS = ["crkfr_create", "crkfr_destroy", "crkfr_set_limiter", "crkfr_set_source", "crkfr_set_state",
           "crkfr_set_update_shape", "crkfr_update_shape_in_use",
           "crkfr_set_alpha", "crkfr_compute_dt", "crkfr_step", "crkfr_advance", "crkfr_get_state",
           "crkfr_get_means", "crkfr_get_alpha", "crkfr_get_diag", "crkfr_nvar", "crkfr_nodes_per_element",
           "crkfr_cfl_in_use", "crkfr_fourier_cfl", "crkfr_set_timing", "crkfr_get_kernel_times",
           "crkfr_last_error", "crkfr_batch_create", "crkfr_batch_destroy", "crkfr_batch_step",
           "crkfr_batch_advance", "crkfr_batch_sync", "crkfr_batch_num_groups", "crkfr_batch_grid",
           "crkfr_batch_autotune", "crkfr_set_mlp", "crkfr_features", "crkfr_mlp_create", "crkfr_mlp_destroy",
           "crkfr_mlp_num_params", "crkfr_mlp_set_params", "crkfr_mlp_get_params", "crkfr_mlp_set_box",
           "crkfr_mlp_get_box", "crkfr_mlp_fit_box", "crkfr_mlp_forward", "crkfr_mlp_loss_grad",
           "crkfr_mlp_train", "crkfr_batch_set_t_end", "crkfr_batch_set_timing", "crkfr_batch_phase_times",
           "crkfr_set_scheme", "crkfr_set_inflow", "crkfr_bind_state", "crkfr_state_ptr",
           "crkfr_set_path", "crkfr_path_in_use", "crkfr_step_static", "crkfr_autotune"]

_lib = None


def lib():
    """Load libcrkfr.so; fails loudly when the HIP library was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: build it with paper_2502_07517_amd/build.py")
        # torch ships a HIP runtime with the same soname as /opt/rocm's; loading
        # torch first makes the library bind to that one runtime, so device
        # pointers and streams are shared (loading it second would map a
        # second runtime into the process)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.crkfr_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]
        L.crkfr_destroy.argtypes = [vp]
        L.crkfr_destroy.restype = None
        L.crkfr_set_limiter.argtypes = [vp, ctypes.POINTER(LimiterOpts)]
        L.crkfr_set_source.argtypes = [vp, ctypes.POINTER(Source)]
        L.crkfr_set_state.argtypes = [vp, vp, ip]
        L.crkfr_bind_state.argtypes = [vp, vp]
        L.crkfr_set_path.argtypes = [vp, ip]
        L.crkfr_step_static.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(LimiterOpts), vp, vp,
                                        ctypes.c_double, vp]
        L.crkfr_path_in_use.argtypes = [vp]
        L.crkfr_set_update_shape.argtypes = [vp, ip]
        L.crkfr_update_shape_in_use.argtypes = [vp]
        L.crkfr_autotune.argtypes = [vp, ip, ctypes.c_char_p, ctypes.POINTER(TuneResult)]
        L.crkfr_state_ptr.argtypes = [vp, ctypes.POINTER(vp)]
        L.crkfr_set_alpha.argtypes = [vp, vp, ip]
        L.crkfr_compute_dt.argtypes = [vp, dp]
        L.crkfr_step.argtypes = [vp, ctypes.c_double]
        L.crkfr_advance.argtypes = [vp, ctypes.c_double, ip]
        L.crkfr_get_state.argtypes = [vp, vp, ip]
        L.crkfr_get_means.argtypes = [vp, vp]
        L.crkfr_get_alpha.argtypes = [vp, vp]
        L.crkfr_get_diag.argtypes = [vp, ctypes.POINTER(Diag)]
        L.crkfr_nvar.argtypes = [vp]
        L.crkfr_nodes_per_element.argtypes = [vp]
        L.crkfr_cfl_in_use.argtypes = [vp]
        L.crkfr_cfl_in_use.restype = ctypes.c_double
        L.crkfr_fourier_cfl.argtypes = [ip, ip, ip, ip, ip, ctypes.c_double]
        L.crkfr_set_scheme.argtypes = [vp, ctypes.POINTER(Scheme)]
        L.crkfr_set_inflow.argtypes = [vp, ctypes.c_void_p, ip, ctypes.c_double, ip]
        L.crkfr_fourier_cfl.restype = ctypes.c_double
        L.crkfr_set_timing.argtypes = [vp, ip]
        L.crkfr_get_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
        L.crkfr_last_error.restype = ctypes.c_char_p
        L.crkfr_batch_create.argtypes = [ctypes.POINTER(vp), ip, vp, ctypes.POINTER(vp)]
        L.crkfr_batch_destroy.argtypes = [vp]
        L.crkfr_batch_destroy.restype = None
        L.crkfr_batch_step.argtypes = [vp]
        L.crkfr_batch_advance.argtypes = [vp, ip]
        L.crkfr_batch_sync.argtypes = [vp]
        L.crkfr_batch_num_groups.argtypes = [vp]
        L.crkfr_batch_grid.argtypes = [vp, ip, ip, ip]
        L.crkfr_batch_autotune.argtypes = [vp, ip]
        L.crkfr_batch_set_t_end.argtypes = [vp, ctypes.c_double]
        L.crkfr_batch_set_timing.argtypes = [vp, ip]
        L.crkfr_batch_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
        fp = ctypes.POINTER(ctypes.c_float)
        L.crkfr_set_mlp.argtypes = [vp, vp]
        L.crkfr_features.argtypes = [vp, vp, vp, ip]
        L.crkfr_mlp_create.argtypes = [ip, ip, ctypes.c_ulonglong, vp, ctypes.POINTER(vp)]
        L.crkfr_mlp_destroy.argtypes = [vp]
        L.crkfr_mlp_destroy.restype = None
        L.crkfr_mlp_num_params.argtypes = [vp]
        L.crkfr_mlp_set_params.argtypes = [vp, vp, ip]
        L.crkfr_mlp_get_params.argtypes = [vp, vp, ip]
        L.crkfr_mlp_set_box.argtypes = [vp, fp, fp]
        L.crkfr_mlp_get_box.argtypes = [vp, fp, fp]
        L.crkfr_mlp_fit_box.argtypes = [vp, vp, ip, ctypes.c_float]
        L.crkfr_mlp_forward.argtypes = [vp, vp, ip, vp]
        L.crkfr_mlp_loss_grad.argtypes = [vp, vp, vp, ip, dp, fp]
        L.crkfr_mlp_train.argtypes = [vp, vp, vp, ip, ip, ip, ctypes.c_float, fp]
        _lib = L
    return _lib


class CrkfrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"crkfr error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise CrkfrError(rc, lib().crkfr_last_error().decode())
    return rc


def _ptr(a):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr()), int(a.is_cuda)
    return ctypes.c_void_p(a.ctypes.data), 0


def fourier_cfl(N, stages=0, system=1, tol=1e-10, dissipation=DISS_D2, points=POINTS_GL):
    return lib().crkfr_fourier_cfl(N, stages, system, dissipation, points, tol)


def make_config(equation, N, nx, ny=1, *, bc=(PERIODIC,) * 4, dtype=FP64, domain=(0.0, 1.0, 0.0, 1.0),
                gamma=1.4, adv=1.0, cfl=0.0, cs=0.98, points=0):
    c = Config()
    c.equation, c.N, c.nx, c.ny = equation, N, nx, ny
    for i in range(4):
        c.bc[i] = bc[i]
    c.dtype = dtype
    c.x0, c.x1, c.y0, c.y1 = domain
    c.gamma, c.adv, c.cfl, c.cs = gamma, adv, cfl, cs
    c.points = points
    return c


def step_static(cfg, u_in, u_out, dt, limiter=None, stream=None):
    """One FP64 step without device allocation (crkfr_step_static): cfg from
    make_config, u_in and u_out contiguous float64 device tensors, limiter a
    dict of set_limiter's options or None."""
    for t in (u_in, u_out):
        if not hasattr(t, "data_ptr") or not t.is_cuda or not t.is_contiguous():
            raise ValueError("u_in and u_out must be contiguous device tensors")
    o = None
    if limiter is not None:
        d = dict(blend=BLEND_OFF, indicator=IND_PAPER, smooth_nbr=1, flux_limiter=0, scaling=0, alpha_min=1e-3,
                 alpha_max=1.0, alpha_const=0.0, eps_rel=0.0, eps_abs=0.0)
        d.update(limiter)
        o = LimiterOpts(d["blend"], d["indicator"], d["smooth_nbr"], d["flux_limiter"], d["scaling"],
                        d["alpha_min"], d["alpha_max"], d["alpha_const"], d["eps_rel"], d["eps_abs"])
    st = ctypes.c_void_p(stream) if stream is not None else None
    _check(lib().crkfr_step_static(ctypes.byref(cfg), ctypes.byref(o) if o is not None else None,
                                   ctypes.c_void_p(u_in.data_ptr()), ctypes.c_void_p(u_out.data_ptr()),
                                   float(dt), st))


class Solver:
    """One cRKFR solver on the current HIP device (see include/crkfr.h)."""

    def __init__(self, equation, N, nx, ny=1, *, bc=(PERIODIC,) * 4, dtype=FP64,
                 domain=(0.0, 1.0, 0.0, 1.0), gamma=1.4, adv=1.0, cfl=0.0, cs=0.98, points=0, stream=None):
        c = Config()
        c.equation, c.N, c.nx, c.ny = equation, N, nx, ny
        for i in range(4):
            c.bc[i] = bc[i]
        c.dtype = dtype
        c.x0, c.x1, c.y0, c.y1 = domain
        c.gamma, c.adv, c.cfl, c.cs = gamma, adv, cfl, cs
        c.points = points
        self.cfg = c
        self.M = NVAR[equation]
        self.dim = 2 if equation in (EULER2D, TENMOM2D) else 1
        self.np = (N + 1) ** self.dim
        self.ne = nx * ny
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        _check(lib().crkfr_create(ctypes.byref(c), st, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().crkfr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self):
        N1 = self.cfg.N + 1
        if self.dim == 2:
            return (self.M, self.cfg.ny, self.cfg.nx, N1, N1)
        return (self.M, self.cfg.nx, N1)

    def set_limiter(self, blend=BLEND_OFF, indicator=IND_PAPER, smooth_nbr=1, flux_limiter=0, scaling=0,
                    alpha_min=1e-3, alpha_max=1.0, alpha_const=0.0, eps_rel=0.0, eps_abs=0.0):
        o = LimiterOpts(blend, indicator, smooth_nbr, flux_limiter, scaling, alpha_min, alpha_max, alpha_const,
                        eps_rel, eps_abs)
        _check(lib().crkfr_set_limiter(self.h, ctypes.byref(o)))

    def set_scheme(self, stages=0, dissipation=DISS_D2, central=CENTRAL_EA):
        o = Scheme(stages, dissipation, central)
        _check(lib().crkfr_set_scheme(self.h, ctypes.byref(o)))

    def set_inflow(self, coeffs, t_ref):
        """coeffs[k][...]: polynomial coefficients of the inflow data in the
        far-field ghost layout (numpy array or device tensor of float64)."""
        if not hasattr(coeffs, "data_ptr"):
            coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        elif not coeffs.is_contiguous() or coeffs.element_size() != 8 or not coeffs.is_floating_point():
            raise ValueError("coeffs must be a contiguous float64 tensor")
        p, dev = _ptr(coeffs)
        _check(lib().crkfr_set_inflow(self.h, p, int(coeffs.shape[0]), float(t_ref), dev))

    def set_source(self, enabled=1, amp=0.0, kappa=0.0, xc=0.0, yc=0.0, gx=0.0, gy=0.0):
        s = Source(enabled, amp, kappa, xc, yc, gx, gy)
        _check(lib().crkfr_set_source(self.h, ctypes.byref(s)))

    def _check_array(self, u, n):
        if hasattr(u, "data_ptr"):
            import torch
            if u.dtype != torch.float64 or not u.is_contiguous() or u.numel() != n:
                raise ValueError(f"expected a contiguous float64 tensor of {n} values")
            return u
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.size != n:
            raise ValueError(f"expected {n} values, got {u.size}")
        return u

    def set_state(self, u):
        u = self._check_array(u, self.M * self.ne * self.np)
        p, dev = _ptr(u)
        rc = _check(lib().crkfr_set_state(self.h, p, dev))
        self._bound = None
        return rc

    def bind_state(self, u):
        """Bind a contiguous float64 device tensor as the state (no copy; the
        caller keeps it alive, see crkfr_bind_state)."""
        if not hasattr(u, "data_ptr") or not u.is_cuda:
            raise ValueError("bind_state needs a device tensor")
        u = self._check_array(u, self.M * self.ne * self.np)
        self._bound = u
        _check(lib().crkfr_bind_state(self.h, ctypes.c_void_p(u.data_ptr())))

    def set_path(self, path):
        """Kernel path of a step: PATH_SPLIT, PATH_TILE, PATH_FACE_UPDATE or PATH_CHECKER (default with the limiter
        chain off: the checkerboard step where it serves, else face-update; split with it on)."""
        _check(lib().crkfr_set_path(self.h, int(path)))

    def path_in_use(self):
        return lib().crkfr_path_in_use(self.h)

    def set_update_shape(self, shape):
        """Workgroup shape of the update for 16-point elements: UPDATE_BLOCK, UPDATE_WAVE, or -1 for the default
        rule (crkfr_set_update_shape)."""
        _check(lib().crkfr_set_update_shape(self.h, int(shape)))

    def update_shape_in_use(self):
        return lib().crkfr_update_shape_in_use(self.h)

    def autotune(self, steps=5, cache=None):
        """Time the kernel paths that serve this configuration and keep the
        fastest (crkfr_autotune); cache: JSON-lines file of tuned
        configurations.  Returns {"path", "update_shape", "from_cache", "ms_per_step"}."""
        r = TuneResult()
        _check(lib().crkfr_autotune(self.h, int(steps), None if cache is None else str(cache).encode(),
                                    ctypes.byref(r)))
        names = ("split", "tile", "face_update", "checker")
        return {"path": r.path, "update_shape": r.update_shape, "from_cache": bool(r.from_cache),
                "ms_per_step": {names[i]: float(r.ms[i]) for i in range(4) if r.ms[i] > 0}}

    def state_ptr(self):
        """Device address of the current FP64 nodal state."""
        p = ctypes.c_void_p()
        _check(lib().crkfr_state_ptr(self.h, ctypes.byref(p)))
        return p.value

    def set_alpha(self, alpha):
        a = self._check_array(alpha, self.ne)
        p, dev = _ptr(a)
        _check(lib().crkfr_set_alpha(self.h, p, dev))

    def compute_dt(self):
        d = ctypes.c_double()
        _check(lib().crkfr_compute_dt(self.h, ctypes.byref(d)))
        return d.value

    def step(self, dt=0.0):
        _check(lib().crkfr_step(self.h, float(dt)))

    def advance(self, t_end, max_steps):
        _check(lib().crkfr_advance(self.h, float(t_end), int(max_steps)))

    def get_state(self, out=None):
        if out is None:
            out = np.empty(self.shape(), dtype=np.float64)
        elif hasattr(out, "data_ptr"):
            self._check_array(out, self.M * self.ne * self.np)
        elif not (out.dtype == np.float64 and out.flags.c_contiguous and out.size == self.M * self.ne * self.np):
            raise ValueError("out must be a contiguous float64 array of the state's size")
        p, dev = _ptr(out)
        _check(lib().crkfr_get_state(self.h, p, dev))
        return out

    def get_means(self):
        out = np.empty((self.M, self.cfg.ny, self.cfg.nx), dtype=np.float64)
        _check(lib().crkfr_get_means(self.h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def get_alpha(self):
        out = np.empty(self.ne, dtype=np.float64)
        _check(lib().crkfr_get_alpha(self.h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def get_diag(self, check=False):
        d = Diag()
        rc = lib().crkfr_get_diag(self.h, ctypes.byref(d))
        if check:
            _check(rc)
        return d.as_dict(), rc

    def cfl(self):
        return lib().crkfr_cfl_in_use(self.h)

    def set_timing(self, on=True):
        _check(lib().crkfr_set_timing(self.h, int(on)))

    def kernel_times(self):
        ms = (ctypes.c_float * 4)()
        _check(lib().crkfr_get_kernel_times(self.h, ms))
        return list(ms)

    def set_mlp(self, mlp):
        """Borrow a network for the learned indicator (None detaches)."""
        self._mlp = mlp
        _check(lib().crkfr_set_mlp(self.h, mlp.h if mlp is not None else None))

    def features(self, device=False):
        """(features [ne][N] float32, indicator alpha [ne] float64) of the
        current state; torch CUDA tensors when device=True."""
        N = self.cfg.N
        if device:
            import torch
            f = torch.empty((self.ne, N), dtype=torch.float32, device="cuda")
            a = torch.empty(self.ne, dtype=torch.float64, device="cuda")
            _check(lib().crkfr_features(self.h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(a.data_ptr()), 1))
            return f, a
        f = np.empty((self.ne, N), dtype=np.float32)
        a = np.empty(self.ne, dtype=np.float64)
        _check(lib().crkfr_features(self.h, ctypes.c_void_p(f.ctypes.data), ctypes.c_void_p(a.ctypes.data), 0))
        return f, a


def _dev_f32(x, cols=None):
    """A contiguous float32 CUDA tensor (device data of the network calls)."""
    import torch
    t = torch.as_tensor(x)
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        t = t.to(device="cuda", dtype=torch.float32).contiguous()
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError(f"expected rows of {cols} features")
    return t


class Mlp:
    """Network of the learned troubled-cell indicator (see include/crkfr.h)."""

    def __init__(self, n_inputs, hidden=16, seed=0, stream=None):
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        _check(lib().crkfr_mlp_create(int(n_inputs), int(hidden), int(seed), st, ctypes.byref(h)))
        self.h = h
        self.n_inputs, self.hidden = int(n_inputs), int(hidden)
        self.dims = [self.n_inputs, self.hidden, self.hidden, 1]

    def close(self):
        if getattr(self, "h", None):
            lib().crkfr_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self):
        return lib().crkfr_mlp_num_params(self.h)

    def get_params(self):
        out = np.empty(self.num_params(), dtype=np.float32)
        _check(lib().crkfr_mlp_get_params(self.h, ctypes.c_void_p(out.ctypes.data), 0))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.num_params():
            raise ValueError("wrong number of parameters")
        _check(lib().crkfr_mlp_set_params(self.h, ctypes.c_void_p(p.ctypes.data), 0))

    def get_box(self):
        lo = (ctypes.c_float * self.n_inputs)()
        hi = (ctypes.c_float * self.n_inputs)()
        _check(lib().crkfr_mlp_get_box(self.h, lo, hi))
        return np.array(lo, dtype=np.float32), np.array(hi, dtype=np.float32)

    def set_box(self, lo, hi):
        lo = (ctypes.c_float * self.n_inputs)(*[float(v) for v in lo])
        hi = (ctypes.c_float * self.n_inputs)(*[float(v) for v in hi])
        _check(lib().crkfr_mlp_set_box(self.h, lo, hi))

    def fit_box(self, x, margin=0.02):
        x = _dev_f32(x, self.n_inputs)
        _check(lib().crkfr_mlp_fit_box(self.h, ctypes.c_void_p(x.data_ptr()), x.shape[0], float(margin)))
        return self.get_box()

    def forward(self, x):
        import torch
        x = _dev_f32(x, self.n_inputs)
        y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().crkfr_mlp_forward(self.h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                       ctypes.c_void_p(y.data_ptr())))
        torch.cuda.synchronize()
        return y

    def loss_grad(self, x, t):
        x = _dev_f32(x, self.n_inputs)
        t = _dev_f32(t).reshape(-1)
        g = np.empty(self.num_params(), dtype=np.float32)
        loss = ctypes.c_double()
        _check(lib().crkfr_mlp_loss_grad(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                         x.shape[0], ctypes.byref(loss),
                                         g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return loss.value, g

    def train(self, x, t, epochs=20, batch=4096, lr=3e-3):
        x = _dev_f32(x, self.n_inputs)
        t = _dev_f32(t).reshape(-1)
        if t.shape[0] != x.shape[0]:
            raise ValueError("x and t need the same number of rows")
        hist = np.empty(int(epochs), dtype=np.float32)
        _check(lib().crkfr_mlp_train(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                     x.shape[0], int(epochs), int(batch), float(lr),
                                     hist.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return hist


class Batch:
    """Many solvers advanced together (see the batch calls of include/crkfr.h)."""

    def __init__(self, solvers, stream=None):
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        _check(lib().crkfr_batch_create(arr, len(self.solvers), st, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().crkfr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        _check(lib().crkfr_batch_step(self.h))

    def advance(self, steps):
        _check(lib().crkfr_batch_advance(self.h, int(steps)))

    def sync(self):
        _check(lib().crkfr_batch_sync(self.h))

    def set_t_end(self, t_end):
        _check(lib().crkfr_batch_set_t_end(self.h, float(t_end)))

    def set_timing(self, on=True):
        _check(lib().crkfr_batch_set_timing(self.h, int(on)))

    def phase_times(self):
        ms = (ctypes.c_float * 4)()
        _check(lib().crkfr_batch_phase_times(self.h, ms))
        return list(ms)

    def num_groups(self):
        return lib().crkfr_batch_num_groups(self.h)

    def grid(self, group, phase, set_to=-1):
        r = lib().crkfr_batch_grid(self.h, group, phase, set_to)
        if r < 0:
            _check(r)
        return r

    def grids(self):
        return [[self.grid(g, ph) for ph in range(4)] for g in range(self.num_groups())]

    def autotune(self, reps=3):
        _check(lib().crkfr_batch_autotune(self.h, int(reps)))
        return self.grids()
