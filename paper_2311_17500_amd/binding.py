"""Thin ctypes binding of libstiga.so (argument marshalling only).

Every computation happens in the HIP library; this module converts Python
arguments into the C structs of include/st_iga.h, passes device pointers of
torch tensors, and turns status codes into exceptions.  There is no fallback:
if the library is missing, ``load`` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstiga.so")

OK, EINVAL, ENOMEM, ENOCONV, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ENOCONV: "ENOCONV", EDEVICE: "EDEVICE", ESTATE: "ESTATE"}

EXPORTS = ["st_iga_default_options", "st_iga_workspace_bytes", "st_iga_setup", "st_iga_linearize",
           "st_iga_set_factors", "st_iga_get_factors", "st_iga_theta_grid", "st_iga_apply", "st_iga_precond",
           "st_iga_residual", "st_iga_w_update", "st_iga_krylov", "st_iga_solve", "st_iga_lift", "st_iga_sizes",
           "st_iga_destroy", "st_iga_last_error", "st_iga_host_query", "st_iga_newton_step", "st_iga_profile",
           "st_iga_profile_read", "st_iga_apply_lowp", "st_iga_precond_lowp", "st_iga_profile_record",
           "st_iga_host_symeig", "st_iga_precond_noalloc", "st_iga_set_stimulus"]


class Problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("p_s", C.c_int32), ("p_t", C.c_int32), ("nknots", C.c_int32 * 4),
                ("knots", C.POINTER(C.c_double) * 4), ("T", C.c_double), ("Cm", C.c_double),
                ("sigma", C.c_double * 3), ("a", C.c_double), ("b", C.c_double), ("c1", C.c_double),
                ("c2", C.c_double), ("de", C.c_double), ("map_kind", C.c_int32 * 3),
                ("map_param", (C.c_double * 3) * 3)]


class Stimulus(C.Structure):
    _fields_ = [("u0_kind", C.c_int32), ("u0_center", C.c_double * 3), ("u0_radius", C.c_double),
                ("u0_value", C.c_double), ("f_kind", C.c_int32), ("f_center", C.c_double * 3),
                ("f_radius", C.c_double), ("f_t0", C.c_double), ("f_t1", C.c_double), ("f_amp", C.c_double),
                ("f_kappa", C.c_double), ("f_velocity", C.c_double * 3)]


class Options(C.Structure):
    _fields_ = [("su", C.c_int32), ("eps_theta", C.c_double), ("eps_react", C.c_double), ("max_rank", C.c_int32),
                ("outer", C.c_int32), ("alpha", C.c_double), ("theta_freeze", C.c_double),
                ("tol_nonlin", C.c_double), ("tol_lin", C.c_double), ("inner_tol", C.c_double),
                ("restart", C.c_int32), ("max_outer", C.c_int32), ("max_krylov", C.c_int32), ("prec", C.c_int32),
                ("lin_forcing", C.c_double), ("coef_slab", C.c_int32), ("reorth", C.c_int32),
                ("graphs", C.c_int32), ("stall_cycles", C.c_int32), ("stall_reduction", C.c_double),
                ("picard_switch", C.c_int32), ("sc_c", C.c_double), ("precond", C.c_int32)]


LOG = 64


class Report(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("krylov_total", C.c_int32), ("refinements", C.c_int32),
                ("krylov", C.c_int32 * LOG), ("rank_theta", C.c_int32 * LOG), ("rank_react", C.c_int32 * LOG),
                ("delta_inf", C.c_double * LOG), ("lin_relres", C.c_double * LOG), ("final_delta_inf", C.c_double),
                ("seconds_linearize", C.c_double), ("seconds_krylov", C.c_double), ("rank_capped", C.c_int32),
                ("lr_relerr_theta", C.c_double * LOG), ("lr_relerr_react", C.c_double * LOG),
                ("switched_at", C.c_int32)]


class StIgaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libstiga.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_2311_17500_amd/build.py")
    lib = C.CDLL(path)
    P, V = C.c_void_p, C.c_void_p
    lib.st_iga_default_options.argtypes = [C.POINTER(Options)]
    lib.st_iga_workspace_bytes.argtypes = [C.POINTER(Problem), C.POINTER(Options)]
    lib.st_iga_workspace_bytes.restype = C.c_size_t
    lib.st_iga_setup.argtypes = [C.POINTER(Problem), C.POINTER(Options), V, C.c_size_t, V, C.POINTER(P)]
    lib.st_iga_linearize.argtypes = [P, V, V, C.c_int32, V]
    lib.st_iga_set_factors.argtypes = [P, C.c_int32, V, V, V, C.c_int32, V, V, V]
    lib.st_iga_get_factors.argtypes = [P, C.POINTER(C.c_int32), V, V, V, C.POINTER(C.c_int32), V, V, V]
    lib.st_iga_theta_grid.argtypes = [P, V, V, V, V]
    lib.st_iga_apply.argtypes = [P, V, V, V]
    lib.st_iga_precond.argtypes = [P, V, V, V]
    lib.st_iga_precond_noalloc.argtypes = [P, V, V, V]
    lib.st_iga_apply_lowp.argtypes = [P, V, V, V]
    lib.st_iga_precond_lowp.argtypes = [P, V, V, V]
    lib.st_iga_residual.argtypes = [P, V, V, V, V]
    lib.st_iga_w_update.argtypes = [P, V, V, V]
    lib.st_iga_krylov.argtypes = [P, V, V, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double), V]
    lib.st_iga_solve.argtypes = [P, C.POINTER(Stimulus), V, V, C.POINTER(Report), V]
    lib.st_iga_lift.argtypes = [P, C.POINTER(Stimulus), V, C.POINTER(C.c_int64)]
    lib.st_iga_set_stimulus.argtypes = [P, C.POINTER(Stimulus)]
    lib.st_iga_sizes.argtypes = [P, C.POINTER(C.c_int64)]
    lib.st_iga_destroy.argtypes = [P]
    lib.st_iga_last_error.argtypes = [P]
    lib.st_iga_last_error.restype = C.c_char_p
    lib.st_iga_newton_step.argtypes = [P, V, V, V, C.c_int32, C.c_double, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double), V]
    lib.st_iga_profile.argtypes = [P, C.c_int32]
    lib.st_iga_profile_read.argtypes = [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32]
    lib.st_iga_profile_record.argtypes = [P, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.st_iga_host_query.argtypes = [C.POINTER(Problem), C.c_int32, C.c_int32, V, C.c_int64, C.POINTER(C.c_int64)]
    lib.st_iga_host_symeig.argtypes = [C.c_int32, V, V, V]
    for name in EXPORTS:
        if name not in ("st_iga_default_options", "st_iga_workspace_bytes", "st_iga_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_problem(prob, knots=None):
    """ctypes Problem (plus the arrays it points to) from a workload description."""
    kn = knots if knots is not None else prob.uniform_knots()
    arrs = [np.ascontiguousarray(k, dtype=np.float64) for k in kn]
    P = Problem()
    P.d, P.p_s, P.p_t = prob.d, prob.p_s, prob.p_t
    for l, a in enumerate(arrs):
        P.nknots[l] = len(a)
        P.knots[l] = a.ctypes.data_as(C.POINTER(C.c_double))
    P.T, P.Cm = prob.T, prob.Cm
    for l, s in enumerate(prob.sigma):
        P.sigma[l] = s
    P.a, P.b, P.c1, P.c2, P.de = prob.a, prob.b, prob.c1, prob.c2, prob.de
    mk = getattr(prob, "map_kind", (0, 0, 0))
    mp = getattr(prob, "map_param", ((0.0, 1.0, 0.0),) * 3)
    for l in range(3):
        P.map_kind[l] = int(mk[l]) if l < len(mk) else 0
        for j in range(3):
            P.map_param[l][j] = float(mp[l][j]) if l < len(mp) else (0.0, 1.0, 0.0)[j]
    return P, arrs


def make_stimulus(prob):
    S = Stimulus()
    S.u0_kind = prob.u0_kind
    for l in range(3):
        S.u0_center[l] = prob.u0_center[l] if l < len(prob.u0_center) else 0.0
    S.u0_radius, S.u0_value = prob.u0_radius, prob.u0_value
    S.f_kind = int(getattr(prob, "f_kind", 0))
    if S.f_kind:
        for l in range(3):
            S.f_center[l] = prob.f_center[l] if l < len(prob.f_center) else 0.0
            S.f_velocity[l] = prob.f_velocity[l] if l < len(prob.f_velocity) else 0.0
        S.f_radius, S.f_t0, S.f_t1 = prob.f_radius, prob.f_t0, prob.f_t1
        S.f_amp, S.f_kappa = prob.f_amp, prob.f_kappa
    return S


def default_options(**kw):
    lib = load()
    O = Options()
    lib.st_iga_default_options(C.byref(O))
    for k, v in kw.items():
        setattr(O, k, v)
    return O


def workspace_bytes(prob, knots=None, **options) -> int:
    """Device workspace one context of this problem needs (host-only call)."""
    lib = load()
    P, keep = make_problem(prob, knots)
    O = default_options(**options)
    return int(lib.st_iga_workspace_bytes(C.byref(P), C.byref(O)))


def host_query(prob, what: int, direction: int, knots=None) -> np.ndarray:
    """Host-only setup data (no GPU), see st_iga_host_query."""
    lib = load()
    P, keep = make_problem(prob, knots)
    n = C.c_int64(0)
    st = lib.st_iga_host_query(C.byref(P), what, direction, None, 0, C.byref(n))
    if st != OK:
        raise StIgaError(st, lib.st_iga_last_error(None).decode())
    out = np.zeros(max(n.value, 1))
    lib.st_iga_host_query(C.byref(P), what, direction, _dptr(out), n.value, C.byref(n))
    return out[: n.value]


def host_symeig(A: np.ndarray):
    """Eigen-decomposition of a symmetric matrix by the library's host solver: (lam ascending, Q)."""
    lib = load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    Q, lam = np.zeros((n, n)), np.zeros(n)
    st = lib.st_iga_host_symeig(n, _dptr(A), _dptr(Q), _dptr(lam))
    if st != OK:
        raise StIgaError(st, lib.st_iga_last_error(None).decode())
    return lam, Q


class Solver:
    """One problem on one GPU: owns a torch workspace and the library context."""

    def __init__(self, prob, knots=None, device="cuda:0", stream=None, **options):
        import torch
        self.torch = torch
        self.lib = load()
        self.prob = prob
        self.P, self._keep = make_problem(prob, knots)
        self.O = default_options(**options)
        nbytes = self.lib.st_iga_workspace_bytes(C.byref(self.P), C.byref(self.O))
        if nbytes == 0:
            raise StIgaError(EINVAL, "invalid problem or options")
        self.device = torch.device(device)
        self.tstream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(self.tstream):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.ctx = C.c_void_p()
        self.stream = self.tstream.cuda_stream
        st = self.lib.st_iga_setup(C.byref(self.P), C.byref(self.O), C.c_void_p(base + off), nbytes, self._s(),
                                   C.byref(self.ctx))
        if st != OK:
            raise StIgaError(st, self.lib.st_iga_last_error(None).decode())
        sz = (C.c_int64 * 9)()
        self.lib.st_iga_sizes(self.ctx, sz)
        self.d, self.n_t, self.N_s, self.N_t = sz[0], sz[4], sz[5], sz[6]
        self.unknowns = sz[7] + (sz[8] << 32)
        self.full = self.N_s * self.n_t
        self.workspace_bytes = nbytes
        if getattr(prob, "f_kind", 0):
            self.set_stimulus(prob)

    def set_stimulus(self, prob):
        """Make the source of `prob` (its f_* fields) the context's f."""
        self._stim = make_stimulus(prob)
        self._chk(self.lib.st_iga_set_stimulus(self.ctx, C.byref(self._stim)))

    def _s(self):
        return C.c_void_p(self.stream)

    def _chk(self, st):
        if st != OK:
            raise StIgaError(st, self.lib.st_iga_last_error(self.ctx).decode())

    @staticmethod
    def _p(t):
        return C.c_void_p(t.data_ptr())

    def vec(self, n=None):
        with self.torch.cuda.stream(self.tstream):
            return self.torch.zeros(self.unknowns if n is None else n, dtype=self.torch.float64, device=self.device)

    def linearize(self, u, w, refresh_theta=True):
        self._chk(self.lib.st_iga_linearize(self.ctx, self._p(u), self._p(w), int(refresh_theta), self._s()))

    def set_factors(self, theta=None, react=None):
        def parts(f):
            if f is None:
                return 0, None, None, None
            U, s, V = (np.ascontiguousarray(a, dtype=np.float64) for a in f)
            return len(s), U, s, V
        rt, Ut, st, Vt = parts(theta)
        rc, Uc, sc, Vc = parts(react)
        self._hold = (Ut, st, Vt, Uc, sc, Vc)
        p = lambda a: _dptr(a) if a is not None else None
        self._chk(self.lib.st_iga_set_factors(self.ctx, rt, p(Ut), p(st), p(Vt), rc, p(Uc), p(sc), p(Vc)))

    def get_factors(self):
        R = self.O.max_rank
        Ut, st, Uc, sc = np.zeros(self.N_t * R), np.zeros(R), np.zeros(self.N_t * R), np.zeros(R)
        Vt, Vc = np.zeros(self.N_s * R), np.zeros(self.N_s * R)
        rt, rc = C.c_int32(0), C.c_int32(0)
        self._chk(self.lib.st_iga_get_factors(self.ctx, C.byref(rt), _dptr(Ut), _dptr(st), _dptr(Vt), C.byref(rc),
                                              _dptr(Uc), _dptr(sc), _dptr(Vc)))
        a, b = rt.value, rc.value
        return ((Ut[: self.N_t * a].reshape(self.N_t, a), st[:a], Vt[: self.N_s * a].reshape(self.N_s, a)),
                (Uc[: self.N_t * b].reshape(self.N_t, b), sc[:b], Vc[: self.N_s * b].reshape(self.N_s, b)))

    def theta_grid(self, u, w):
        out = self.vec()
        self._chk(self.lib.st_iga_theta_grid(self.ctx, self._p(u), self._p(w), self._p(out), self._s()))
        return out

    def apply(self, x, y=None):
        y = self.vec() if y is None else y
        self._chk(self.lib.st_iga_apply(self.ctx, self._p(x), self._p(y), self._s()))
        return y

    def precond(self, r, z=None):
        z = self.vec() if z is None else z
        self._chk(self.lib.st_iga_precond(self.ctx, self._p(r), self._p(z), self._s()))
        return z

    def precond_noalloc(self, r, z=None):
        """z = A-hat^{-1} r through the allocation-free entry point (z must be
        given to keep the call itself free of allocations)."""
        z = self.vec() if z is None else z
        self._chk(self.lib.st_iga_precond_noalloc(self.ctx, self._p(r), self._p(z), self._s()))
        return z

    def apply_lowp(self, x, y=None):
        y = self.vec() if y is None else y
        self._chk(self.lib.st_iga_apply_lowp(self.ctx, self._p(x), self._p(y), self._s()))
        return y

    def precond_lowp(self, r, z=None):
        z = self.vec() if z is None else z
        self._chk(self.lib.st_iga_precond_lowp(self.ctx, self._p(r), self._p(z), self._s()))
        return z

    def residual(self, u, w):
        r = self.vec()
        self._chk(self.lib.st_iga_residual(self.ctx, self._p(u), self._p(w), self._p(r), self._s()))
        return r

    def w_update(self, u):
        w = self.vec(self.full)
        self._chk(self.lib.st_iga_w_update(self.ctx, self._p(u), self._p(w), self._s()))
        return w

    def krylov(self, b, tol=1e-10, x=None):
        x = self.vec() if x is None else x
        it, rr = C.c_int32(0), C.c_double(0)
        self._chk(self.lib.st_iga_krylov(self.ctx, self._p(b), self._p(x), tol, C.byref(it), C.byref(rr), self._s()))
        return x, it.value, rr.value

    def newton_step(self, u_in, u_out, w, refresh_theta=True, tol=1e-8):
        it, rr, dinf = C.c_int32(0), C.c_double(0), C.c_double(0)
        self._chk(self.lib.st_iga_newton_step(self.ctx, self._p(u_in), self._p(u_out), self._p(w),
                                              int(refresh_theta), tol, C.byref(it), C.byref(rr), C.byref(dinf),
                                              self._s()))
        return it.value, rr.value, dinf.value

    KCLASSES = ["gather", "time_mix", "arrowhead", "multidot", "update_norm", "pointwise_ionic", "maxima",
                "banded", "expand", "dense_fd", "coefficient"]
    FNAMES = ["gather_scalar", "gather_v4", "gather_rows", "time_mix", "dense_mode_mfma", "arrowhead",
              "multidot", "update_norm", "pointwise_ionic", "mode_max", "gather_sweep", "coef_fused",
              "quad_fused", "sweep_dual", "time_core", "react_point", "band_solve"]

    def profile(self, on=True):
        self._chk(self.lib.st_iga_profile(self.ctx, int(on)))

    def profile_records(self):
        """[(function name, ms, algorithmic bytes, algorithmic flops)] of every launch since the last reset."""
        out, i = [], 0
        fn, ms, by, fl = C.c_int32(0), C.c_double(0), C.c_double(0), C.c_double(0)
        while self.lib.st_iga_profile_record(self.ctx, i, C.byref(fn), C.byref(ms), C.byref(by), C.byref(fl)) == OK:
            name = self.FNAMES[fn.value % 32] + "<" + ["f64", "f32", "bf16"][fn.value // 32] + ">"
            out.append((name, ms.value, by.value, fl.value))
            i += 1
        return out

    def profile_read(self, reset=True):
        """{class: (ms, launches, algorithmic bytes, algorithmic flops)} since the last reset; per kernel
        function under "fn:<name><<precision>>"."""
        out = {}
        for k, name in enumerate(self.KCLASSES):
            ms, n, by, fl = C.c_double(0), C.c_int64(0), C.c_double(0), C.c_double(0)
            self._chk(self.lib.st_iga_profile_read(self.ctx, k, C.byref(ms), C.byref(n), C.byref(by), C.byref(fl), 0))
            out[name] = (ms.value, n.value, by.value, fl.value)
        for q, pn in enumerate(["f64", "f32", "bf16"]):
            for f, fname in enumerate(self.FNAMES):
                ms, n, by, fl = C.c_double(0), C.c_int64(0), C.c_double(0), C.c_double(0)
                self._chk(self.lib.st_iga_profile_read(self.ctx, 100 + f + 32 * q, C.byref(ms), C.byref(n),
                                                       C.byref(by), C.byref(fl), 0))
                if n.value:
                    out[f"fn:{fname}<{pn}>"] = (ms.value, n.value, by.value, fl.value)
        if reset:
            self._chk(self.lib.st_iga_profile_read(self.ctx, 0, None, None, None, None, 1))
        return out

    def lift(self):
        c0 = np.zeros(self.N_s)
        cnt = C.c_int64(0)
        S = make_stimulus(self.prob)
        self._chk(self.lib.st_iga_lift(self.ctx, C.byref(S), _dptr(c0), C.byref(cnt)))
        return c0, cnt.value

    def solve(self):
        u, w = self.vec(self.full), self.vec(self.full)
        rep = Report()
        S = make_stimulus(self.prob)
        self._chk(self.lib.st_iga_solve(self.ctx, C.byref(S), self._p(u), self._p(w), C.byref(rep), self._s()))
        return u, w, rep

    def close(self):
        if self.ctx:
            self.lib.st_iga_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
