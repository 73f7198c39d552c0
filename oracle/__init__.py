"""ctypes front-end of the plain C oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The HIP library and its Python binding never
import this package.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORC_LIBPATH selects another build of the same sources (the sanitizer
# build of the CPU test job); the default is the plain one.
_LIBPATH = os.environ.get("ORC_LIBPATH") or os.path.join(_HERE, "liboracle.so")
_lib = None

FREE, RECORD, REPLAY = 0, 1, 2
EXPRB42, PEXPRB43, EXPRB53, EPI3, EPI2, EXPRB42M, EXPRB32 = 0, 1, 2, 3, 4, 5, 6
METHODS = {"exprb42": EXPRB42, "pexprb43": PEXPRB43, "exprb53": EXPRB53, "epi3": EPI3,
           "epi2": EPI2, "exprb42m": EXPRB42M, "exprb32": EXPRB32}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class Swe(C.Structure):
    _fields_ = [("n", C.c_int), ("radius", C.c_double), ("omega", C.c_double),
                ("gravity", C.c_double), ("gamma_h", C.c_double), ("dt_e", C.c_double),
                ("nu", C.c_double), ("xyz", _dp), ("deg", _ip), ("nbr", _ip),
                ("area", _dp), ("len", _dp), ("dist", _dp), ("nrm", _dp), ("tng", _dp),
                ("cor", _dp), ("work", _dp), ("hs", _dp)]


class Attempt(C.Structure):
    _fields_ = [("tau", C.c_double), ("m", C.c_int32), ("flags", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("a", C.POINTER(Attempt)), ("len", C.c_int), ("cap", C.c_int), ("pos", C.c_int)]

    def entries(self):
        return [(self.a[i].tau, self.a[i].m, self.a[i].flags) for i in range(self.len)]

    def as_array(self):
        """(len, 3) float64 array: tau, m, flags."""
        e = self.entries()
        return np.array(e, dtype=np.float64).reshape(-1, 3)


class PhiOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("m_init", C.c_int), ("m_max", C.c_int),
                ("delta", C.c_double), ("gamma", C.c_double), ("max_attempts", C.c_int),
                ("mode", C.c_int), ("sched", C.POINTER(Schedule)), ("tape", C.c_void_p)]


class PhiStats(C.Structure):
    _fields_ = [(k, C.c_int) for k in ("attempts", "rejected", "accepted", "matvecs", "expms",
                                       "sum_m", "max_m", "last_m", "rec_matvecs")]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepState(C.Structure):
    _fields_ = [("m_warm", C.c_int * 3), ("have_prev", C.c_int), ("u_prev", _dp),
                ("f_prev", _dp), ("calls", PhiStats * 3)]


RHS_FN = C.CFUNCTYPE(None, C.c_void_p, _dp, _dp)
JV_FN = C.CFUNCTYPE(None, C.c_void_p, _dp, _dp, _dp)
MATVEC_FN = C.CFUNCTYPE(None, C.c_void_p, _dp, _dp)


class Problem(C.Structure):
    _fields_ = [("n", C.c_int), ("rhs", RHS_FN), ("jv", JV_FN), ("ctx", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIBPATH)
        L.orc_swe_init.argtypes = [C.POINTER(Swe), C.c_int, _dp, _ip, _ip, _dp, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_swe_free.argtypes = [C.POINTER(Swe)]
        for f in ("orc_rhs",):
            getattr(L, f).argtypes = [C.POINTER(Swe), _dp, _dp]
        for f in ("orc_jv", "orc_jtv", "orc_ktv"):
            getattr(L, f).argtypes = [C.POINTER(Swe), _dp, _dp, _dp]
        L.orc_phi_vjp_dense.argtypes = [C.c_int, _dp, C.c_int, C.POINTER(_dp), C.c_int, _dp,
                                        C.POINTER(_dp), C.POINTER(_dp), C.POINTER(_dp), _dp,
                                        C.POINTER(PhiOpts), C.POINTER(PhiStats),
                                        C.POINTER(PhiStats)]
        L.orc_step_vjp.argtypes = [C.POINTER(Swe), C.c_int, _dp, C.c_double, _dp, _dp,
                                   C.POINTER(PhiOpts), C.POINTER(PhiStats)]
        L.orc_diagnostics.argtypes = [C.POINTER(Swe), _dp, _dp]
        L.orc_swe_set_topography.argtypes = [C.POINTER(Swe), _dp]
        L.orc_div.argtypes = [C.POINTER(Swe), _dp, _dp, _dp, _dp]
        L.orc_grad.argtypes = [C.POINTER(Swe), _dp, _dp, _dp, _dp]
        L.orc_curl.argtypes = [C.POINTER(Swe), _dp, _dp, _dp, _dp]
        L.orc_lap.argtypes = [C.POINTER(Swe), _dp, _dp]
        L.orc_expm.argtypes = [C.c_int, _dp, _dp]
        L.orc_expm.restype = C.c_int
        L.orc_phi_default_opts.argtypes = [C.POINTER(PhiOpts)]
        L.orc_phi_combo.argtypes = [C.c_int, MATVEC_FN, C.c_void_p, C.c_int, C.POINTER(_dp),
                                    C.c_int, _dp, C.POINTER(_dp), C.POINTER(PhiOpts), _ip,
                                    C.POINTER(PhiStats)]
        L.orc_phi_combo_dense.argtypes = [C.c_int, _dp, C.c_int, C.POINTER(_dp), C.c_int, _dp,
                                          C.POINTER(_dp), C.POINTER(PhiOpts), _ip,
                                          C.POINTER(PhiStats)]
        L.orc_step_state_init.argtypes = [C.POINTER(StepState), C.c_int]
        L.orc_step_state_free.argtypes = [C.POINTER(StepState)]
        L.orc_step.argtypes = [C.POINTER(Problem), C.c_int, _dp, C.c_double,
                               C.POINTER(StepState), C.POINTER(PhiOpts)]
        L.orc_swe_problem.argtypes = [C.POINTER(Swe), C.POINTER(Problem)]
        L.orc_phi_cost.argtypes = [C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                                   C.c_double]
        L.orc_phi_cost.restype = C.c_double
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's independent cell loops (results do not depend
    on the count: every sum keeps its serial order)."""
    lib().orc_set_threads(int(n))


def get_threads():
    return lib().orc_get_threads()


def phi_cost(tau, m, p, remaining, n, hnorm):
    """eq. cost: the controller's work estimate C(tau, m) (Sec. 4.3)."""
    return lib().orc_phi_cost(float(tau), int(m), int(p), float(remaining), float(n),
                              float(hnorm))


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def opts(tol=1e-10, m_init=1, m_max=40, delta=1.4, gamma=0.8, max_attempts=10000,
         mode=FREE, sched=None):
    o = PhiOpts()
    lib().orc_phi_default_opts(C.byref(o))
    o.tol, o.m_init, o.m_max, o.delta, o.gamma = tol, m_init, m_max, delta, gamma
    o.max_attempts, o.mode = max_attempts, mode
    o.sched = C.pointer(sched) if sched is not None else None
    return o


def new_schedule():
    return Schedule()


def schedule_from_array(arr):
    """Build a replay schedule from an (len, 3) array of (tau, m, flags)."""
    arr = np.asarray(arr, dtype=np.float64).reshape(-1, 3)
    s = Schedule()
    buf = (Attempt * max(1, len(arr)))()
    for i, (t, m, f) in enumerate(arr):
        buf[i].tau, buf[i].m, buf[i].flags = float(t), int(m), int(f)
    s.a = C.cast(buf, C.POINTER(Attempt))
    s.len = s.cap = len(arr)
    s.pos = 0
    s._keep = buf
    return s


def expm(A):
    A = _f64(A)
    K = A.shape[0]
    X = np.empty_like(A)
    s = lib().orc_expm(K, _ptr(A), _ptr(X))
    return X, s


def _vec_array(vs, n):
    arr = (_dp * len(vs))()
    keep = []
    for i, v in enumerate(vs):
        if v is None:
            arr[i] = _dp()
        else:
            a = _f64(v)
            assert a.shape == (n,)
            keep.append(a)
            arr[i] = _ptr(a)
    return arr, keep


def phi_combo_dense(A, vs, rho, o=None, m_warm=0):
    """W_i = sum_l rho_i^l phi_l(rho_i A) v_l with a dense A (list vs, None = 0)."""
    A = _f64(A)
    n = A.shape[0]
    p = len(vs) - 1
    va, keep = _vec_array(vs, n)
    rho = _f64(rho)
    outs = [np.zeros(n) for _ in rho]
    oa = (_dp * len(outs))(*[_ptr(w) for w in outs])
    st = PhiStats()
    mw = C.c_int(m_warm)
    o = o if o is not None else opts()
    rc = lib().orc_phi_combo_dense(n, _ptr(A), p, va, len(rho), _ptr(rho), oa, C.byref(o),
                                   C.byref(mw), C.byref(st))
    if rc:
        raise RuntimeError("orc_phi_combo_dense failed: %d" % rc)
    return outs, st.asdict(), mw.value


def phi_vjp_dense(A, vs, rho, wbars, o=None):
    """Forward W_i and the adjoint of one phi-combination with a dense A:
    returns (W list, vbar list (p+1), Abar (n x n), forward stats, adjoint stats)."""
    A = _f64(A)
    n = A.shape[0]
    p = len(vs) - 1
    va, keep = _vec_array(vs, n)
    rho = _f64(rho)
    outs = [np.zeros(n) for _ in rho]
    oa = (_dp * len(outs))(*[_ptr(w) for w in outs])
    wb = [_f64(w) for w in wbars]
    wba = (_dp * len(wb))(*[_ptr(w) for w in wb])
    vb = [np.zeros(n) for _ in range(p + 1)]
    vba = (_dp * len(vb))(*[_ptr(w) for w in vb])
    Abar = np.zeros((n, n))
    fs, ast = PhiStats(), PhiStats()
    o = o if o is not None else opts()
    rc = lib().orc_phi_vjp_dense(n, _ptr(A), p, va, len(rho), _ptr(rho), wba, oa, vba,
                                 _ptr(Abar), C.byref(o), C.byref(fs), C.byref(ast))
    if rc:
        raise RuntimeError("orc_phi_vjp_dense failed: %d" % rc)
    return outs, vb, Abar, fs.asdict(), ast.asdict()


class SWE:
    """The oracle's shallow-water model on one mesh."""

    def __init__(self, mesh, gamma_h=4e-4, radius=6.371e6, omega=7.292e-5,
                 gravity=9.80616, dt_e=240.0):
        self.mesh = mesh
        self.n = len(mesh["xyz"])
        self.N = 4 * self.n
        self._xyz = _f64(mesh["xyz"])
        self._deg = np.ascontiguousarray(mesh["deg"], dtype=np.int32)
        self._nbr = np.ascontiguousarray(mesh["nbr"], dtype=np.int32)
        self._cor = _f64(mesh["corners"])
        self.s = Swe()
        rc = lib().orc_swe_init(C.byref(self.s), self.n, _ptr(self._xyz),
                                self._deg.ctypes.data_as(_ip), self._nbr.ctypes.data_as(_ip),
                                _ptr(self._cor), radius, omega, gravity, gamma_h, dt_e)
        if rc:
            raise RuntimeError("orc_swe_init failed %d" % rc)
        self.problem = Problem()
        lib().orc_swe_problem(C.byref(self.s), C.byref(self.problem))

    def __del__(self):
        try:
            lib().orc_swe_free(C.byref(self.s))
        except Exception:
            pass

    # geometry views
    @property
    def area(self):
        return np.ctypeslib.as_array(self.s.area, (self.n,)).copy()

    @property
    def nu(self):
        return self.s.nu

    def edge_len(self):
        return np.ctypeslib.as_array(self.s.len, (self.n, 6)).copy()

    def edge_dist(self):
        return np.ctypeslib.as_array(self.s.dist, (self.n, 6)).copy()

    def edge_nrm(self):
        return np.ctypeslib.as_array(self.s.nrm, (self.n, 6, 3)).copy()

    # operators
    def div(self, fx, fy, fz):
        o = np.empty(self.n)
        lib().orc_div(C.byref(self.s), _ptr(_f64(fx)), _ptr(_f64(fy)), _ptr(_f64(fz)), _ptr(o))
        return o

    def grad(self, psi):
        gx, gy, gz = np.empty(self.n), np.empty(self.n), np.empty(self.n)
        lib().orc_grad(C.byref(self.s), _ptr(_f64(psi)), _ptr(gx), _ptr(gy), _ptr(gz))
        return np.stack([gx, gy, gz], 1)

    def curl(self, ux, uy, uz):
        o = np.empty(self.n)
        lib().orc_curl(C.byref(self.s), _ptr(_f64(ux)), _ptr(_f64(uy)), _ptr(_f64(uz)), _ptr(o))
        return o

    def lap(self, psi):
        o = np.empty(self.n)
        lib().orc_lap(C.byref(self.s), _ptr(_f64(psi)), _ptr(o))
        return o

    def rhs(self, u):
        u = _f64(u)
        f = np.empty(self.N)
        lib().orc_rhs(C.byref(self.s), _ptr(u), _ptr(f))
        return f

    def jv(self, u, v):
        u, v = _f64(u), _f64(v)
        o = np.empty(self.N)
        lib().orc_jv(C.byref(self.s), _ptr(u), _ptr(v), _ptr(o))
        return o

    def jtv(self, u, w):
        u, w = _f64(u), _f64(w)
        o = np.empty(self.N)
        lib().orc_jtv(C.byref(self.s), _ptr(u), _ptr(w), _ptr(o))
        return o

    def ktv(self, a, b):
        """K(a, b) = grad_u <a, J(u) b>."""
        a, b = _f64(a), _f64(b)
        o = np.empty(self.N)
        lib().orc_ktv(C.byref(self.s), _ptr(a), _ptr(b), _ptr(o))
        return o

    def set_topography(self, hs):
        """Surface topography h_s (n values, metres; None: flat)."""
        if hs is None:
            lib().orc_swe_set_topography(C.byref(self.s), None)
        else:
            hs = _f64(hs)
            assert hs.shape == (self.n,)
            lib().orc_swe_set_topography(C.byref(self.s), _ptr(hs))

    def diagnostics(self, u):
        """Mass, total energy and potential enstrophy of u (Sec. 6)."""
        o = np.empty(3)
        lib().orc_diagnostics(C.byref(self.s), _ptr(_f64(u)), _ptr(o))
        return {"mass": o[0], "energy": o[1], "enstrophy": o[2]}

    def step_vjp(self, method, u, dt, ubar, o=None):
        """(d u_{n+1} / d u_n)^T ubar for one step from u (exprb42); pass
        replay opts to follow a recorded forward.  Returns (ubar_n, stats of
        the two adjoint calls)."""
        u, ubar = _f64(u), _f64(ubar)
        out = np.empty(self.N)
        st = (PhiStats * 2)()
        o = o if o is not None else opts()
        rc = lib().orc_step_vjp(C.byref(self.s), METHODS[method], _ptr(u), dt, _ptr(ubar),
                                _ptr(out), C.byref(o), st)
        if rc:
            raise RuntimeError("orc_step_vjp failed: %d" % rc)
        return out, [st[0].asdict(), st[1].asdict()]

    def dense_jacobian(self, u):
        J = np.empty((self.N, self.N))
        e = np.zeros(self.N)
        for k in range(self.N):
            e[k] = 1.0
            J[:, k] = self.jv(u, e)
            e[k] = 0.0
        return J

    def phi_combo(self, u, dt, vs, rho, o=None, m_warm=0):
        """W_i = sum_l rho_i^l phi_l(rho_i dt J(u)) v_l (Alg. 1)."""
        u = _f64(u)
        p = len(vs) - 1
        va, keep = _vec_array(vs, self.N)
        rho = _f64(rho)
        outs = [np.zeros(self.N) for _ in rho]
        oa = (_dp * len(outs))(*[_ptr(w) for w in outs])
        tmp_u = u

        def mv(ctx, x, y):
            lib().orc_jv(C.byref(self.s), _ptr(tmp_u), x, y)
            ya = np.ctypeslib.as_array(y, (self.N,))
            ya *= dt

        cb = MATVEC_FN(mv)
        st = PhiStats()
        mw = C.c_int(m_warm)
        o = o if o is not None else opts()
        rc = lib().orc_phi_combo(self.N, cb, None, p, va, len(rho), _ptr(rho), oa, C.byref(o),
                                 C.byref(mw), C.byref(st))
        if rc:
            raise RuntimeError("orc_phi_combo failed: %d" % rc)
        return outs, st.asdict(), mw.value


def exprb42_loss_grad(swe, u0, dt, steps, obs_step, obs_cell, obs_val, tol=1e-10, m_max=40,
                      progress=None):
    """Loss L = 1/2 sum_k (h[obs_cell_k] after step obs_step_k - obs_val_k)^2
    over an exprb42 trajectory of `steps` steps from u0, and dL/du0 by
    per-step vector-Jacobian products on the recorded schedule.
    progress(phase, k), if given, is called after each forward and reverse
    step.  Returns (L, grad, schedules)."""
    obs_step = np.asarray(obs_step, dtype=np.int64)
    obs_cell = np.asarray(obs_cell, dtype=np.int64)
    obs_val = np.asarray(obs_val, dtype=np.float64)
    n = swe.n
    us = [np.array(u0, dtype=np.float64)]
    scheds = []
    st = swe_stepper(swe, "exprb42")
    for k in range(steps):
        sch = new_schedule()
        us.append(st.step(us[-1], dt, opts(tol=tol, m_max=m_max, mode=RECORD, sched=sch)))
        scheds.append(sch.as_array())
        if progress:
            progress("forward", k + 1)
    loss = 0.0
    res = []
    for k in range(steps + 1):
        sel = obs_step == k
        r = us[k][3 * n + obs_cell[sel]] - obs_val[sel]
        res.append((obs_cell[sel], r))
        loss += 0.5 * float(r @ r)
    g = np.zeros(swe.N)
    for k in range(steps, 0, -1):
        c, r = res[k]
        np.add.at(g, 3 * n + c, r)
        g, _ = swe.step_vjp("exprb42", us[k - 1], dt, g,
                            opts(tol=tol, m_max=m_max, mode=REPLAY,
                                 sched=schedule_from_array(scheds[k - 1])))
        if progress:
            progress("reverse", k)
    c, r = res[0]
    np.add.at(g, 3 * n + c, r)
    return loss, g, scheds


class Stepper:
    """Runs one of the schemes with the oracle (keeps warm starts and epi3
    history across steps)."""

    def __init__(self, problem_n, problem, method, owner=None):
        self.n = problem_n
        self.problem = problem
        self._owner = owner          # keeps the model (and its C state) alive
        self.method = METHODS[method] if isinstance(method, str) else method
        self.state = StepState()
        lib().orc_step_state_init(C.byref(self.state), self.n)

    def __del__(self):
        try:
            lib().orc_step_state_free(C.byref(self.state))
        except Exception:
            pass

    def step(self, u, dt, o=None):
        u = np.array(u, dtype=np.float64, copy=True)
        o = o if o is not None else opts()
        rc = lib().orc_step(C.byref(self.problem), self.method, _ptr(u), dt,
                            C.byref(self.state), C.byref(o))
        if rc:
            raise RuntimeError("orc_step failed: %d" % rc)
        return u

    def call_stats(self):
        return [self.state.calls[i].asdict() for i in range(3)]


def swe_stepper(swe, method):
    return Stepper(swe.N, swe.problem, method, owner=swe)


class CallbackProblem:
    """An ODE u' = f(u) given by Python callables (for scheme-order pins)."""

    def __init__(self, n, f, jac):
        self.n = n

        def rhs(ctx, u, out):
            ua = np.ctypeslib.as_array(u, (n,))
            np.ctypeslib.as_array(out, (n,))[:] = f(ua)

        def jv(ctx, u, v, out):
            ua = np.ctypeslib.as_array(u, (n,))
            va = np.ctypeslib.as_array(v, (n,))
            np.ctypeslib.as_array(out, (n,))[:] = jac(ua) @ va

        self._rhs = RHS_FN(rhs)
        self._jv = JV_FN(jv)
        self.problem = Problem(n, self._rhs, self._jv, None)

    def stepper(self, method):
        return Stepper(self.n, self.problem, method, owner=self)
