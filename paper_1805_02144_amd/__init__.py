"""Python binding of libexprb (HIP, gfx950): argument marshalling only.

Every arithmetic step runs in the library's HIP kernels.  PyTorch is used
for device memory (tensors are passed by data_ptr) and for the current HIP
stream.  There is no CPU fallback: importing works without a GPU, but any
call needs the built library and a visible GPU, and fails loudly otherwise.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libexprb.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, ENAN, ESTATE, ESCHED = 0, -1, -2, -3, -4, -5, -6, -7
FREE, RECORD, REPLAY = 0, 1, 2
METHODS = {"exprb42": 0, "pexprb43": 1, "exprb53": 2, "epi3": 3, "epi2": 4, "exprb42m": 5}
MMAX_LIMIT = 44
PMAX = 4

EXPORTS = ["xrb_default_params", "xrb_create", "xrb_destroy", "xrb_set_stream", "xrb_sync",
           "xrb_last_error", "xrb_n_cells", "xrb_rhs", "xrb_jv", "xrb_phi_combo", "xrb_step",
           "xrb_diagnostics", "xrb_set_topography", "xrb_autotune",
           "xrb_step_stats", "xrb_reset_history", "xrb_schedule_mode", "xrb_schedule_set",
           "xrb_schedule_get", "xrb_profile", "xrb_profile_get", "xrb_step_batch", "xrb_jtv",
           "xrb_ktv", "xrb_step_vjp", "xrb_step_tableau", "xrb_mesh_info",
           "xrb_schedule_set_member", "xrb_schedule_get_member", "xrb_profile_overhead",
           "xrb_jv_static", "xrb_step_batch_capture", "xrb_graph_launch"]

KERNELS = ["jv_iom2", "lap", "iom2_update", "controller", "combine", "jv_other", "rhs", "vec", "upd_lap"]

_dp = C.POINTER(C.c_double)


TAB_CALLS, TAB_OUT, TAB_STAGES = 3, 2, 2


class Tableau(C.Structure):
    """xrb_tableau: a general exponential Rosenbrock scheme as phi-combination
    calls (see include/exprb.h)."""
    _fields_ = [("ncalls", C.c_int), ("p", C.c_int * TAB_CALLS), ("ns", C.c_int * TAB_CALLS),
                ("rho", (C.c_double * TAB_OUT) * TAB_CALLS),
                ("vc", ((C.c_double * (1 + TAB_STAGES)) * (PMAX + 1)) * TAB_CALLS),
                ("nstages", C.c_int), ("stage_call", C.c_int * TAB_STAGES),
                ("uc", ((C.c_double * TAB_OUT) * TAB_CALLS) * TAB_STAGES),
                ("un1", (C.c_double * TAB_OUT) * TAB_CALLS)]


def make_tableau(calls, stages, un1):
    """Build a Tableau.  calls: list of dicts {"p", "rho": [..], "v": {l: {"v": c, "D2": c,
    "D3": c}}}; stages: list of (call index, {(c, o): coef}) defining U2, U3; un1: {(c, o): coef}."""
    T = Tableau()
    T.ncalls = len(calls)
    for c, cl in enumerate(calls):
        T.p[c] = cl["p"]
        T.ns[c] = len(cl["rho"])
        for o, r in enumerate(cl["rho"]):
            T.rho[c][o] = r
        for l, terms in cl.get("v", {}).items():
            for name, coef in terms.items():
                q = {"v": 0, "D2": 1, "D3": 2}[name]
                T.vc[c][l][q] = coef
    T.nstages = len(stages)
    for st, (c, terms) in enumerate(stages):
        T.stage_call[st] = c
        for (cc, o), coef in terms.items():
            T.uc[st][cc][o] = coef
    for (cc, o), coef in un1.items():
        T.un1[cc][o] = coef
    return T


# The schemes of Sec. 4.4 (eqs. 3.11-3.13) and the third-order exprb32 in
# the tableau form; the outputs carry rho^l, so exprb53's U3 rescales its
# phi_3 terms by (27/25) 2^3 and (729/125) (10/9)^3.
TABLEAUS = {
    "exprb42": make_tableau(
        [{"p": 1, "rho": [0.75], "v": {1: {"v": 1.0}}},
         {"p": 3, "rho": [1.0], "v": {1: {"v": 1.0}, 3: {"D2": 32.0 / 9.0}}}],
        [(0, {(0, 0): 1.0})], {(1, 0): 1.0}),
    "pexprb43": make_tableau(
        [{"p": 1, "rho": [0.5, 1.0], "v": {1: {"v": 1.0}}},
         {"p": 4, "rho": [1.0], "v": {3: {"D2": 16.0, "D3": -2.0}, 4: {"D2": -48.0, "D3": 12.0}}}],
        [(0, {(0, 0): 1.0}), (0, {(0, 1): 1.0})], {(0, 1): 1.0, (1, 0): 1.0}),
    "exprb53": make_tableau(
        [{"p": 1, "rho": [0.5, 0.9], "v": {1: {"v": 1.0}}},
         {"p": 3, "rho": [0.5, 0.9], "v": {3: {"D2": 1.0}}},
         {"p": 4, "rho": [1.0], "v": {1: {"v": 1.0}, 3: {"D2": 18.0, "D3": -250.0 / 81.0},
                                      4: {"D2": -60.0, "D3": 500.0 / 27.0}}}],
        [(0, {(0, 0): 1.0}), (1, {(0, 1): 1.0, (1, 0): 216.0 / 25.0, (1, 1): 8.0})],
        {(2, 0): 1.0}),
    "exprb32": make_tableau(
        [{"p": 1, "rho": [1.0], "v": {1: {"v": 1.0}}},
         {"p": 3, "rho": [1.0], "v": {3: {"D2": 2.0}}}],
        [(0, {(0, 0): 1.0})], {(0, 0): 1.0, (1, 0): 1.0}),
}


class Mesh(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("xyz", _dp), ("deg", C.POINTER(C.c_int32)),
                ("nbr", C.POINTER(C.c_int32)), ("corners", _dp)]


class Params(C.Structure):
    _fields_ = [("radius", C.c_double), ("omega", C.c_double), ("gravity", C.c_double),
                ("gamma_h", C.c_double), ("dt_e", C.c_double), ("tol", C.c_double),
                ("m_init", C.c_int32), ("m_max", C.c_int32), ("delta", C.c_double),
                ("gamma", C.c_double), ("max_attempts", C.c_int32), ("lanes", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("single_us", C.c_double * 4), ("batch_us", C.c_double * 4),
                ("lanes", C.c_int32), ("lanes_batch", C.c_int32), ("nm_batch", C.c_int32),
                ("jv_cand", C.c_int32 * 4), ("jv_single_us", C.c_double * 4),
                ("jv_batch_us", C.c_double * 4), ("jv_block", C.c_int32),
                ("jv_block_batch", C.c_int32), ("lap_cand", C.c_int32 * 3),
                ("lap_us", C.c_double * 3), ("lap_block", C.c_int32), ("lap_grid", C.c_int32)]


class PhiStats(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("attempts", "rejected", "accepted", "matvecs", "expms",
                                         "sum_m", "max_m", "last_m", "rec_matvecs")]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libexprb.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libexprb.so is not built: run paper_1805_02144_amd/build.py "
                               "(or __graft_entry__.build())")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so the process holds a single runtime (loading the library
        # first can leave two, and device allocation fails)
        import torch  # noqa: F401
        L = C.CDLL(LIBPATH)
        vp = C.c_void_p
        L.xrb_default_params.argtypes = [C.POINTER(Params)]
        L.xrb_create.argtypes = [C.POINTER(Mesh), C.POINTER(Params), vp, C.POINTER(vp)]
        L.xrb_destroy.argtypes = [vp]
        L.xrb_set_stream.argtypes = [vp, vp]
        L.xrb_sync.argtypes = [vp]
        L.xrb_last_error.argtypes = [vp]
        L.xrb_last_error.restype = C.c_char_p
        L.xrb_n_cells.argtypes = [vp]
        L.xrb_n_cells.restype = C.c_int64
        L.xrb_mesh_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(_dp), C.POINTER(_dp)]
        L.xrb_rhs.argtypes = [vp, vp, vp]
        L.xrb_jv.argtypes = [vp, vp, vp, vp]
        L.xrb_jv_static.argtypes = [vp, vp, vp, vp]
        L.xrb_jtv.argtypes = [vp, vp, vp, vp]
        L.xrb_ktv.argtypes = [vp, vp, vp, vp]
        L.xrb_diagnostics.argtypes = [vp, vp, _dp]
        L.xrb_set_topography.argtypes = [vp, _dp]
        L.xrb_autotune.argtypes = [vp, C.c_int, C.POINTER(TuneResult)]
        L.xrb_step_vjp.argtypes = [vp, C.c_int, vp, C.c_double, _dp, C.c_int, vp, vp,
                                   C.POINTER(PhiStats)]
        L.xrb_phi_combo.argtypes = [vp, C.c_double, vp, C.c_int, C.POINTER(vp), C.c_int, _dp,
                                    C.POINTER(vp), C.POINTER(PhiStats)]
        L.xrb_step.argtypes = [vp, C.c_int, vp, C.c_double]
        L.xrb_step_batch.argtypes = [vp, C.c_int, C.c_int, vp, _dp, C.POINTER(PhiStats)]
        L.xrb_step_batch_capture.argtypes = [vp, C.c_int, C.c_int, vp, _dp]
        L.xrb_graph_launch.argtypes = [vp]
        L.xrb_step_tableau.argtypes = [vp, C.POINTER(Tableau), vp, C.c_double]
        L.xrb_step_stats.argtypes = [vp, C.POINTER(PhiStats)]
        L.xrb_reset_history.argtypes = [vp]
        L.xrb_schedule_mode.argtypes = [vp, C.c_int]
        L.xrb_schedule_set.argtypes = [vp, _dp, C.c_int]
        L.xrb_schedule_get.argtypes = [vp, _dp, C.c_int, C.POINTER(C.c_int)]
        L.xrb_schedule_set_member.argtypes = [vp, C.c_int, _dp, C.c_int]
        L.xrb_schedule_get_member.argtypes = [vp, C.c_int, _dp, C.c_int, C.POINTER(C.c_int)]
        L.xrb_profile.argtypes = [vp, C.c_int]
        L.xrb_profile_overhead.argtypes = [vp, C.c_int, _dp]
        L.xrb_profile_get.argtypes = [vp, C.c_int, _dp, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]
        for f in EXPORTS:
            if f not in ("xrb_last_error", "xrb_n_cells"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def default_params(**kw):
    p = Params()
    lib().xrb_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class ExprbError(RuntimeError):
    pass


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libexprb needs a visible GPU (torch.cuda.is_available() is False)")
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    """One library context: mesh geometry on the GPU plus workspaces."""

    def __init__(self, mesh, device="cuda:0", **params):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self._xyz = np.ascontiguousarray(mesh["xyz"], dtype=np.float64)
        self._deg = np.ascontiguousarray(mesh["deg"], dtype=np.int32)
        self._nbr = np.ascontiguousarray(mesh["nbr"], dtype=np.int32)
        self._cor = np.ascontiguousarray(mesh["corners"], dtype=np.float64)
        self.n = len(self._xyz)
        self.N = 4 * self.n
        m = Mesh(self.n, self._xyz.ctypes.data_as(_dp),
                 self._deg.ctypes.data_as(C.POINTER(C.c_int32)),
                 self._nbr.ctypes.data_as(C.POINTER(C.c_int32)), self._cor.ctypes.data_as(_dp))
        self.params = default_params(**params)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            self._check(lib().xrb_create(C.byref(m), C.byref(self.params), C.c_void_p(stream),
                                         C.byref(h)), None)
        self.h = h

    def _check(self, rc, h="self"):
        if rc != OK:
            msg = lib().xrb_last_error(self.h if h == "self" else None)
            raise ExprbError("libexprb error %d: %s" % (rc, msg.decode() if msg else ""))

    def close(self):
        if getattr(self, "h", None):
            lib().xrb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        lib().xrb_set_stream(self.h, C.c_void_p(s))

    def _vec(self, x):
        t = self.torch.as_tensor(x, dtype=self.torch.float64, device=self.device)
        t = t.contiguous()
        if t.numel() != self.N:
            raise ValueError("vector of length %d expected" % self.N)
        return t

    def empty(self):
        return self.torch.empty(self.N, dtype=self.torch.float64, device=self.device)

    def sync(self):
        """Wait for the context's stream; raises the first device-side failure
        latched since the previous sync."""
        self._check(lib().xrb_sync(self.h))

    def mesh_info(self):
        """(n_cells, centres [n, 3], areas [n] in m^2) as the library holds them."""
        n = C.c_int64()
        xyz, area = _dp(), _dp()
        self._check(lib().xrb_mesh_info(self.h, C.byref(n), C.byref(xyz), C.byref(area)))
        k = n.value
        return (k, np.ctypeslib.as_array(xyz, (k, 3)).copy(),
                np.ctypeslib.as_array(area, (k,)).copy())

    def rhs(self, u):
        self._stream()
        u = self._vec(u)
        f = self.empty()
        self._check(lib().xrb_rhs(self.h, _ptr(u), _ptr(f)))
        return f

    def jv(self, u, v):
        self._stream()
        u, v = self._vec(u), self._vec(v)
        out = self.empty()
        self._check(lib().xrb_jv(self.h, _ptr(u), _ptr(v), _ptr(out)))
        return out

    def jv_static(self, u, v, out=None):
        """J(u) v through the entry point that allocates nothing (its
        intermediates live in the library's static device scratch); `out`
        may be given so that the caller allocates nothing either."""
        self._stream()
        u, v = self._vec(u), self._vec(v)
        if out is None:
            out = self.empty()
        elif not (self.torch.is_tensor(out) and out.dtype == self.torch.float64
                  and out.device == self.torch.device(self.device) and out.is_contiguous()
                  and out.numel() == self.N):
            raise ValueError("out: a contiguous float64 tensor of length %d on %s expected"
                             % (self.N, self.device))
        self._check(lib().xrb_jv_static(self.h, _ptr(u), _ptr(v), _ptr(out)))
        return out

    def jtv(self, u, w):
        """J(u)^T w."""
        self._stream()
        u, w = self._vec(u), self._vec(w)
        out = self.empty()
        self._check(lib().xrb_jtv(self.h, _ptr(u), _ptr(w), _ptr(out)))
        return out

    def ktv(self, a, b):
        """K(a, b) = grad_u <a, J(u) b>."""
        self._stream()
        a, b = self._vec(a), self._vec(b)
        out = self.empty()
        self._check(lib().xrb_ktv(self.h, _ptr(a), _ptr(b), _ptr(out)))
        return out

    def autotune(self, nm_batch=16):
        """Time the stencil launch shapes on this grid and keep the fastest
        bitwise-consistent lanes pair, then the fastest block shapes (see
        xrb_autotune)."""
        self._stream()
        r = TuneResult()
        self._check(lib().xrb_autotune(self.h, int(nm_batch), C.byref(r)))
        jv = [c for c in r.jv_cand if c > 0]
        return {"single_us": dict(zip((1, 2, 4, 8), r.single_us)),
                "batch_us": dict(zip((1, 2, 4, 8), r.batch_us)),
                "lanes": r.lanes, "lanes_batch": r.lanes_batch, "nm_batch": r.nm_batch,
                "jv_threads_single_us": {c: r.jv_single_us[k] for k, c in enumerate(jv)},
                "jv_threads_batch_us": {c: r.jv_batch_us[k] for k, c in enumerate(jv)},
                "jv_block": r.jv_block, "jv_block_batch": r.jv_block_batch,
                "lap_us": {c: r.lap_us[k] for k, c in enumerate(r.lap_cand) if c > 0},
                "lap_block": r.lap_block, "lap_grid": r.lap_grid}

    def set_topography(self, hs):
        """Surface topography h_s (n values in metres, host; None: flat)."""
        if hs is None:
            self._check(lib().xrb_set_topography(self.h, None))
            return
        self._hs = np.ascontiguousarray(hs, dtype=np.float64)
        if self._hs.shape != (self.n,):
            raise ValueError("h_s of length %d expected" % self.n)
        self._check(lib().xrb_set_topography(self.h, self._hs.ctypes.data_as(_dp)))

    def diagnostics(self, u):
        """Mass, total energy and potential enstrophy of u (Sec. 6)."""
        self._stream()
        u = self._vec(u)
        o = np.empty(3)
        self._check(lib().xrb_diagnostics(self.h, _ptr(u), o.ctypes.data_as(_dp)))
        return {"mass": float(o[0]), "energy": float(o[1]), "enstrophy": float(o[2])}

    def step_vjp(self, method, u, dt, ubar, sched=None, return_stats=False):
        """(d u_{n+1}/d u_n)^T ubar for one step from u; sched: that step's
        recorded (tau, m, flags) rows (None: recompute with the free
        controller from a cold start)."""
        self._stream()
        u, ubar = self._vec(u), self._vec(ubar)
        out = self.empty()
        mid = METHODS[method] if isinstance(method, str) else int(method)
        if sched is not None and len(sched):
            a = np.ascontiguousarray(np.asarray(sched, dtype=np.float64).reshape(-1, 3))
            sp, sl = a.ctypes.data_as(_dp), len(a)
        else:
            a, sp, sl = None, None, 0
        st = (PhiStats * 2)()
        self._check(lib().xrb_step_vjp(self.h, mid, _ptr(u), float(dt), sp, sl, _ptr(ubar),
                                       _ptr(out), st if return_stats else None))
        if return_stats:
            return out, [st[0].asdict(), st[1].asdict()]
        return out

    def phi_combo(self, u, dt, vs, rho, return_stats=False):
        """W_i = sum_l rho_i^l phi_l(rho_i dt J(u)) v_l (vs: list, None = 0)."""
        self._stream()
        u = self._vec(u)
        keep = [None if v is None else self._vec(v) for v in vs]
        va = (C.c_void_p * len(vs))(*[None if v is None else v.data_ptr() for v in keep])
        outs = [self.empty() for _ in rho]
        oa = (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        r = np.ascontiguousarray(rho, dtype=np.float64)
        st = PhiStats()
        self._check(lib().xrb_phi_combo(self.h, float(dt), _ptr(u), len(vs) - 1, va, len(outs),
                                        r.ctypes.data_as(_dp), oa, C.byref(st)))
        return (outs, st.asdict()) if return_stats else outs

    def step(self, method, u, dt):
        """Advance u (a float64 device tensor, updated in place) by one step."""
        self._stream()
        if not (u.is_contiguous() and u.dtype == self.torch.float64 and u.numel() == self.N
                and u.device == self.device):
            raise ValueError("u must be a contiguous float64 tensor of length 4N on the device")
        mid = METHODS[method] if isinstance(method, str) else int(method)
        self._check(lib().xrb_step(self.h, mid, _ptr(u), float(dt)))
        return u

    def step_tableau(self, tab, u, dt):
        """Advance u (float64 device tensor, in place) by one step of a scheme
        given as a Tableau (or a name in TABLEAUS)."""
        self._stream()
        if not (u.is_contiguous() and u.dtype == self.torch.float64 and u.numel() == self.N
                and u.device == self.device):
            raise ValueError("u must be a contiguous float64 tensor of length 4N on the device")
        T = TABLEAUS[tab] if isinstance(tab, str) else tab
        self._check(lib().xrb_step_tableau(self.h, C.byref(T), _ptr(u), float(dt)))
        return u

    def step_batch(self, method, U, dts, return_stats=False):
        """One step for every member of U (float64 device tensor [nm, 4N],
        updated in place) with per-member step sizes dts."""
        self._stream()
        if not (U.is_contiguous() and U.dtype == self.torch.float64 and U.dim() == 2
                and U.shape[1] == self.N and U.device == self.device):
            raise ValueError("U must be a contiguous float64 [nm, 4N] tensor on the device")
        nm = U.shape[0]
        d = np.ascontiguousarray(dts, dtype=np.float64)
        if d.shape != (nm,):
            raise ValueError("one step size per member expected")
        mid = METHODS[method] if isinstance(method, str) else int(method)
        st = (PhiStats * (3 * nm))()
        self._check(lib().xrb_step_batch(self.h, mid, nm, _ptr(U), d.ctypes.data_as(_dp), st))
        if return_stats:
            return U, [[st[3 * k + c].asdict() for c in range(3)] for k in range(nm)]
        return U

    _gstream = None

    def step_batch_capture(self, method, U, dts):
        """Capture one replayed batched step of U (float64 device tensor
        [nm, 4N]) with step sizes dts as a HIP graph (xrb_step_batch_capture;
        the context must be in REPLAY mode with per-member schedules).  The
        capture runs on a side stream of this context (a graph cannot be
        captured on the null stream); U and dts stay baked into the graph."""
        if not (U.is_contiguous() and U.dtype == self.torch.float64 and U.dim() == 2
                and U.shape[1] == self.N and U.device == self.device):
            raise ValueError("U must be a contiguous float64 [nm, 4N] tensor on the device")
        nm = U.shape[0]
        d = np.ascontiguousarray(dts, dtype=np.float64)
        if d.shape != (nm,):
            raise ValueError("one step size per member expected")
        mid = METHODS[method] if isinstance(method, str) else int(method)
        if self._gstream is None:
            self._gstream = self.torch.cuda.Stream(device=self.device)
        self._gstream.wait_stream(self.torch.cuda.current_stream(self.device))
        lib().xrb_set_stream(self.h, C.c_void_p(self._gstream.cuda_stream))
        try:
            self._check(lib().xrb_step_batch_capture(self.h, mid, nm, _ptr(U), d.ctypes.data_as(_dp)))
        finally:
            self._stream()
        self._graph_keep = (U, d)
        return U

    def graph_launch(self):
        """Run the captured batched step (xrb_graph_launch) and wait for it."""
        if self._gstream is None:
            raise ValueError("nothing captured")
        cur = self.torch.cuda.current_stream(self.device)
        self._gstream.wait_stream(cur)
        lib().xrb_set_stream(self.h, C.c_void_p(self._gstream.cuda_stream))
        try:
            self._check(lib().xrb_graph_launch(self.h))
        finally:
            self._stream()
        cur.wait_stream(self._gstream)

    def step_stats(self):
        st = (PhiStats * 3)()
        self._check(lib().xrb_step_stats(self.h, st))
        return [s.asdict() for s in st]

    def reset_history(self):
        self._check(lib().xrb_reset_history(self.h))

    def schedule_mode(self, mode):
        self._check(lib().xrb_schedule_mode(self.h, int(mode)))

    def schedule_set(self, arr):
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).reshape(-1, 3))
        self._check(lib().xrb_schedule_set(self.h, a.ctypes.data_as(_dp), len(a)))

    def schedule_set_member(self, k, arr):
        """Replay schedule of ensemble member k (rows tau, m, flags)."""
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).reshape(-1, 3))
        self._check(lib().xrb_schedule_set_member(self.h, int(k), a.ctypes.data_as(_dp), len(a)))

    def schedule_get_member(self, k):
        """Schedule recorded for ensemble member k."""
        n = C.c_int()
        self._check(lib().xrb_schedule_get_member(self.h, int(k), None, 0, C.byref(n)))
        a = np.zeros((max(1, n.value), 3))
        self._check(lib().xrb_schedule_get_member(self.h, int(k), a.ctypes.data_as(_dp),
                                                  n.value, C.byref(n)))
        return a[:n.value]

    def profile(self, every=1):
        """Time every `every`-th launch of each kernel with HIP events
        (counters zeroed); every = 0 disables."""
        self._check(lib().xrb_profile(self.h, int(every)))

    def profile_overhead(self, reps=200):
        """Microseconds one event pair adds to a timed launch (xrb_profile_overhead)."""
        self._stream()
        us = C.c_double()
        self._check(lib().xrb_profile_overhead(self.h, int(reps), C.byref(us)))
        return us.value

    def profile_get(self):
        """{kernel: (device ms over the timed launches, timed launches, all launches)}."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms = C.c_double()
            cnt = C.c_int64()
            allc = C.c_int64()
            self._check(lib().xrb_profile_get(self.h, k, C.byref(ms), C.byref(cnt),
                                              C.byref(allc)))
            out[name] = (ms.value, cnt.value, allc.value)
        return out

    def schedule_get(self):
        n = C.c_int()
        self._check(lib().xrb_schedule_get(self.h, None, 0, C.byref(n)))
        a = np.zeros((max(1, n.value), 3))
        self._check(lib().xrb_schedule_get(self.h, a.ctypes.data_as(_dp), n.value, C.byref(n)))
        return a[:n.value]


def _trajectory_function():
    torch = _torch()

    class _Trajectory(torch.autograd.Function):
        """States u_0..u_K of K steps of a scheme, differentiable in u_0.
        Forward: each step runs in RECORD mode and its schedule is kept with a
        checkpoint of its input state.  Backward: for k = K..1,
        g <- vjp(u_{k-1}, g) + dL/du_{k-1}, each VJP replaying step k's
        schedule (xrb_step_vjp recomputes the step on the device)."""

        @staticmethod
        def forward(fctx, u0, ctx, dts, method):
            states = [u0.detach().clone()]
            scheds = []
            u = u0.detach().clone()
            ctx.reset_history()
            for dt in dts:
                ctx.schedule_set(np.zeros((0, 3)))
                ctx.schedule_mode(RECORD)
                try:
                    ctx.step(method, u, float(dt))
                finally:
                    ctx.schedule_mode(FREE)
                scheds.append(ctx.schedule_get())
                states.append(u.clone())
            fctx.ctx, fctx.dts, fctx.method, fctx.scheds = ctx, list(dts), method, scheds
            fctx.save_for_backward(*states[:-1])
            return torch.stack(states)

        @staticmethod
        def backward(fctx, grad):
            states = fctx.saved_tensors
            g = grad[-1].contiguous()
            for k in range(len(fctx.dts), 0, -1):
                g = fctx.ctx.step_vjp(fctx.method, states[k - 1], fctx.dts[k - 1], g,
                                      sched=fctx.scheds[k - 1])
                g = g + grad[k - 1]
            return g, None, None, None

    return _Trajectory


_TRAJ = None


def trajectory(ctx, u0, dts, method="exprb42"):
    """Run len(dts) steps from u0 (float64 device tensor of length 4N) and
    return the states [K+1, 4N]; with u0.requires_grad the result is
    differentiable in u0 (backward by per-step vector-Jacobian products on the
    recorded schedules; exprb42 only)."""
    global _TRAJ
    if method != "exprb42":
        raise ValueError("trajectory gradients are available for exprb42")
    if _TRAJ is None:
        _TRAJ = _trajectory_function()
    return _TRAJ.apply(u0, ctx, list(dts), method)
