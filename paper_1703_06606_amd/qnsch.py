"""ctypes binding of ``libqnsch_hip.so`` (the C ABI of ``include/qnsch.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
Importing this module does not need a GPU; creating a context does.  If the
library has not been built the binding raises instead of falling back.
"""
import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(PKG, "libqnsch_hip.so")

OK, EINVAL, ENOMEM, ENOCONV, EDIVERGED, EDEVICE, EBUSY = 0, -1, -2, -3, -4, -5, -6
WALL, PERIODIC = 0, 1
FP64, MIXED = 0, 1
PRIMITIVE, PROJECTION = 0, 1

# every exported symbol declared in include/qnsch.h
SYMBOLS = ("qnsch_default_opts", "qnsch_create", "qnsch_destroy", "qnsch_last_error", "qnsch_levels",
           "qnsch_set_state", "qnsch_set_iterate", "qnsch_get_state", "qnsch_step", "qnsch_begin_step", "qnsch_vcycle",
           "qnsch_accelerate",
           "qnsch_residual", "qnsch_halfsweep", "qnsch_end_step", "qnsch_lin_apply", "qnsch_mass", "qnsch_energy",
           "qnsch_dissipation", "qnsch_diagnostics", "qnsch_stats",
           "qnsch_synchronize", "qnsch_set_allocator", "qnsch_graphs", "qnsch_profile", "qnsch_profile_ops", "qnsch_profile_read", "qnsch_profile_breakdown", "qnsch_copy_probe",
           "qnsch_footprint", "qnsch_server_create", "qnsch_server_destroy", "qnsch_server_last_error", "qnsch_server_submit",
           "qnsch_server_progress", "qnsch_server_poll", "qnsch_server_result", "qnsch_server_stats",
           "qnsch_server_latency",
           "qnsch_default_eta", "qnsch_residual_noalloc", "qnsch_residual_noalloc_error")


# operation classes of qnsch_profile_breakdown, in the library's numbering
OP_NAMES = ("begin", "restrict_n", "residual0", "residual", "halfsweep", "restrict", "coarse_solve",
            "prolong", "step_end", "restore", "mx_restrict_n", "mx_halfsweep", "mx_restrict", "mx_coarse_solve",
            "mx_prolong", "mx_update", "dissipation", "diagnostics", "pj_final", "smooth", "mx_smooth", "residual_acc",
            "accelerate", "fused_sweep", "mx_fused_sweep")


class QnschError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("qnsch error %d: %s" % (code, msg))
        self.code = code


class Grid(C.Structure):
    _fields_ = [("m1", C.c_int32), ("m2", C.c_int32), ("Lx", C.c_double), ("Ly", C.c_double),
                ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("levels", C.c_int32)]


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rho1", "rho2", "visc1", "visc2", "Re", "We", "inv_Fr", "Pe", "M",
                                           "eps", "eta", "mob_reg", "rho_ref")]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("tol", C.c_double), ("max_vcycles", C.c_int32), ("nu1", C.c_int32),
                ("nu2", C.c_int32), ("nu_coarse", C.c_int32), ("vanka_omega", C.c_double),
                ("smoother", C.c_int32), ("scheme", C.c_int32), ("coarse_omega", C.c_double),
                ("accel", C.c_int32), ("blocking", C.c_int32)]


HIST = 128  # QNSCH_HIST


class StepStats(C.Structure):
    _fields_ = [("vcycles", C.c_int32), ("res", C.c_double * 5), ("res0", C.c_double * 5), ("step_ms", C.c_double),
                ("hist_len", C.c_int32), ("hist", (C.c_double * 5) * HIST), ("dissipation", C.c_double * 5)]


_lib = None
# qnsch_alloc_fn / qnsch_free_fn
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)
# every pair of callbacks ever given to the library, kept alive for the
# process: a context calls the functions it was created with until it is
# destroyed, also after the allocator was changed
_allocators = []


def lib():
    """Load the HIP library; raises if it is missing (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError("libqnsch_hip.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB)
        P = C.POINTER(C.c_double)
        vp = C.c_void_p
        L.qnsch_default_opts.argtypes = [C.POINTER(Opts)]
        L.qnsch_default_opts.restype = None
        L.qnsch_default_eta.argtypes = [C.c_double, C.c_double]
        L.qnsch_default_eta.restype = C.c_double
        L.qnsch_create.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.POINTER(Opts), vp, C.POINTER(vp)]
        L.qnsch_destroy.argtypes = [vp]
        L.qnsch_destroy.restype = None
        L.qnsch_last_error.argtypes = [vp]
        L.qnsch_last_error.restype = C.c_char_p
        L.qnsch_levels.argtypes = [vp]
        L.qnsch_set_state.argtypes = [vp, P, P, P, P, P]
        L.qnsch_set_iterate.argtypes = [vp, P, P, P, P, P]
        L.qnsch_get_state.argtypes = [vp, P, P, P, P, P]
        L.qnsch_step.argtypes = [vp, C.c_double]
        L.qnsch_begin_step.argtypes = [vp, C.c_double]
        L.qnsch_vcycle.argtypes = [vp]
        L.qnsch_accelerate.argtypes = [vp]
        L.qnsch_residual.argtypes = [vp, P, P]
        L.qnsch_halfsweep.argtypes = [vp, C.c_int]
        L.qnsch_end_step.argtypes = [vp]
        L.qnsch_lin_apply.argtypes = [vp, P, P]
        L.qnsch_mass.argtypes = [vp, P]
        L.qnsch_energy.argtypes = [vp, P]
        L.qnsch_dissipation.argtypes = [vp, P]
        L.qnsch_diagnostics.argtypes = [vp, P]
        L.qnsch_stats.argtypes = [vp, C.POINTER(StepStats)]
        L.qnsch_synchronize.argtypes = [vp]
        L.qnsch_graphs.argtypes = [vp, C.c_int]
        L.qnsch_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
        L.qnsch_profile.argtypes = [vp, C.c_int]
        L.qnsch_profile_ops.argtypes = [vp, C.c_uint64]
        L.qnsch_profile_read.argtypes = [vp, P]
        L.qnsch_profile_breakdown.argtypes = [vp, C.POINTER(C.c_int32), P, C.c_int32]
        L.qnsch_copy_probe.argtypes = [C.c_size_t, C.c_int, P]
        L.qnsch_residual_noalloc.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_double] + [vp] * 8 + [vp, P]
        L.qnsch_residual_noalloc_error.argtypes = []
        L.qnsch_residual_noalloc_error.restype = C.c_char_p
        L.qnsch_footprint.argtypes = [C.POINTER(Grid), C.POINTER(Opts)]
        L.qnsch_footprint.restype = C.c_size_t
        L.qnsch_server_create.argtypes = [C.c_size_t, C.c_int32, C.c_int32, vp, C.POINTER(vp)]
        L.qnsch_server_destroy.argtypes = [vp]
        L.qnsch_server_destroy.restype = None
        L.qnsch_server_last_error.argtypes = [vp]
        L.qnsch_server_last_error.restype = C.c_char_p
        L.qnsch_server_submit.argtypes = [vp, C.POINTER(Grid), C.POINTER(Params), C.POINTER(Opts), P, C.c_int32,
                                          C.c_double, C.POINTER(C.c_uint64)]
        L.qnsch_server_progress.argtypes = [vp, C.c_int32]
        L.qnsch_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.qnsch_server_result.argtypes = [vp, C.c_uint64, P, P, P, P, P, P, P, P, C.POINTER(C.c_int32), P]
        L.qnsch_server_stats.argtypes = [vp, P]
        L.qnsch_server_latency.argtypes = [vp, P, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def set_allocator(alloc=None, free=None):
    """device memory of contexts created from now on: alloc(bytes) -> int
    device address (256-byte aligned, 0 on failure) and free(address, bytes),
    or both None for hipMalloc / hipFree (qnsch_set_allocator)"""
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        rc = lib().qnsch_set_allocator(ALLOC_FN(), FREE_FN(), None)
    else:
        cbs = (ALLOC_FN(lambda n, user: alloc(n) or None), FREE_FN(lambda ptr, n, user: free(ptr, n)))
        _allocators.append(cbs)
        rc = lib().qnsch_set_allocator(cbs[0], cbs[1], None)
    if rc != OK:
        raise QnschError(rc, "qnsch_set_allocator failed")


def copy_probe(n_doubles, reps=20):
    """{GB/s, ms per copy} of a plain device copy kernel of n doubles"""
    out = np.zeros(2)
    rc = lib().qnsch_copy_probe(n_doubles, reps, _ptr(out))
    if rc != OK:
        raise QnschError(rc, "copy probe failed")
    return float(out[0]), float(out[1])


def residual_noalloc(grid, params, dt, w, wn, stream=None):
    """qnsch_residual_noalloc: the residual norms of the iterate w (device
    pointers to c, mu, p, u, v) with the time-n data wn (device pointers to
    c, u, v), without allocating; returns the five norms"""
    g, p, _ = _structs(grid, params, None)
    out = np.zeros(5)
    ptrs = [C.c_void_p(int(w[k])) for k in ("c", "mu", "p", "u", "v")] + \
           [C.c_void_p(int(wn[k])) for k in ("c", "u", "v")]
    rc = lib().qnsch_residual_noalloc(C.byref(g), C.byref(p), float(dt), *ptrs,
                                      C.c_void_p(stream) if stream else None, _ptr(out))
    if rc != OK:
        raise QnschError(rc, lib().qnsch_residual_noalloc_error().decode())
    return out


def default_eta(rho1, rho2):
    """interface ratio parameter of sec. 8.1 for the density pair"""
    return float(lib().qnsch_default_eta(C.c_double(rho1), C.c_double(rho2)))


def default_opts():
    o = Opts()
    lib().qnsch_default_opts(C.byref(o))
    return {n: getattr(o, n) for n, _ in Opts._fields_}


class Solver:
    """One simulation on the GPU.  Fields are (m2, m1) numpy arrays; u[j, i]
    is the west face of cell (i, j), v[j, i] its south face."""

    def __init__(self, grid, params, opts=None, stream=None):
        self.m1, self.m2 = int(grid["m1"]), int(grid["m2"])
        g = Grid(self.m1, self.m2, grid["Lx"], grid["Ly"], grid["bcx"], grid["bcy"], grid.get("levels", 0))
        p = Params(*[float(params[n]) for n, _ in Params._fields_])
        o = None
        if opts is not None:
            d = default_opts()
            d.update(opts)
            o = Opts(*[d[n] for n, _ in Opts._fields_])
        h = C.c_void_p()
        rc = lib().qnsch_create(C.byref(g), C.byref(p), C.byref(o) if o is not None else None,
                                C.c_void_p(stream) if stream else None, C.byref(h))
        if rc != OK:
            raise QnschError(rc, "qnsch_create rejected the configuration")
        self.h = h
        self._L = lib()  # kept for __del__, which may run after the module's globals are cleared

    def __del__(self):
        if getattr(self, "h", None) and getattr(self, "_L", None) is not None:
            self._L.qnsch_destroy(self.h)
            self.h = None

    def _chk(self, rc):
        if rc != OK:
            raise QnschError(rc, lib().qnsch_last_error(self.h).decode())
        return rc

    @property
    def levels(self):
        return lib().qnsch_levels(self.h)

    def _f(self, a):
        return None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.m2, self.m1)

    def set_state(self, c, mu=None, p=None, u=None, v=None):
        arrs = [self._f(a) for a in (c, mu, p, u, v)]
        self._chk(lib().qnsch_set_state(self.h, *[_ptr(a) for a in arrs]))

    def get_state(self):
        out = [np.zeros((self.m2, self.m1)) for _ in range(5)]
        self._chk(lib().qnsch_get_state(self.h, *[_ptr(a) for a in out]))
        return dict(zip(("c", "mu", "p", "u", "v"), out))

    def step(self, dt, check=True):
        rc = lib().qnsch_step(self.h, dt)
        if check:
            self._chk(rc)
        return rc

    def begin_step(self, dt):
        self._chk(lib().qnsch_begin_step(self.h, dt))

    def vcycle(self):
        self._chk(lib().qnsch_vcycle(self.h))

    def accelerate(self):
        self._chk(lib().qnsch_accelerate(self.h))

    def residual(self):
        r = np.zeros((5, self.m2, self.m1))
        n = np.zeros(5)
        self._chk(lib().qnsch_residual(self.h, _ptr(r), _ptr(n)))
        return r, n

    def halfsweep(self, colour):
        self._chk(lib().qnsch_halfsweep(self.h, colour))

    def end_step(self):
        self._chk(lib().qnsch_end_step(self.h))

    def lin_apply(self, dw):
        """J(w) dw at the current iterate (mixed-precision contexts), shape
        (5, m2, m1)"""
        dw = np.ascontiguousarray(dw, dtype=np.float64).reshape(5, self.m2, self.m1)
        out = np.zeros_like(dw)
        self._chk(lib().qnsch_lin_apply(self.h, _ptr(dw), _ptr(out)))
        return out

    def mass(self):
        out = np.zeros(2)
        self._chk(lib().qnsch_mass(self.h, _ptr(out)))
        return out

    def energy(self):
        out = np.zeros(5)
        self._chk(lib().qnsch_energy(self.h, _ptr(out)))
        return out

    def dissipation(self):
        out = np.zeros(5)
        self._chk(lib().qnsch_dissipation(self.h, _ptr(out)))
        return out

    def diagnostics(self):
        """dict: rising velocity V_c, integral of c, max and L2 norm of the
        discrete divergence, highest/lowest c = 1/2 crossing, crossing in
        the first column, integral of the divergence"""
        out = np.zeros(8)
        self._chk(lib().qnsch_diagnostics(self.h, _ptr(out)))
        return dict(zip(("V_c", "c_integral", "div_max", "div_l2", "y_top", "y_bottom", "y_col0", "div_integral"),
                        out))

    def stats(self):
        s = StepStats()
        self._chk(lib().qnsch_stats(self.h, C.byref(s)))
        hist = np.array([list(s.hist[k]) for k in range(s.hist_len)]).reshape(s.hist_len, 5)
        return dict(vcycles=s.vcycles, res=list(s.res), res0=list(s.res0), step_ms=s.step_ms, hist=hist,
                    dissipation=np.array(list(s.dissipation)))

    def synchronize(self):
        self._chk(lib().qnsch_synchronize(self.h))

    def graphs(self, enable):
        """replay each cycle's fixed launches as a captured HIP graph, or
        launch them one by one (the default)"""
        self._chk(lib().qnsch_graphs(self.h, int(bool(enable))))

    def profile(self, mode):
        """0 off, 1 (or True) finest half-sweeps, 2 every launch"""
        self._chk(lib().qnsch_profile(self.h, int(mode)))

    def profile_read(self):
        out = np.zeros(2)
        self._chk(lib().qnsch_profile_read(self.h, _ptr(out)))
        return int(out[0]), float(out[1])

    def profile_ops(self, names):
        """time every launch of the named operations (OP_NAMES) on every level,
        with the kernels' own timestamps where an operation is one kernel"""
        mask = 0
        for n in names:
            mask |= 1 << OP_NAMES.index(n)
        self._chk(lib().qnsch_profile_ops(self.h, mask))

    def profile_breakdown(self, by_level=False):
        """launches and milliseconds timed since profile(2) or profile_ops:
        {operation name + "_fine" or "_coarse": (launches, ms)}, or with
        by_level {(operation name, level): (launches, ms)}"""
        cap = 16 * len(OP_NAMES)
        kinds = (C.c_int32 * cap)()
        out = np.zeros(2 * cap)
        n = lib().qnsch_profile_breakdown(self.h, kinds, _ptr(out), cap)
        if n < 0:
            self._chk(n)
        res = {}
        for k in range(min(n, cap)):
            t = kinds[k]
            op, lev = OP_NAMES[t // 16], t % 16
            key = (op, lev) if by_level else op + ("_coarse" if lev else "_fine")
            a, b = res.get(key, (0, 0.0))
            res[key] = (a + int(out[2 * k]), b + float(out[2 * k + 1]))
        return res

    def set_iterate(self, c, mu=None, p=None, u=None, v=None):
        arrs = [self._f(a) for a in (c, mu, p, u, v)]
        self._chk(lib().qnsch_set_iterate(self.h, *[_ptr(a) for a in arrs]))

    def set_time_n_and_iterate(self, wn, w, dt):
        """time-n data from the state dict wn, then the iterate w"""
        self.set_state(*[wn.get(k) for k in ("c", "mu", "p", "u", "v")])
        self.begin_step(dt)
        self.set_iterate(*[w.get(k) for k in ("c", "mu", "p", "u", "v")])


def _structs(grid, params, opts):
    g = Grid(int(grid["m1"]), int(grid["m2"]), grid["Lx"], grid["Ly"], grid["bcx"], grid["bcy"], grid.get("levels", 0))
    p = Params(*[float(params[n]) for n, _ in Params._fields_])
    o = None
    if opts is not None:
        d = default_opts()
        d.update(opts)
        o = Opts(*[d[n] for n, _ in Opts._fields_])
    return g, p, o


def footprint(grid, opts=None):
    """device bytes of a context of this grid (and precision)"""
    g, _, o = _structs(grid, dict((n, 1.0) for n, _ in Params._fields_), opts)
    return int(lib().qnsch_footprint(C.byref(g), C.byref(o) if o is not None else None))


class Server:
    """Continuous-batching server of many simulations (qnsch_server_*)."""

    def __init__(self, hbm_budget, max_slots, lanes=3, stream=None):
        h = C.c_void_p()
        rc = lib().qnsch_server_create(int(hbm_budget), int(max_slots), int(lanes),
                                       C.c_void_p(stream) if stream else None, C.byref(h))
        if rc != OK:
            raise QnschError(rc, "qnsch_server_create failed")
        self.h = h
        self._L = lib()
        self.shapes = {}

    def __del__(self):
        if getattr(self, "h", None) and getattr(self, "_L", None) is not None:
            self._L.qnsch_server_destroy(self.h)
            self.h = None

    def submit(self, grid, params, opts, c0, nsteps, dt):
        g, p, o = _structs(grid, params, opts)
        c0 = np.ascontiguousarray(c0, dtype=np.float64).reshape(int(grid["m2"]), int(grid["m1"]))
        rid = C.c_uint64()
        rc = lib().qnsch_server_submit(self.h, C.byref(g), C.byref(p), C.byref(o) if o is not None else None,
                                       _ptr(c0), int(nsteps), float(dt), C.byref(rid))
        if rc != OK:
            raise QnschError(rc, "submit rejected")
        self.shapes[rid.value] = (int(grid["m2"]), int(grid["m1"]), int(nsteps))
        return rid.value

    def progress(self, max_ticks=1):
        rc = lib().qnsch_server_progress(self.h, int(max_ticks))
        if rc < 0:
            raise QnschError(rc, lib().qnsch_server_last_error(self.h).decode())
        return rc

    def poll(self, rid):
        st, status = C.c_int32(), C.c_int32()
        self_rc = lib().qnsch_server_poll(self.h, C.c_uint64(rid), C.byref(st), C.byref(status))
        if self_rc != OK:
            raise QnschError(self_rc, "unknown request")
        return st.value, status.value

    def result(self, rid):
        m2, m1, ns = self.shapes[rid]
        f = [np.zeros((m2, m1)) for _ in range(5)]
        mass, en, ms = np.zeros((ns, 2)), np.zeros((ns, 5)), np.zeros(ns)
        vc = (C.c_int32 * ns)()
        times = np.zeros(2)
        rc = lib().qnsch_server_result(self.h, C.c_uint64(rid), *[_ptr(a) for a in f], _ptr(mass), _ptr(en), _ptr(ms),
                                       vc, _ptr(times))
        out = dict(zip(("c", "mu", "p", "u", "v"), f))
        out.update(status=rc, mass=mass, energy=en, step_ms=ms, vcycles=np.array(vc[:]), wait_ms=times[0],
                   total_ms=times[1])
        return out

    def latency(self):
        """(p50 step ms, p99 step ms, cell-steps/s)"""
        out = np.zeros(3)
        rc = lib().qnsch_server_latency(self.h, _ptr(out[0:]), _ptr(out[1:]), _ptr(out[2:]))
        if rc != OK:
            raise QnschError(rc, "latency failed")
        return float(out[0]), float(out[1]), float(out[2])

    def stats(self):
        out = np.zeros(12)
        self_rc = lib().qnsch_server_stats(self.h, _ptr(out))
        if self_rc != OK:
            raise QnschError(self_rc, "stats failed")
        keys = ("p50_ms", "p99_ms", "cell_steps", "wall_s", "cell_steps_per_s", "steps", "launches", "ticks",
                "host_admit_ms", "host_finish_ms", "host_wait_ms", "contexts_created")
        return dict(zip(keys, out))
