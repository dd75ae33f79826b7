"""ctypes binding of the FP64 CPU oracle (``libqnsch_oracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU package.  The oracle itself is
plain C in ``qnsch_oracle.c``; this file only marshals arguments.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libqnsch_oracle.so")
SRC = os.path.join(HERE, "qnsch_oracle.c")

WALL, PERIODIC = 0, 1
OK, ENOCONV, EDIVERGED = 0, -3, -4
MAXV = 200


def build():
    """Compile the oracle (gcc, FP64, no fast-math; OpenMP over the
    independent cells of a colour, results independent of the thread count)."""
    cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-Wall", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)


class _Grid(C.Structure):
    _fields_ = [("m1", C.c_int), ("m2", C.c_int), ("Lx", C.c_double), ("Ly", C.c_double),
                ("bcx", C.c_int), ("bcy", C.c_int), ("levels", C.c_int)]


class _Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rho1", "rho2", "visc1", "visc2", "Re", "We", "inv_Fr",
                                           "Pe", "M", "eps", "eta", "mob_reg", "rho_ref")]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_vcycles", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("nu_coarse", C.c_int), ("vanka_omega", C.c_double), ("smoother", C.c_int),
                ("scheme", C.c_int), ("coarse_omega", C.c_double), ("accel", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Opts)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_levels.argtypes = [C.c_void_p]
        L.orc_set_state.argtypes = [C.c_void_p, P, P, P, P, P]
        L.orc_get_state.argtypes = [C.c_void_p, P, P, P, P, P]
        L.orc_begin_step.argtypes = [C.c_void_p, C.c_double]
        L.orc_residual.argtypes = [C.c_void_p, P, P]
        L.orc_halfsweep.argtypes = [C.c_void_p, C.c_int]
        L.orc_vcycle.argtypes = [C.c_void_p]
        L.orc_accelerate.argtypes = [C.c_void_p]
        L.orc_accel_coeffs.argtypes = [C.c_void_p, P]
        L.orc_solve.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_double]
        L.orc_stats.argtypes = [C.c_void_p, P]
        L.orc_mass.argtypes = [C.c_void_p, P]
        L.orc_energy.argtypes = [C.c_void_p, P]
        L.orc_dissipation.argtypes = [C.c_void_p, P]
        L.orc_velocity_np1.argtypes = [C.c_void_p, P, P]
        L.orc_diagnostics.argtypes = [C.c_void_p, P]
        L.orc_num_unknowns.argtypes = [C.c_void_p]
        L.orc_dense.argtypes = [C.c_void_p, P, P]
        L.orc_add_unknowns.argtypes = [C.c_void_p, P]
        L.orc_jvp.argtypes = [C.c_void_p, P, P]
        L.orc_material.argtypes = [C.c_void_p, C.c_double, C.c_double, P]
        L.orc_threads.argtypes = [C.c_int]
        L.orc_restrict.argtypes = [C.c_void_p, C.c_int, P, P]
        L.orc_prolong.argtypes = [C.c_void_p, C.c_int, P, P]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def threads(n=0):
    """set the oracle's thread count (n > 0); returns the count in use"""
    return lib().orc_threads(int(n))


class Oracle:
    """One simulation on the CPU oracle.  Fields are numpy arrays of shape
    (m2, m1) (row j, column i); u[j, i] is the west face of cell (i, j) and
    v[j, i] the south face."""

    def __init__(self, grid, params, opts):
        self.m1, self.m2 = grid["m1"], grid["m2"]
        g = _Grid(grid["m1"], grid["m2"], grid["Lx"], grid["Ly"], grid["bcx"], grid["bcy"], grid.get("levels", 0))
        p = _Params(*[float(params[n]) for n, _ in _Params._fields_])
        o = _Opts(opts["tol"], opts["max_vcycles"], opts["nu1"], opts["nu2"], opts["nu_coarse"], opts["vanka_omega"],
                  opts.get("smoother", 1), opts.get("scheme", 0), opts.get("coarse_omega", 0.0), opts.get("accel", 2))
        self.h = lib().orc_create(C.byref(g), C.byref(p), C.byref(o))
        if not self.h:
            raise ValueError("oracle rejected the grid")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    @property
    def levels(self):
        return lib().orc_levels(self.h)

    def _f(self, a):
        return None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.m2, self.m1)

    def set_state(self, c, mu=None, p=None, u=None, v=None):
        arrs = [self._f(a) for a in (c, mu, p, u, v)]
        lib().orc_set_state(self.h, *[_ptr(a) for a in arrs])

    def get_state(self):
        out = [np.zeros((self.m2, self.m1)) for _ in range(5)]
        lib().orc_get_state(self.h, *[_ptr(a) for a in out])
        return dict(zip(("c", "mu", "p", "u", "v"), out))

    def begin_step(self, dt):
        lib().orc_begin_step(self.h, dt)

    def residual(self):
        r = np.zeros((5, self.m2, self.m1))
        n = np.zeros(5)
        lib().orc_residual(self.h, _ptr(r), _ptr(n))
        return r, n

    def halfsweep(self, colour):
        lib().orc_halfsweep(self.h, colour)

    def vcycle(self):
        lib().orc_vcycle(self.h)

    def accelerate(self):
        lib().orc_accelerate(self.h)

    def accel_coeffs(self):
        """coefficients of the pending combination (the used ones)"""
        g = np.zeros(3)
        n = lib().orc_accel_coeffs(self.h, _ptr(g))
        return g[:n].copy()

    def solve(self):
        return lib().orc_solve(self.h)

    def step(self, dt):
        return lib().orc_step(self.h, dt)

    def stats(self):
        hist = np.zeros((MAXV + 1, 5))
        nv = lib().orc_stats(self.h, _ptr(hist))
        return nv, hist[: nv + 1].copy()

    def mass(self):
        out = np.zeros(2)
        lib().orc_mass(self.h, _ptr(out))
        return out

    def energy(self):
        out = np.zeros(5)
        lib().orc_energy(self.h, _ptr(out))
        return out

    def dissipation(self):
        out = np.zeros(5)
        lib().orc_dissipation(self.h, _ptr(out))
        return out

    def velocity_np1(self):
        """projection scheme: the velocity of time n+1 of the current iterate"""
        u, v = np.zeros((self.m2, self.m1)), np.zeros((self.m2, self.m1))
        lib().orc_velocity_np1(self.h, _ptr(u), _ptr(v))
        return u, v

    def diagnostics(self):
        out = np.zeros(8)
        lib().orc_diagnostics(self.h, _ptr(out))
        return dict(zip(("V_c", "c_integral", "div_max", "div_l2", "y_top", "y_bottom", "y_col0", "div_integral"),
                        out))

    def dense(self, jacobian=True):
        n = lib().orc_num_unknowns(self.h)
        N = np.zeros(n)
        J = np.zeros((n, n)) if jacobian else None
        lib().orc_dense(self.h, _ptr(N), _ptr(J))
        return N, J

    def add_unknowns(self, dx):
        dx = np.ascontiguousarray(dx, dtype=np.float64)
        lib().orc_add_unknowns(self.h, _ptr(dx))

    def material(self, c1, c0):
        out = np.zeros(6)
        lib().orc_material(self.h, c1, c0, _ptr(out))
        return dict(zip(("rho", "visc", "mob", "F", "g", "r"), out))

    def set_time_n_and_iterate(self, wn, w, dt):
        """time-n data from the state dict wn, then the iterate w (both dicts
        of c, mu, p, u, v), ready for residual evaluation at step size dt"""
        self.set_state(*[wn.get(k) for k in ("c", "mu", "p", "u", "v")])
        self.begin_step(dt)
        self.set_state(*[w.get(k) for k in ("c", "mu", "p", "u", "v")])

    def level_shape(self, l):
        """(m2, m1) of level l"""
        return self.m2 >> l, self.m1 >> l

    def restrict(self, l, fine):
        """the V-cycle's restriction of 5 fields of level l (shape (5, m2_l, m1_l))
        to level l + 1"""
        f = np.ascontiguousarray(fine, dtype=np.float64).reshape((5,) + self.level_shape(l))
        out = np.zeros((5,) + self.level_shape(l + 1))
        lib().orc_restrict(self.h, l, _ptr(f), _ptr(out))
        return out

    def prolong(self, l, e, fine=None):
        """fine + P e: the V-cycle's prolongation of a correction e of level
        l + 1 (shape (5, m2_l+1, m1_l+1)) added to 5 fields of level l"""
        e = np.ascontiguousarray(e, dtype=np.float64).reshape((5,) + self.level_shape(l + 1))
        out = np.zeros((5,) + self.level_shape(l)) if fine is None else \
            np.array(fine, dtype=np.float64).reshape((5,) + self.level_shape(l))
        lib().orc_prolong(self.h, l, _ptr(e), _ptr(out))
        return out

    def jvp(self, d):
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(5, self.m2, self.m1)
        out = np.zeros_like(d)
        lib().orc_jvp(self.h, _ptr(d), _ptr(out))
        return out
