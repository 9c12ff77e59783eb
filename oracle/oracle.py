"""ctypes view of the FP64 CPU oracle in ``oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product path never imports
it.  The oracle follows arXiv 2512.20252 step by step (Sections 2-4); see the
header of ``oracle.c`` for the layout and the per-function citations.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

GEOMETRY = {"none": 0, "circle": 1, "ellipse": 2, "airfoil": 3, "sphere": 4}
OUTER = {"freestream": 0, "periodic": 1, "walls": 2, "specular": 3}
RULE = {"midpoint": 0, "trapezoid": 1, "stretched": 2, "refined": 3}
WEIGHTS = {"cell": 0, "jacobian": 1}
# "f32_absolute" selects how the library stores FP32 values; the FP64 oracle
# has no such choice and ignores it
FLAGS = {"no_cutcell": 1, "no_upwind": 2, "implicit": 4, "face_limit": 8, "naive": 16, "no_aux": 32,
         "f32_absolute": 0}

CL_GAS, CL_SOLID, CL_CUT_G, CL_CUT_S = 0, 1, 2, 3


def build(verbose=False):
    """Compile the oracle with plain IEEE semantics (no contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-shared", "-fPIC", "-o", LIB_PATH, SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)


class _Case(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("outer", ctypes.c_int), ("vn", ctypes.c_int * 3),
                ("vlo", ctypes.c_double * 3), ("vhi", ctypes.c_double * 3), ("vrule", ctypes.c_int),
                ("gkind", ctypes.c_int), ("gcen", ctypes.c_double * 3), ("gsize", ctypes.c_double * 3),
                ("aoa", ctypes.c_double), ("Kn", ctypes.c_double), ("Ma", ctypes.c_double),
                ("Pr", ctypes.c_double), ("gam", ctypes.c_double), ("alpha", ctypes.c_double),
                ("Tw", ctypes.c_double), ("cfl", ctypes.c_double), ("omega", ctypes.c_double),
                ("avhs", ctypes.c_double), ("flags", ctypes.c_int), ("lid_u", ctypes.c_double),
                ("vstretch", ctypes.c_double), ("Uw", ctypes.c_double * 3), ("Ow", ctypes.c_double * 3),
                ("vref_amp", ctypes.c_double), ("vref_width", ctypes.c_double), ("vref_centre", ctypes.c_double * 3),
                ("vweights", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        L.or_create.restype = vp
        L.or_create.argtypes = [ctypes.POINTER(_Case), ip]
        L.or_destroy.argtypes = [vp]
        for name in ("or_init_freestream",):
            getattr(L, name).argtypes = [vp, dp, dp, ctypes.c_double]
        L.or_set_state.argtypes = [vp, dp, dp]
        L.or_get_state.argtypes = [vp, dp, dp]
        L.or_step.argtypes = [vp, ctypes.c_int]
        L.or_moments.argtypes = [vp, dp]
        L.or_tau.argtypes = [vp, dp]
        L.or_next_dt.argtypes = [vp]
        L.or_next_dt.restype = ctypes.c_double
        L.or_clock.argtypes = [vp, dp]
        L.or_forces.argtypes = [vp, dp, dp, dp]
        L.or_info.argtypes = [vp, ip]
        L.or_velocity.argtypes = [vp, dp, dp]
        L.or_freestream.argtypes = [vp, dp, dp]
        L.or_mu0.argtypes = [vp]
        L.or_mu0.restype = ctypes.c_double
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_threads.argtypes = []
        L.or_threads.restype = ctypes.c_int
        L.or_index_sets.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_uint8)]
        L.or_pair_geometry.argtypes = [vp, dp, dp]
        L.or_fill_debug.argtypes = [vp] + [dp] * 7
        L.or_weights.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp]
        L.or_weights.restype = ctypes.c_int
        L.or_cell_moments.argtypes = [vp, dp, dp, dp]
        L.or_shakhov.argtypes = [vp, dp, dp, dp]
        L.or_maxwellian.argtypes = [vp, ctypes.c_double, dp, ctypes.c_double, dp, dp]
        L.or_cut_sets.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_uint8), dp]
        L.or_wall_distribution.argtypes = [vp, dp, dp, dp, dp, dp]
        L.or_wall_distribution.restype = ctypes.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _case_struct(case):
    c = _Case()
    d = case["dim"]
    c.dim = d
    for a in range(3):
        c.n[a] = case["n"][a] if a < d else 1
        c.lo[a] = case["lo"][a] if a < d else 0.0
        c.hi[a] = case["hi"][a] if a < d else 1.0
        c.vn[a] = case["vn"][a] if a < d else 1
        c.vlo[a] = case["vlo"][a] if a < d else 0.0
        c.vhi[a] = case["vhi"][a] if a < d else 0.0
        c.gcen[a] = case.get("center", (0.0, 0.0, 0.0))[a] if a < len(case.get("center", ())) else 0.0
        c.gsize[a] = case.get("size", (0.0, 0.0, 0.0))[a] if a < len(case.get("size", ())) else 0.0
    c.outer = OUTER[case.get("outer", "freestream")]
    c.vrule = RULE[case.get("rule", "midpoint")]
    c.gkind = GEOMETRY[case.get("geometry", "none")]
    c.aoa = case.get("aoa", 0.0)
    c.Kn, c.Ma, c.Pr, c.gam = case["Kn"], case["Ma"], case["Pr"], case["gamma"]
    c.alpha, c.Tw, c.cfl = case["alpha"], case["Tw"], case.get("cfl", 0.5)
    c.omega, c.avhs = case.get("omega_vhs", 0.81), case.get("a_vhs", 1.0)
    fl = 0
    for f in case.get("flags", ()):
        fl |= FLAGS[f]
    c.flags = fl
    c.lid_u = case.get("lid_u", 0.0)
    c.vstretch = case.get("vstretch", 0.0)
    Uw, Ow = case.get("U_w", (0.0, 0.0, 0.0)), case.get("Omega_w", (0.0, 0.0, 0.0))
    for a in range(3):
        c.Uw[a] = Uw[a] if a < len(Uw) else 0.0
        c.Ow[a] = Ow[a] if a < len(Ow) else 0.0
    c.vref_amp = case.get("vref_amp", 0.0)
    c.vref_width = case.get("vref_width", 1.0)
    rc = case.get("vref_centre", (0.0, 0.0, 0.0))
    for a in range(3):
        c.vref_centre[a] = rc[a] if a < len(rc) else 0.0
    c.vweights = WEIGHTS[case.get("vweights", "cell")]
    return c


def threads():
    """OpenMP threads the oracle's cell loops run on."""
    return int(lib().or_threads())


def set_threads(n):
    """Run the oracle's cell loops on n OpenMP threads from now on."""
    lib().or_set_threads(int(n))


class Oracle:
    """One oracle solve: geometry built at construction, state stepped on call."""

    def __init__(self, case):
        self.case = dict(case)
        self._c = _case_struct(case)
        err = ctypes.c_int(0)
        self._h = lib().or_create(ctypes.byref(self._c), ctypes.byref(err))
        if not self._h:
            raise ValueError(f"oracle: geometry rejected (code {err.value})")
        info = (ctypes.c_int * 7)()
        lib().or_info(self._h, info)
        self.dim, self.Nc, self.NV, self.NA, self.npairs, self.nfluid, self.nghost = list(info)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    # state ---------------------------------------------------------------
    def init_freestream(self, u=None, amp=0.0):
        u0 = _f64(u[0]).reshape(-1) if u is not None else None
        u1 = _f64(u[1]).reshape(-1) if (u is not None and self.NA == 2) else None
        lib().or_init_freestream(self._h, _dp(u0), _dp(u1), amp)

    def set_state(self, f):
        f0 = _f64(f[0]).reshape(-1)
        f1 = _f64(f[1]).reshape(-1) if self.NA == 2 else None
        lib().or_set_state(self._h, _dp(f0), _dp(f1))

    def get_state(self):
        f0 = np.empty((self.Nc, self.NV))
        f1 = np.empty((self.Nc, self.NV)) if self.NA == 2 else None
        lib().or_get_state(self._h, _dp(f0), _dp(f1))
        return (f0, f1) if self.NA == 2 else (f0,)

    def step(self, n=1):
        lib().or_step(self._h, int(n))

    # outputs -------------------------------------------------------------
    def moments(self):
        out = np.empty((self.Nc, 8))
        lib().or_moments(self._h, _dp(out))
        return out

    def tau(self):
        out = np.empty(self.Nc)
        lib().or_tau(self._h, _dp(out))
        return out

    def next_dt(self):
        return lib().or_next_dt(self._h)

    def clock(self):
        out = np.empty(3)
        lib().or_clock(self._h, _dp(out))
        return {"dt": out[0], "time": out[1], "step": int(out[2])}

    def forces(self):
        F = np.empty(3)
        cdcl = np.empty(2)
        wall = np.empty((max(self.npairs, 1), 17))
        lib().or_forces(self._h, _dp(F), _dp(cdcl), _dp(wall))
        return F, cdcl[0], cdcl[1], wall[: self.npairs]

    def velocity(self):
        xi = np.empty((self.NV, 3))
        w = np.empty(self.NV)
        lib().or_velocity(self._h, _dp(xi), _dp(w))
        return xi, w

    def freestream(self):
        f0 = np.empty(self.NV)
        f1 = np.empty(self.NV) if self.NA == 2 else None
        lib().or_freestream(self._h, _dp(f0), _dp(f1))
        return (f0, f1) if self.NA == 2 else (f0,)

    def mu0(self):
        return lib().or_mu0(self._h)

    def index_sets(self):
        solid = np.empty(self.Nc, dtype=np.uint8)
        pint = np.empty((max(self.npairs, 1), 32), dtype=np.int32)
        cls = np.empty((max(self.npairs, 1), self.NV), dtype=np.uint8)
        lib().or_index_sets(self._h, solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            pint.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            cls.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return {"solid": solid, "pairs": pint[: self.npairs], "cls": cls[: self.npairs]}

    def pair_geometry(self):
        g = np.empty((max(self.npairs, 1), 9))
        wg = np.empty((max(self.npairs, 1), self.NV))
        lib().or_pair_geometry(self._h, _dp(g), _dp(wg))
        return {"xw": g[: self.npairs, 0:3], "nw": g[: self.npairs, 3:6], "xsp": g[: self.npairs, 6:9],
                "wg": wg[: self.npairs]}

    def fill_debug(self):
        shp = (self.NA, max(self.npairs, 1), self.NV)
        arrs = [np.empty(shp) for _ in range(6)]
        rhow = np.empty(max(self.npairs, 1))
        lib().or_fill_debug(self._h, *[_dp(a) for a in arrs], _dp(rhow))
        names = ["fsp", "fgc", "fiw", "fw", "ghost", "face"]
        out = {n: a[:, : self.npairs] for n, a in zip(names, arrs)}
        out["rhow"] = rhow[: self.npairs]
        return out

    def weights(self, ip, k):
        w = np.empty(26)
        ns = lib().or_weights(self._h, int(ip), int(k), _dp(w))
        return w[:ns]

    def cell_moments(self, f0, f1=None):
        out = np.empty(8)
        lib().or_cell_moments(self._h, _dp(_f64(f0)), _dp(_f64(f1) if f1 is not None else None), _dp(out))
        return out

    def shakhov(self, mom8):
        g0 = np.empty(self.NV)
        g1 = np.empty(self.NV)
        lib().or_shakhov(self._h, _dp(_f64(mom8)), _dp(g0), _dp(g1))
        return (g0, g1) if self.NA == 2 else (g0,)

    def maxwellian(self, rho, U, T):
        g0 = np.empty(self.NV)
        g1 = np.empty(self.NV)
        U3 = _f64(list(U) + [0.0] * (3 - len(U)))
        lib().or_maxwellian(self._h, rho, _dp(U3), T, _dp(g0), _dp(g1) if self.NA == 2 else None)
        return (g0, g1) if self.NA == 2 else (g0,)

    def cut_sets(self, n):
        n3 = _f64(list(n) + [0.0] * (3 - len(n)))
        cls = np.empty(self.NV, dtype=np.uint8)
        wg = np.empty(self.NV)
        lib().or_cut_sets(self._h, _dp(n3), cls.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _dp(wg))
        return cls, wg

    def wall_distribution(self, n, fi):
        """Wall density and wall distribution at one wall point with unit
        normal n (into the gas) for incident arrays fi = (h, b) or (f,)."""
        n3 = _f64(list(n) + [0.0] * (3 - len(n)))
        f0 = _f64(fi[0])
        f1 = _f64(fi[1]) if self.NA == 2 else None
        w0 = np.empty(self.NV)
        w1 = np.empty(self.NV) if self.NA == 2 else None
        rw = lib().or_wall_distribution(self._h, _dp(n3), _dp(f0), _dp(f1), _dp(w0), _dp(w1))
        return rw, ((w0, w1) if self.NA == 2 else (w0,))


def residual(m_prev, m_next):
    """Convergence residual of Section 4 between the moment fields of two
    consecutive steps (rows rho, U[3], T, q[3]; NaN rows for solid cells):
    for each conservative variable W_i = rho, rho U_x, rho U_y, rho U_z,
    rho E with rho E = rho |U|^2 / 2 + 3 rho T / 4 (p = rho T / 2),
    res_i = sqrt(sum_j (W_i^{n+1} - W_i^n)^2) / sum_j |W_i^{n+1}| over the
    fluid cells j (0 where the variable vanishes everywhere); returns the
    five values and their maximum."""
    def cons(m):
        rho, U, T = m[:, 0], m[:, 1:4], m[:, 4]
        return np.column_stack([rho, rho[:, None] * U, rho * (0.5 * (U * U).sum(axis=1) + 0.75 * T)])
    ok = np.isfinite(m_next[:, 0])
    a, b = cons(m_prev[ok]), cons(m_next[ok])
    num = np.sqrt(((b - a) ** 2).sum(axis=0))
    den = np.abs(b).sum(axis=0)
    res = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return res, float(res.max())
