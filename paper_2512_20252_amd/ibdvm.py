"""Python binding of libibdvm.so (argument marshalling only).

Every step of the solve runs in the library's HIP kernels; this module turns
case dicts into the C structs of ``include/ibdvm.h``, allocates the device
workspace as a torch uint8 tensor, passes the current torch stream and copies
host arrays in and out.  It raises if the library is missing: there is no
fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibdvm.so")

OK, E_INVALID_ARG, E_GEOMETRY, E_NO_MEMORY, E_DEVICE, E_UNSTABLE, E_UNSUPPORTED, E_STATE, E_CANCELLED = range(9)
GEOMETRY = {"none": 0, "circle": 1, "ellipse": 2, "airfoil": 3, "sphere": 4}
OUTER = {"freestream": 0, "periodic": 1, "walls": 2, "specular": 3}
RULE = {"midpoint": 0, "trapezoid": 1, "stretched": 2, "refined": 3}
WEIGHTS = {"cell": 0, "jacobian": 1}
PRECISION = {"f64": 0, "f32": 1}
FLAGS = {"no_cutcell": 1 << 0, "no_upwind": 1 << 1, "implicit": 1 << 2, "face_limit": 1 << 3, "naive": 1 << 4,
         "no_aux": 1 << 5, "f32_absolute": 1 << 6, "host_only": 1 << 8}

c_int32, c_double, c_size_t, c_void_p = ctypes.c_int32, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p


class Grid(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("n", c_int32 * 3), ("lo", c_double * 3), ("hi", c_double * 3),
                ("outer_bc", c_int32), ("lid_u", c_double)]


class VGrid(ctypes.Structure):
    _fields_ = [("n", c_int32 * 3), ("lo", c_double * 3), ("hi", c_double * 3), ("rule", c_int32),
                ("stretch", c_double), ("refine_amp", c_double), ("refine_width", c_double),
                ("refine_centre", c_double * 3), ("weights", c_int32)]


class Geom(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("center", c_double * 3), ("size", c_double * 3), ("aoa_rad", c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("cfl", c_double), ("omega_vhs", c_double), ("a_vhs", c_double),
                ("flags", ctypes.c_uint32), ("workspace", c_void_p), ("workspace_bytes", c_size_t),
                ("stream", c_void_p), ("U_w", c_double * 3), ("Omega_w", c_double * 3)]


class WallPoint(ctypes.Structure):
    _fields_ = [("xw", c_double * 3), ("nw", c_double * 3), ("rho_w", c_double), ("p_w", c_double),
                ("tau_w", c_double * 3), ("q_n", c_double), ("C_p", c_double), ("T_s", c_double),
                ("u_s", c_double * 3)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", c_int32), ("converged", c_int32), ("steps", ctypes.c_int64),
                ("C_D", c_double), ("C_L", c_double), ("t_submit", c_double), ("t_admit", c_double),
                ("t_done", c_double), ("updates", ctypes.c_int64), ("tile", c_int32 * 3)]


class IbdvmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ibdvm error {code}: {msg}")
        self.code = code


_lib = None
EXPORTS = ["ibdvm_footprint", "ibdvm_create", "ibdvm_destroy", "ibdvm_info", "ibdvm_init_freestream",
           "ibdvm_set_state", "ibdvm_get_state", "ibdvm_step", "ibdvm_moments", "ibdvm_surface_forces",
           "ibdvm_clock", "ibdvm_index_sets", "ibdvm_pair_geometry", "ibdvm_wall_state", "ibdvm_batch_step",
           "ibdvm_profile", "ibdvm_profile_read", "ibdvm_set_tile", "ibdvm_get_tile", "ibdvm_autotune",
           "ibdvm_last_error", "ibdvm_init_freestream_hashed", "ibdvm_graph_create", "ibdvm_batch_graph_create", "ibdvm_graph_launch",
           "ibdvm_graph_destroy", "ibdvm_server_create", "ibdvm_server_submit", "ibdvm_server_poll",
           "ibdvm_server_info", "ibdvm_server_clock", "ibdvm_server_error", "ibdvm_server_destroy", "ibdvm_set_stream",
           "ibdvm_server_set_fusion", "ibdvm_residual", "ibdvm_server_cancel", "ibdvm_stream_copy",
           "ibdvm_surface_forces_static", "ibdvm_checkpoint_bytes", "ibdvm_checkpoint", "ibdvm_restore"]
_NOT_STATUS = ("ibdvm_destroy", "ibdvm_last_error", "ibdvm_graph_destroy", "ibdvm_server_clock",
               "ibdvm_server_error", "ibdvm_server_destroy")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        dp = P(c_double)
        L.ibdvm_footprint.argtypes = [P(Grid), P(VGrid), P(Geom), P(Opts), P(c_size_t)]
        L.ibdvm_create.argtypes = [P(Grid), P(VGrid), P(Geom), c_double, c_double, c_double, c_double, c_double,
                                   c_double, P(Opts), P(c_void_p)]
        L.ibdvm_destroy.argtypes = [c_void_p]
        L.ibdvm_destroy.restype = None
        L.ibdvm_info.argtypes = [c_void_p, P(ctypes.c_int64)]
        L.ibdvm_init_freestream.argtypes = [c_void_p, dp, dp, c_double]
        L.ibdvm_set_state.argtypes = [c_void_p, dp, dp]
        L.ibdvm_get_state.argtypes = [c_void_p, dp, dp]
        L.ibdvm_step.argtypes = [c_void_p, c_int32]
        L.ibdvm_moments.argtypes = [c_void_p, c_void_p, c_int32]
        L.ibdvm_surface_forces.argtypes = [c_void_p, dp, dp, dp, P(WallPoint), c_int32, P(c_int32)]
        L.ibdvm_clock.argtypes = [c_void_p, dp, dp, P(ctypes.c_int64)]
        L.ibdvm_index_sets.argtypes = [c_void_p, P(ctypes.c_uint8), P(ctypes.c_int32), P(ctypes.c_uint8)]
        L.ibdvm_pair_geometry.argtypes = [c_void_p, dp, dp]
        L.ibdvm_wall_state.argtypes = [c_void_p, dp, dp, dp]
        L.ibdvm_batch_step.argtypes = [P(c_void_p), c_int32, c_int32]
        L.ibdvm_profile.argtypes = [c_void_p, c_int32]
        L.ibdvm_profile_read.argtypes = [c_void_p, P(c_double), P(ctypes.c_int64)]
        L.ibdvm_set_tile.argtypes = [c_void_p, c_int32, c_int32, c_int32]
        L.ibdvm_get_tile.argtypes = [c_void_p, P(c_int32)]
        L.ibdvm_autotune.argtypes = [c_void_p, c_int32, P(c_int32)]
        L.ibdvm_last_error.argtypes = []
        L.ibdvm_last_error.restype = ctypes.c_char_p
        L.ibdvm_init_freestream_hashed.argtypes = [c_void_p, ctypes.c_uint64, c_double]
        L.ibdvm_graph_create.argtypes = [c_void_p, c_int32, P(c_void_p)]
        L.ibdvm_batch_graph_create.argtypes = [P(c_void_p), c_int32, c_int32, P(c_void_p)]
        L.ibdvm_set_stream.argtypes = [c_void_p, c_void_p]
        L.ibdvm_residual.argtypes = [c_void_p, P(c_double)]
        L.ibdvm_server_set_fusion.argtypes = [c_void_p, ctypes.c_int64]
        L.ibdvm_graph_launch.argtypes = [c_void_p]
        L.ibdvm_graph_destroy.argtypes = [c_void_p]
        L.ibdvm_graph_destroy.restype = None
        L.ibdvm_server_create.argtypes = [c_void_p, c_size_t, c_int32, c_int32, P(c_void_p)]
        L.ibdvm_server_submit.argtypes = [c_void_p, P(Grid), P(VGrid), P(Geom), c_double, c_double, c_double,
                                          c_double, c_double, c_double, P(Opts), ctypes.c_uint64, c_double,
                                          c_double, ctypes.c_int64, dp, P(ctypes.c_int64)]
        L.ibdvm_server_poll.argtypes = [c_void_p, c_int32, P(Result), c_int32, P(c_int32)]
        L.ibdvm_server_info.argtypes = [c_void_p, P(ctypes.c_int64)]
        L.ibdvm_server_cancel.argtypes = [c_void_p, ctypes.c_int64]
        L.ibdvm_stream_copy.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
        L.ibdvm_surface_forces_static.argtypes = [c_void_p, c_void_p, c_int32]
        L.ibdvm_checkpoint_bytes.argtypes = [c_void_p, P(c_size_t)]
        L.ibdvm_checkpoint.argtypes = [c_void_p, c_void_p, c_size_t]
        L.ibdvm_restore.argtypes = [c_void_p, c_void_p, c_size_t]
        L.ibdvm_server_clock.argtypes = [c_void_p]
        L.ibdvm_server_clock.restype = c_double
        L.ibdvm_server_error.argtypes = [c_void_p]
        L.ibdvm_server_error.restype = ctypes.c_char_p
        L.ibdvm_server_destroy.argtypes = [c_void_p]
        L.ibdvm_server_destroy.restype = None
        for name in EXPORTS:
            if name not in _NOT_STATUS:
                getattr(L, name).restype = c_int32
        _lib = L
    return _lib


def check(code):
    if code != OK:
        raise IbdvmError(code, lib().ibdvm_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(c_double)) if a is not None else None


def structs(case, precision="f64", flags=(), workspace=0, nbytes=0, stream=0):
    d = case["dim"]
    g = Grid()
    g.dim = d
    v = VGrid()
    for a in range(3):
        g.n[a] = case["n"][a] if a < d else 1
        g.lo[a] = case["lo"][a] if a < d else 0.0
        g.hi[a] = case["hi"][a] if a < d else 1.0
        v.n[a] = case["vn"][a] if a < d else 1
        v.lo[a] = case["vlo"][a] if a < d else 0.0
        v.hi[a] = case["vhi"][a] if a < d else 0.0
    g.outer_bc = OUTER[case.get("outer", "freestream")]
    g.lid_u = case.get("lid_u", 0.0)
    v.rule = RULE[case.get("rule", "midpoint")]
    v.stretch = case.get("vstretch", 0.0)
    v.refine_amp = case.get("vref_amp", 0.0)
    v.refine_width = case.get("vref_width", 1.0)
    rc = case.get("vref_centre", (0.0, 0.0, 0.0))
    for a in range(3):
        v.refine_centre[a] = rc[a] if a < len(rc) else 0.0
    v.weights = WEIGHTS[case.get("vweights", "cell")]
    ge = Geom()
    ge.kind = GEOMETRY[case.get("geometry", "none")]
    cen, size = case.get("center", (0, 0, 0)), case.get("size", (0, 0, 0))
    for a in range(3):
        ge.center[a] = cen[a] if a < len(cen) else 0.0
        ge.size[a] = size[a] if a < len(size) else 0.0
    ge.aoa_rad = case.get("aoa", 0.0)
    o = Opts()
    o.precision = PRECISION[precision]
    o.cfl = case.get("cfl", 0.5)
    o.omega_vhs = case.get("omega_vhs", 0.81)
    o.a_vhs = case.get("a_vhs", 1.0)
    fl = 0
    for f in tuple(case.get("flags", ())) + tuple(flags):
        fl |= FLAGS[f]
    o.flags = fl
    o.workspace = workspace
    o.workspace_bytes = nbytes
    o.stream = stream
    Uw, Ow = case.get("U_w", (0.0, 0.0, 0.0)), case.get("Omega_w", (0.0, 0.0, 0.0))
    for a in range(3):
        o.U_w[a] = Uw[a] if a < len(Uw) else 0.0
        o.Omega_w[a] = Ow[a] if a < len(Ow) else 0.0
    return g, v, ge, o


def footprint(case, precision="f64"):
    g, v, ge, o = structs(case, precision)
    n = c_size_t(0)
    check(lib().ibdvm_footprint(ctypes.byref(g), ctypes.byref(v), ctypes.byref(ge), ctypes.byref(o), ctypes.byref(n)))
    return int(n.value)


class Solver:
    """One resident solve.  ``workspace`` may be a caller-provided device
    tensor (uint8, >= footprint bytes); otherwise one is allocated with torch
    on the current device.  ``host_only`` builds the geometry tables only."""

    def __init__(self, case, precision="f64", host_only=False, workspace=None, stream=None):
        self.case = dict(case)
        self.precision = precision
        self.host_only = host_only
        self.workspace = None
        ws_ptr, nbytes, sptr = 0, 0, 0
        if not host_only:
            import torch
            nbytes = footprint(case, precision)
            if workspace is None:
                workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            self.workspace = workspace
            ws_ptr, nbytes = workspace.data_ptr(), workspace.numel()
            self.stream = stream if stream is not None else torch.cuda.current_stream()
            sptr = self.stream.cuda_stream
        g, v, ge, o = structs(case, precision, ("host_only",) if host_only else (), ws_ptr, nbytes, sptr)
        h = c_void_p(0)
        check(lib().ibdvm_create(ctypes.byref(g), ctypes.byref(v), ctypes.byref(ge), case["Kn"], case["Ma"],
                                 case["Pr"], case["gamma"], case["alpha"], case["Tw"], ctypes.byref(o),
                                 ctypes.byref(h)))
        self._h = h
        self._lib = lib()  # held so that destruction at interpreter exit needs no module global
        info = (ctypes.c_int64 * 7)()
        check(lib().ibdvm_info(self._h, info))
        self.dim, self.Nc, self.NV, self.NA, self.npairs, self.nfluid, self.nghost = [int(x) for x in info]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ibdvm_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    # state --------------------------------------------------------------
    def init_freestream(self, u=None, amp=0.0):
        u0 = np.ascontiguousarray(u[0], dtype=np.float64).reshape(-1) if u is not None else None
        u1 = np.ascontiguousarray(u[1], dtype=np.float64).reshape(-1) if (u is not None and self.NA == 2) else None
        check(lib().ibdvm_init_freestream(self._h, _dp(u0), _dp(u1), float(amp)))

    def set_stream(self, stream):
        """Rebind to another torch stream (after the queued work finished)."""
        self.stream = stream
        check(lib().ibdvm_set_stream(self._h, c_void_p(stream.cuda_stream if stream is not None else 0)))

    def init_freestream_hashed(self, seed, amp):
        check(lib().ibdvm_init_freestream_hashed(self._h, int(seed), float(amp)))

    def set_state(self, f):
        f0 = np.ascontiguousarray(f[0], dtype=np.float64).reshape(-1)
        f1 = np.ascontiguousarray(f[1], dtype=np.float64).reshape(-1) if self.NA == 2 else None
        check(lib().ibdvm_set_state(self._h, _dp(f0), _dp(f1)))

    def get_state(self):
        f0 = np.empty((self.Nc, self.NV))
        f1 = np.empty((self.Nc, self.NV)) if self.NA == 2 else None
        check(lib().ibdvm_get_state(self._h, _dp(f0), _dp(f1)))
        return (f0, f1) if self.NA == 2 else (f0,)

    def checkpoint(self):
        """A checkpoint record of the solve (host bytes): ibdvm_checkpoint."""
        n = c_size_t()
        check(lib().ibdvm_checkpoint_bytes(self._h, ctypes.byref(n)))
        rec = np.empty(n.value, dtype=np.uint8)
        check(lib().ibdvm_checkpoint(self._h, rec.ctypes.data_as(c_void_p), n.value))
        return rec

    def restore(self, record):
        """Resume from a checkpoint record: ibdvm_restore."""
        rec = np.ascontiguousarray(record, dtype=np.uint8)
        check(lib().ibdvm_restore(self._h, rec.ctypes.data_as(c_void_p), rec.size))

    def step(self, n=1):
        check(lib().ibdvm_step(self._h, int(n)))

    # outputs ------------------------------------------------------------
    def moments(self):
        out = np.empty((self.Nc, 8))
        check(lib().ibdvm_moments(self._h, out.ctypes.data, 0))
        return out

    def moments_device(self, out):
        """Enqueue the moments into a device float64 tensor of shape (cells, 8)."""
        check(lib().ibdvm_moments(self._h, out.data_ptr(), 1))

    def clock(self):
        dt, t, s = c_double(0), c_double(0), ctypes.c_int64(0)
        check(lib().ibdvm_clock(self._h, ctypes.byref(dt), ctypes.byref(t), ctypes.byref(s)))
        return {"dt": dt.value, "time": t.value, "step": int(s.value)}

    def surface_forces(self):
        F = np.empty(3)
        cd, cl = c_double(0), c_double(0)
        cap = max(self.npairs, 1)
        pts = (WallPoint * cap)()
        n = c_int32(0)
        check(lib().ibdvm_surface_forces(self._h, _dp(F), ctypes.byref(cd), ctypes.byref(cl), pts, cap,
                                         ctypes.byref(n)))
        wall = np.array([list(p.xw) + list(p.nw) + [p.rho_w, p.p_w] + list(p.tau_w) + [p.q_n, p.C_p, p.T_s]
                         + list(p.u_s) for p in pts[: n.value]]).reshape(-1, 17)
        return F, cd.value, cl.value, wall

    def surface_forces_static(self, out, cap):
        """Enqueue the allocation-free surface forces into the device float64
        tensor out (at least 5 + 17 cap elements) on the solve's stream."""
        assert out.numel() >= 5 + 17 * cap
        check(lib().ibdvm_surface_forces_static(self._h, out.data_ptr(), int(cap)))

    def residual(self):
        """Convergence residual of the last step: per variable (rho, rho U[3],
        rho E) and the maximum."""
        r = np.empty(6)
        check(lib().ibdvm_residual(self._h, _dp(r)))
        return r[:5], float(r[5])

    def wall_state(self):
        ghost = np.empty((self.NA, max(self.npairs, 1), self.NV))
        face = np.empty_like(ghost)
        rhow = np.empty(max(self.npairs, 1))
        check(lib().ibdvm_wall_state(self._h, _dp(ghost), _dp(face), _dp(rhow)))
        return {"ghost": ghost[:, : self.npairs], "face": face[:, : self.npairs], "rhow": rhow[: self.npairs]}

    def profile(self, enable=True):
        check(lib().ibdvm_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        ms = (c_double * 2)()
        cnt = (ctypes.c_int64 * 2)()
        check(lib().ibdvm_profile_read(self._h, ms, cnt))
        return {"update_ms": ms[0], "update_launches": int(cnt[0]), "fill_ms": ms[1], "fill_launches": int(cnt[1])}

    def set_tile(self, V, TX, LY):
        check(lib().ibdvm_set_tile(self._h, int(V), int(TX), int(LY)))

    def get_tile(self):
        out = (c_int32 * 3)()
        check(lib().ibdvm_get_tile(self._h, out))
        return tuple(out)

    def autotune(self, reps=3):
        out = (c_int32 * 3)()
        check(lib().ibdvm_autotune(self._h, int(reps), out))
        return tuple(out)

    def index_sets(self):
        solid = np.empty(self.Nc, dtype=np.uint8)
        pint = np.empty((max(self.npairs, 1), 32), dtype=np.int32)
        cls = np.empty((max(self.npairs, 1), self.NV), dtype=np.uint8)
        check(lib().ibdvm_index_sets(self._h, solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                     pint.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     cls.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return {"solid": solid, "pairs": pint[: self.npairs], "cls": cls[: self.npairs]}

    def pair_geometry(self):
        g = np.empty((max(self.npairs, 1), 9))
        wg = np.empty((max(self.npairs, 1), self.NV))
        check(lib().ibdvm_pair_geometry(self._h, _dp(g), _dp(wg)))
        return {"xw": g[: self.npairs, 0:3], "nw": g[: self.npairs, 3:6], "xsp": g[: self.npairs, 6:9],
                "wg": wg[: self.npairs]}


def stream_copy(src, dst, stream=None):
    """Enqueue the library's streaming copy of the torch tensor src into dst
    (same byte size) on stream (default: the current stream)."""
    import torch
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    s = stream if stream is not None else torch.cuda.current_stream()
    check(lib().ibdvm_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, s.cuda_stream))


def batch_step(solvers, n):
    arr = (c_void_p * len(solvers))(*[s.handle for s in solvers])
    check(lib().ibdvm_batch_step(arr, len(solvers), int(n)))


class Graph:
    """nsteps captured steps of one solver, or of the fused steps of several
    solvers sharing a stream (a list), replayed on their stream."""

    def __init__(self, solver, nsteps):
        self.solver = solver
        h = c_void_p(0)
        if isinstance(solver, (list, tuple)):
            arr = (c_void_p * len(solver))(*[s.handle for s in solver])
            check(lib().ibdvm_batch_graph_create(arr, len(solver), int(nsteps), ctypes.byref(h)))
        else:
            check(lib().ibdvm_graph_create(solver.handle, int(nsteps), ctypes.byref(h)))
        self._h = h
        self._lib = lib()  # held so that destruction at interpreter exit needs no module global

    def launch(self):
        check(lib().ibdvm_graph_launch(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ibdvm_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Server:
    """Continuous batching of 2D solves in one device workspace (a torch
    uint8 tensor of ``nbytes``)."""

    def __init__(self, nbytes, max_active=4, steps_per_replay=100, fuse_below=None, workspace_ptr=None):
        """workspace_ptr: an existing device buffer of nbytes (256-byte
        aligned) instead of a torch allocation."""
        if workspace_ptr is None:
            import torch
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            ptr, nbytes = self.workspace.data_ptr(), self.workspace.numel()
        else:
            self.workspace, ptr = None, int(workspace_ptr)
        h = c_void_p(0)
        code = lib().ibdvm_server_create(ptr, int(nbytes), int(max_active), int(steps_per_replay), ctypes.byref(h))
        if code != OK:
            raise IbdvmError(code, "server_create")
        self._h = h
        self._lib = lib()  # held so that destruction at interpreter exit needs no module global
        self._outs = {}
        if fuse_below is not None:
            self._check(lib().ibdvm_server_set_fusion(self._h, int(fuse_below)))

    def _check(self, code):
        if code != OK:
            raise IbdvmError(code, lib().ibdvm_server_error(self._h).decode())

    def submit(self, case, precision="f32", seed=0, amp=1e-3, tol=1e-6, max_steps=200000, keep_moments=False):
        g, v, ge, o = structs(case, precision)
        out = None
        if keep_moments:
            out = np.empty((int(np.prod(case["n"][: case["dim"]])), 8))
        rid = ctypes.c_int64(0)
        self._check(lib().ibdvm_server_submit(self._h, ctypes.byref(g), ctypes.byref(v), ctypes.byref(ge),
                                              case["Kn"], case["Ma"], case["Pr"], case["gamma"], case["alpha"],
                                              case["Tw"], ctypes.byref(o), int(seed), float(amp), float(tol),
                                              int(max_steps), _dp(out), ctypes.byref(rid)))
        self._outs[rid.value] = out
        return rid.value

    def poll(self, block=False, cap=64):
        res = (Result * cap)()
        n = c_int32(0)
        self._check(lib().ibdvm_server_poll(self._h, 1 if block else 0, res, cap, ctypes.byref(n)))
        out = []
        for r in res[: n.value]:
            d = {k: getattr(r, k) for k, _ in Result._fields_ if k != "tile"}
            d["tile"] = tuple(r.tile)
            d["moments"] = self._outs.pop(r.id, None)
            out.append(d)
        return out

    def cancel(self, rid):
        self._check(lib().ibdvm_server_cancel(self._h, int(rid)))

    def info(self):
        a = (ctypes.c_int64 * 5)()
        self._check(lib().ibdvm_server_info(self._h, a))
        return dict(zip(("queued", "active", "finished", "bytes_used", "bytes_total"), [int(x) for x in a]))

    def clock(self):
        return lib().ibdvm_server_clock(self._h)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ibdvm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
