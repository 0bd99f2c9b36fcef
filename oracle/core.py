"""ctypes wrapper of the C oracle (``oracle.c``).  Test infrastructure only.

Arrays cross the boundary as C-contiguous NumPy arrays; every function
returns NumPy arrays and raises ``OracleError`` on a non-zero status.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

OK, E_ARG, E_MESH, E_STATE, E_NUMERIC = 0, -1, -2, -3, -7
BC_WALL, BC_TRANSMIT = 0, 1
GUESS_TR, GUESS_GIVEN = 0, 1
KIND_INTERIOR, KIND_WALL, KIND_TRANSMIT = 0, 1, 2


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double),
                ("newton_tol", C.c_double), ("level_margin", C.c_double),
                ("max_levels", C.c_int32), ("order", C.c_int32),
                ("newton_max_iter", C.c_int32), ("boundary", C.c_int32),
                ("reclassify", C.c_int32), ("time_order", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("subiterations", C.c_int64), ("cell_updates", C.c_int64),
                ("face_solves", C.c_int64), ("newton_updates", C.c_int64),
                ("newton_fallbacks", C.c_int64), ("vacuum_faces", C.c_int64),
                ("cells_per_level", C.c_int64 * 8),
                ("theta", C.c_int32), ("phase", C.c_int32),
                ("dt_min", C.c_double), ("t_reached", C.c_double),
                ("wall_impulse", C.c_double * 3)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["cells_per_level"] = list(self.cells_per_level)
        d["wall_impulse"] = list(self.wall_impulse)
        return d


class RiemannOut(C.Structure):
    _fields_ = [("p_star", C.c_double), ("u_star", C.c_double),
                ("newton_updates", C.c_int32), ("fallback", C.c_int32),
                ("vacuum", C.c_int32)]


def params(gamma=1.4, cfl=0.5, newton_tol=1e-12, level_margin=1e-9, max_levels=3,
           order=1, newton_max_iter=50, boundary=BC_WALL, reclassify=1, time_order=1):
    return Params(gamma, cfl, newton_tol, level_margin, max_levels, order,
                  newton_max_iter, boundary, reclassify, time_order)


_libs = {}
_variant = "seq"


def select(variant):
    """Library for the objects made from now on: "seq" (the sequential
    parity reference, the default) or "omp" (the same source built with
    OpenMP: same bits, all host threads; for timing the CPU baseline)."""
    global _variant
    if variant not in ("seq", "omp"):
        raise ValueError(variant)
    _variant = variant


def threads():
    """Threads the selected library's loops run on."""
    return int(lib().orc_threads())


def lib(variant=None):
    variant = variant or _variant
    if variant not in _libs:
        path = _build.build(force=False, openmp=(variant == "omp"))
        L = C.CDLL(path)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        i8p = C.POINTER(C.c_int8)
        L.orc_mesh_build.argtypes = [C.c_int64, dp, C.c_int64, i64p, C.POINTER(P)]
        L.orc_mesh_free.argtypes = [P]
        L.orc_mesh_free.restype = None
        L.orc_mesh_counts.argtypes = [P, i64p, i64p, i64p]
        L.orc_mesh_geometry.argtypes = [P, dp, dp, i64p, i64p, dp, dp, i64p]
        L.orc_riemann_solve.argtypes = [C.c_double, dp, dp, C.c_double, C.c_int32,
                                        C.c_int32, C.c_double, C.POINTER(RiemannOut)]
        L.orc_riemann_sample.argtypes = [C.c_double, dp, dp, C.POINTER(RiemannOut),
                                         C.c_double, dp]
        L.orc_face_flux.argtypes = [C.c_double, dp, dp, dp, C.c_int32, C.c_double,
                                    C.c_int32, C.c_int32, C.c_double, dp,
                                    C.POINTER(RiemannOut)]
        L.orc_face_flux_moving.argtypes = [C.c_double, dp, dp, dp, C.c_double, C.c_int32,
                                           C.c_double, C.c_int32, dp, C.POINTER(RiemannOut)]
        L.orc_state_motion.argtypes = [P, dp]
        L.orc_state_volumes.argtypes = [P, dp]
        L.orc_gradients.argtypes = [P, C.POINTER(Params), dp, dp, dp]
        L.orc_classify.argtypes = [P, C.POINTER(Params), dp, dp, i8p, dp,
                                   C.POINTER(C.c_int32)]
        L.orc_state_new.argtypes = [P, C.POINTER(Params), dp, C.POINTER(P)]
        L.orc_state_free.argtypes = [P]
        L.orc_state_free.restype = None
        L.orc_state_set.argtypes = [P, dp, dp, i8p, C.c_int32, C.c_int32, C.c_double,
                                    C.c_double]
        L.orc_advance.argtypes = [P, C.c_int64]
        L.orc_state_read.argtypes = [P, dp, dp, i8p]
        L.orc_state_stats.argtypes = [P, C.POINTER(Stats)]
        L.orc_subiteration_level.argtypes = [C.c_int64, C.c_int32]
        L.orc_subiteration_level.restype = C.c_int32
        L.orc_threads.argtypes = []
        L.orc_threads.restype = C.c_int32
        _libs[variant] = L
    return _libs[variant]


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _i64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64)) if a is not None else None


def _i8(a):
    return a.ctypes.data_as(C.POINTER(C.c_int8)) if a is not None else None


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


class Mesh:
    """Faces and FP64 geometry of a tetrahedral mesh (positively oriented tets)."""

    def __init__(self, nodes, tets):
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int64)
        self._L = lib()
        h = C.c_void_p()
        _check(self._L.orc_mesh_build(nodes.shape[0], _d(nodes), tets.shape[0], _i64(tets),
                                    C.byref(h)), "orc_mesh_build")
        self._h = h
        nc, nf, nb = C.c_int64(), C.c_int64(), C.c_int64()
        self._L.orc_mesh_counts(h, C.byref(nc), C.byref(nf), C.byref(nb))
        self.n_cells, self.n_faces, self.n_boundary = nc.value, nf.value, nb.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.orc_mesh_free(h)
            self._h = None

    def geometry(self):
        nc, nf = self.n_cells, self.n_faces
        g = dict(vol=np.empty(nc), centroid=np.empty((nc, 3)),
                 face_L=np.empty(nf, np.int64), face_R=np.empty(nf, np.int64),
                 face_area=np.empty((nf, 3)), face_centroid=np.empty((nf, 3)),
                 cell_faces=np.empty((nc, 4), np.int64))
        _check(self._L.orc_mesh_geometry(self._h, _d(g["vol"]), _d(g["centroid"]),
                                       _i64(g["face_L"]), _i64(g["face_R"]),
                                       _d(g["face_area"]), _d(g["face_centroid"]),
                                       _i64(g["cell_faces"])), "orc_mesh_geometry")
        return g


def riemann_solve(wl, wr, gamma=1.4, tol=1e-12, max_iter=50, guess=None):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    out = RiemannOut()
    mode = GUESS_TR if guess is None else GUESS_GIVEN
    _check(lib().orc_riemann_solve(gamma, _d(wl), _d(wr), tol, max_iter, mode,
                                   0.0 if guess is None else float(guess), C.byref(out)),
           "orc_riemann_solve")
    return out


def riemann_sample(wl, wr, rs, xi, gamma=1.4):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    w = np.empty(3)
    side = lib().orc_riemann_sample(gamma, _d(wl), _d(wr), C.byref(rs), float(xi), _d(w))
    return w, side


def face_flux(wl, wr, area, kind=KIND_INTERIOR, gamma=1.4, tol=1e-12, max_iter=50,
              guess=None):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr if wr is not None else wl, dtype=np.float64)
    area = np.ascontiguousarray(area, dtype=np.float64)
    flux = np.empty(5)
    out = RiemannOut()
    mode = GUESS_TR if guess is None else GUESS_GIVEN
    _check(lib().orc_face_flux(gamma, _d(wl), _d(wr), _d(area), kind, tol, max_iter, mode,
                               0.0 if guess is None else float(guess), _d(flux),
                               C.byref(out)), "orc_face_flux")
    return flux, out


def face_flux_moving(wl, wr, area, xi, kind=KIND_INTERIOR, gamma=1.4, tol=1e-12, max_iter=50):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr if wr is not None else wl, dtype=np.float64)
    area = np.ascontiguousarray(area, dtype=np.float64)
    flux = np.empty(5)
    out = RiemannOut()
    _check(lib().orc_face_flux_moving(gamma, _d(wl), _d(wr), _d(area), float(xi), kind, tol,
                                      max_iter, _d(flux), C.byref(out)), "orc_face_flux_moving")
    return flux, out


def gradients(mesh, prim, prm=None):
    prm = prm or params(order=2)
    prim = np.ascontiguousarray(prim, dtype=np.float64)
    raw = np.empty((mesh.n_cells, 3, 5))
    lim = np.empty((mesh.n_cells, 3, 5))
    _check(mesh._L.orc_gradients(mesh._h, C.byref(prm), _d(prim), _d(raw), _d(lim)),
           "orc_gradients")
    return raw, lim


def classify(mesh, cons, prm):
    cons = np.ascontiguousarray(cons, dtype=np.float64)
    dt = np.empty(mesh.n_cells)
    lev = np.empty(mesh.n_cells, np.int8)
    dtmin = C.c_double()
    theta = C.c_int32()
    _check(mesh._L.orc_classify(mesh._h, C.byref(prm), _d(cons), _d(dt), _i8(lev),
                              C.byref(dtmin), C.byref(theta)), "orc_classify")
    return dt, lev, dtmin.value, theta.value


class State:
    """The oracle's solver: conserved state, accumulators, levels, schedule."""

    def __init__(self, mesh, prim, prm):
        self.mesh = mesh
        self.prm = prm
        prim = np.ascontiguousarray(prim, dtype=np.float64)
        self._L = mesh._L
        h = C.c_void_p()
        _check(self._L.orc_state_new(mesh._h, C.byref(prm), _d(prim), C.byref(h)),
               "orc_state_new")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.orc_state_free(h)
            self._h = None

    def set(self, cons, accum, levels, phase, theta, dt_min, t=0.0):
        cons = np.ascontiguousarray(cons, dtype=np.float64)
        accum = np.ascontiguousarray(accum, dtype=np.float64)
        levels = np.ascontiguousarray(levels, dtype=np.int8)
        _check(self._L.orc_state_set(self._h, _d(cons), _d(accum), _i8(levels), phase, theta,
                                   dt_min, t), "orc_state_set")

    def advance(self, n):
        _check(self._L.orc_advance(self._h, int(n)), "orc_advance")

    def read(self):
        n = self.mesh.n_cells
        cons = np.empty((n, 5))
        accum = np.empty((n, 5))
        lev = np.empty(n, np.int8)
        _check(self._L.orc_state_read(self._h, _d(cons), _d(accum), _i8(lev)), "orc_state_read")
        return cons, accum, lev

    def motion(self, node_vel):
        """Node velocities [n_nodes][3] of a moving mesh (ALE, geometric
        conservation law)."""
        v = np.ascontiguousarray(node_vel, dtype=np.float64)
        _check(self._L.orc_state_motion(self._h, _d(v)), "orc_state_motion")

    def volumes(self):
        vol = np.empty(self.mesh.n_cells)
        _check(self._L.orc_state_volumes(self._h, _d(vol)), "orc_state_volumes")
        return vol

    def stats(self):
        st = Stats()
        _check(self._L.orc_state_stats(self._h, C.byref(st)), "orc_state_stats")
        return st.as_dict()


def subiteration_level(s, theta):
    """Level computed in subiteration s = 1..2^theta (Alg. 2)."""
    return lib().orc_subiteration_level(int(s), int(theta))


def prim_to_cons(prim, gamma=1.4):
    """Ideal-gas conversion on arrays [n][5] (rho,u,v,w,p) -> (rho, m, E)."""
    prim = np.asarray(prim, dtype=np.float64)
    out = np.empty_like(prim)
    out[:, 0] = prim[:, 0]
    out[:, 1:4] = prim[:, :1] * prim[:, 1:4]
    out[:, 4] = prim[:, 4] / (gamma - 1.0) + 0.5 * prim[:, 0] * (prim[:, 1:4] ** 2).sum(1)
    return out


def cons_to_prim(cons, gamma=1.4):
    cons = np.asarray(cons, dtype=np.float64)
    out = np.empty_like(cons)
    out[:, 0] = cons[:, 0]
    out[:, 1:4] = cons[:, 1:4] / cons[:, :1]
    out[:, 4] = (gamma - 1.0) * (cons[:, 4] - 0.5 * (cons[:, 1:4] ** 2).sum(1) / cons[:, 0])
    return out
