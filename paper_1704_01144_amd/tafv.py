"""Python binding of the tafv C-ABI (``include/tafv.h``), argument
marshalling only: every step of the method runs in the HIP library.

The functions carry the C names (``tafv_create``, ``tafv_mesh_upload``, ...)
and take NumPy arrays for host buffers; ``Solver`` is a small convenience
wrapper over them.  There is no CPU fallback: importing this module raises
if ``libtafv.so`` is missing.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtafv.so")

OK, E_ARG, E_MESH, E_STATE, E_ORDER, E_DEVICE, E_OOM, E_NUMERIC, E_MLP = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, FP32_FLUX = 0, 1
GUESS_TR, GUESS_MLP = 0, 1
BC_WALL, BC_TRANSMIT = 0, 1
SCATTER_COLOUR, SCATTER_GATHER = 0, 1
ORDER_CALLER, ORDER_MORTON = 0, 1


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEALLOC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TafvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tafv error {code}: {msg}")
        self.code = code


class tafv_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("newton_tol", C.c_double),
                ("level_margin", C.c_double), ("max_levels", C.c_int32), ("order", C.c_int32),
                ("precision", C.c_int32), ("guess", C.c_int32), ("boundary", C.c_int32),
                ("newton_max_iter", C.c_int32), ("reclassify", C.c_int32),
                ("scatter", C.c_int32), ("cell_order", C.c_int32),
                ("guess_stats", C.c_int32), ("guess_gate", C.c_double),
                ("batch", C.c_int32), ("guess_strength", C.c_double),
                ("time_order", C.c_int32), ("fuse_faces", C.c_int32),
                ("pipeline_chunks", C.c_int32)]


class tafv_stats(C.Structure):
    _fields_ = [("subiterations", C.c_int64), ("cell_updates", C.c_int64),
                ("face_solves", C.c_int64), ("newton_updates", C.c_int64),
                ("newton_fallbacks", C.c_int64), ("vacuum_faces", C.c_int64),
                ("cells_per_level", C.c_int64 * 8), ("theta", C.c_int32), ("phase", C.c_int32),
                ("dt_min", C.c_double), ("t_reached", C.c_double),
                ("wall_impulse", C.c_double * 3), ("guess_faces", C.c_int64),
                ("guess_newton_updates", C.c_int64), ("guess_rejected", C.c_int64),
                ("guess_used", C.c_int64), ("guess_evaluated", C.c_int64),
                ("newton_hist", (C.c_int64 * 8) * 3),
                ("newton_hist_long_updates", C.c_int64 * 3)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["cells_per_level"] = list(self.cells_per_level)
        d["wall_impulse"] = list(self.wall_impulse)
        d["newton_hist"] = [list(row) for row in self.newton_hist]
        d["newton_hist_long_updates"] = list(self.newton_hist_long_updates)
        return d


def _one_hip_runtime():
    """PyTorch's ROCm wheels carry their own HIP runtime, whose library has
    the same soname as the system's.  Loaded before PyTorch, libtafv.so
    would bring in the system runtime, PyTorch would then load its own next
    to it, and the second runtime to initialise finds no device.  Loading
    PyTorch first (when it is installed) makes libtafv.so bind to PyTorch's
    runtime, so that the process has one."""
    import importlib.util
    if importlib.util.find_spec("torch") is not None:
        import torch  # noqa: F401


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    _one_hip_runtime()
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    dp, i64p, i8p, i32p = (C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int8),
                           C.POINTER(C.c_int32))
    fp = C.POINTER(C.c_float)
    sig = {
        "tafv_params_default": [C.POINTER(tafv_params)],
        "tafv_create": [C.c_int, C.POINTER(tafv_params), P, C.POINTER(P)],
        "tafv_destroy": [P],
        "tafv_set_allocator": [P, ALLOC_FN, DEALLOC_FN, P],
        "tafv_mesh_upload": [P, C.c_int64, dp, C.c_int64, i64p, i32p],
        "tafv_mesh_params": [P, C.c_int32, C.c_int32],
        "tafv_mesh_motion": [P, C.c_int32, dp],
        "tafv_volume_read": [P, C.c_int32, dp],
        "tafv_mesh_inspect": [C.c_int64, dp, C.c_int64, i64p, i64p, i64p, i32p, i32p, i8p, dp,
                              i32p, dp],
        "tafv_state_init": [P, C.c_int32, dp],
        "tafv_advance": [P, C.c_int64, C.POINTER(tafv_stats)],
        "tafv_advance_group": [C.POINTER(P), C.c_int32, C.c_int64, C.c_int32,
                               C.POINTER(tafv_stats)],
        "tafv_state_reset": [P, C.c_int32],
        "tafv_mesh_stats": [P, C.c_int32, C.POINTER(tafv_stats)],
        "tafv_state_read": [P, C.c_int32, dp, i8p],
        "tafv_checkpoint_read": [P, C.c_int32, dp, dp, i8p, i32p, i32p, dp, dp],
        "tafv_checkpoint_write": [P, C.c_int32, dp, dp, i8p, C.c_int32, C.c_int32, C.c_double,
                                  C.c_double],
        "tafv_profile_enable": [P, C.c_int32],
        "tafv_guess_config": [P, C.c_int32, C.c_double, C.c_double, C.c_int32],
        "tafv_mlp_set": [P, fp, C.c_int64],
        "tafv_mlp_get": [P, fp, C.c_int64],
        "tafv_mlp_forward": [P, fp, C.c_int64, fp],
        "tafv_mlp_grad": [P, fp, fp, C.c_int64, fp, fp],
        "tafv_mlp_grad_noalloc": [P, fp, fp, C.c_int64, fp, fp],
        "tafv_mlp_train": [P, fp, fp, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_uint64, fp],
        "tafv_facelog_config": [P, C.c_int64, C.c_double, C.c_uint64],
        "tafv_facelog_read": [P, fp, C.c_int64, i64p],
        "tafv_profile_read": [P, C.c_int32, dp, i64p, i64p, C.POINTER(C.c_char_p), i32p],
        "tafv_batch_config": [P, C.c_int32, C.c_int32, C.c_char_p],
        "tafv_batch_info": [P, i32p, C.c_int32],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.tafv_last_error.argtypes = [P]
    L.tafv_last_error.restype = C.c_char_p
    L.tafv_device_buffers.argtypes = [P]
    L.tafv_device_buffers.restype = C.c_int64
    return L


lib = _load()

# every symbol the header declares (checked by the CPU tests)
EXPORTS = ["tafv_params_default", "tafv_create", "tafv_destroy", "tafv_last_error",
           "tafv_set_allocator", "tafv_device_buffers",
           "tafv_mesh_upload", "tafv_mesh_inspect", "tafv_mesh_params", "tafv_state_init",
           "tafv_state_reset", "tafv_advance", "tafv_advance_group",
           "tafv_mesh_stats", "tafv_state_read", "tafv_checkpoint_read", "tafv_checkpoint_write",
           "tafv_profile_enable", "tafv_profile_read", "tafv_guess_config", "tafv_mlp_set", "tafv_mlp_get",
           "tafv_mlp_forward", "tafv_mlp_grad", "tafv_mlp_grad_noalloc", "tafv_mlp_train",
           "tafv_facelog_config",
           "tafv_facelog_read", "tafv_batch_config", "tafv_batch_info", "tafv_mesh_motion",
           "tafv_volume_read"]
MLP_PARAMS = 1313
MLP_GRAD_NOALLOC_MAX_ROWS = 65536


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, ctx=None):
    if rc != OK:
        msg = lib.tafv_last_error(ctx)
        raise TafvError(rc, msg.decode() if msg else "")


def tafv_params_default(**overrides):
    p = tafv_params()
    _check(lib.tafv_params_default(C.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def tafv_create(device=0, params=None, hip_stream=None):
    params = params or tafv_params_default()
    h = C.c_void_p()
    _check(lib.tafv_create(device, C.byref(params), C.c_void_p(hip_stream or 0), C.byref(h)))
    return h


def tafv_destroy(ctx):
    _check(lib.tafv_destroy(ctx))


def tafv_set_allocator(ctx, alloc=None, dealloc=None):
    """Route the context's device memory through Python callables:
    alloc(nbytes) -> device pointer as an int (0 when it cannot) and
    dealloc(ptr).  Both None restores hipMalloc / hipFree.  Returns the
    ctypes wrappers, which must stay alive as long as the context."""
    if (alloc is None) != (dealloc is None):
        raise ValueError("give both alloc and dealloc, or neither")
    if alloc is None:
        _check(lib.tafv_set_allocator(ctx, ALLOC_FN(), DEALLOC_FN(), None), ctx)
        return None

    def _alloc(n, _user):
        try:
            return int(alloc(int(n)) or 0)
        except Exception:  # an exception must not cross into the library
            return 0

    def _dealloc(ptr, _user):
        dealloc(int(ptr))

    keep = (ALLOC_FN(_alloc), DEALLOC_FN(_dealloc))
    _check(lib.tafv_set_allocator(ctx, keep[0], keep[1], None), ctx)
    return keep


def torch_allocator(device=0, stream=None):
    """alloc/dealloc callables over PyTorch's caching allocator on `device`
    and `stream` (a torch.cuda.Stream or raw stream handle; None: the
    current stream), for tafv_set_allocator."""
    import torch

    def alloc(n):
        try:
            return torch.cuda.caching_allocator_alloc(n, device, stream)
        except RuntimeError:  # out of memory
            return 0

    def dealloc(ptr):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, dealloc


def tafv_device_buffers(ctx):
    return int(lib.tafv_device_buffers(ctx))


def tafv_mesh_upload(ctx, nodes, tets):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int64)
    mid = C.c_int32()
    _check(lib.tafv_mesh_upload(ctx, nodes.shape[0], _d(nodes), tets.shape[0],
                                tets.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(mid)), ctx)
    return mid.value


def tafv_mesh_inspect(nodes, tets):
    """Host-only mesh preprocessing (no device): faces, colours, geometry."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int64)
    t64 = tets.ctypes.data_as(C.POINTER(C.c_int64))
    nf, nb, ncol = C.c_int64(), C.c_int64(), C.c_int32()
    _check(lib.tafv_mesh_inspect(nodes.shape[0], _d(nodes), tets.shape[0], t64, C.byref(nf),
                                 C.byref(nb), C.byref(ncol), None, None, None, None, None))
    fc = np.empty((nf.value, 2), np.int32)
    col = np.empty(nf.value, np.int8)
    area = np.empty((nf.value, 3))
    nbr = np.empty((tets.shape[0], 4), np.int32)
    coef = np.empty((tets.shape[0], 3, 4))
    _check(lib.tafv_mesh_inspect(nodes.shape[0], _d(nodes), tets.shape[0], t64, C.byref(nf),
                                 C.byref(nb), C.byref(ncol),
                                 fc.ctypes.data_as(C.POINTER(C.c_int32)),
                                 col.ctypes.data_as(C.POINTER(C.c_int8)), _d(area),
                                 nbr.ctypes.data_as(C.POINTER(C.c_int32)), _d(coef)))
    return dict(n_faces=nf.value, n_boundary=nb.value, n_colours=ncol.value, face_cells=fc,
                face_colour=col, face_area=area, cell_neighbours=nbr, recon_coef=coef)


def tafv_mesh_params(ctx, mesh_id, max_levels):
    _check(lib.tafv_mesh_params(ctx, mesh_id, max_levels), ctx)


def tafv_state_init(ctx, mesh_id, prim):
    prim = np.ascontiguousarray(prim, dtype=np.float64)
    _check(lib.tafv_state_init(ctx, mesh_id, _d(prim)), ctx)


def tafv_state_reset(ctx, mesh_id):
    _check(lib.tafv_state_reset(ctx, mesh_id), ctx)


def tafv_advance(ctx, n):
    st = tafv_stats()
    _check(lib.tafv_advance(ctx, int(n), C.byref(st)), ctx)
    return st.as_dict()


def tafv_advance_group(ctxs, n, workers=4, stats=True):
    """Advance the contexts together (one host worker per `workers` share of
    them); returns the summed counters, or None with stats=False."""
    arr = (C.c_void_p * len(ctxs))(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    st = tafv_stats() if stats else None
    rc = lib.tafv_advance_group(arr, len(ctxs), int(n), int(workers),
                                C.byref(st) if stats else None)
    if rc != OK:
        bad = None
        for c in ctxs:  # the failing context holds the message
            msg = lib.tafv_last_error(c)
            if msg:
                bad = msg
                break
        raise TafvError(rc, (bad or lib.tafv_last_error(None) or b"").decode())
    return st.as_dict() if stats else None


def tafv_advance_async(ctx, n):
    """tafv_advance without reading the counters back (no stream sync at the end)."""
    _check(lib.tafv_advance(ctx, int(n), None), ctx)


def tafv_mesh_stats(ctx, mesh_id):
    st = tafv_stats()
    _check(lib.tafv_mesh_stats(ctx, mesh_id, C.byref(st)), ctx)
    return st.as_dict()


def tafv_state_read(ctx, mesh_id, n_cells):
    cons = np.empty((n_cells, 5))
    lev = np.empty(n_cells, np.int8)
    _check(lib.tafv_state_read(ctx, mesh_id, _d(cons), lev.ctypes.data_as(C.POINTER(C.c_int8))),
           ctx)
    return cons, lev


def tafv_checkpoint_read(ctx, mesh_id, n_cells):
    cons = np.empty((n_cells, 5))
    acc = np.empty((n_cells, 5))
    lev = np.empty(n_cells, np.int8)
    phase, theta = C.c_int32(), C.c_int32()
    dtmin, t = C.c_double(), C.c_double()
    _check(lib.tafv_checkpoint_read(ctx, mesh_id, _d(cons), _d(acc),
                                    lev.ctypes.data_as(C.POINTER(C.c_int8)), C.byref(phase),
                                    C.byref(theta), C.byref(dtmin), C.byref(t)), ctx)
    return dict(cons=cons, accum=acc, levels=lev, phase=phase.value, theta=theta.value,
                dt_min=dtmin.value, t=t.value)


def tafv_checkpoint_write(ctx, mesh_id, cons, accum, levels, phase, theta, dt_min, t):
    cons = np.ascontiguousarray(cons, dtype=np.float64)
    accum = np.ascontiguousarray(accum, dtype=np.float64)
    levels = np.ascontiguousarray(levels, dtype=np.int8)
    _check(lib.tafv_checkpoint_write(ctx, mesh_id, _d(cons), _d(accum),
                                     levels.ctypes.data_as(C.POINTER(C.c_int8)), phase, theta,
                                     dt_min, t), ctx)


def _f(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def tafv_guess_config(ctx, guess, gate=0.0, stats=1, strength=0.0):
    _check(lib.tafv_guess_config(ctx, int(guess), float(gate), float(strength), int(stats)), ctx)


def tafv_mlp_set(ctx, params):
    params = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib.tafv_mlp_set(ctx, _f(params), params.size), ctx)


def tafv_mlp_get(ctx):
    out = np.empty(MLP_PARAMS, np.float32)
    _check(lib.tafv_mlp_get(ctx, _f(out), out.size), ctx)
    return out


def tafv_mlp_forward(ctx, x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty(x.shape[0], np.float32)
    _check(lib.tafv_mlp_forward(ctx, _f(x), x.shape[0], _f(y)), ctx)
    return y


def tafv_mlp_grad(ctx, x, t):
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    g = np.empty(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    _check(lib.tafv_mlp_grad(ctx, _f(x), _f(t), x.shape[0], _f(g), _f(loss)), ctx)
    return g, float(loss[0])


def tafv_mlp_grad_noalloc(ctx, x, t):
    """tafv_mlp_grad without device allocation (library scratch, at most
    MLP_GRAD_NOALLOC_MAX_ROWS rows)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    g = np.empty(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    _check(lib.tafv_mlp_grad_noalloc(ctx, _f(x), _f(t), x.shape[0], _f(g), _f(loss)), ctx)
    return g, float(loss[0])


def tafv_mlp_train(ctx, x, t, epochs=20, batch=4096, lr=1e-3, seed=0):
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    loss = np.zeros(max(epochs, 1), np.float32)
    _check(lib.tafv_mlp_train(ctx, _f(x), _f(t), x.shape[0], epochs, batch, lr, seed, _f(loss)),
           ctx)
    return loss[:epochs]


def tafv_facelog_config(ctx, capacity, rate, seed=0):
    _check(lib.tafv_facelog_config(ctx, int(capacity), float(rate), int(seed)), ctx)


def tafv_facelog_read(ctx, cap):
    rows = np.empty((max(cap, 1), 7), np.float32)
    n = C.c_int64()
    _check(lib.tafv_facelog_read(ctx, _f(rows), int(cap), C.byref(n)), ctx)
    return rows[:n.value]


def tafv_mesh_motion(ctx, mesh_id, node_vel):
    v = np.ascontiguousarray(node_vel, dtype=np.float64)
    _check(lib.tafv_mesh_motion(ctx, mesh_id, _d(v)), ctx)


def tafv_volume_read(ctx, mesh_id, n_cells):
    vol = np.empty(n_cells)
    _check(lib.tafv_volume_read(ctx, mesh_id, _d(vol)), ctx)
    return vol


def tafv_profile_enable(ctx, on=True):
    _check(lib.tafv_profile_enable(ctx, 1 if on else 0), ctx)


def tafv_profile_read(ctx):
    n = 16
    ms = np.zeros(n)
    launches = np.zeros(n, np.int64)
    items = np.zeros(n, np.int64)
    names = (C.c_char_p * n)()
    ncls = C.c_int32()
    _check(lib.tafv_profile_read(ctx, n, _d(ms), launches.ctypes.data_as(C.POINTER(C.c_int64)),
                                 items.ctypes.data_as(C.POINTER(C.c_int64)), names,
                                 C.byref(ncls)), ctx)
    return {names[k].decode(): dict(ms=float(ms[k]), launches=int(launches[k]),
                                    items=int(items[k])) for k in range(ncls.value)}


def tafv_batch_config(ctx, graph=1, autotune=1, tune_cache=None):
    path = tune_cache.encode() if tune_cache else None
    _check(lib.tafv_batch_config(ctx, int(graph), int(autotune), path), ctx)


def tafv_batch_info(ctx):
    """Launch settings of the batched kernels: (blocks, unit groups per grab,
    threads per block) of the gradient, flux and cell kernels, and where
    they came from."""
    a = (C.c_int32 * 10)()
    _check(lib.tafv_batch_info(ctx, a, 10), ctx)
    v = list(a)
    return dict(grad=tuple(v[0:3]), flux=tuple(v[3:6]), cells=tuple(v[6:9]),
                source={0: "default", 1: "tuned", 2: "cache"}[v[9]])


class Solver:
    """One context with one or more meshes."""

    def __init__(self, device=0, hip_stream=None, allocator=None, **params):
        """allocator: None (hipMalloc), or (alloc, dealloc) callables for
        tafv_set_allocator, e.g. torch_allocator(device, stream)."""
        self.params = tafv_params_default(**params)
        self.ctx = tafv_create(device, self.params, hip_stream)
        self.n_cells = []
        self._alloc_keep = None
        if allocator is not None:
            try:
                self._alloc_keep = tafv_set_allocator(self.ctx, *allocator)
            except Exception:
                self.close()
                raise

    def upload(self, nodes, tets, max_levels=None):
        mid = tafv_mesh_upload(self.ctx, nodes, tets)
        self.n_cells.append(len(tets))
        if max_levels is not None:
            tafv_mesh_params(self.ctx, mid, max_levels)
        return mid

    def init(self, prim, mesh_id=0):
        tafv_state_init(self.ctx, mesh_id, prim)

    def advance(self, n):
        return tafv_advance(self.ctx, n)

    def reset(self, mesh_id=0):
        tafv_state_reset(self.ctx, mesh_id)

    def read(self, mesh_id=0):
        return tafv_state_read(self.ctx, mesh_id, self.n_cells[mesh_id])

    def stats(self, mesh_id=0):
        return tafv_mesh_stats(self.ctx, mesh_id)

    def motion(self, node_vel, mesh_id=0):
        tafv_mesh_motion(self.ctx, mesh_id, node_vel)

    def volumes(self, mesh_id=0):
        return tafv_volume_read(self.ctx, mesh_id, self.n_cells[mesh_id])

    def checkpoint(self, mesh_id=0):
        return tafv_checkpoint_read(self.ctx, mesh_id, self.n_cells[mesh_id])

    def restore(self, ck, mesh_id=0):
        tafv_checkpoint_write(self.ctx, mesh_id, ck["cons"], ck["accum"], ck["levels"],
                              ck["phase"], ck["theta"], ck["dt_min"], ck["t"])

    def close(self):
        if self.ctx:
            tafv_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
