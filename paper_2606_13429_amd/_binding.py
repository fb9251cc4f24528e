"""ctypes binding of libdcg.so (include/dcg.h): argument marshalling only.

Every function keeps the name of its C entry point.  Vector arguments are
torch tensors on the GPU (or raw device addresses as ints); the binding
checks dtype, device, contiguity and length, passes ``data_ptr()`` and the
current torch stream, and raises DCGError for negative status codes.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libdcg.so is not built (%s); run `python paper_2606_13429_amd/build.py` "
        "or __graft_entry__.build() first" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ types
DCG_OK, DCG_NOT_CONVERGED, DCG_PENDING = 0, 1, 2
DCG_EINVAL, DCG_ENOMEM, DCG_EDEVICE, DCG_EAGAIN, DCG_ENOTFOUND, DCG_EBREAKDOWN = -1, -2, -3, -4, -5, -6
DCG_FP64, DCG_MIXED = 0, 1
DCG_OUTER_CG, DCG_OUTER_FCG1, DCG_OUTER_FCG, DCG_OUTER_GMRES = 0, 1, 2, 3
DCG_INNER_MG, DCG_INNER_EXACT, DCG_INNER_NONE = 0, 1, 2
(DCG_OP_ASTAR, DCG_OP_ZT, DCG_OP_Z, DCG_OP_ADIVZ, DCG_OP_DEFLATED, DCG_OP_INNER, DCG_OP_LAPLACE,
 DCG_OP_RAS, DCG_OP_RESTRICT, DCG_OP_PROLONG, DCG_OP_COARSE, DCG_OP_WCYCLE, DCG_OP_RAS_BATCH,
 DCG_OP_WCYCLE_BATCH, DCG_OP_OMG_APPLY, DCG_OP_OMG_LEVEL, DCG_OP_OMG_RAS, DCG_OP_OMG_RESTRICT,
 DCG_OP_OMG_PROLONG, DCG_OP_OMG_COARSE, DCG_OP_OMG_WCYCLE) = range(21)
BATCH = 16   # vectors of the _BATCH operators and requests per serving batch
(DCG3D_OP_ASTAR, DCG3D_OP_ZT, DCG3D_OP_Z, DCG3D_OP_DEFLATED, DCG3D_OP_REDUCED, DCG3D_OP_INNER,
 DCG3D_OP_ADIVZ) = range(7)
DCG3D_MAX_N, DCG3D_DEFAULT_MAX_INNER, DCG3D_MAX_HOST_BLOCKS_N = 64, 20000, 16
DCG3D_INNER_FDM, DCG3D_INNER_PCG, DCG3D_INNER_NONE, DCG3D_INNER_MG = 0, 1, 2, 3
(DCG3D_MG_LAPLACE, DCG3D_MG_RAS, DCG3D_MG_RESTRICT, DCG3D_MG_PROLONG, DCG3D_MG_COARSE,
 DCG3D_MG_WCYCLE) = range(6)


class dcg_mesh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("penalty", ctypes.c_double),
                ("pre", ctypes.c_int32), ("post", ctypes.c_int32)]


class dcg_options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("outer", ctypes.c_int), ("c_F", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("max_inner", ctypes.c_int32),
                ("x0_given", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("max_pending", ctypes.c_int32),
                ("c_A", ctypes.c_double), ("m_max", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("ras_group", ctypes.c_int32), ("smooth3d", ctypes.c_int32),
                ("outer_mg", ctypes.c_int32)]


class dcg_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("total_wcycles", ctypes.c_int32), ("inner_solves", ctypes.c_int32),
                ("inner_per_outer", ctypes.c_double), ("rel_res_recurrence", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_queue_ms", ctypes.c_double),
                ("restarts", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_h = ctypes.c_void_p
_vp = ctypes.c_void_p
_P = ctypes.POINTER

_SIGS = {
    "dcg_defaults": (None, [_P(dcg_mesh), _P(dcg_options)]),
    "dcg_setup": (ctypes.c_int, [_P(dcg_mesh), ctypes.c_double, ctypes.c_double, _P(dcg_options), _P(_h)]),
    "dcg_solve": (ctypes.c_int, [_h, _vp, _vp, ctypes.c_double, _P(dcg_stats), _vp]),
    "dcg_apply": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "dcg_apply_noalloc": (ctypes.c_int, [_h, ctypes.c_int, _vp, _vp, _vp]),
    "dcg_noalloc_bytes": (ctypes.c_int64, []),
    "dcg_num_levels": (ctypes.c_int32, [ctypes.c_int32]),
    "dcg_host_assemble": (ctypes.c_int, [_P(dcg_mesh), ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double),
                                         ctypes.c_int64, _P(ctypes.c_int32), ctypes.c_int64, _P(ctypes.c_int64)]),
    "dcg_bdf2_rhs": (ctypes.c_int, [_h, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp]),
    "dcg_kernel_timing": (ctypes.c_int, [_h, ctypes.c_int32]),
    "dcg_kernel_timing_read": (ctypes.c_int, [_h, _P(ctypes.c_double), _P(ctypes.c_int64)]),
    "dcg_kernel_timing_read_astar": (ctypes.c_int, [_h, _P(ctypes.c_double), _P(ctypes.c_int64)]),
    "dcg_server_create": (ctypes.c_int, [_P(dcg_options), _P(_h)]),
    "dcg_server_prepare": (ctypes.c_int, [_h, _P(dcg_mesh)]),
    "dcg_submit": (ctypes.c_int, [_h, _P(dcg_mesh), ctypes.c_double, ctypes.c_double, _vp, _vp,
                                  ctypes.c_double, _P(ctypes.c_uint64)]),
    "dcg_poll": (ctypes.c_int, [_h, ctypes.c_uint64, _P(dcg_stats)]),
    "dcg_server_counters": (ctypes.c_int, [_h, _P(ctypes.c_int64), _P(ctypes.c_int64)]),
    "dcg_server_group_bytes": (ctypes.c_int64, [_P(dcg_mesh), ctypes.c_int]),
    "dcg_server_destroy": (ctypes.c_int, [_h]),
    "dcg_destroy": (ctypes.c_int, [_h]),
    "dcg_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "dcg_last_error": (ctypes.c_char_p, [_h]),
    "dcg_clear_cache": (None, []),
    "dcg3d_setup": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int32, _P(dcg_options), _P(_h)]),
    "dcg3d_solve": (ctypes.c_int, [_h, _vp, _vp, ctypes.c_double, _P(dcg_stats)]),
    "dcg3d_apply": (ctypes.c_int, [_h, ctypes.c_int, _vp, _vp, ctypes.c_double]),
    "dcg3d_destroy": (ctypes.c_int, [_h]),
    "dcg3d_kernel_timing": (ctypes.c_int, [_h, ctypes.c_int32]),
    "dcg3d_kernel_timing_read": (ctypes.c_int, [_h, _P(ctypes.c_double), _P(ctypes.c_int64)]),
    "dcg3d_last_error": (ctypes.c_char_p, [_h]),
    "dcg3d_host_blocks": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                         _P(ctypes.c_double)]),
    "dcg3d_mg_apply": (ctypes.c_int, [_h, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]),
    "dcg_host_outer_mg": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double), ctypes.c_int64]),
    "dcg3d_mg_levels": (ctypes.c_int, [_h, _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    "dcg3d_host_mg": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, _P(ctypes.c_double)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class DCGError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (dcg_strerror(status), status, message))
        self.status = status


def _check(status, handle=None):
    if status < 0:
        raise DCGError(status, dcg_last_error(handle))
    return status


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    import torch
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ API
def dcg_defaults():
    m, o = dcg_mesh(), dcg_options()
    _lib.dcg_defaults(ctypes.byref(m), ctypes.byref(o))
    return m, o


def dcg_num_levels(n):
    return _lib.dcg_num_levels(n)


def dcg_strerror(status):
    return _lib.dcg_strerror(status).decode()


def dcg_last_error(handle=None):
    return _lib.dcg_last_error(handle).decode()


def dcg_setup(mesh, dt, nu=1.0, opt=None):
    h = _h()
    _check(_lib.dcg_setup(ctypes.byref(mesh), dt, nu, ctypes.byref(opt) if opt is not None else None,
                          ctypes.byref(h)))
    return h


def dcg_solve(handle, b, x, tol, stream=None):
    """Returns (status, dcg_stats); raises DCGError on negative status."""
    n = None
    st = dcg_stats()
    status = _lib.dcg_solve(handle, _ptr(b, _f64(), n, "b"), _ptr(x, _f64(), n, "x"), tol,
                            ctypes.byref(st), _stream(stream))
    _check(status, handle)
    return status, st


def dcg_apply(handle, op, level, inp, in2, out, stream=None):
    return _check(_lib.dcg_apply(handle, op, level, _ptr(inp, name="in"), _ptr(in2, name="in2"),
                                 _ptr(out, name="out"), _stream(stream)), handle)


def dcg_apply_noalloc(handle, op, inp, out, stream=None):
    return _check(_lib.dcg_apply_noalloc(handle, op, _ptr(inp, name="in"), _ptr(out, name="out"),
                                         _stream(stream)), handle)


def dcg_noalloc_bytes():
    return _lib.dcg_noalloc_bytes()


def dcg_host_outer_mg(n, penalty, dt, nu, level, which):
    """Host copy of a class table of the outer multigrid (no device call):
    which 0 the operator table (9, 5, 16, 16), 1 the RAS update table
    (49, 16, 208), 2 the coarsest inverse (1024, 1024), 3 and 4 tables 0 and
    1 in the MFMA operand order, (9, 20, 64) and (49, 52, 64)."""
    import numpy as np
    shape = {0: (9, 5, 16, 16), 1: (49, 16, 208), 2: (1024, 1024), 3: (9, 20, 64), 4: (49, 52, 64)}[which]
    out = np.empty(shape, dtype=np.float64)
    _check(_lib.dcg_host_outer_mg(n, penalty, dt, nu, level, which, out.ctypes.data_as(_P(ctypes.c_double)),
                                  out.size))
    return out


def dcg_host_assemble(mesh, which, level=0):
    """Returns (values as a flat numpy float64 array, int32 columns or None)."""
    import numpy as np
    need = ctypes.c_int64()
    _check(_lib.dcg_host_assemble(ctypes.byref(mesh), which, level, None, 0, None, 0, ctypes.byref(need)))
    vals = np.empty(need.value, dtype=np.float64)
    ne = mesh.n * mesh.n
    ncols = {0: ne * 5, 1: ne * 5, 3: None, 4: None}.get(which)
    if which == 3:
        nk = mesh.n >> (dcg_num_levels(mesh.n) - level)
        ncols = nk * nk * 5
    elif which == 4:
        ncols = vals.size // (128 * 128) * 32
    cols = np.empty(ncols, dtype=np.int32) if ncols else None
    _check(_lib.dcg_host_assemble(
        ctypes.byref(mesh), which, level, vals.ctypes.data_as(_P(ctypes.c_double)), vals.size,
        cols.ctypes.data_as(_P(ctypes.c_int32)) if cols is not None else None,
        cols.size if cols is not None else 0, None))
    return vals, cols


def dcg_bdf2_rhs(handle, s1, s2, F, c, f, x0, stream=None):
    return _check(_lib.dcg_bdf2_rhs(handle, _ptr(s1, _f64(), name="s1"), _ptr(s2, _f64(), name="s2"),
                                    _ptr(F, _f64(), name="F"), c, _ptr(f, _f64(), name="f"),
                                    _ptr(x0, _f64(), name="x0"), _stream(stream)), handle)


def dcg_kernel_timing(handle, enable):
    return _check(_lib.dcg_kernel_timing(handle, int(enable)), handle)


def dcg_kernel_timing_read(handle):
    """Returns (total milliseconds, launches) of the timed kernel."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(_lib.dcg_kernel_timing_read(handle, ctypes.byref(ms), ctypes.byref(n)), handle)
    return ms.value, n.value


def dcg_server_create(opt=None):
    s = _h()
    _check(_lib.dcg_server_create(ctypes.byref(opt) if opt is not None else None, ctypes.byref(s)))
    return s


def dcg_server_prepare(server, mesh):
    return _check(_lib.dcg_server_prepare(server, ctypes.byref(mesh)))


def dcg_submit(server, mesh, dt, nu, b, x, tol):
    """Returns the ticket; raises DCGError (e.g. DCG_EAGAIN) on negative status."""
    t = ctypes.c_uint64()
    N = 16 * mesh.n * mesh.n
    _check(_lib.dcg_submit(server, ctypes.byref(mesh), dt, nu, _ptr(b, _f64(), N, "b"),
                           _ptr(x, _f64(), N, "x"), tol, ctypes.byref(t)))
    return t.value


def dcg_poll(server, ticket):
    """Returns (status, dcg_stats); status DCG_PENDING while running.  A
    failed request returns its negative status (no exception) with the
    message in dcg_last_error(); an unknown ticket raises DCGError."""
    st = dcg_stats()
    status = _lib.dcg_poll(server, ticket, ctypes.byref(st))
    if status == DCG_ENOTFOUND:
        raise DCGError(status, dcg_last_error())
    return status, st


def dcg_server_group_bytes(mesh, prec=DCG_MIXED):
    return _lib.dcg_server_group_bytes(ctypes.byref(mesh), prec)


def dcg_server_counters(server):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.dcg_server_counters(server, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def dcg_server_destroy(server):
    return _lib.dcg_server_destroy(server)


def dcg_destroy(handle):
    return _lib.dcg_destroy(handle)


def dcg_clear_cache():
    _lib.dcg_clear_cache()


def _f64():
    import torch
    return torch.float64


# ------------------------------------------------------------------ 3D solver
def _check3(status, handle=None):
    if status < 0:
        msg = _lib.dcg3d_last_error(handle)
        raise DCGError(status, msg.decode() if msg else "")
    return status


def _sync_torch_stream():
    # the 3D entry points run on the legacy default stream: order them after
    # work torch queued on another current stream
    import torch
    cs = torch.cuda.current_stream()
    if cs.cuda_stream != 0:
        cs.synchronize()


def dcg3d_setup(n, penalty, dt, nu=1.0, opt=None, inner=DCG3D_INNER_FDM):
    h = _h()
    _check3(_lib.dcg3d_setup(n, penalty, dt, nu, inner, ctypes.byref(opt) if opt is not None else None,
                             ctypes.byref(h)))
    return h


def dcg3d_solve(handle, b, x, tol):
    """Returns (status, dcg_stats); raises DCGError on negative status."""
    st = dcg_stats()
    _sync_torch_stream()
    status = _lib.dcg3d_solve(handle, _ptr(b, _f64(), None, "b"), _ptr(x, _f64(), None, "x"), tol,
                              ctypes.byref(st))
    _check3(status, handle)
    return status, st


def dcg3d_apply(handle, op, inp, out, tol=0.0):
    _sync_torch_stream()
    return _check3(_lib.dcg3d_apply(handle, op, _ptr(inp, _f64(), None, "in"), _ptr(out, _f64(), None, "out"),
                                    tol), handle)


def dcg3d_destroy(handle):
    return _lib.dcg3d_destroy(handle)


def dcg3d_last_error(handle=None):
    msg = _lib.dcg3d_last_error(handle)
    return msg.decode() if msg else ""


def dcg3d_host_blocks(n, penalty, dt, which):
    """Host copy of the assembled 3D blocks (no device call): a flat float64 array."""
    import numpy as np
    ne = n ** 3
    N = 2 * n
    size = {0: 7 * ne * 576, 1: 7 * ne * 64, 2: ne * 64, 3: 64, 4: 2 * (N * N + N)}[which]
    out = np.empty(size, dtype=np.float64)
    _check3(_lib.dcg3d_host_blocks(n, penalty, dt, which, out.ctypes.data_as(_P(ctypes.c_double))))
    return out


def dcg3d_mg_apply(handle, op, level, inp, inp2, out):
    """One level operator of the 3D multigrid hierarchy (inp2 may be None)."""
    _sync_torch_stream()
    return _check3(_lib.dcg3d_mg_apply(handle, op, level, _ptr(inp, _f64(), None, "in"),
                                       _ptr(inp2, _f64(), None, "in2"), _ptr(out, _f64(), None, "out")),
                   handle)


def dcg3d_mg_levels(handle):
    """(J, coarsest cubes per side) of a DCG3D_INNER_MG handle."""
    J, c = ctypes.c_int32(), ctypes.c_int32()
    _check3(_lib.dcg3d_mg_levels(handle, ctypes.byref(J), ctypes.byref(c)), handle)
    return J.value, c.value


def dcg3d_host_mg(n, penalty, levels, level, which, coarsest=None):
    """Host copy of a class table of the 3D multigrid hierarchy (no device
    call): which 0 the operator table (27, 7, 8, 8), 1 the RAS update table
    (343, 8, 200), 2 the coarsest inverse (m, m); ``coarsest`` (cubes per
    side of level 1) sizes the latter."""
    import numpy as np
    if which == 2:
        m = 8 * coarsest ** 3
        shape = (m, m)
    else:
        shape = {0: (27, 7, 8, 8), 1: (343, 8, 200)}[which]
    out = np.empty(shape, dtype=np.float64)
    _check3(_lib.dcg3d_host_mg(n, penalty, levels, level, which, out.ctypes.data_as(_P(ctypes.c_double))))
    return out


def dcg3d_kernel_timing(handle, enable):
    return _check3(_lib.dcg3d_kernel_timing(handle, int(bool(enable))), handle)


def dcg3d_kernel_timing_read(handle):
    """Returns (total ms, launches) of the timed Laplacian launches."""
    ms, k = ctypes.c_double(), ctypes.c_int64()
    _check3(_lib.dcg3d_kernel_timing_read(handle, ctypes.byref(ms), ctypes.byref(k)), handle)
    return ms.value, k.value


def dcg_kernel_timing_read_astar(handle):
    """Returns (total ms, launches) of the timed A* launches of the CG outer loop."""
    ms, k = ctypes.c_double(), ctypes.c_int64()
    _check(_lib.dcg_kernel_timing_read_astar(handle, ctypes.byref(ms), ctypes.byref(k)), handle)
    return ms.value, k.value
