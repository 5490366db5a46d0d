"""ctypes binding of libmx (include/mx.h): argument marshalling only.

Every step of the solver runs inside libmx (host C++ for topology, gfx950 HIP kernels for all
numerical work on the device).  Device buffers are torch tensors (complex128 / any dtype with the
right byte size), passed by data pointer; streams are torch HIP streams.  If the library is not
built, every entry point raises -- there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmx.so")

MX_OK, MX_EINVAL, MX_ENOMEM, MX_EDEVICE, MX_EPIVOT, MX_ENAN, MX_ESTALL = 0, -1, -2, -3, -4, -5, -6
MX_EHBM, MX_ETIMEOUT = -7, -8
MX_BC_PEC, MX_BC_IMPEDANCE = 0, 1
MX_AS, MX_RAS, MX_ORAS = 0, 1, 2
MX_C128, MX_C64 = 0, 1
KINDS = {"as": MX_AS, "ras": MX_RAS, "oras": MX_ORAS}
PRECISIONS = {"c128": MX_C128, "c64": MX_C64}

# every symbol declared in include/mx.h
SYMBOLS = [
    "mx_last_error", "mx_version", "mx_ctx_create", "mx_ctx_destroy", "mx_mesh_box",
    "mx_mesh_sizes", "mx_mesh_export", "mx_mesh_destroy", "mx_matrix_assemble", "mx_matrix_sizes",
    "mx_matrix_export", "mx_matrix_destroy", "mx_spmv", "mx_rhs_gaussian", "mx_partition_box",
    "mx_partition_sizes", "mx_partition_export", "mx_partition_destroy", "mx_precond_setup",
    "mx_precond_apply", "mx_precond_get_info", "mx_precond_stage", "mx_precond_export_perm", "mx_precond_export_diag",
    "mx_precond_check", "mx_precond_destroy", "mx_gmres", "mx_selftest", "mx_local_problem",
    "mx_precond_sweep_timing", "mx_precond_autotune", "mx_server_create", "mx_server_submit",
    "mx_server_wait", "mx_server_solution", "mx_server_release", "mx_server_stats",
    "mx_server_destroy", "mx_matrix_upload", "mx_precond_plan", "mx_precond_materialize",
    "mx_selftest_host", "mx_gmres_noalloc", "mx_precond_add_coarse", "mx_precond_coarse_export",
    "mx_coarse_operators", "mx_weight_assemble", "mx_gmres_weighted", "mx_precond_plan_coarse",
    "mx_precond_tune_factor", "mx_server_batch_stats", "mx_matrix_assemble_order",
    "mx_mesh_order2_sizes", "mx_mesh_order2_export", "mx_partition_order2_export",
    "mx_weight_assemble_order", "mx_precond_add_coarse_box", "mx_precond_plan_coarse_box",
    "mx_coarse_operators_box", "mx_server_inject_enomem",
]


class MxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libmx error %d: %s" % (code, msg))
        self.code = code


# factor_schedule values of mx_precond_opts (mx.h)
FACTOR_SCHEDULES = {"auto": 0, "one_stream": 1, "lookahead": 2}
# combine values of mx_precond_add_coarse (mx.h)
COARSE = {"additive": 0, "hybrid": 1, "deflation": 2}


class PrecondOpts(C.Structure):
    _fields_ = [("kind", C.c_int), ("xi_prec", C.c_double), ("precision", C.c_int),
                ("sweep_grid", C.c_int), ("sub_begin", C.c_int),
                ("sub_end", C.c_int), ("pool_limit", C.c_int64), ("factor_schedule", C.c_int32),
                ("factor_width", C.c_int32)]


class PrecondInfo(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("tile", C.c_int32), ("n_local_total", C.c_int64),
                ("max_local", C.c_int64), ("max_blocks", C.c_int64), ("tiles", C.c_int64),
                ("factor_bytes", C.c_int64), ("env_entries", C.c_int64), ("env_flops", C.c_double),
                ("tile_flops", C.c_double), ("apply_bytes", C.c_int64), ("sweep_bytes", C.c_int64),
                ("t_host_setup", C.c_double),
                ("t_upload", C.c_double), ("t_factor", C.c_double), ("pack_bytes", C.c_int64),
                ("t_pack", C.c_double), ("factor_groups", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iters", C.c_int), ("flexible", C.c_int),
                ("fixed_iters", C.c_int), ("spmv_c64", C.c_int), ("rtol", C.c_double),
                ("graph", C.c_int)]


class GmresStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int), ("converged", C.c_int),
                ("relres_true", C.c_double), ("relres_est", C.c_double), ("t_solve", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("slots", C.c_int), ("kind", C.c_int),
                ("precision", C.c_int), ("layers", C.c_int), ("restart", C.c_int),
                ("max_iters", C.c_int), ("flexible", C.c_int), ("spmv_c64", C.c_int),
                ("rtol", C.c_double), ("batch_applies", C.c_int), ("batch_window_us", C.c_int)]


class Request(C.Structure):
    _fields_ = [("n", C.c_int), ("p", C.c_int), ("k", C.c_double), ("xi", C.c_double),
                ("center", C.c_double * 3), ("pol", C.c_double * 3), ("sigma", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("converged", C.c_int),
                ("relres_true", C.c_double), ("n_dof", C.c_int64), ("footprint_bytes", C.c_uint64),
                ("t_queue", C.c_double), ("t_host", C.c_double), ("t_device", C.c_double),
                ("t_total", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
P = C.c_void_p
I32P = np.ctypeslib.ndpointer(np.int32, flags="C")
I64P = np.ctypeslib.ndpointer(np.int64, flags="C")
I8P = np.ctypeslib.ndpointer(np.int8, flags="C")
F64P = np.ctypeslib.ndpointer(np.float64, flags="C")


def load(path=LIB_PATH):
    """Loads libmx.so (built by paper_1711_03789_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmx.so not built: run `python -m paper_1711_03789_amd.build` "
                           "(there is no CPU fallback)")
    lib = C.CDLL(path)
    sig = {
        "mx_last_error": (C.c_char_p, []),
        "mx_version": (C.c_int, []),
        "mx_ctx_create": (C.c_int, [C.c_int, C.POINTER(P)]),
        "mx_ctx_destroy": (None, [P]),
        "mx_mesh_box": (C.c_int, [C.c_int] * 3 + [C.c_double] * 3 + [C.POINTER(P)]),
        "mx_mesh_sizes": (C.c_int, [P] + [C.POINTER(C.c_int64)] * 4),
        "mx_mesh_export": (C.c_int, [P, P, P, P, P, P]),
        "mx_mesh_destroy": (None, [P]),
        "mx_matrix_assemble": (C.c_int, [P, P, C.c_double, C.c_double, C.c_int, C.POINTER(P)]),
        "mx_matrix_assemble_order": (C.c_int, [P, P, C.c_int, C.c_double, C.c_double, C.c_int,
                                               C.POINTER(P)]),
        "mx_weight_assemble_order": (C.c_int, [P, P, C.c_int, C.c_double, C.c_int, C.POINTER(P)]),
        "mx_mesh_order2_sizes": (C.c_int, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "mx_mesh_order2_export": (C.c_int, [P, P, P, P]),
        "mx_partition_order2_export": (C.c_int, [P, P, C.c_int, P, P, P]),
        "mx_matrix_sizes": (C.c_int, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "mx_matrix_export": (C.c_int, [P, P, P, P]),
        "mx_matrix_destroy": (None, [P]),
        "mx_spmv": (C.c_int, [P, P, P, P, P]),
        "mx_rhs_gaussian": (C.c_int, [P, C.c_int, F64P, F64P, C.c_double, P]),
        "mx_partition_box": (C.c_int, [P, C.c_int, C.c_int, C.c_int, P, P, P, C.c_int, C.POINTER(P)]),
        "mx_partition_sizes": (C.c_int, [P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
        "mx_partition_export": (C.c_int, [P, C.c_int, P, P, P, P]),
        "mx_partition_destroy": (None, [P]),
        "mx_precond_setup": (C.c_int, [P, P, P, P, C.POINTER(PrecondOpts), C.POINTER(P)]),
        "mx_precond_plan": (C.c_int, [P, P, P, P, C.POINTER(PrecondOpts), C.POINTER(P),
                                      C.POINTER(C.c_uint64)]),
        "mx_precond_materialize": (C.c_int, [P, P, P]),
        "mx_precond_stage": (C.c_int, [P, P]),
        "mx_matrix_upload": (C.c_int, [P, P]),
        "mx_precond_apply": (C.c_int, [P, P, P, P, P]),
        "mx_precond_get_info": (C.c_int, [P, C.POINTER(PrecondInfo)]),
        "mx_precond_export_perm": (C.c_int, [P, C.c_int, C.c_int64, P, P]),
        "mx_precond_export_diag": (C.c_int, [P, C.c_int, C.c_int64, P]),
        "mx_precond_check": (C.c_int, [P]),
        "mx_precond_add_coarse": (C.c_int, [P, P, P, P, C.c_int, C.c_int, P]),
        "mx_precond_plan_coarse": (C.c_int, [P, P, P, C.c_int, C.c_int]),
        "mx_precond_tune_factor": (C.c_int, [P, P, P, P, C.POINTER(PrecondOpts), P, C.POINTER(C.c_int32),
                                             C.POINTER(C.c_int32), C.POINTER(C.c_double), P]),
        "mx_precond_coarse_export": (C.c_int, [P] + [C.POINTER(C.c_int64)] * 3 + [P] * 6),
        "mx_coarse_operators": (C.c_int, [P, P, C.c_int] + [C.POINTER(C.c_int64)] * 3 + [P] * 6),
        "mx_coarse_operators_box": (C.c_int, [P, P] + [C.c_int] * 4 + [C.POINTER(C.c_int64)] * 3
                                    + [P] * 6),
        "mx_precond_add_coarse_box": (C.c_int, [P, P, P, P] + [C.c_int] * 5 + [P]),
        "mx_precond_plan_coarse_box": (C.c_int, [P, P, P] + [C.c_int] * 5),
        "mx_precond_autotune": (C.c_int, [P, P, P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "mx_server_create": (C.c_int, [C.c_int, C.POINTER(ServerOpts), C.POINTER(P)]),
        "mx_server_submit": (C.c_int, [P, C.POINTER(Request), C.POINTER(C.c_uint64)]),
        "mx_server_wait": (C.c_int, [P, C.c_uint64, C.c_double, C.POINTER(Result)]),
        "mx_server_solution": (C.c_int, [P, C.c_uint64, P, C.c_int64]),
        "mx_server_release": (C.c_int, [P, C.c_uint64]),
        "mx_server_stats": (C.c_int, [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                      C.POINTER(C.c_int)]),
        "mx_server_destroy": (None, [P]),
        "mx_server_batch_stats": (C.c_int, [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
        "mx_server_inject_enomem": (C.c_int, [P, C.c_int]),
        "mx_precond_sweep_timing": (C.c_int, [P, C.c_int, C.POINTER(C.c_int64),
                                              C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "mx_precond_destroy": (None, [P]),
        "mx_gmres": (C.c_int, [P, P, P, P, P, C.POINTER(GmresOpts), C.POINTER(GmresStats), P, P]),
        "mx_weight_assemble": (C.c_int, [P, P, C.c_double, C.c_int, C.POINTER(P)]),
        "mx_gmres_weighted": (C.c_int, [P, P, P, P, P, P, C.POINTER(GmresOpts), C.POINTER(GmresStats),
                                        P, P]),
        "mx_gmres_noalloc": (C.c_int, [P, P, P, P, P, C.POINTER(GmresOpts), C.POINTER(GmresStats), P,
                                       P]),
        "mx_selftest": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "mx_selftest_host": (C.c_int, [C.c_int64, C.c_int64, C.c_int, C.POINTER(C.c_int64)]),
        "mx_local_problem": (C.c_int, [P, P, P, C.POINTER(PrecondOpts), C.c_int,
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64), P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != MX_OK:
        raise MxError(rc, _lib.mx_last_error().decode())


def _ptr(a):
    """Raw pointer of a numpy array (host) or a torch tensor (host or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


def _dvec(t, n, what):
    """Device pointer of `t`, which must be a contiguous torch tensor on the GPU holding n
    complex128 values (16 n bytes; any dtype of that byte size).  The kernels index such vectors
    up to n without knowing their allocation, so a wrong size is refused here (MX_EINVAL).  None
    passes through; the library reports it."""
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise MxError(MX_EINVAL, "%s: expected a torch tensor on the GPU" % what)
    if not t.is_contiguous():
        raise MxError(MX_EINVAL, "%s: tensor must be contiguous" % what)
    nb = t.numel() * t.element_size()
    if nb != 16 * n:
        raise MxError(MX_EINVAL, "%s: %d bytes, expected complex128[%d] (%d bytes)"
                      % (what, nb, n, 16 * n))
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None  # the library reports the missing device itself
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _h(obj):
    return obj.h if obj is not None else None


class Context:
    def __init__(self, device=0):
        load()
        h = P()
        _check(_lib.mx_ctx_create(device, C.byref(h)))
        self.h, self.device = h, device

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mx_ctx_destroy(self.h)
        self.h = None

    __del__ = close

    def selftest(self):
        e64, e32 = C.c_double(), C.c_double()
        _check(_lib.mx_selftest(self.h, C.byref(e64), C.byref(e32)))
        return e64.value, e32.value


class Mesh:
    def __init__(self, nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
        load()
        h = P()
        _check(_lib.mx_mesh_box(nx, ny, nz, lx, ly, lz, C.byref(h)))
        self.h = h
        a = [C.c_int64() for _ in range(4)]
        _check(_lib.mx_mesh_sizes(h, *[C.byref(x) for x in a]))
        self.n_vert, self.n_tet, self.n_edge, self.n_bface = [x.value for x in a]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mx_mesh_destroy(self.h)
        self.h = None

    def export(self):
        tv = np.zeros((self.n_tet, 4), np.int32)
        ev = np.zeros((self.n_edge, 2), np.int32)
        te = np.zeros((self.n_tet, 6), np.int32)
        ts = np.zeros((self.n_tet, 6), np.int8)
        bf = np.zeros((self.n_bface, 3), np.int32)
        _check(_lib.mx_mesh_export(self.h, _ptr(tv), _ptr(ev), _ptr(te), _ptr(ts), _ptr(bf)))
        return {"tet_vert": tv, "edge_vert": ev, "tet_edge": te, "tet_edge_sign": ts, "bface_vert": bf}

    def order2(self):
        """Order-2 numbering: face vertex triples, faces of every tetrahedron, boundary DOFs."""
        nf, nd = C.c_int64(), C.c_int64()
        _check(_lib.mx_mesh_order2_sizes(self.h, C.byref(nf), C.byref(nd)))
        fv = np.zeros((nf.value, 3), np.int32)
        tf = np.zeros((self.n_tet, 4), np.int32)
        db = np.zeros(nd.value, np.uint8)
        _check(_lib.mx_mesh_order2_export(self.h, _ptr(fv), _ptr(tf), _ptr(db)))
        return {"n_face": nf.value, "n_dof": nd.value, "face_vert": fv, "tet_face": tf,
                "dof_boundary": db.astype(bool)}

    def rhs_gaussian(self, center, pol, sigma, bc=MX_BC_IMPEDANCE):
        f = np.zeros(self.n_edge, np.complex128)
        _check(_lib.mx_rhs_gaussian(self.h, bc, np.asarray(center, np.float64),
                                    np.asarray(pol, np.float64), sigma, _ptr(f)))
        return f


class Matrix:
    def __init__(self, ctx, mesh, k, xi, bc=MX_BC_IMPEDANCE, order=1):
        load()
        h = P()
        if order == 1:
            _check(_lib.mx_matrix_assemble(ctx.h if ctx is not None else None, mesh.h, k, xi, bc,
                                           C.byref(h)))
        else:
            _check(_lib.mx_matrix_assemble_order(ctx.h if ctx is not None else None, mesh.h, order,
                                                 k, xi, bc, C.byref(h)))
        self.h, self.k, self.xi, self.bc, self.order = h, k, xi, bc, order
        n, nnz = C.c_int64(), C.c_int64()
        _check(_lib.mx_matrix_sizes(h, C.byref(n), C.byref(nnz)))
        self.n, self.nnz = n.value, nnz.value

    @classmethod
    def weight(cls, ctx, mesh, k, bc=MX_BC_IMPEDANCE, order=1):
        """D_k = K + k^2 M, the weight of weighted GMRES (mx_weight_assemble[_order])."""
        load()
        self = cls.__new__(cls)
        h = P()
        if order == 1:
            _check(_lib.mx_weight_assemble(ctx.h if ctx is not None else None, mesh.h, k, bc,
                                           C.byref(h)))
        else:
            _check(_lib.mx_weight_assemble_order(ctx.h if ctx is not None else None, mesh.h, order,
                                                 k, bc, C.byref(h)))
        self.h, self.k, self.xi, self.bc, self.order = h, k, 0.0, bc, order
        n, nnz = C.c_int64(), C.c_int64()
        _check(_lib.mx_matrix_sizes(h, C.byref(n), C.byref(nnz)))
        self.n, self.nnz = n.value, nnz.value
        return self

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mx_matrix_destroy(self.h)
        self.h = None

    def upload(self, ctx):
        _check(_lib.mx_matrix_upload(ctx.h, self.h))

    def export(self):
        rp = np.zeros(self.n + 1, np.int64)
        col = np.zeros(self.nnz, np.int32)
        val = np.zeros(self.nnz, np.complex128)
        _check(_lib.mx_matrix_export(self.h, _ptr(rp), _ptr(col), _ptr(val)))
        return rp, col, val

    def spmv(self, ctx, x, y, stream=None):
        _check(_lib.mx_spmv(ctx.h, self.h, _dvec(x, self.n, "x"), _dvec(y, self.n, "y"),
                            _stream(stream)))


class Partition:
    def __init__(self, mesh, px, py, pz, layers, cx=None, cy=None, cz=None):
        load()
        h = P()
        arrs = [None if c is None else np.ascontiguousarray(c, np.int32) for c in (cx, cy, cz)]
        self._cuts = arrs
        _check(_lib.mx_partition_box(mesh.h, px, py, pz, *[_ptr(a) for a in arrs], layers, C.byref(h)))
        self.h = h
        self.n_edge = mesh.n_edge

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mx_partition_destroy(self.h)
        self.h = None

    def export(self, kind):
        kind = KINDS.get(kind, kind)
        n, tot = C.c_int32(), C.c_int64()
        _check(_lib.mx_partition_sizes(self.h, kind, C.byref(n), C.byref(tot)))
        off = np.zeros(n.value + 1, np.int64)
        l2g = np.zeros(tot.value, np.int32)
        owner = np.zeros(self.n_edge, np.int32)
        nt = np.zeros(n.value, np.int64)
        _check(_lib.mx_partition_export(self.h, kind, _ptr(off), _ptr(l2g), _ptr(owner), _ptr(nt)))
        return {"offsets": off, "loc2glob": l2g, "owner": owner, "n_tet": nt,
                "sets": [l2g[off[i]:off[i + 1]] for i in range(n.value)]}

    def export_order2(self, mesh, kind):
        """Order-2 local DOF sets and owners (mx_partition_order2_export)."""
        kind = KINDS.get(kind, kind)
        n, tot = C.c_int32(), C.c_int64()
        _check(_lib.mx_partition_sizes(self.h, kind, C.byref(n), C.byref(tot)))
        off = np.zeros(n.value + 1, np.int64)
        _check(_lib.mx_partition_order2_export(mesh.h, self.h, kind, _ptr(off), None, None))
        nf, nd = C.c_int64(), C.c_int64()
        _check(_lib.mx_mesh_order2_sizes(mesh.h, C.byref(nf), C.byref(nd)))
        l2g = np.zeros(off[-1], np.int32)
        owner = np.zeros(nd.value, np.int32)
        _check(_lib.mx_partition_order2_export(mesh.h, self.h, kind, _ptr(off), _ptr(l2g), _ptr(owner)))
        return {"offsets": off, "owner": owner, "sets": [l2g[off[i]:off[i + 1]] for i in range(n.value)]}


def selftest_host(n_items, fail_item=-1, fail_code=MX_EINVAL):
    """Host thread-pool error path (no device): returns (status, items run before a failure)."""
    load()
    ran = C.c_int64()
    rc = _lib.mx_selftest_host(n_items, fail_item, fail_code, C.byref(ran))
    return rc, ran.value


def _coarse_csr(fn, n_fine):
    import scipy.sparse as sp
    n, nr, na = C.c_int64(), C.c_int64(), C.c_int64()
    _check(fn(C.byref(n), C.byref(nr), C.byref(na), None, None, None, None, None, None))
    rp, rc, rv = np.zeros(n.value + 1, np.int64), np.zeros(nr.value, np.int32), np.zeros(nr.value)
    ap, ac = np.zeros(n.value + 1, np.int64), np.zeros(na.value, np.int32)
    av = np.zeros(na.value, np.complex128)
    _check(fn(C.byref(n), C.byref(nr), C.byref(na), _ptr(rp), _ptr(rc), _ptr(rv), _ptr(ap), _ptr(ac),
              _ptr(av)))
    return (sp.csr_matrix((rv, rc, rp), shape=(n.value, n_fine)),
            sp.csr_matrix((av, ac, ap), shape=(n.value, n.value)))


def coarse_operators(mesh, A, ratio=None, box=None, nq=12):
    """Host-only (R0, A0) of the coarse level for A on mesh: the nested mesh of `ratio`
    (mx_coarse_operators) or a coarse box mesh of box = (cnx, cny, cnz) cubes with an nq-point
    rule per fine edge (mx_coarse_operators_box)."""
    load()
    if box is not None:
        return _coarse_csr(lambda *a: _lib.mx_coarse_operators_box(mesh.h, A.h, *map(int, box),
                                                                   int(nq), *a), A.n)
    return _coarse_csr(lambda *a: _lib.mx_coarse_operators(mesh.h, A.h, int(ratio), *a), A.n)


def local_problem(mesh, A, part, l, kind="oras", xi_prec=None):
    """Host-only: local matrix of subdomain l (CSR in local numbering) and its RCM order."""
    load()
    o = PrecondOpts(KINDS.get(kind, kind), A.xi if xi_prec is None else xi_prec, MX_C128, 0, 0, 0, 0)
    n, nnz = C.c_int64(), C.c_int64()
    _check(_lib.mx_local_problem(mesh.h, A.h, part.h, C.byref(o), l, C.byref(n), C.byref(nnz),
                                 None, None, None, None, None))
    rp = np.zeros(n.value + 1, np.int64)
    col = np.zeros(nnz.value, np.int32)
    val = np.zeros(nnz.value, np.complex128)
    perm = np.zeros(n.value, np.int32)
    first = np.zeros(n.value, np.int32)
    _check(_lib.mx_local_problem(mesh.h, A.h, part.h, C.byref(o), l, C.byref(n), C.byref(nnz),
                                 _ptr(rp), _ptr(col), _ptr(val), _ptr(perm), _ptr(first)))
    return {"rowptr": rp, "col": col, "val": val, "perm": perm, "first": first}


class Precond:
    """plan_only=True runs only the host half (mx_precond_plan); call materialize() before use."""

    def __init__(self, ctx, A, mesh, part, kind="oras", xi_prec=None, precision="c128",
                 sweep_grid=0, share=None, plan_only=False, pool_limit=0, schedule="auto",
                 width=0):
        load()
        s0, s1 = share if share is not None else (0, 0)
        o = PrecondOpts(KINDS.get(kind, kind), A.xi if xi_prec is None else xi_prec,
                        PRECISIONS.get(precision, precision), sweep_grid, s0, s1, pool_limit,
                        FACTOR_SCHEDULES.get(schedule, schedule), width)
        h = P()
        self.device_bytes = None
        if plan_only:
            nb = C.c_uint64()
            _check(_lib.mx_precond_plan(_h(ctx), A.h, mesh.h, part.h, C.byref(o), C.byref(h),
                                        C.byref(nb)))
            self.device_bytes = nb.value
        else:
            _check(_lib.mx_precond_setup(ctx.h, A.h, mesh.h, part.h, C.byref(o), C.byref(h)))
        self.h, self.ctx, self.n = h, ctx, A.n

    def stage(self, ctx):
        """Host-to-device copies of the setup's device half (any host thread; optional)."""
        _check(_lib.mx_precond_stage(ctx.h, self.h))

    def materialize(self, ctx, stream=None):
        _check(_lib.mx_precond_materialize(ctx.h, self.h, _stream(stream)))
        self.ctx = ctx

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mx_precond_destroy(self.h)
        self.h = None

    def info(self):
        inf = PrecondInfo()
        _check(_lib.mx_precond_get_info(self.h, C.byref(inf)))
        return inf.as_dict()

    def apply(self, v, z, stream=None):
        _check(_lib.mx_precond_apply(_h(self.ctx), self.h, _dvec(v, self.n, "v"),
                                     _dvec(z, self.n, "z"), _stream(stream)))

    def check(self):
        _check(_lib.mx_precond_check(self.h))

    def add_coarse(self, ctx, A, mesh, ratio=None, combine="additive", stream=None, box=None, nq=12):
        """Two-level form; A and mesh are the ones P was built from.  The nested coarse mesh of
        `ratio` (mx_precond_add_coarse) or a coarse box mesh of box = (cnx, cny, cnz) cubes with
        an nq-point rule per fine edge (mx_precond_add_coarse_box)."""
        if box is not None:
            _check(_lib.mx_precond_add_coarse_box(ctx.h, self.h, A.h, mesh.h, *map(int, box), int(nq),
                                                  COARSE.get(combine, combine), _stream(stream)))
        else:
            _check(_lib.mx_precond_add_coarse(ctx.h, self.h, A.h, mesh.h, int(ratio),
                                              COARSE.get(combine, combine), _stream(stream)))
        self._coarse_A = A  # the library borrows A

    def plan_coarse(self, A, mesh, ratio=None, combine="additive", box=None, nq=12):
        """Host half of add_coarse (mx_precond_plan_coarse[_box]); any host thread."""
        if box is not None:
            _check(_lib.mx_precond_plan_coarse_box(self.h, A.h, mesh.h, *map(int, box), int(nq),
                                                   COARSE.get(combine, combine)))
        else:
            _check(_lib.mx_precond_plan_coarse(self.h, A.h, mesh.h, int(ratio),
                                               COARSE.get(combine, combine)))
        self._coarse_A = A

    def coarse_export(self):
        """(R0, A0) as scipy CSR matrices (coarse edges x fine edges, coarse x coarse)."""
        return _coarse_csr(lambda *a: _lib.mx_precond_coarse_export(self.h, *a), self.n)

    def autotune(self, stream=None):
        """Picks the fastest sweep grid; returns (grid, ms per application)."""
        g, ms = C.c_int32(), C.c_double()
        _check(_lib.mx_precond_autotune(_h(self.ctx), self.h, _stream(stream), C.byref(g), C.byref(ms)))
        return g.value, ms.value

    def sweep_timing(self, enable):
        """enable=True starts per-launch event timing of the sweep kernels; enable=False stops
        and returns (applications, forward_ms_total, backward_ms_total)."""
        n, a, b = C.c_int64(), C.c_double(), C.c_double()
        _check(_lib.mx_precond_sweep_timing(self.h, 1 if enable else 0, C.byref(n), C.byref(a),
                                            C.byref(b)))
        return n.value, a.value, b.value

    def perm(self, l, n_local):
        perm = np.zeros(n_local, np.int32)
        first = np.zeros(n_local, np.int32)
        _check(_lib.mx_precond_export_perm(self.h, l, n_local, _ptr(perm), _ptr(first)))
        return perm, first

    def diag(self, l, n_local):
        d = np.zeros(n_local, np.complex128)
        _check(_lib.mx_precond_export_diag(self.h, l, n_local, _ptr(d)))
        return d


def tune_factor(ctx, A, mesh, part, kind="oras", xi_prec=None, precision="c128", stream=None):
    """Factorisation tuner (mx_precond_tune_factor): returns (schedule, width, best ms, ms of the
    five candidates: one stream, look-ahead with widths 1..4)."""
    o = PrecondOpts(KINDS.get(kind, kind), A.xi if xi_prec is None else xi_prec,
                    PRECISIONS.get(precision, precision), 0, 0, 0, 0, 0, 0)
    bs, bw, ms = C.c_int32(), C.c_int32(), C.c_double()
    each = np.zeros(5)
    _check(_lib.mx_precond_tune_factor(ctx.h, A.h, mesh.h, part.h, C.byref(o), _stream(stream),
                                       C.byref(bs), C.byref(bw), C.byref(ms), _ptr(each)))
    return bs.value, bw.value, ms.value, each.tolist()


def gmres(ctx, A, Pc, b, x, restart=50, rtol=1e-6, max_iters=1000, flexible=False,
          fixed_iters=0, spmv_c64=False, history=False, stream=None, noalloc=False, weight=None,
          graph=False):
    """noalloc=True calls mx_gmres_noalloc (fixed per-GPU workspace, no device allocation);
    weight=D (a Matrix.weight) calls mx_gmres_weighted (residual minimised in the D-norm)."""
    o = GmresOpts(restart, max_iters, int(flexible), fixed_iters, int(spmv_c64), rtol, int(graph))
    st = GmresStats()
    hist = np.zeros(max(max_iters, fixed_iters) + 2, np.float64) if history else None
    if weight is not None:
        _check(_lib.mx_gmres_weighted(ctx.h, A.h, Pc.h if Pc is not None else None, weight.h,
                                      _dvec(b, A.n, "b"), _dvec(x, A.n, "x"), C.byref(o),
                                      C.byref(st), _ptr(hist), _stream(stream)))
        out = st.as_dict()
        if history:
            out["history"] = hist[: st.iters + 1].copy()
        return out
    fn = _lib.mx_gmres_noalloc if noalloc else _lib.mx_gmres
    _check(fn(ctx.h, A.h, Pc.h if Pc is not None else None, _dvec(b, A.n, "b"),
                         _dvec(x, A.n, "x"),
                         C.byref(o), C.byref(st), _ptr(hist), _stream(stream)))
    out = st.as_dict()
    if history:
        out["history"] = hist[: st.iters + 1].copy()
    return out


class Server:
    """Continuous-batching solve server (include/mx.h, mx_server_*)."""

    def __init__(self, device=0, slots=4, hbm_budget=0, kind="oras", precision="c64", layers=2,
                 restart=50, max_iters=1000, flexible=True, spmv_c64=False, rtol=1e-6,
                 batch_applies=True, batch_window_us=0):
        load()
        o = ServerOpts(hbm_budget, slots, KINDS.get(kind, kind), PRECISIONS.get(precision, precision),
                       layers, restart, max_iters, int(flexible), int(spmv_c64), rtol,
                       int(batch_applies), batch_window_us)
        h = P()
        _check(_lib.mx_server_create(device, C.byref(o), C.byref(h)))
        self.h = h
        self.sizes = {}

    def submit(self, n, p, k, xi, center=(0.5, 0.5, 0.5), pol=(1.0, 0.0, 0.0), sigma=0.1):
        r = Request(n, p, k, xi, (C.c_double * 3)(*center), (C.c_double * 3)(*pol), sigma)
        t = C.c_uint64()
        _check(_lib.mx_server_submit(self.h, C.byref(r), C.byref(t)))
        return t.value

    def wait(self, ticket, timeout=-1.0):
        res = Result()
        _check(_lib.mx_server_wait(self.h, ticket, timeout, C.byref(res)))
        out = res.as_dict()
        if res.status != MX_OK:
            out["error"] = _lib.mx_last_error().decode()
        return out

    def solution(self, ticket, n_dof):
        x = np.zeros(n_dof, np.complex128)
        _check(_lib.mx_server_solution(self.h, ticket, _ptr(x), n_dof))
        return x

    def release(self, ticket):
        _check(_lib.mx_server_release(self.h, ticket))

    def stats(self):
        b, pk, ma = C.c_uint64(), C.c_uint64(), C.c_int()
        _check(_lib.mx_server_stats(self.h, C.byref(b), C.byref(pk), C.byref(ma)))
        nb, na = C.c_uint64(), C.c_uint64()
        _check(_lib.mx_server_batch_stats(self.h, C.byref(nb), C.byref(na)))
        return {"budget": b.value, "peak_used": pk.value, "max_admitted": ma.value,
                "batches": nb.value, "batched_applications": na.value}

    def inject_enomem(self, n):
        """Test hook: the next n device phases fail once after their setup and are retried."""
        _check(_lib.mx_server_inject_enomem(self.h, int(n)))

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mx_server_destroy(self.h)
        self.h = None

    __del__ = close
