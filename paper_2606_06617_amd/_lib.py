"""ctypes binding of libpswflr.so (include/pswflr.h), argument marshalling only.

Every step of the path runs in the library's HIP kernels; this module only
converts Python values and torch tensors into the C structs and device
pointers the ABI expects.  Importing it fails loudly when the library has
not been built (there is no fallback).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpswflr.so")

MAX_CHANNELS = 64
FLAG_CHECK_INPUTS = 1

OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "workspace", 4: "device error",
          5: "out of memory", 6: "internal error"}


class Params(ctypes.Structure):
    _fields_ = [
        ("n_channels", ctypes.c_int32),
        ("p", ctypes.c_int32 * MAX_CHANNELS),
        ("box", ctypes.c_double * 3),
        ("r_c", ctypes.c_double),
        ("c", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("grid", ctypes.c_int32 * 3),
        ("support", ctypes.c_int32),
        ("c_spread", ctypes.c_double),
        ("tile", ctypes.c_int32 * 3),
        ("flags", ctypes.c_uint32),
        ("cell", ctypes.c_double * 9),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("c", ctypes.c_double), ("r_c", ctypes.c_double), ("k_c", ctypes.c_double),
        ("c_spread", ctypes.c_double), ("eta", ctypes.c_double),
        ("h", ctypes.c_double * 3),
        ("volume", ctypes.c_double),
        ("grid", ctypes.c_int32 * 3),
        ("support", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("kz_keep", ctypes.c_int32),
        ("ny_keep", ctypes.c_int32),
        ("tile", ctypes.c_int32 * 3),
        ("cg_spread", ctypes.c_int32),
        ("cg_gather", ctypes.c_int32),
        ("xcols", ctypes.c_int64),
        ("max_atoms", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_size_t),
        ("grid_offset", ctypes.c_size_t),
        ("self_coef", ctypes.c_double * MAX_CHANNELS),
        ("zero_coef", ctypes.c_double * MAX_CHANNELS),
        ("cell", ctypes.c_double * 9),
    ]


class IO(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int64),
        ("pos", ctypes.c_void_p),
        ("q", ctypes.c_void_p),
        ("energy", ctypes.c_void_p),
        ("forces", ctypes.c_void_p),
        ("virial", ctypes.c_void_p),
        ("potential", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load libpswflr.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libpswflr.so is not built (expected at %s); run "
            "`python -m paper_2606_06617_amd.build` first -- there is no CPU fallback" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    L.pswflr_plan_create.argtypes = [ctypes.POINTER(Params), i64, ctypes.POINTER(vp)]
    L.pswflr_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.pswflr_plan_destroy.argtypes = [vp]
    L.pswflr_execute.argtypes = [vp, vp, vp, sz, i64, vp, vp, vp, vp, vp, vp]
    L.pswflr_backward.argtypes = [vp, vp, vp, sz, i64, vp, vp, vp, vp, vp]
    L.pswflr_execute_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
    L.pswflr_realspace.argtypes = [vp, vp, vp, sz, i64, vp, vp, vp, vp, vp, vp]
    L.pswflr_force_vjp.argtypes = [vp, vp, vp, sz, i64, vp, vp, vp, vp, vp]
    L.pswflr_cell_gradient.argtypes = [vp, vp, vp, vp]
    L.pswflr_batch_workspace.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                         ctypes.POINTER(sz)]
    L.pswflr_execute_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(IO), vp, vp, sz]
    L.pswflr_execute_batch_flat.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(i64), vp, vp, vp, vp,
                                            vp, vp, vp, vp, sz]
    L.pswflr_backward_batch_flat.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(i64), vp, vp, vp, vp,
                                             vp, vp, vp, sz]
    L.pswflr_profile_enable.argtypes = [vp, ctypes.c_int]
    L.pswflr_profile_stages.argtypes = [vp, ctypes.c_uint32]
    L.pswflr_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.pswflr_status_string.argtypes = [ctypes.c_int]
    L.pswflr_status_string.restype = ctypes.c_char_p
    L.pswflr_last_error.argtypes = [ctypes.c_char_p, sz]
    for name in ("pswflr_plan_create", "pswflr_plan_info", "pswflr_plan_destroy", "pswflr_execute",
                 "pswflr_execute_noalloc", "pswflr_realspace", "pswflr_force_vjp", "pswflr_cell_gradient",
                 "pswflr_backward", "pswflr_batch_workspace", "pswflr_execute_batch",
                 "pswflr_execute_batch_flat", "pswflr_backward_batch_flat",
                 "pswflr_profile_enable", "pswflr_profile_stages", "pswflr_profile_read"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class PswflrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def check(status):
    if status != OK:
        buf = ctypes.create_string_buffer(512)
        lib().pswflr_last_error(buf, 512)
        raise PswflrError(status, buf.value.decode(errors="replace"))


def make_params(box, ps, r_c, c=0.0, tol=1e-5, grid=None, support=0, c_spread=0.0, tile=None, flags=0):
    prm = Params()
    ps = list(ps)
    if not 1 <= len(ps) <= MAX_CHANNELS:
        raise ValueError("between 1 and %d channels" % MAX_CHANNELS)
    prm.n_channels = len(ps)
    for i, p in enumerate(ps):
        prm.p[i] = int(p)
    rows = [list(r) if hasattr(r, "__len__") else None for r in box]
    if len(rows) == 3 and all(r is not None and len(r) == 3 for r in rows):
        # a 3x3 cell (lattice vectors as rows)
        for a in range(3):
            for b in range(3):
                prm.cell[3 * a + b] = float(rows[a][b])
    elif len(rows) == 3 and all(r is None for r in rows):
        for a in range(3):
            prm.box[a] = float(box[a])
    else:
        raise ValueError("box must be 3 edges or a 3x3 cell (rows: lattice vectors)")
    for a in range(3):
        prm.grid[a] = int(grid[a]) if grid is not None else 0
    prm.r_c = float(r_c)
    prm.c = float(c or 0.0)
    prm.tol = float(tol or 0.0)
    prm.support = int(support or 0)
    prm.c_spread = float(c_spread or 0.0)
    for a in range(3):
        prm.tile[a] = int(tile[a]) if tile is not None else 0
    prm.flags = int(flags)
    return prm
