"""ctypes declarations of the C ABI in include/idugks.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libidugks.so")

BC_WALL, BC_FARFIELD, BC_PERIODIC = 0, 1, 2
GAUSS_HERMITE, NEWTON_COTES = 0, 1
BGK, SHAKHOV = 0, 1
FP64, FP32_MIXED = 0, 1
EXPLICIT, IMPLICIT = 0, 1
SWEEPS_AUTO, SWEEPS_LEVELS, SWEEPS_HYPERPLANES = 0, 1, 2

STATUS = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_DIVERGED",
          5: "E_NOT_CONVERGED", 6: "E_STATE"}


class IdugksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"idugks {STATUS.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("ni", C.c_int32), ("nj", C.c_int32),
        ("xn", C.POINTER(C.c_double)), ("yn", C.POINTER(C.c_double)),
        ("bc", C.c_int32 * 4),
        ("wall_u", C.c_double * 4), ("wall_v", C.c_double * 4), ("wall_T", C.c_double * 4),
        ("far_rho", C.c_double), ("far_u", C.c_double), ("far_v", C.c_double), ("far_T", C.c_double),
        ("quad", C.c_int32), ("nvx", C.c_int32), ("nvy", C.c_int32), ("vmax", C.c_double),
        ("model", C.c_int32), ("Kn", C.c_double), ("Pr", C.c_double), ("omega", C.c_double),
        ("K", C.c_int32),
        ("cfl_phys", C.c_double), ("cfl_imp", C.c_double), ("limiter", C.c_int32),
        ("precision", C.c_int32),
        ("init_rho", C.c_double), ("init_u", C.c_double), ("init_v", C.c_double),
        ("init_T", C.c_double), ("predictor", C.c_int32), ("relax_sweeps", C.c_int32),
        ("cfl_start", C.c_double), ("cfl_growth", C.c_double),
        ("nnodes", C.c_int32), ("ncells", C.c_int32),
        ("cell_nodes", C.POINTER(C.c_int32)), ("side_tag", C.POINTER(C.c_int32)),
        ("sweep_order", C.c_int32), ("diverge_iters", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [("nc", C.c_int32), ("nv", C.c_int32), ("nvp", C.c_int32), ("nf", C.c_int32),
                ("nwall", C.c_int32), ("nvx", C.c_int32), ("nvy", C.c_int32),
                ("precision", C.c_int32), ("dt", C.c_double), ("M0", C.c_double),
                ("iterations", C.c_int64)]


_D = C.POINTER(C.c_double)
_P = C.c_void_p
_SIGS = {
    "idugks_describe": (C.c_int, [C.POINTER(Config), _D, _D, _D, _D, _D, C.POINTER(C.c_int32),
                                  _D, _D, _D, _D, _D]),
    "idugks_workspace_size": (C.c_int, [C.POINTER(Config), C.POINTER(C.c_size_t)]),
    "idugks_init": (C.c_int, [C.POINTER(Config), _P, C.c_size_t, _P, C.POINTER(_P)]),
    "idugks_init_noalloc": (C.c_int, [C.POINTER(Config), _P, C.POINTER(_P)]),
    "idugks_get_info": (C.c_int, [_P, C.POINTER(Info)]),
    "idugks_velocities": (C.c_int, [_P, _D, _D, _D]),
    "idugks_step": (C.c_int, [_P, C.c_int32, C.c_int32, _D]),
    "idugks_solve": (C.c_int, [_P, C.c_double, C.c_int32, C.POINTER(C.c_int32), _D]),
    "idugks_residual": (C.c_int, [_P, _D]),
    "idugks_moments": (C.c_int, [_P, _P, C.c_int32]),
    "idugks_flux": (C.c_int, [_P, _P, C.c_int32]),
    "idugks_macro_residual": (C.c_int, [_P, _P, C.c_int32]),
    "idugks_face_moments": (C.c_int, [_P, _P, _P, C.c_int32]),
    "idugks_predict": (C.c_int, [_P, _P, _P, C.c_int32]),
    "idugks_get_state": (C.c_int, [_P, _P, C.c_int32]),
    "idugks_set_state": (C.c_int, [_P, _P, C.c_int32]),
    "idugks_vjp": (C.c_int, [_P, _P, _P, _D, C.c_int32]),
    "idugks_objective": (C.c_int, [_P, C.c_int32, _D, _P, _D, C.c_int32]),
    "idugks_adjoint": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int32, _D, _D,
                                 C.POINTER(C.c_int32), _D, _P, C.c_int32]),
    "idugks_num_kernels": (C.c_int32, []),
    "idugks_kernel_name": (C.c_char_p, [C.c_int32]),
    "idugks_profile": (C.c_int, [_P, C.c_int32, C.c_int32, _D, C.POINTER(C.c_int64)]),
    "idugks_profile_mask": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_uint32, _D, C.POINTER(C.c_int64)]),
    "idugks_last_error": (C.c_char_p, []),
    "idugks_destroy": (None, [_P]),
}
EXPORTED = tuple(_SIGS)
NOALLOC_MAX_BYTES = 64 << 20   # IDUGKS_NOALLOC_MAX_BYTES
_lib = None


def library_path():
    return _LIB_PATH


def load_library():
    """Load the in-tree libidugks.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_1709_01819_amd.build` (no fallback exists)")
    # The workspace and stream come from PyTorch, so the library must bind to the HIP
    # runtime PyTorch loads (same soname).  Importing torch first makes the dynamic linker
    # resolve the library's libamdhip64.so.7 to that one; loaded the other way round, the
    # process holds two HIP runtimes and the library's one sees no device.
    import torch  # noqa: F401
    lib = C.CDLL(_LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def make_config(cfg):
    """Build the C struct from a config dict; returns (struct, keep-alive arrays).

    A "mesh" entry (xn, yn, cell_nodes [nc, 4], side_tag [nc, 4]) selects an unstructured
    mesh; "sweep_order" (SWEEPS_AUTO, SWEEPS_LEVELS, SWEEPS_HYPERPLANES) how the sweeps walk
    the cell order; "diverge_iters" the consecutive residual growths after which a solve
    stops as diverged (0: off)."""
    import numpy as np
    mesh = cfg.get("mesh")
    src = cfg if mesh is None else mesh
    xn = np.ascontiguousarray(src["xn"], dtype=np.float64)
    yn = np.ascontiguousarray(src["yn"], dtype=np.float64)
    c = Config()
    c.struct_size = C.sizeof(Config)
    keep = [xn, yn]
    if mesh is None:
        c.ni, c.nj = cfg["ni"], cfg["nj"]
    else:
        cn = np.ascontiguousarray(mesh["cell_nodes"], dtype=np.int32)
        tg = np.ascontiguousarray(mesh["side_tag"], dtype=np.int32)
        if cn.ndim != 2 or cn.shape[1] != 4 or tg.shape != cn.shape:
            raise ValueError("cell_nodes and side_tag must both be [ncells, 4]")
        c.ni, c.nj = 0, 0
        c.nnodes, c.ncells = len(xn), cn.shape[0]
        c.cell_nodes = cn.ctypes.data_as(C.POINTER(C.c_int32))
        c.side_tag = tg.ctypes.data_as(C.POINTER(C.c_int32))
        keep += [cn, tg]
    c.sweep_order = int(cfg.get("sweep_order", SWEEPS_AUTO))
    c.diverge_iters = int(cfg.get("diverge_iters", 0))
    c.xn, c.yn = xn.ctypes.data_as(_D), yn.ctypes.data_as(_D)
    for s in range(4):
        c.bc[s] = cfg["bc"][s]
        c.wall_u[s] = cfg["wall_u"][s]
        c.wall_v[s] = cfg["wall_v"][s]
        c.wall_T[s] = cfg["wall_T"][s]
    for k in ("far_rho", "far_u", "far_v", "far_T", "quad", "nvx", "nvy", "vmax", "model", "Kn",
              "Pr", "omega", "K", "cfl_phys", "cfl_imp", "limiter", "precision", "init_rho",
              "init_u", "init_v", "init_T"):
        setattr(c, k, cfg[k])
    c.predictor = cfg.get("predictor", 0)
    c.relax_sweeps = cfg.get("relax_sweeps", 0)
    c.cfl_start = cfg.get("cfl_start", 0.0)
    c.cfl_growth = cfg.get("cfl_growth", 1.0)
    return c, tuple(keep)


def describe(cfg):
    """Host-only description of a configuration (velocity set, dt, geometry); no GPU needed."""
    import numpy as np
    lib = load_library()
    c, keep = make_config(cfg)
    nv = cfg["nvx"] * cfg["nvy"]
    nc = cfg["ni"] * cfg["nj"] if cfg.get("mesh") is None else len(cfg["mesh"]["cell_nodes"])
    out = {k: np.zeros(nv) for k in ("xi", "eta", "w")}
    out["dt"] = np.zeros(1)
    out["area"] = np.zeros(nc)
    out["nb"] = np.zeros(4 * nc, np.int32)
    for k in ("nx", "ny", "S", "ax", "ay"):
        out[k] = np.zeros(4 * nc)
    d = lambda k: out[k].ctypes.data_as(_D)
    rc = lib.idugks_describe(C.byref(c), d("xi"), d("eta"), d("w"), d("dt"), d("area"),
                             out["nb"].ctypes.data_as(C.POINTER(C.c_int32)), d("nx"), d("ny"),
                             d("S"), d("ax"), d("ay"))
    if rc:
        raise IdugksError(rc, lib.idugks_last_error().decode())
    for k in ("nb", "nx", "ny", "S", "ax", "ay"):
        out[k] = out[k].reshape(nc, 4)
    out["dt"] = float(out["dt"][0])
    return out
