"""ctypes binding of the C oracle (``idugks_oracle.c``).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the benchmark).
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "idugks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_sanitized(out_path):
    """The oracle compiled with AddressSanitizer and UndefinedBehaviorSanitizer (host code,
    serial: no OpenMP; the first error aborts), for a test that loads it in a child process
    through IDUGKS_ORACLE_LIB with the ASan runtime preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", out_path, _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    return out_path


def build(force=True):
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP over independent loops)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrcMesh(C.Structure):
    _fields_ = [
        ("nnodes", C.c_int32), ("xn", C.POINTER(C.c_double)), ("yn", C.POINTER(C.c_double)),
        ("ncells", C.c_int32), ("cell_nodes", C.POINTER(C.c_int32)),
        ("side_tag", C.POINTER(C.c_int32)),
    ]


class OrcConfig(C.Structure):
    _fields_ = [
        ("ni", C.c_int32), ("nj", C.c_int32),
        ("xn", C.POINTER(C.c_double)), ("yn", C.POINTER(C.c_double)),
        ("bc", C.c_int32 * 4),
        ("wall_u", C.c_double * 4), ("wall_v", C.c_double * 4), ("wall_T", C.c_double * 4),
        ("far_rho", C.c_double), ("far_u", C.c_double), ("far_v", C.c_double), ("far_T", C.c_double),
        ("quad", C.c_int32), ("nvx", C.c_int32), ("nvy", C.c_int32), ("vmax", C.c_double),
        ("model", C.c_int32), ("Kn", C.c_double), ("Pr", C.c_double), ("omega", C.c_double),
        ("K", C.c_int32),
        ("cfl_phys", C.c_double), ("cfl_imp", C.c_double), ("limiter", C.c_int32),
        ("init_rho", C.c_double), ("init_u", C.c_double), ("init_v", C.c_double),
        ("init_T", C.c_double), ("predictor", C.c_int32), ("relax_sweeps", C.c_int32),
        ("cfl_start", C.c_double), ("cfl_growth", C.c_double),
    ]


_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_P = C.c_void_p


def load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("IDUGKS_ORACLE_LIB")  # another build of the same source
    if path is None:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
    lib = C.CDLL(path)
    sig = {
        "orc_create": (C.c_int, [C.POINTER(OrcConfig), C.POINTER(_P)]),
        "orc_create_mesh": (C.c_int, [C.POINTER(OrcConfig), C.POINTER(OrcMesh), C.POINTER(_P)]),
        "orc_destroy": (None, [_P]),
        "orc_last_error": (C.c_char_p, []),
        "orc_sizes": (None, [_P, _I]),
        "orc_dt": (C.c_double, [_P]),
        "orc_quadrature_1d": (C.c_int, [C.c_int32, C.c_int32, C.c_double, _D, _D]),
        "orc_velocities": (None, [_P, _D, _D, _D]),
        "orc_cells": (None, [_P, _D, _D, _D]),
        "orc_cell_sides": (None, [_P, _I, _D, _D, _D, _D, _D, _D, _D]),
        "orc_get_state": (None, [_P, _D]),
        "orc_set_state": (None, [_P, _D]),
        "orc_equilibrium": (None, [_P, _D, _D, _D, _D]),
        "orc_moments_of": (None, [_P, _D, _D, _D]),
        "orc_heat_flux_of": (None, [_P, _D, _D, _D]),
        "orc_moments": (None, [_P, _D]),
        "orc_barplus": (None, [_P, _D]),
        "orc_flux": (C.c_int, [_P, _D]),
        "orc_face_moments": (C.c_int, [_P, _D, _D]),
        "orc_macro_residual": (C.c_int, [_P, _D]),
        "orc_predict": (C.c_int, [_P, _D, _D]),
        "orc_micro_operator": (C.c_int, [_P, C.c_int32, _D, _D]),
        "orc_micro_sweep": (C.c_int, [_P, C.c_int32, _D, _D]),
        "orc_explicit_step": (C.c_int, [_P, C.c_int32, _D]),
        "orc_implicit_step": (C.c_int, [_P, C.c_int32, _D]),
        "orc_solve": (C.c_int, [_P, C.c_double, C.c_int32, _I, _D]),
        "orc_residual": (C.c_int, [_P, _D]),
        "orc_gradients": (C.c_int, [_P, _D, _D]),
        "orc_lsq_gradient": (C.c_int, [_P, _D, C.c_int32, _D, _D]),
        "orc_faces": (None, [_P, _I, _I, _I, _I, _D, _D, _D, _D, _D]),
        "orc_face_flux": (C.c_int, [_P, _D]),
        "orc_macro_sweep_rhs": (C.c_int, [_P, _D, _D]),
        "orc_implicit_detail": (C.c_int, [_P, _D, _D, _D]),
        "orc_set_first_order": (None, [_P, C.c_int32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(_D)


def quadrature_1d(quad, n, vmax=0.0):
    lib = load()
    x = np.zeros(n)
    w = np.zeros(n)
    rc = lib.orc_quadrature_1d(quad, n, vmax, _dp(x), _dp(w))
    if rc:
        raise ValueError(lib.orc_last_error().decode())
    return x, w


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Oracle:
    """One problem instance of the CPU reference."""

    def __init__(self, cfg):
        """cfg: a workload dict; with a "mesh" entry (xn, yn, cell_nodes [nc, 4], side_tag
        [nc, 4]) the problem lives on that unstructured mesh and ni, nj, xn, yn are unused."""
        lib = load()
        self._lib = lib
        mesh = cfg.get("mesh")
        c = OrcConfig()
        if mesh is None:
            self._xn = np.ascontiguousarray(cfg["xn"], dtype=np.float64)
            self._yn = np.ascontiguousarray(cfg["yn"], dtype=np.float64)
            c.ni, c.nj = cfg["ni"], cfg["nj"]
            c.xn, c.yn = _dp(self._xn), _dp(self._yn)
        else:
            self._xn = np.ascontiguousarray(mesh["xn"], dtype=np.float64)
            self._yn = np.ascontiguousarray(mesh["yn"], dtype=np.float64)
            self._cn = np.ascontiguousarray(mesh["cell_nodes"], dtype=np.int32)
            self._tag = np.ascontiguousarray(mesh["side_tag"], dtype=np.int32)
            assert self._cn.shape == self._tag.shape and self._cn.shape[1] == 4
            m = OrcMesh()
            m.nnodes, m.ncells = len(self._xn), self._cn.shape[0]
            m.xn, m.yn = _dp(self._xn), _dp(self._yn)
            m.cell_nodes = self._cn.ctypes.data_as(_I)
            m.side_tag = self._tag.ctypes.data_as(_I)
        for s in range(4):
            c.bc[s] = cfg["bc"][s]
            c.wall_u[s] = cfg["wall_u"][s]
            c.wall_v[s] = cfg["wall_v"][s]
            c.wall_T[s] = cfg["wall_T"][s]
        for k in ("far_rho", "far_u", "far_v", "far_T", "quad", "nvx", "nvy", "vmax", "model",
                  "Kn", "Pr", "omega", "K", "cfl_phys", "cfl_imp", "limiter", "init_rho",
                  "init_u", "init_v", "init_T"):
            setattr(c, k, cfg[k])
        c.predictor = cfg.get("predictor", 0)
        c.relax_sweeps = cfg.get("relax_sweeps", 0)
        c.cfl_start = cfg.get("cfl_start", 0.0)
        c.cfl_growth = cfg.get("cfl_growth", 1.0)
        h = _P()
        if mesh is None:
            rc = lib.orc_create(C.byref(c), C.byref(h))
        else:
            rc = lib.orc_create_mesh(C.byref(c), C.byref(m), C.byref(h))
        if rc:
            raise OracleError(rc, lib.orc_last_error().decode())
        self._h = h
        sz = (C.c_int32 * 4)()
        lib.orc_sizes(h, sz)
        self.nc, self.nv, self.nf, self.nwall = list(sz)
        self.ni, self.nj = (cfg["ni"], cfg["nj"]) if mesh is None else (self.nc, 1)
        self.cfg = cfg

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def _check(self, rc):
        if rc:
            raise OracleError(rc, self._lib.orc_last_error().decode())

    # geometry and velocities
    @property
    def dt(self):
        return self._lib.orc_dt(self._h)

    def velocities(self):
        xi, eta, w = np.zeros(self.nv), np.zeros(self.nv), np.zeros(self.nv)
        self._lib.orc_velocities(self._h, _dp(xi), _dp(eta), _dp(w))
        return xi, eta, w

    def cells(self):
        a, x, y = np.zeros(self.nc), np.zeros(self.nc), np.zeros(self.nc)
        self._lib.orc_cells(self._h, _dp(a), _dp(x), _dp(y))
        return a, x, y

    def cell_sides(self):
        n = 4 * self.nc
        nb = np.zeros(n, np.int32)
        arrs = [np.zeros(n) for _ in range(7)]
        self._lib.orc_cell_sides(self._h, nb.ctypes.data_as(_I), *[_dp(a) for a in arrs])
        keys = ("nx", "ny", "S", "dx", "dy", "ax", "ay")
        out = {k: a.reshape(self.nc, 4) for k, a in zip(keys, arrs)}
        out["nb"] = nb.reshape(self.nc, 4)
        return out

    # state
    def get_state(self):
        f = np.zeros((2, self.nc, self.nv))
        self._lib.orc_get_state(self._h, _dp(f))
        return f

    def set_state(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(2, self.nc, self.nv)
        self._lib.orc_set_state(self._h, _dp(f))

    # gas model
    def equilibrium(self, W, q=(0.0, 0.0)):
        W = np.ascontiguousarray(W, dtype=np.float64)
        q = np.ascontiguousarray(q, dtype=np.float64)
        G, H = np.zeros(self.nv), np.zeros(self.nv)
        self._lib.orc_equilibrium(self._h, _dp(W), _dp(q), _dp(G), _dp(H))
        return G, H

    def moments_of(self, G, H):
        G = np.ascontiguousarray(G, dtype=np.float64)
        H = np.ascontiguousarray(H, dtype=np.float64)
        W = np.zeros(4)
        self._lib.orc_moments_of(self._h, _dp(G), _dp(H), _dp(W))
        return W

    def heat_flux_of(self, G, H):
        G = np.ascontiguousarray(G, dtype=np.float64)
        H = np.ascontiguousarray(H, dtype=np.float64)
        q = np.zeros(2)
        self._lib.orc_heat_flux_of(self._h, _dp(G), _dp(H), _dp(q))
        return q

    def moments(self):
        out = np.zeros((self.nc, 8))
        self._lib.orc_moments(self._h, _dp(out))
        return out

    # the method
    def barplus(self):
        out = np.zeros((2, self.nc, self.nv))
        self._lib.orc_barplus(self._h, _dp(out))
        return out

    def flux(self):
        M = np.zeros((2, self.nc, self.nv))
        self._check(self._lib.orc_flux(self._h, _dp(M)))
        return M

    def face_moments(self):
        Wf = np.zeros((self.nf, 4))
        rw = np.zeros(self.nf)
        self._check(self._lib.orc_face_moments(self._h, _dp(Wf), _dp(rw)))
        return Wf, rw

    def macro_residual(self):
        MW = np.zeros((self.nc, 4))
        self._check(self._lib.orc_macro_residual(self._h, _dp(MW)))
        return MW

    def predict(self):
        Ws = np.zeros((self.nc, 4))
        dti = np.zeros(self.nc)
        self._check(self._lib.orc_predict(self._h, _dp(Ws), _dp(dti)))
        return Ws, dti

    def micro_operator(self, v):
        D = np.zeros(self.nc)
        Cc = np.zeros((self.nc, 4))
        self._check(self._lib.orc_micro_operator(self._h, v, _dp(D), _dp(Cc)))
        return D, Cc

    def micro_sweep(self, v, rhs):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        out = np.zeros(self.nc)
        self._check(self._lib.orc_micro_sweep(self._h, v, _dp(rhs), _dp(out)))
        return out

    def explicit_step(self, n=1):
        r = C.c_double(0.0)
        self._check(self._lib.orc_explicit_step(self._h, n, C.byref(r)))
        return r.value

    def implicit_step(self, n=1):
        r = C.c_double(0.0)
        self._check(self._lib.orc_implicit_step(self._h, n, C.byref(r)))
        return r.value

    def solve(self, tol, max_iter):
        it = C.c_int32(0)
        r = C.c_double(0.0)
        rc = self._lib.orc_solve(self._h, tol, max_iter, C.byref(it), C.byref(r))
        if rc and rc != 5:
            self._check(rc)
        return it.value, r.value, rc == 0

    def residual(self):
        out = np.zeros(4)
        self._check(self._lib.orc_residual(self._h, _dp(out)))
        return out

    # intermediate quantities (pins of individual steps)
    def gradients(self):
        sx = np.zeros((2, self.nc, self.nv))
        sy = np.zeros((2, self.nc, self.nv))
        self._check(self._lib.orc_gradients(self._h, _dp(sx), _dp(sy)))
        return sx, sy

    def lsq_gradient(self, phi, limiter):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.nc)
        gx, gy = np.zeros(self.nc), np.zeros(self.nc)
        self._check(self._lib.orc_lsq_gradient(self._h, _dp(phi), int(limiter), _dp(gx), _dp(gy)))
        return gx, gy

    def faces(self):
        ints = [np.zeros(self.nf, np.int32) for _ in range(4)]
        dbl = [np.zeros(self.nf) for _ in range(5)]
        self._lib.orc_faces(self._h, *[a.ctypes.data_as(_I) for a in ints], *[_dp(a) for a in dbl])
        keys = ("L", "R", "type", "side", "nx", "ny", "S", "mx", "my")
        return dict(zip(keys, ints + dbl))

    def face_flux(self):
        F = np.zeros((2, self.nf, self.nv))
        self._check(self._lib.orc_face_flux(self._h, _dp(F)))
        return F

    def macro_sweep_rhs(self, rhs):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64).reshape(self.nc, 4)
        dW = np.zeros((self.nc, 4))
        self._check(self._lib.orc_macro_sweep_rhs(self._h, _dp(rhs), _dp(dW)))
        return dW

    def implicit_detail(self):
        ds = np.zeros((2, self.nc, self.nv))
        dr = np.zeros(self.nf)
        r = C.c_double(0.0)
        self._check(self._lib.orc_implicit_detail(self._h, _dp(ds), _dp(dr), C.byref(r)))
        return ds, dr, r.value

    def set_first_order(self, on=True):
        """Analysis switch: reconstruction without the gradient (first-order residual)."""
        self._lib.orc_set_first_order(self._h, 1 if on else 0)
