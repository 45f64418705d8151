"""Python front end of the C ABI: workspace and stream from PyTorch, everything else in HIP."""
import ctypes as C

import numpy as np

from .abi import IMPLICIT, IdugksError, Info, load_library, make_config

_D = C.POINTER(C.c_double)


def _dp(a):
    return a.ctypes.data_as(_D)


class Solver:
    """One IDUGKS problem on one GPU (see include/idugks.h for the semantics of each call)."""

    def __init__(self, cfg, device="cuda:0", stream=None, static_workspace=False):
        """static_workspace: take the workspace from the library's static scratch array
        (idugks_init_noalloc; nothing is allocated) instead of a torch buffer."""
        import torch
        self._lib = load_library()
        self.cfg = cfg
        self.device = torch.device(device)
        c, keep = make_config(cfg)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                self._check(self._lib.idugks_init_noalloc(C.byref(c), C.c_void_p(self.stream.cuda_stream),
                                                          C.byref(h)))
        else:
            nbytes = C.c_size_t(0)
            self._check(self._lib.idugks_workspace_size(C.byref(c), C.byref(nbytes)))
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self._check(self._lib.idugks_init(C.byref(c), C.c_void_p(self.workspace.data_ptr()),
                                              nbytes.value, C.c_void_p(self.stream.cuda_stream),
                                              C.byref(h)))
        del keep
        self._h = h
        info = self.info()
        self.nc, self.nv, self.nf = info.nc, info.nv, info.nf
        self.dt = info.dt

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.idugks_destroy(h)
            self._h = None

    def close(self):
        self.__del__()

    def _check(self, rc):
        if rc:
            raise IdugksError(rc, self._lib.idugks_last_error().decode())

    def info(self):
        i = Info()
        self._check(self._lib.idugks_get_info(self._h, C.byref(i)))
        return i

    def velocities(self):
        xi, eta, w = (np.zeros(self.nv) for _ in range(3))
        self._check(self._lib.idugks_velocities(self._h, _dp(xi), _dp(eta), _dp(w)))
        return xi, eta, w

    def step(self, mode=IMPLICIT, n=1):
        r = C.c_double(0.0)
        self._check(self._lib.idugks_step(self._h, mode, n, C.byref(r)))
        return r.value

    def solve(self, tol, max_iter):
        it = C.c_int32(0)
        r = C.c_double(0.0)
        rc = self._lib.idugks_solve(self._h, tol, max_iter, C.byref(it), C.byref(r))
        if rc not in (0, 5):
            self._check(rc)
        return it.value, r.value, rc == 0

    def residual(self):
        out = np.zeros(4)
        self._check(self._lib.idugks_residual(self._h, _dp(out)))
        return out

    def moments(self):
        out = np.zeros((self.nc, 8))
        self._check(self._lib.idugks_moments(self._h, C.c_void_p(out.ctypes.data), 1))
        return out

    def flux(self):
        M = np.zeros((2, self.nc, self.nv))
        self._check(self._lib.idugks_flux(self._h, C.c_void_p(M.ctypes.data), 1))
        return M

    def face_moments(self):
        Wf = np.zeros((self.nf, 4))
        rw = np.zeros(self.nf)
        self._check(self._lib.idugks_face_moments(self._h, C.c_void_p(Wf.ctypes.data),
                                                  C.c_void_p(rw.ctypes.data), 1))
        return Wf, rw

    def macro_residual(self):
        MW = np.zeros((self.nc, 4))
        self._check(self._lib.idugks_macro_residual(self._h, C.c_void_p(MW.ctypes.data), 1))
        return MW

    def predict(self):
        Ws = np.zeros((self.nc, 4))
        dti = np.zeros(self.nc)
        self._check(self._lib.idugks_predict(self._h, C.c_void_p(Ws.ctypes.data),
                                             C.c_void_p(dti.ctypes.data), 1))
        return Ws, dti

    def get_state(self):
        f = np.zeros((2, self.nc, self.nv))
        self._check(self._lib.idugks_get_state(self._h, C.c_void_p(f.ctypes.data), 1))
        return f

    def set_state(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(2, self.nc, self.nv)
        self._check(self._lib.idugks_set_state(self._h, C.c_void_p(f.ctypes.data), 1))

    # sensitivities (BGK, no limiter, FP64): theta = (lid speed, wall temperature, Kn)
    def vjp(self, lam):
        """(lam^T dR/df, lam^T dR/dtheta) at the current state; lam [2, nc, nv]."""
        lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(2, self.nc, self.nv)
        fb = np.zeros((2, self.nc, self.nv))
        tb = np.zeros(3)
        self._check(self._lib.idugks_vjp(self._h, C.c_void_p(lam.ctypes.data),
                                         C.c_void_p(fb.ctypes.data), _dp(tb), 1))
        return fb, tb

    def objective(self, which):
        """(J, dJ/df, dJ/dtheta at fixed f); which 0: lid x-momentum flux, 1: wall heat flux."""
        J = np.zeros(1)
        g = np.zeros((2, self.nc, self.nv))
        t = np.zeros(3)
        self._check(self._lib.idugks_objective(self._h, which, _dp(J), C.c_void_p(g.ctypes.data),
                                               _dp(t), 1))
        return float(J[0]), g, t

    def adjoint(self, which, tol=1e-10, max_iter=10000, want_lam=False):
        """Steady sensitivity at the current (converged) state:
        (J, dJ/dtheta, iterations, last relative change, multipliers or None)."""
        J = np.zeros(1)
        grad = np.zeros(3)
        it = C.c_int32(0)
        res = np.zeros(1)
        lam = np.zeros((2, self.nc, self.nv)) if want_lam else None
        self._check(self._lib.idugks_adjoint(self._h, which, tol, max_iter, _dp(J), _dp(grad),
                                             C.byref(it), _dp(res),
                                             C.c_void_p(lam.ctypes.data) if want_lam else None, 1))
        return float(J[0]), grad, it.value, float(res[0]), lam

    def kernel_names(self):
        n = self._lib.idugks_num_kernels()
        return [self._lib.idugks_kernel_name(k).decode() for k in range(n)]

    def profile(self, mode=IMPLICIT, n=1, kernels=None):
        """Per-kernel HIP-event milliseconds over n steps: {name: (ms_total, launches)}.

        kernels: names of the kernels to bracket with events (default all); the others run
        without events and report (0.0, 0)."""
        names = self.kernel_names()
        nk = len(names)
        mask = 0xFFFFFFFF if kernels is None else sum(1 << names.index(k) for k in kernels)
        ms = np.zeros(nk)
        cnt = np.zeros(nk, dtype=np.int64)
        self._check(self._lib.idugks_profile_mask(self._h, mode, n, mask, _dp(ms),
                                                  cnt.ctypes.data_as(C.POINTER(C.c_int64))))
        return {name: (float(ms[k]), int(cnt[k])) for k, name in enumerate(names)}
