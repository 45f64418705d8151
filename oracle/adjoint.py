"""Steady residual, wall objectives and their sensitivities: a plain PyTorch (CPU, float64)
reference.

TEST INFRASTRUCTURE ONLY: used by the tests and nothing else; the product path never
imports it.

Paper: Pan, Zhong & Zhuo, arXiv:1709.01819.  The steady state of both the explicit scheme
(Eq. 21) and the implicit scheme (Eq. 22-32) is the zero of the residual

    R_i(v) = M_i(v) - (2 Omega_i / (2 tau_i + dt)) (phi~_i(v) - phi_eq,i(v)),

M_i(v) = -sum_k S_k (xi.n_k) phi_k(v) the interface flux of Eq. 11-19 and 23, with the
collision term scaled by the cell area (the form that follows from Eq. 10 and Eq. 21).  This
module writes R(f; theta) out with plain tensor operations, in the paper's order: cell
moments and equilibria (Eq. 2, 4), phi-bar-plus (Eq. 10, 12), least-squares gradient (Eq. 15),
upwind reconstruction at each face back-traced by h xi (Eq. 13-14), diffuse walls with the
density of zero normal mass flux (Eq. 34), face moments and equilibria, the Eq. 18 blend and
the flux (Eq. 19).  Scope: BGK, no limiter.  The parameters are

    theta = (U_lid, T_w, Kn): tangential speed of the j+ wall, temperature of every wall
                              (a common value), Knudsen number (mu_ref = Kn / sqrt(pi)).

Objectives, from the wall-face distributions phi_k of Eq. 18 (n_k pointing out of the gas):
    J1 = sum over j+ wall faces of S_k sum_v w xi_x (xi.n_k) G_k        (lid x-momentum flux)
    J2 = sum over wall faces of S_k sum_v w (xi.n_k) (|xi - U_w|^2 G_k + H_k)/2   (heat flux)

Derivatives are those of this function, taken by torch.autograd (a library primitive).
Sensitivities of J at a steady state of a closed domain use the Lagrange form of the
constrained steady problem (R = 0 and total mass sum_i Omega_i rho_i = M0):

    A^T lam + mu l_M = dJ/df,   dJ/dtheta = dJ/dtheta|_f - lam^T dR/dtheta,

A = dR/df; l_M = Omega_i w_v on G (mass), and lam is fixed by l_L^T lam = 0 with
l_L = w_v on G, the left null vector of A (the residual conserves mass exactly).  On small
problems the bordered system is solved densely.
"""
import math

import numpy as np
import torch

from .oracle import Oracle

BC_WALL, BC_FARFIELD, BC_PERIODIC = 0, 1, 2
F_INTERIOR, F_SELF, F_WALL, F_FAR = 0, 1, 2, 3
LID_SIDE = 3


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


class SteadyResidual:
    """R(f; theta) of one configuration (a workload dict; geometry and velocities come from
    the C oracle, which is pinned separately)."""

    def __init__(self, cfg):
        if cfg["model"] != 0 or cfg["limiter"] != 0:
            raise ValueError("the sensitivity reference covers BGK without limiter")
        self.cfg = cfg
        o = Oracle(cfg)
        self.nc, self.nv = o.nc, o.nv
        xi, eta, w = o.velocities()
        self.xi, self.eta, self.w = _t(xi), _t(eta), _t(w)
        area, _, _ = o.cells()
        self.area = _t(area)
        sd = o.cell_sides()
        self.nb = torch.as_tensor(sd["nb"], dtype=torch.long)
        for k in ("nx", "ny", "S", "dx", "dy", "ax", "ay"):
            setattr(self, "s_" + k, _t(sd[k]))
        self.dt = o.dt
        self.h = 0.5 * self.dt
        self.K = cfg["K"]
        self.omega = cfg["omega"]
        self.closed = all(b != BC_FARFIELD for b in cfg["bc"])
        self._faces(cfg)
        self.theta0 = torch.tensor([cfg["wall_u"][LID_SIDE], self._common_wall_T(cfg), cfg["Kn"]],
                                   dtype=torch.float64)

    @staticmethod
    def _common_wall_T(cfg):
        Ts = {cfg["wall_T"][s] for s in range(4) if cfg["bc"][s] == BC_WALL}
        if len(Ts) > 1:
            raise ValueError("walls must share one temperature")
        return Ts.pop() if Ts else 1.0

    def _faces(self, cfg):
        """One entry per face: cells and sides of both ends, type, normal from L to R."""
        L, sL, R, sR, typ = [], [], [], [], []
        nb = self.nb.numpy()
        for c in range(self.nc):
            for s in range(4):
                j = nb[c, s]
                if j >= 0:
                    if s in (1, 3):  # each interior / periodic face once, from its "+" side
                        L.append(c); sL.append(s); R.append(j); sR.append(s ^ 1)
                        typ.append(F_SELF if j == c else F_INTERIOR)
                else:
                    L.append(c); sL.append(s); R.append(-1); sR.append(s)
                    typ.append(F_WALL if cfg["bc"][s] == BC_WALL else F_FAR)
        self.fL = torch.tensor(L)
        self.fsL = torch.tensor(sL)
        self.fR = torch.tensor(R)
        self.fsR = torch.tensor(sR)
        self.ftype = torch.tensor(typ)
        self.fnx = self.s_nx[self.fL, self.fsL]
        self.fny = self.s_ny[self.fL, self.fsL]
        self.fS = self.s_S[self.fL, self.fsL]
        un = self.xi[None, :] * self.fnx[:, None] + self.eta[None, :] * self.fny[:, None]
        tie = un.abs() <= 1e-12 * (self.xi.abs() + self.eta.abs())[None, :]
        self.fun = torch.where(tie, torch.zeros_like(un), un)   # normal speed, ties exactly 0

    # ---- gas model (Eq. 2, 4; discrete-conservation correction) -------------------------
    def rt_of(self, W):
        U, V = W[..., 1] / W[..., 0], W[..., 2] / W[..., 0]
        return (2.0 * W[..., 3] / W[..., 0] - U * U - V * V) / (self.K + 2)

    def equilibrium(self, W):
        """Conservative Maxwellian pair (G, H) [..., nv] with the moments W [..., 4]."""
        rho = W[..., 0:1]
        U, V = W[..., 1:2] / rho, W[..., 2:3] / rho
        RT = self.rt_of(W)[..., None]
        lam = 0.5 / RT
        cx, cy = self.xi - U, self.eta - V
        GM = rho * lam / math.pi * torch.exp(-lam * (cx * cx + cy * cy))
        psi = torch.stack([torch.ones_like(cx), self.xi.expand_as(cx), self.eta.expand_as(cx),
                           0.5 * (self.xi * self.xi + self.eta * self.eta) + 0.5 * self.K * RT], -1)
        wG = self.w * GM
        A = torch.einsum("...v,...va,...vb->...ab", wG, psi, psi)
        m0 = torch.einsum("...v,...va->...a", wG, psi)
        beta = torch.linalg.solve(A, (W - m0)[..., None])[..., 0]
        G = GM * (1.0 + torch.einsum("...va,...a->...v", psi, beta))
        return G, self.K * RT * G

    def moments(self, G, H):
        x, y, w = self.xi, self.eta, self.w
        return torch.stack([(w * G).sum(-1), (w * x * G).sum(-1), (w * y * G).sum(-1),
                            0.5 * (w * ((x * x + y * y) * G + H)).sum(-1)], -1)

    def tau(self, W, Kn):
        RT = self.rt_of(W)
        return Kn / math.sqrt(math.pi) * (2.0 * RT) ** self.omega / (W[..., 0] * RT)

    def wall_maxwellian(self, s, theta):
        """Conservative Maxwellian of side s at unit density (Section 2.3) and K RT_w."""
        u = theta[0] if s == LID_SIDE else torch.tensor(self.cfg["wall_u"][s], dtype=torch.float64)
        v = torch.tensor(self.cfg["wall_v"][s], dtype=torch.float64)
        T = theta[1]
        RT = 0.5 * T
        W = torch.stack([torch.ones((), dtype=torch.float64), u, v,
                         0.5 * (u * u + v * v) + 0.5 * (self.K + 2) * RT])
        g, _ = self.equilibrium(W)
        return g, self.K * RT

    # ---- the residual -----------------------------------------------------------------
    def evaluate(self, f, theta):
        """Residual R [2, nc, nv] and the face distributions phi_k [2, nf, nv]."""
        G, H = f[0], f[1]
        Kn = theta[2]
        W = self.moments(G, H)
        EG, EH = self.equilibrium(W)
        tau = self.tau(W, Kn)[:, None]
        a = (2.0 * tau - self.h) / (2.0 * tau + self.dt)
        b = 3.0 * self.h / (2.0 * tau + self.dt)
        bp = torch.stack([a * G + b * EG, a * H + b * EH])          # phi-bar-plus
        # least-squares gradient (Eq. 15) over the interior and periodic neighbours
        nb = self.nb.clamp(min=0)
        diff = bp[:, nb, :] - bp[:, :, None, :]                       # [2, nc, 4, nv]
        mask = (self.nb >= 0).to(torch.float64)[None, :, :, None]
        sx = (self.s_ax[None, :, :, None] * mask * diff).sum(2)
        sy = (self.s_ay[None, :, :, None] * mask * diff).sum(2)
        # upwind reconstruction at the faces (Eq. 13-14)
        un = self.fun
        upL = (un > 0) | (self.ftype != F_INTERIOR)[:, None]
        u = torch.where(upL, self.fL[:, None], self.fR.clamp(min=0)[:, None])
        us = torch.where(upL, self.fsL[:, None], self.fsR[:, None])
        rx = self.s_dx[u, us] - self.h * self.xi
        ry = self.s_dy[u, us] - self.h * self.eta
        vv = torch.arange(self.nv)[None, :]
        fb = bp[:, u, vv] + sx[:, u, vv] * rx + sy[:, u, vv] * ry   # [2, nf, nv]
        # diffuse walls (Eq. 34) and the free stream
        fbG, fbH = fb[0], fb[1]
        wall_rows = torch.nonzero(self.ftype == F_WALL)[:, 0]
        far_rows = torch.nonzero(self.ftype == F_FAR)[:, 0]
        fbG = fbG.clone()
        fbH = fbH.clone()
        if len(wall_rows):
            side = self.fsL[wall_rows]
            gws, krts = {}, {}
            for s in sorted(set(side.tolist())):
                gws[s], krts[s] = self.wall_maxwellian(s, theta)
            g = torch.stack([gws[s] for s in side.tolist()])
            krt = torch.stack([krts[s] for s in side.tolist()])[:, None]
            unw = un[wall_rows]
            num = (self.w * torch.clamp(unw, min=0) * fbG[wall_rows]).sum(-1)
            den = (self.w * torch.clamp(unw, max=0) * g).sum(-1)
            rho_w = (-num / den)[:, None]
            inc = unw <= 0
            fbG[wall_rows] = torch.where(inc, rho_w * g, fbG[wall_rows])
            fbH[wall_rows] = torch.where(inc, rho_w * krt * g, fbH[wall_rows])
        if len(far_rows):
            Wi = torch.tensor([self.cfg["far_rho"], self.cfg["far_rho"] * self.cfg["far_u"],
                               self.cfg["far_rho"] * self.cfg["far_v"], 0.0], dtype=torch.float64)
            Wi[3] = 0.5 * self.cfg["far_rho"] * (self.cfg["far_u"] ** 2 + self.cfg["far_v"] ** 2
                                                 + (self.K + 2) * 0.5 * self.cfg["far_T"])
            gi, hi = self.equilibrium(Wi)
            inc = un[far_rows] < 0
            fbG[far_rows] = torch.where(inc, gi, fbG[far_rows])
            fbH[far_rows] = torch.where(inc, hi, fbH[far_rows])
        # face records and the Eq. 18 blend
        Wk = self.moments(fbG, fbH)
        Wk = torch.where((self.ftype == F_SELF)[:, None], W[self.fL], Wk)   # unused, kept finite
        EkG, EkH = self.equilibrium(Wk)
        t2 = 2.0 * self.tau(Wk, Kn)[:, None]
        phG = (t2 * fbG + self.h * EkG) / (t2 + self.h)
        phH = (t2 * fbH + self.h * EkH) / (t2 + self.h)
        live = (self.ftype != F_SELF).to(torch.float64)[:, None]
        FG = live * self.fS[:, None] * un * phG
        FH = live * self.fS[:, None] * un * phH
        # M_i = -sum_k S (xi.n_out) phi_k (Eq. 23): n points out of L and into R
        M = torch.zeros(2, self.nc, self.nv, dtype=torch.float64)
        F = torch.stack([FG, FH])
        M = M.index_add(1, self.fL, -F)
        inner = torch.nonzero(self.fR >= 0)[:, 0]
        M = M.index_add(1, self.fR[inner], F[:, inner])
        c = 2.0 * self.area[:, None] / (2.0 * tau + self.dt)
        R = M - c[None] * (f - torch.stack([EG, EH]))
        return R, torch.stack([phG, phH]), M

    def residual(self, f, theta=None):
        return self.evaluate(f, self.theta0 if theta is None else theta)[0]

    # ---- objectives ------------------------------------------------------------------
    def objective(self, which, f, theta=None):
        theta = self.theta0 if theta is None else theta
        _, ph, _ = self.evaluate(f, theta)
        walls = torch.nonzero(self.ftype == F_WALL)[:, 0]
        un = self.fun[walls]
        S = self.fS[walls][:, None]
        side = self.fsL[walls]
        if which == 0:
            lid = side == LID_SIDE
            return (S[lid] * self.w * self.xi * un[lid] * ph[0, walls][lid]).sum()
        uw = torch.stack([theta[0] if s == LID_SIDE else torch.tensor(self.cfg["wall_u"][s], dtype=torch.float64)
                          for s in side.tolist()])[:, None]
        vw = torch.tensor([self.cfg["wall_v"][s] for s in side.tolist()], dtype=torch.float64)[:, None]
        c2 = (self.xi - uw) ** 2 + (self.eta - vw) ** 2
        return (S * self.w * un * 0.5 * (c2 * ph[0, walls] + ph[1, walls])).sum()

    # ---- derivatives -------------------------------------------------------------------
    def vjp(self, f, lam, theta=None):
        """(lam^T dR/df, lam^T dR/dtheta) at f."""
        theta = (self.theta0 if theta is None else theta).clone().requires_grad_(True)
        f = torch.as_tensor(f, dtype=torch.float64).clone().requires_grad_(True)
        R = self.residual(f, theta)
        gf, gt = torch.autograd.grad(R, (f, theta), torch.as_tensor(lam, dtype=torch.float64))
        return gf, gt

    def objective_grad(self, which, f, theta=None):
        """(J, dJ/df, dJ/dtheta at fixed f)."""
        theta = (self.theta0 if theta is None else theta).clone().requires_grad_(True)
        f = torch.as_tensor(f, dtype=torch.float64).clone().requires_grad_(True)
        J = self.objective(which, f, theta)
        gf, gt = torch.autograd.grad(J, (f, theta))
        return J.item(), gf, gt

    def jacobian(self, f, theta=None):
        """Dense dR/df [n, n] (small problems only)."""
        theta = self.theta0 if theta is None else theta
        f = torch.as_tensor(f, dtype=torch.float64)
        n = f.numel()
        Jm = torch.autograd.functional.jacobian(lambda x: self.residual(x.reshape(f.shape), theta).reshape(-1),
                                                f.reshape(-1), vectorize=True)
        return Jm.reshape(n, n)

    def mass_vectors(self):
        """l_M (total mass: Omega_i w_v on G) and l_L (left null vector: w_v on G)."""
        lM = torch.zeros(2, self.nc, self.nv, dtype=torch.float64)
        lL = torch.zeros_like(lM)
        lM[0] = self.area[:, None] * self.w[None, :]
        lL[0] = self.w[None, :].expand(self.nc, -1)
        return lM, lL

    def adjoint_dense(self, which, f, theta=None):
        """Steady sensitivity by a dense solve of the bordered adjoint system (closed
        domains).  Returns (J, dJ/dtheta, lam, mu)."""
        theta = self.theta0 if theta is None else theta
        f = torch.as_tensor(f, dtype=torch.float64)
        J, gJ, tJ = self.objective_grad(which, f, theta)
        A = self.jacobian(f, theta).numpy()
        n = A.shape[0]
        lM, lL = (v.reshape(-1).numpy() for v in self.mass_vectors())
        B = np.zeros((n + 1, n + 1))
        B[:n, :n] = A.T
        B[:n, n] = lM
        B[n, :n] = lL
        rhs = np.concatenate([gJ.reshape(-1).numpy(), [0.0]])
        sol = np.linalg.solve(B, rhs)
        lam = torch.as_tensor(sol[:n]).reshape(f.shape)
        _, tR = self.vjp(f, lam, theta)
        return J, (tJ - tR).numpy(), lam, sol[n]
