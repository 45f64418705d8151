"""Pins of the sensitivity reference (oracle/adjoint.py).

The PyTorch residual is checked against the C oracle's flux and explicit step; its
derivatives against central differences of the residual; the steady sensitivities against
central differences of fully converged C-oracle solves (the definition of dJ/dtheta)."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Oracle
from oracle.adjoint import SteadyResidual

SMALL = {
    "cavity_tanh": lambda: wl.shrink(wl.case("cavity_kn1"), 5, 4, 6),
    "couette": lambda: wl.shrink(wl.case("couette"), nj=8, nv=6),
    "box": lambda: wl.periodic_box(n=4, nv=6),
    "cavity_nc": lambda: wl.shrink(wl.cavity(n=6, nv=9, quad=wl.NEWTON_COTES, vmax=4.0, Kn=0.5), 5, 6, 9),
}


def _perturbed(cfg, seed):
    o = Oracle(cfg)
    f = o.get_state() * wl.perturbation((2, o.nc, o.nv), seed)
    o.set_state(f)
    return o, f


@pytest.mark.parametrize("name", list(SMALL))
def test_residual_matches_c_oracle(name):
    cfg = SMALL[name]()
    o, f = _perturbed(cfg, 11)
    M = o.flux()
    sr = SteadyResidual(cfg)
    R, _, Mt = sr.evaluate(torch.tensor(f), sr.theta0)
    assert np.abs(Mt.numpy() - M).max() <= 1e-13 * np.abs(M).max()
    # the residual is the explicit update scaled by Omega / dt (Eq. 21)
    o.explicit_step(1)
    area, _, _ = o.cells()
    Rc = (o.get_state() - f) * area[None, :, None] / o.dt
    assert np.abs(R.numpy() - Rc).max() <= 1e-12 * np.abs(Rc).max()


@pytest.mark.parametrize("name", ["cavity_tanh", "couette", "cavity_nc"])
def test_vjp_matches_central_differences(name):
    cfg = SMALL[name]()
    _, f = _perturbed(cfg, 12)
    sr = SteadyResidual(cfg)
    f = torch.tensor(f)
    rng = np.random.default_rng(5)
    lam = torch.tensor(rng.standard_normal(f.shape))
    d = torch.tensor(rng.standard_normal(f.shape)) * f
    gf, gt = sr.vjp(f, lam)
    eps = 1e-6
    fd = (lam * (sr.residual(f + eps * d) - sr.residual(f - eps * d))).sum().item() / (2 * eps)
    assert abs(fd - (gf * d).sum().item()) <= 1e-7 * abs(fd)
    for m in range(3):
        e = torch.zeros(3, dtype=torch.float64)
        e[m] = 1e-6
        fdt = (lam * (sr.residual(f, sr.theta0 + e) - sr.residual(f, sr.theta0 - e))).sum().item() / 2e-6
        assert abs(fdt - gt[m].item()) <= 1e-6 * max(abs(fdt), 1e-3 * np.abs(gt.numpy()).max())


def test_residual_conserves_mass_exactly():
    """w on G is a left null vector of dR/df and of dR/dtheta (walls are impermeable)."""
    cfg = SMALL["cavity_tanh"]()
    _, f = _perturbed(cfg, 13)
    sr = SteadyResidual(cfg)
    f = torch.tensor(f)
    _, lL = sr.mass_vectors()
    gf, gt = sr.vjp(f, lL)
    scale = sr.vjp(f, torch.ones_like(f))[0].abs().max().item()
    assert gf.abs().max().item() <= 1e-12 * scale
    assert np.abs(gt.numpy()).max() <= 1e-12 * scale


def test_objectives_vanish_at_rest():
    cfg = SMALL["cavity_tanh"]()
    cfg["wall_u"] = [0.0] * 4
    sr = SteadyResidual(cfg)
    f = torch.tensor(Oracle(cfg).get_state())
    assert abs(sr.objective(0, f).item()) <= 1e-15
    assert abs(sr.objective(1, f).item()) <= 1e-15


def _cfg_at(base, th):
    c = dict(base)
    c["wall_u"], c["wall_T"] = list(base["wall_u"]), list(base["wall_T"])
    c["wall_u"][3] = th[0]
    for s in range(4):
        if c["bc"][s] == wl.BC_WALL:
            c["wall_T"][s] = th[1]
    c["Kn"] = th[2]
    return c


def _steady(cfg):
    o = Oracle(cfg)
    it, res, ok = o.solve(1e-15, 20000)
    assert ok, (it, res)
    return torch.tensor(o.get_state())


@pytest.mark.parametrize("which", [0, 1])
def test_steady_sensitivity_matches_converged_differences(which):
    base = wl.shrink(wl.case("cavity_kn1"), 4, 4, 6)
    sr = SteadyResidual(base)
    f = _steady(base)
    J, dJ, lam, _ = sr.adjoint_dense(which, f)
    th0 = sr.theta0.numpy()
    for m in range(3):
        h = 1e-5 * max(1.0, abs(th0[m]))
        vals = []
        for sgn in (1, -1):
            th = th0.copy()
            th[m] += sgn * h
            c = _cfg_at(base, th)
            vals.append(SteadyResidual(c).objective(which, _steady(c)).item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - dJ[m]) <= 1e-8 * np.abs(dJ).max(), (m, fd, dJ[m])
