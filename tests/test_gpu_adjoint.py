"""GPU sensitivities against the PyTorch reference (oracle/adjoint.py) through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Oracle
from oracle.adjoint import SteadyResidual

pytestmark = pytest.mark.gpu

CASES = {
    "cavity_tanh": lambda: wl.shrink(wl.case("cavity_kn1"), 5, 4, 6),
    "couette": lambda: wl.shrink(wl.case("couette"), nj=8, nv=6),
    "box": lambda: wl.periodic_box(n=4, nv=6),
    "cavity_nc": lambda: wl.shrink(wl.cavity(n=6, nv=9, quad=wl.NEWTON_COTES, vmax=4.0, Kn=0.5), 5, 6, 9),
    "cavity_ragged": lambda: wl.shrink(wl.case("cavity_kn1"), 7, 9, 11),
}


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _pair(cfg, seed, amp=0.1):
    from paper_1709_01819_amd import Solver
    o = Oracle(cfg)
    f = o.get_state() * wl.perturbation((2, o.nc, o.nv), seed, amp)
    g = Solver(cfg)
    g.set_state(f)
    return g, SteadyResidual(cfg), f


@pytest.mark.parametrize("name", list(CASES))
def test_vjp_parity(name):
    g, sr, f = _pair(CASES[name](), seed=21)
    lam = np.random.default_rng(4).standard_normal(f.shape)
    fb, tb = g.vjp(lam)
    fo, to = sr.vjp(torch.tensor(f), torch.tensor(lam))
    assert _rel(fb, fo.numpy()) <= 1e-12, _rel(fb, fo.numpy())
    assert _rel(tb, to.numpy()) <= 1e-11, (tb, to.numpy())


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("name", ["cavity_tanh", "cavity_nc", "cavity_ragged"])
def test_objective_parity(name, which):
    g, sr, f = _pair(CASES[name](), seed=22)
    J, dJ, tJ = g.objective(which)
    Jo, dJo, tJo = sr.objective_grad(which, torch.tensor(f))
    # the wall heat flux is a difference of inflow and outflow energy fluxes: the bound is
    # relative to the size of the summed terms
    scale = np.abs(dJo.numpy() * f).sum()
    assert abs(J - Jo) <= 1e-12 * scale, (J, Jo, scale)
    assert _rel(dJ, dJo.numpy()) <= 1e-12
    assert _rel(tJ, tJo.numpy()) <= 1e-11, (tJ, tJo.numpy())


def test_vjp_parity_full_size():
    """The 64x64 tanh cavity at Kn = 1 with 28x28 velocities, perturbed state."""
    g, sr, f = _pair(wl.case("cavity_kn1"), seed=23, amp=0.05)
    lam = np.random.default_rng(6).standard_normal(f.shape)
    fb, tb = g.vjp(lam)
    fo, to = sr.vjp(torch.tensor(f), torch.tensor(lam))
    assert _rel(fb, fo.numpy()) <= 1e-12, _rel(fb, fo.numpy())
    assert _rel(tb, to.numpy()) <= 1e-11, (tb, to.numpy())
    J, dJ, tJ = g.objective(1)
    Jo, dJo, tJo = sr.objective_grad(1, torch.tensor(f))
    assert abs(J - Jo) <= 1e-12 * np.abs(dJo.numpy() * f).sum()
    assert _rel(dJ, dJo.numpy()) <= 1e-12


@pytest.mark.parametrize("which", [0, 1])
def test_adjoint_matches_dense_reference(which):
    """Converged tiny cavity: the iterated adjoint equals the dense bordered solve."""
    from paper_1709_01819_amd import Solver
    cfg = wl.shrink(wl.case("cavity_kn1"), 4, 4, 6)
    g = Solver(cfg)
    it, res, ok = g.solve(1e-15, 20000)
    assert ok
    f = g.get_state()
    sr = SteadyResidual(cfg)
    Jo, dJo, lamo, _ = sr.adjoint_dense(which, torch.tensor(f))
    J, grad, its, r, lam = g.adjoint(which, 1e-13, 20000, want_lam=True)
    assert abs(J - Jo) <= 1e-12 * np.abs(sr.objective_grad(which, torch.tensor(f))[1].numpy() * f).sum()
    assert _rel(grad, dJo) <= 1e-9, (grad, dJo, its, r)
    # the multipliers are unique up to multiples of w on G
    _, lL = sr.mass_vectors()
    lL = lL.numpy()

    def proj(x):
        return x - lL * (x * lL).sum() / (lL * lL).sum()
    assert _rel(proj(lam), proj(lamo.numpy())) <= 1e-8


def test_adjoint_full_size_matches_finite_differences():
    """Lid-driven cavity, 64x64 tanh mesh, GH 28x28, BGK, Kn = 1: adjoint dJ/dtheta for both
    objectives against central differences (h = 1e-6) of converged GPU solves."""
    from paper_1709_01819_amd import Solver
    from paper_1709_01819_amd.sensitivity import config_at
    base = wl.case("cavity_kn1")
    theta0 = np.array([base["wall_u"][3], base["wall_T"][0], base["Kn"]])

    def steady(th):
        s = Solver(config_at(base, th))
        it, res, ok = s.solve(1e-14, 20000)
        assert ok, (it, res)
        return s

    s0 = steady(theta0)
    grads = {}
    for which in (0, 1):
        J, grad, its, r, _ = s0.adjoint(which, 1e-12, 50000)
        grads[which] = (J, grad)
    for m in range(3):
        h = 1e-6
        Jp, Jm = [], []
        for sgn, acc in ((1, Jp), (-1, Jm)):
            th = theta0.copy()
            th[m] += sgn * h
            s = steady(th)
            acc.extend(s.objective(w)[0] for w in (0, 1))
            del s
        for which in (0, 1):
            fd = (Jp[which] - Jm[which]) / (2 * h)
            scale = np.abs(grads[which][1]).max()
            assert abs(fd - grads[which][1][m]) <= 1e-6 * scale, (which, m, fd, grads[which][1])


def test_autograd_function_matches_adjoint():
    from paper_1709_01819_amd.sensitivity import SteadyObjective
    cfg = wl.shrink(wl.case("cavity_kn1"), 4, 4, 6)
    theta = torch.tensor([0.16, 1.0, 1.0], dtype=torch.float64, requires_grad=True)
    J = SteadyObjective.apply(theta, cfg, 1)
    (gr,) = torch.autograd.grad(J, theta)
    sr = SteadyResidual(cfg)
    o = Oracle(cfg)
    o.solve(1e-15, 20000)
    Jo, dJo, _, _ = sr.adjoint_dense(1, torch.tensor(o.get_state()))
    assert abs(J.item() - Jo) <= 1e-10 * abs(Jo)
    assert _rel(gr.numpy(), dJo) <= 1e-8
