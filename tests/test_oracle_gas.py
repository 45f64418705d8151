"""Pins of the oracle's gas model: moments (Eq. 4-5), equilibrium (Eq. 2, Eq. 20).

- conservation of the collision operator on the discrete velocity set (the
  equilibrium has exactly the conserved moments it is built from);
- the equilibrium at rest on a Gauss-Hermite grid reduces to the closed-form
  Maxwellian rho exp(-|xi|^2)/pi (that quadrature is exact for it);
- a moving, heated Maxwellian on a fine grid is barely touched by the
  discrete-conservation correction (it equals Eq. 2 reduced by Eq. 5);
- the Shakhov equilibrium carries the heat flux (1 - Pr) q (continuous identity
  of the Shakhov model) and no extra mass, momentum or energy.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import Oracle


def _tiny(quad, nv, model, vmax=0.0):
    K = 1 if model == wl.SHAKHOV else 3
    Pr = 2.0 / 3.0 if model == wl.SHAKHOV else 1.0
    return Oracle(wl.cavity(n=3, stretch=None, nv=nv, quad=quad, vmax=vmax, model=model, Pr=Pr,
                            K=K, Kn=0.1))


def _W(rho, U, V, T, K):
    RT = 0.5 * T
    return np.array([rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V + (K + 2) * RT)])


GRIDS = [(wl.GAUSS_HERMITE, 12, 0.0), (wl.GAUSS_HERMITE, 28, 0.0), (wl.NEWTON_COTES, 41, 4.0),
         (wl.NEWTON_COTES, 40, 6.0)]


@pytest.mark.parametrize("model", [wl.BGK, wl.SHAKHOV])
@pytest.mark.parametrize("quad,nv,vmax", GRIDS)
def test_collision_conserves(model, quad, nv, vmax):
    o = _tiny(quad, nv, model, vmax)
    K = o.cfg["K"]
    for seed in range(10):
        rng = np.random.default_rng(1709 + seed)
        W0 = _W(rng.uniform(0.5, 2.0), rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3),
                rng.uniform(0.6, 1.6), K)
        G0, H0 = o.equilibrium(W0)
        noise = wl.perturbation((2, o.nv), seed)
        G, H = G0 * noise[0], H0 * noise[1]
        W = o.moments_of(G, H)
        q = o.heat_flux_of(G, H)
        Ge, He = o.equilibrium(W, q)
        We = o.moments_of(Ge, He)
        scale = np.array([W[0], W[0], W[0], W[3]])
        assert np.max(np.abs(We - W) / scale) <= 1e-14


def test_equilibrium_at_rest_is_closed_form():
    o = _tiny(wl.GAUSS_HERMITE, 16, wl.BGK)
    xi, eta, w = o.velocities()
    for rho in (0.7, 1.0, 1.3):
        G, H = o.equilibrium(_W(rho, 0.0, 0.0, 1.0, 3))
        ref = rho / math.pi * np.exp(-(xi ** 2 + eta ** 2))
        assert np.max(np.abs(G - ref)) <= 1e-14 * ref.max()
        # H = K RT G with K = 3, RT = 1/2
        assert np.max(np.abs(H - 1.5 * ref)) <= 1e-14 * ref.max()


def test_moving_maxwellian_matches_eq2():
    o = _tiny(wl.GAUSS_HERMITE, 28, wl.BGK)
    xi, eta, w = o.velocities()
    rho, U, V, T = 1.1, 0.12, -0.07, 1.25
    G, H = o.equilibrium(_W(rho, U, V, T, 3))
    lam = 1.0 / T  # lambda = 1/(2RT), R = 1/2
    ref = rho * lam / math.pi * np.exp(-lam * ((xi - U) ** 2 + (eta - V) ** 2))
    assert np.max(np.abs(G - ref)) <= 1e-9 * ref.max()
    assert np.max(np.abs(H - 3 * 0.5 * T * G)) <= 1e-14 * H.max()


def test_shakhov_heat_flux_identity():
    o = _tiny(wl.GAUSS_HERMITE, 28, wl.SHAKHOV)
    Pr = 2.0 / 3.0
    cases = [(1.0, 0.01, -0.02, 1.0, (0.01, 0.02)), (1.2, 0.05, 0.03, 1.1, (-0.02, 0.01)),
             (0.9, 0.0, 0.0, 1.0, (0.1, 0.0)), (1.0, -0.04, 0.02, 0.9, (0.0, -0.05))]
    for rho, U, V, T, q in cases:
        W = _W(rho, U, V, T, 1)
        G, H = o.equilibrium(W, q)
        qq = o.heat_flux_of(G, H)
        q = np.array(q)
        assert np.max(np.abs(qq - (1 - Pr) * q)) <= 1e-12 * np.abs(q).max()
        assert np.max(np.abs(o.moments_of(G, H) - W)) <= 1e-14 * W[3]
    # BGK equilibria carry no heat flux
    G, H = o.equilibrium(_W(1.0, 0.03, 0.01, 1.05, 1), (0.0, 0.0))
    assert np.max(np.abs(o.heat_flux_of(G, H))) <= 1e-13
