"""Pins of the oracle's point-relaxation predictor (CPU only).

The paper names a point relaxation scheme beside LU-SGS for the prediction step (its
conclusions) without a formula; the reading here relaxes the same system
(L + D + U) dW = M_W of Eq. 29-31 point by point: dW = D^-1 M_W, then Jacobi sweeps.

- With no sweeps the prediction is a per-cell scaling of M_W (no coupling between
  cells), by 1/D with D = Omega/dt_imp + (1/2) sum lambda S = (Omega/dt_imp)(1 + CFL/2)
  on a periodic box (no wall faces; sum lambda S = CFL Omega/dt_imp by the definition of
  dt_imp).
- The predictor only changes the path to the steady state, not the state: LU-SGS and
  point relaxation converge to the same fields.
"""
import numpy as np

import workloads as wl
from oracle import Oracle


def _perturbed(cfg, seed=7, amp=0.05):
    o = Oracle(cfg)
    f = o.get_state()
    o.set_state(f * wl.perturbation(f.shape, seed, amp))
    return o


def test_point_implicit_step_is_the_diagonal_scaling():
    cfg = dict(wl.periodic_box(n=6, nv=6), predictor=1, relax_sweeps=0)
    o = _perturbed(cfg)
    f = o.get_state()
    W = np.array([o.moments_of(f[0, c], f[1, c]) for c in range(o.nc)])
    MW = o.macro_residual()
    Ws, dti = o.predict()
    area, _, _ = o.cells()
    dW = Ws - W
    kappa = dti / (area * (1.0 + cfg["cfl_imp"] / 2.0))
    scale = np.max(np.abs(MW))
    assert scale > 0
    assert np.max(np.abs(dW - kappa[:, None] * MW)) <= 1e-12 * np.max(np.abs(kappa)) * scale


def test_point_relaxation_reaches_the_lusgs_steady_state():
    base = wl.cavity(n=8, nj=6, stretch=1.5, nv=6, Kn=0.3)
    fields = []
    for extra in ({}, {"predictor": 1, "relax_sweeps": 2}):
        o = Oracle(dict(base, **extra))
        it, res, ok = o.solve(1e-12, 20000)
        assert ok, (extra, it, res)
        fields.append(o.moments()[:, :4])
    ref = np.max(np.abs(fields[0]), axis=0)
    assert np.all(np.max(np.abs(fields[1] - fields[0]), axis=0) <= 1e-8 * ref)


def test_relaxation_sweeps_change_the_prediction():
    cfg = wl.cavity(n=6, stretch=None, nv=6, Kn=0.3)
    preds = []
    for k in (0, 1, 4):
        o = _perturbed(dict(cfg, predictor=1, relax_sweeps=k))
        preds.append(o.predict()[0])
    assert np.max(np.abs(preds[1] - preds[0])) > 0
    assert np.max(np.abs(preds[2] - preds[1])) > 0
