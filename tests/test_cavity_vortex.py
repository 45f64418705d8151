"""Pins of the vortex-centre extraction used by the Re = 1000 cavity check (CPU only).

The extraction is checked on polynomial stream functions whose centre, stream function
value and vorticity are known in closed form: psi = -A g(x) g(y), g(t) = t^2 (1 - t),
vanishes on all four walls, has its extremum at (2/3, 2/3) with psi = -A (4/27)^2 and
vorticity -laplacian(psi) = -16 A / 27 there; mirroring x -> 1 - x moves the centre to
(1/3, 2/3).
"""
import os

import numpy as np
import pytest

from cavity_vortex import centre, load_golden, stream_function, vortex_metrics

HERE = os.path.dirname(os.path.abspath(__file__))


def _field(n, A, mirror=False):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    y = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, y)
    if mirror:
        X = 1.0 - X
    g, dg = X ** 2 * (1 - X), 2 * X - 3 * X ** 2
    gy, dgy = Y ** 2 * (1 - Y), 2 * Y - 3 * Y ** 2
    u = -A * g * dgy                               # d psi / dy
    v = A * dg * gy * (-1.0 if mirror else 1.0)    # -d psi / dx
    return u, v


@pytest.mark.parametrize("mirror", [False, True])
def test_polynomial_vortex_centre(mirror):
    n, A = 128, 3.0
    u, v = _field(n, A, mirror)
    m = vortex_metrics(u.ravel(), v.ravel(), n, n, 1.0)
    xc = 1.0 / 3.0 if mirror else 2.0 / 3.0
    assert abs(m["primary_x"] - xc) < 2e-3
    assert abs(m["primary_y"] - 2.0 / 3.0) < 2e-3
    assert m["primary_psi"] == pytest.approx(-A * (4.0 / 27.0) ** 2, rel=2e-3)
    assert m["primary_omega"] == pytest.approx(16.0 * A / 27.0, rel=2e-3)


def test_stream_function_is_second_order_and_vanishes_on_the_walls():
    errs = []
    for n in (32, 64):
        u, _ = _field(n, 1.0)
        h = 1.0 / n
        psi = stream_function(u, h)
        x = (np.arange(n) + 0.5) * h
        X, Y = np.meshgrid(x, x)
        exact = -(X ** 2 * (1 - X)) * (Y ** 2 * (1 - Y))
        errs.append(np.max(np.abs(psi - exact)))
        # the top row sits half a cell below the lid, where psi is O(h)
        assert abs(psi[-1]).max() < 2 * h
    assert errs[0] / errs[1] > 3.5


def test_secondary_extremum_is_refined_to_the_true_maximum():
    n = 64
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    psi = np.exp(-((X - 0.11) ** 2 + (Y - 0.09) ** 2) / 0.002)
    val, xc, yc = centre(psi, h, +1, (0.0, 0.3), (0.0, 0.3))
    assert abs(xc - 0.11) < 0.2 * h and abs(yc - 0.09) < 0.2 * h
    assert val == pytest.approx(1.0, rel=1e-2)


def test_golden_table_holds_the_ten_quantities():
    g = load_golden(os.path.join(HERE, "golden", "cavity_re1000_table1.txt"))
    assert len(g) == 10
    assert g["primary_psi"] < 0 < g["left_psi_e4"]
