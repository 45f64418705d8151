"""Converged fields of the HIP path against the converged oracle on shrunk copies of the two
large workloads (same physics, smaller mesh and velocity set):

  Kn = 10 lid-driven cavity: Shakhov (Pr = 2/3, K = 1), Newton-Cotes velocities on [-4, 4]^2,
  CFL 1000 (Section 3.2), 24^2 cells, 17^2 velocities;
  Mach 5 cylinder: Shakhov, Kn = 0.1, Venkatakrishnan limiter, far field, O-grid to 15 radii,
  Newton-Cotes on [-15, 15]^2 (Section 3.3) with the start-up ramp of the implicit CFL,
  24 x 32 cells, 40^2 velocities.

The FP64 form must reach the residual at the oracle's iteration and match its fields to
1e-10 of each field's largest magnitude.  The FP32-bulk / FP64-moment form must match to
1e-5.  Rounding the stored FP32 state to its last bit each iteration leaves a floor in the
relative density change of about 1e-8 at Kn = 10 (the transport sweeps carry each cell's
rounding downstream almost undamped), so there the FP32 form iterates to its floor (below
5e-8) and FP64 iterations finish the solve from that state (mixed-precision refinement),
which must reach the FP64 fixed point like the oracle started from the same state.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import Oracle

pytestmark = pytest.mark.gpu

TOL = 1e-8


def _solver(cfg):
    from paper_1709_01819_amd import Solver
    return Solver(cfg)


def _kn10():
    return dict(wl.shrink(wl.case("cavity_kn10"), ni=24, nj=24, nv=17), precision=wl.FP64,
                cfl_imp=1000.0)


def _cylinder():
    return dict(wl.shrink(wl.case("cylinder_ma5"), ni=24, nj=32, nv=40), precision=wl.FP64)


CASES = {"kn10_cavity": _kn10, "ma5_cylinder": _cylinder}


@pytest.fixture(scope="module", params=list(CASES))
def converged(request):
    cfg = CASES[request.param]()
    o = Oracle(cfg)
    it, res, ok = o.solve(TOL, 4000)
    assert ok, (it, res)
    print(f"{request.param}: oracle converged in {it} iterations")
    return request.param, cfg, it, o.moments()


def _field_errors(mg, mo):
    # rho, U, V, T, each relative to its largest magnitude (at least 1)
    return [float(np.max(np.abs(mg[:, k] - mo[:, k])) / max(1.0, np.abs(mo[:, k]).max())) for k in range(4)]


def test_fp64_converged_fields(converged):
    name, cfg, it_o, mo = converged
    g = _solver(cfg)
    it_g, res, ok = g.solve(TOL, 4000)
    assert ok and it_g == it_o, (it_g, it_o, res)
    errs = _field_errors(g.moments(), mo)
    print(f"{name} FP64: max field errors rho, U, V, T {errs}")
    assert max(errs) <= 1e-10


FLOOR32 = 5e-8


def test_fp32_mixed_converged_fields_and_refinement(converged):
    name, cfg, it_o, mo = converged
    g = _solver(dict(cfg, precision=wl.FP32_MIXED))
    it_g, res, ok = g.solve(TOL, max(1500, 4 * it_o))
    errs = _field_errors(g.moments(), mo)
    print(f"{name} FP32-mixed: {it_g} iterations (oracle {it_o}), res {res:.3e}, "
          f"max field errors rho, U, V, T {errs}")
    assert ok or res <= FLOOR32
    assert max(errs) <= 1e-5
    # refinement: FP64 iterations from the FP32 state reach the FP64 fixed point
    f32 = g.get_state()
    o = Oracle(cfg)
    o.set_state(f32)
    it_o2, res_o2, ok_o2 = o.solve(TOL, 4000)
    h = _solver(cfg)
    h.set_state(f32)
    it_h, res_h, ok_h = h.solve(TOL, 4000)
    errs2 = _field_errors(h.moments(), o.moments())
    print(f"{name} refinement: {it_h} FP64 iterations from the FP32 state (oracle {it_o2}), "
          f"max field errors {errs2}")
    assert ok_o2 and ok_h and it_h == it_o2
    assert max(errs2) <= 1e-10
