"""Parity of the HIP path with the CPU oracle, through the C ABI (needs an MI355X).

Inputs are seeded and identical on both sides: the oracle's initial equilibrium times
1 + 0.1 U(-1, 1) noise (workloads.perturbation).  FP64 results must agree to 1e-12 of
the largest magnitude of each compared array per step (the two sides sum in different
orders and the GPU contracts to FMA), converged fields to 1e-10.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import Oracle

pytestmark = pytest.mark.gpu


def _solver(cfg):
    from paper_1709_01819_amd import Solver
    return Solver(cfg)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def _rel_species(a, b):
    return max(_rel(a[s], b[s]) for s in range(2))


def _pair(cfg, seed=None, amp=0.1):
    o, g = Oracle(cfg), _solver(cfg)
    if seed is not None:
        f = o.get_state()
        f = f * wl.perturbation(f.shape, seed, amp)
        o.set_state(f)
        g.set_state(f)
    return o, g


CASES = {
    "couette": lambda: wl.case("couette"),
    "cavity_tanh": lambda: wl.cavity(n=12, nj=10, stretch=1.5, nv=8, Kn=0.075),
    "cavity_shakhov_nc": lambda: wl.cavity(n=10, stretch=None, nv=13, quad=wl.NEWTON_COTES,
                                           vmax=4.0, Kn=1.0, model=wl.SHAKHOV, Pr=2 / 3, K=1),
    "cylinder_limiter": lambda: wl.cylinder(ni=8, nj=12, rmax=6.0, nv=16, vmax=12.0, Kn=0.1,
                                            precision=wl.FP64),
    "periodic_box": lambda: wl.periodic_box(n=5, nv=8),
    # 91^2 = 8281 velocities: the flux kernel splits them into chunks of 4160 and 4121 and
    # combines the per-chunk macroscopic residuals
    "cavity_shakhov_chunked": lambda: wl.cavity(n=6, stretch=None, nv=91, quad=wl.NEWTON_COTES,
                                                vmax=4.0, Kn=1.0, model=wl.SHAKHOV, Pr=2 / 3, K=1),
    "cylinder_chunked": lambda: wl.cylinder(ni=6, nj=8, rmax=6.0, nv=91, vmax=12.0, Kn=0.1,
                                            precision=wl.FP64),
}


@pytest.mark.parametrize("name", ["couette", "cavity_shakhov_nc", "cylinder_limiter"])
def test_velocity_set_and_initial_state(name):
    cfg = CASES[name]()
    o, g = _pair(cfg)
    for a, b in zip(g.velocities(), o.velocities()):
        assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, np.abs(b).max())
    # the GPU builds equilibria in a central basis, the oracle in the raw basis: at Mach 5
    # the raw Gram matrix has condition ~1e5, hence 1e-12 rather than 1e-14
    assert _rel_species(g.get_state(), o.get_state()) <= 1e-12
    assert abs(g.dt - o.dt) <= 1e-15 * o.dt
    mo_g, mo_o = g.moments(), o.moments()
    assert np.max(np.abs(mo_g[:, :5] - mo_o[:, :5])) <= 1e-12


def test_state_roundtrip_is_exact():
    cfg = CASES["cavity_tanh"]()
    o, g = _pair(cfg, seed=2)
    assert np.array_equal(g.get_state(), o.get_state())


@pytest.mark.parametrize("name", list(CASES))
def test_flux_parity(name):
    o, g = _pair(CASES[name](), seed=1)
    Mg, Mo = g.flux(), o.flux()
    assert _rel_species(Mg, Mo) <= 1e-12, _rel_species(Mg, Mo)
    MWg, MWo = g.macro_residual(), o.macro_residual()
    for a in range(4):
        assert _rel(MWg[:, a], MWo[:, a]) <= 1e-11


# wide meshes: the macro LU-SGS workgroup then takes two lanes per cell (each lane the i or
# the j sides and two of the four components) instead of four
PRED_CASES = dict(CASES, cavity_80=lambda: wl.cavity(n=80, stretch=1.5, nv=4, Kn=0.075),
                  cavity_120=lambda: wl.cavity(n=120, stretch=1.5, nv=4, Kn=0.075))
# the point-relaxation predictor (Jacobi sweeps of the macroscopic system)
RELAX_CASES = {
    "cavity_tanh_relax0": lambda: dict(CASES["cavity_tanh"](), predictor=1, relax_sweeps=0),
    "cavity_tanh_relax3": lambda: dict(CASES["cavity_tanh"](), predictor=1, relax_sweeps=3),
    "couette_relax2": lambda: dict(CASES["couette"](), predictor=1, relax_sweeps=2),
    "cylinder_limiter_relax1": lambda: dict(CASES["cylinder_limiter"](), predictor=1, relax_sweeps=1),
    "periodic_box_relax4": lambda: dict(CASES["periodic_box"](), predictor=1, relax_sweeps=4),
}
PRED_CASES.update(RELAX_CASES)
# the start-up ramp of the implicit CFL (3, 15, 75, 375, then 1000; on the chunked cylinder
# the macro rows come from their own launch)
RAMP_CASES = {
    "cavity_tanh_ramp": lambda: dict(CASES["cavity_tanh"](), cfl_start=3.0, cfl_growth=5.0),
    "cylinder_chunked_ramp": lambda: dict(CASES["cylinder_chunked"](), cfl_start=0.5, cfl_growth=3.0),
}
PRED_CASES.update(RAMP_CASES)


@pytest.mark.parametrize("name", ["couette", "cavity_tanh", "cavity_shakhov_nc", "cylinder_limiter",
                                  "cavity_80", "cavity_120"] + list(RELAX_CASES))
def test_predictor_parity(name):
    o, g = _pair(PRED_CASES[name](), seed=3)
    Wg, dg = g.predict()
    Wo, do = o.predict()
    assert _rel(dg, do) <= 1e-13
    for a in range(4):
        assert _rel(Wg[:, a], Wo[:, a]) <= 1e-12


@pytest.mark.parametrize("name", list(CASES) + ["cavity_tanh_relax3", "cylinder_limiter_relax1"]
                         + list(RAMP_CASES))
def test_implicit_step_parity(name):
    o, g = _pair(PRED_CASES[name](), seed=4)
    for n in (1, 4):
        ro = o.implicit_step(n)
        rg = g.step(wl.IMPLICIT, n)
        assert _rel_species(g.get_state(), o.get_state()) <= 1e-12
        assert abs(rg - ro) <= 1e-9 * ro + 1e-15


@pytest.mark.parametrize("name", list(RAMP_CASES))
def test_cfl_ramp_predictor_after_steps(name):
    """The implicit time steps of the prediction follow the ramp's iteration count on both
    sides, and set_state restarts the ramp."""
    o, g = _pair(PRED_CASES[name](), seed=9)
    o.implicit_step(2)
    g.step(wl.IMPLICIT, 2)
    assert _rel(g.predict()[1], o.predict()[1]) <= 1e-12
    f = o.get_state()
    o.set_state(f)
    g.set_state(f)
    assert _rel(g.predict()[1], o.predict()[1]) <= 1e-13


@pytest.mark.parametrize("name", ["couette", "cavity_tanh", "cylinder_limiter"])
def test_explicit_step_parity(name):
    o, g = _pair(CASES[name](), seed=5)
    o.explicit_step(3)
    g.step(wl.EXPLICIT, 3)
    assert _rel_species(g.get_state(), o.get_state()) <= 1e-12


def test_couette_converged_fields():
    cfg = wl.case("couette")
    o, g = _pair(cfg)
    it_o, r_o, ok_o = o.solve(1e-8, 2000)
    it_g, r_g, ok_g = g.solve(1e-8, 2000)
    assert ok_o and ok_g and it_o == it_g
    assert np.max(np.abs(g.moments()[:, :4] - o.moments()[:, :4])) <= 1e-10


def test_cavity_c2_full_size_steps():
    """The benchmark workload (64^2 tanh cavity, GH 28^2, Kn = 0.075) at full size."""
    cfg = wl.case("cavity_kn0.075")
    o, g = _pair(cfg, seed=6, amp=0.02)
    assert _rel_species(g.flux(), o.flux()) <= 1e-12
    o.implicit_step(2)
    g.step(wl.IMPLICIT, 2)
    assert _rel_species(g.get_state(), o.get_state()) <= 1e-12


def test_kn10_cavity_128_history_and_divergence():
    """The Kn = 10 Shakhov cavity on its 128^2 mesh (17^2 velocities here) at CFL 1000
    diverges after about two dozen iterations; the HIP path follows the oracle's residual
    history step by step and fails at the same iteration (a property of the method as
    read, not of either implementation)."""
    from paper_1709_01819_amd.abi import IdugksError
    from oracle.oracle import OracleError
    cfg = dict(wl.shrink(wl.case("cavity_kn10"), ni=128, nj=128, nv=17), precision=wl.FP64,
               cfl_imp=1000.0)
    o, g = _pair(cfg)
    ro, rg, fail_o, fail_g = [], [], None, None
    for it in range(1, 41):
        if fail_o is None:
            try:
                ro.append(o.implicit_step(1))
            except OracleError:
                fail_o = it
        if fail_g is None:
            try:
                rg.append(g.step(wl.IMPLICIT, 1))
            except IdugksError:
                fail_g = it
        if it == 12:
            assert _rel_species(g.get_state(), o.get_state()) <= 1e-10
        if fail_o and fail_g:
            break
    assert fail_o is not None and fail_o == fail_g
    np.testing.assert_allclose(rg[:20], ro[:20], rtol=1e-6)
    # with diverge_iters the solve stops on the residual's growth, at the first iteration
    # where it has grown that many times in a row (found in the oracle's history), while
    # the state is still physical
    n_div = 3
    grown, stop = 0, None
    for k in range(1, len(ro)):
        grown = grown + 1 if ro[k] > ro[k - 1] else 0
        if grown >= n_div:
            stop = k + 1
            break
    assert stop is not None and stop < fail_o
    s = _solver(dict(cfg, diverge_iters=n_div))  # from the same initial state
    with pytest.raises(IdugksError, match="residual grew"):
        s.solve(1e-12, 40)
    assert s.info().iterations == stop
    assert np.all(np.isfinite(s.get_state()))


def _local_errors(a, b):
    """Errors of a against b on local scales: per velocity relative to that velocity's
    largest magnitude over the cells (the tails of a wide velocity set), per cell relative
    to that cell's largest magnitude over the velocities (low-density regions), and
    element by element wherever the value is at least 1e-20 of the field's largest."""
    d, m = np.abs(a - b), np.abs(b)
    per_v = float((d.max(0) / m.max(0)).max())
    per_c = float((d.max(1) / m.max(1)).max())
    big = m >= 1e-20 * m.max()
    elem = float((d[big] / m[big]).max())
    return per_v, per_c, elem


# FP64: the two sides differ in summation order and in the basis of the equilibrium
# correction (central here, raw in the oracle, whose Gram matrix reaches a condition of
# about 1e5 at Mach 5: 1e-16 x 1e5 = 1e-11).  Values below 1e-20 of the largest are sums
# of neighbour terms many orders larger, so only the scaled checks cover them.  The wide
# velocity set: 65^2 Newton-Cotes points on [-12, 12]^2 around the ramped cylinder.
LOCAL_CASES = {
    "cylinder_wide_ramp": lambda: dict(wl.cylinder(ni=6, nj=8, rmax=6.0, nv=65, vmax=12.0, Kn=0.1,
                                                   precision=wl.FP64), cfl_start=0.5, cfl_growth=3.0),
}


@pytest.mark.parametrize("name", ["couette", "cavity_tanh", "cavity_shakhov_nc", "cylinder_limiter",
                                  "cylinder_wide_ramp"])
def test_step_parity_on_local_scales(name):
    cfg = LOCAL_CASES[name]() if name in LOCAL_CASES else CASES[name]()
    o, g = _pair(cfg, seed=14, amp=0.02)
    for _ in range(2):
        o.implicit_step(1)
        g.step(wl.IMPLICIT, 1)
    fo, fg = o.get_state(), g.get_state()
    for s in range(2):
        per_v, per_c, elem = _local_errors(fg[s], fo[s])
        print(f"{name} species {s}: per velocity {per_v:.2e}, per cell {per_c:.2e}, element {elem:.2e}")
        assert per_v <= 1e-11 and per_c <= 1e-11
        assert elem <= 1e-6


@pytest.mark.parametrize("name", ["cavity_kn10", "cylinder_ma5"])
def test_full_size_fp32_step(name):
    """The two large workloads in their FP32-mixed benchmark form at full size: the 128^2
    cavity with 101^2 Newton-Cotes velocities (Shakhov, Kn = 10) and the 96 x 160 O-grid
    cylinder with 100^2 velocities (Shakhov, limiter, far field, Ma 5, first step of its
    CFL ramp); about 1.6e8 cell-velocity pairs each, two velocity chunks in the flux,
    level-scheduled sweeps over 160 velocity slices.  One implicit iteration from a seeded
    perturbation against the FP64 oracle, to the FP32 bar of the small cases."""
    cfg = wl.case(name)
    assert cfg["precision"] == wl.FP32_MIXED
    o, g = _pair(cfg, seed=12, amp=0.02)
    o.implicit_step(1)
    g.step(wl.IMPLICIT, 1)
    fo = o.get_state()
    fg = g.get_state()
    for s in range(2):
        assert _rel(fg[s], fo[s]) <= 2e-6


# ------------------------------------------------------------------ full C2, converged
@pytest.fixture(scope="module")
def c2_oracle_converged():
    """FP64 oracle on the 64^2 / GH 28^2 cavity (Kn = 0.075, CFL 1000) to Res < 1e-8."""
    o = Oracle(wl.case("cavity_kn0.075"))
    it, res, ok = o.solve(1e-8, 2000)
    assert ok
    return it, o.moments()


def test_c2_fp64_converged_fields(c2_oracle_converged):
    it_o, mo = c2_oracle_converged
    g = _solver(wl.case("cavity_kn0.075"))
    it_g, res, ok = g.solve(1e-8, 2000)
    assert ok and it_g == it_o
    mg = g.moments()
    for k in range(4):   # rho, U, V, T
        assert np.max(np.abs(mg[:, k] - mo[:, k])) <= 1e-10


def test_c2_fp32_mixed_converged_fields(c2_oracle_converged):
    """FP32 distributions/fluxes/sweeps, FP64 moments and predictor: stated bound 1e-5."""
    it_o, mo = c2_oracle_converged
    g = _solver(wl.case("cavity_kn0.075", precision=wl.FP32_MIXED))
    it_g, res, ok = g.solve(1e-8, 2000)
    assert ok and abs(it_g - it_o) <= 0.25 * it_o
    mg = g.moments()
    errs = [float(np.max(np.abs(mg[:, k] - mo[:, k]))) for k in range(4)]
    print("FP32-mixed converged max abs errors rho, U, V, T:", errs)
    assert max(errs) <= 1e-5


# 181^2 velocities on 5 x 4 cells: the FP32 sweeps take two velocities per lane (1024
# slices of 2 x 16, the last one ragged)
FP32_CASES = dict(CASES, cavity_shakhov_vpl2=lambda: wl.cavity(
    n=5, nj=4, stretch=None, nv=181, quad=wl.NEWTON_COTES, vmax=4.0, Kn=1.0, model=wl.SHAKHOV,
    Pr=2 / 3, K=1))


@pytest.mark.parametrize("name", ["cavity_tanh", "cavity_shakhov_nc", "cylinder_limiter",
                                  "cavity_shakhov_vpl2"])
def test_fp32_mixed_step_close_to_fp64_oracle(name):
    cfg = FP32_CASES[name]()
    cfg["precision"] = wl.FP32_MIXED
    o, g = _pair(cfg, seed=8)
    o.implicit_step(2)
    g.step(wl.IMPLICIT, 2)
    assert _rel_species(g.get_state(), o.get_state()) <= 2e-6
