"""Level-scheduled sweeps and unstructured meshes on the GPU (needs an MI355X).

1. On structured meshes the level-scheduled sweeps (sweep_order LEVELS) take the same cells
   in the same order as the i+j hyperplane sweeps: the micro sweeps do the same
   arithmetic per cell, the macro sweep sums its sides in another order, so the two paths
   agree to rounding (FP64 1e-13, FP32-mixed a few units of the last place).
2. Hybrid quadrilateral/triangle cavities with jittered nodes, in row order and in a seeded
   random cell order (many irregular levels), BGK and Shakhov with the limiter: every step
   against the oracle at the FP64 bar of the structured parity tests (1e-12 of the largest
   magnitude per step, 1e-10 for converged fields), FP32-mixed at 1e-5.
3. The Kn 10 cavity on the 28928-cell hybrid mesh with 101^2 velocities (the benchmark's
   unstructured workload) at full size: one implicit iteration against the FP64 oracle.
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


def _seeded(f, seed, amp=0.1):
    return f * wl.perturbation(f.shape, seed, amp)


# ------------------------------------------------------------ 1. levels = hyperplanes
STRUCT = {
    "cavity_bgk": lambda: wl.cavity(n=24, nj=20, stretch=1.5, nv=12, Kn=0.075),
    "cavity_shakhov_nc_limiter": lambda: dict(
        wl.cavity(n=20, stretch=None, nv=13, quad=wl.NEWTON_COTES, vmax=4.0, Kn=1.0,
                  model=wl.SHAKHOV, Pr=2 / 3, K=1), limiter=1),
    "couette": lambda: wl.couette(nj=32, nv=12),
    "cylinder": lambda: wl.cylinder(ni=12, nj=16, rmax=6.0, nv=16, vmax=6.0, Ma=1.5, Kn=0.1,
                                    precision=wl.FP64),
}


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32_MIXED], ids=["fp64", "fp32"])
@pytest.mark.parametrize("name", list(STRUCT))
def test_level_sweeps_match_hyperplane_sweeps(name, prec):
    cfg = dict(STRUCT[name](), precision=prec)
    a = _solver(dict(cfg, sweep_order=wl.SWEEPS_HYPERPLANES))
    b = _solver(dict(cfg, sweep_order=wl.SWEEPS_LEVELS))
    f0 = _seeded(a.get_state(), 21, 0.05)
    a.set_state(f0)
    b.set_state(f0)
    tol = 1e-13 if prec == wl.FP64 else 1e-6
    for k in range(4):
        ra, rb = a.step(wl.IMPLICIT, 1), b.step(wl.IMPLICIT, 1)
        fa, fb = a.get_state(), b.get_state()
        print(f"{name} step {k}: residuals {ra:.6e} {rb:.6e}, state difference {_rel_species(fb, fa):.2e}")
        assert _rel_species(fb, fa) <= tol
        assert abs(ra - rb) <= 1e3 * tol * abs(ra)


# The level micro sweeps read a neighbour's increment from an LDS ring of the last 256
# (FP32) or 128 (FP64) positions when every level fits it and the neighbour is close
# enough, else from memory.  Levels of 200 (FP32) or 100 (FP64) cells: in the middle of
# the mesh only part of the previous level is close enough, so one level reads both ways;
# against the hyperplane sweeps.  Levels of 140 (FP64) or 260 (FP32) cells, larger than
# the ring: every neighbour comes from memory; against the hyperplane sweeps, and (260^2,
# too large for the hyperplane macro sweep) against the oracle at the FP32 step bar.
RING = {"fp32_partial_window": (200, wl.FP32_MIXED), "fp64_partial_window": (100, wl.FP64),
        "fp64_levels_above_ring": (140, wl.FP64)}


def _ring_cfg(n, prec):
    return dict(wl.cavity(n=n, stretch=None, nv=8, Kn=0.075, precision=prec),
                sweep_order=wl.SWEEPS_LEVELS)


@pytest.mark.parametrize("name", list(RING))
def test_level_sweeps_ring_window_edges(name):
    n, prec = RING[name]
    cfg = _ring_cfg(n, prec)
    a = _solver(dict(cfg, sweep_order=wl.SWEEPS_HYPERPLANES))
    b = _solver(cfg)
    f0 = _seeded(a.get_state(), 23, 0.05)
    a.set_state(f0)
    b.set_state(f0)
    tol = 1e-13 if prec == wl.FP64 else 1e-6
    for k in range(3):
        ra, rb = a.step(wl.IMPLICIT, 1), b.step(wl.IMPLICIT, 1)
        d = _rel_species(b.get_state(), a.get_state())
        print(f"{name} step {k}: residuals {ra:.6e} {rb:.6e}, state difference {d:.2e}")
        assert d <= tol
        assert abs(ra - rb) <= 1e3 * tol * abs(ra)


def test_level_sweeps_levels_above_ring_fp32_against_oracle():
    o, g = _pair(_ring_cfg(260, wl.FP32_MIXED), seed=24, amp=0.05)
    for k in range(2):
        ro, rg = o.implicit_step(1), g.step(wl.IMPLICIT, 1)
        d = _rel_species(g.get_state(), o.get_state())
        print(f"260^2 FP32 step {k}: res {ro:.6e} / {rg:.6e}, state {d:.2e}")
        assert d <= 2e-6


# ------------------------------------------------------------ 2. hybrid meshes vs the oracle
def _hyb_bgk():
    return wl.hybrid_cavity(n=16, nq=3, nv=12, jitter=0.15, seed=1, Kn=0.075)


def _hyb_random():
    c = _hyb_bgk()
    return wl.with_mesh(c, wl.renumbered(c["mesh"], 9))


def _hyb_shakhov():
    return dict(wl.hybrid_cavity(n=14, nq=2, nv=13, jitter=0.2, seed=2, quad=wl.NEWTON_COTES,
                                 vmax=4.0, Kn=1.0, model=wl.SHAKHOV, Pr=2 / 3, K=1), limiter=1)


def _hyb_farfield():
    c = wl.hybrid_cavity(n=12, nq=2, nv=12, jitter=0.2, seed=3, Kn=0.2)
    c.update(bc=[wl.BC_FARFIELD, wl.BC_WALL, wl.BC_FARFIELD, wl.BC_FARFIELD],
             far_rho=1.0, far_u=0.2, far_v=0.05, far_T=1.0, init_u=0.2, init_v=0.05)
    return c


HYB = {"hybrid_bgk": _hyb_bgk, "hybrid_random_order": _hyb_random,
       "hybrid_shakhov_nc_limiter": _hyb_shakhov, "hybrid_farfield_wall": _hyb_farfield}


def _pair(cfg, seed, amp=0.1):
    o, g = Oracle(cfg), _solver(cfg)
    f = _seeded(o.get_state(), seed, amp)
    o.set_state(f)
    g.set_state(f)
    return o, g


@pytest.mark.parametrize("name", list(HYB))
def test_hybrid_geometry_and_initial_state(name):
    cfg = HYB[name]()
    o, g = Oracle(cfg), _solver(cfg)
    assert (g.nc, g.nv, g.nf) == (o.nc, o.nv, o.nf)
    assert abs(g.dt - o.dt) <= 1e-14 * o.dt  # the velocity sets agree to rounding
    assert _rel_species(g.get_state(), o.get_state()) <= 1e-14


@pytest.mark.parametrize("name", list(HYB))
def test_hybrid_flux_face_and_predictor_parity(name):
    o, g = _pair(HYB[name](), seed=31)
    assert _rel_species(g.flux(), o.flux()) <= 1e-12
    Wg, rg = g.face_moments()
    Wo, ro = o.face_moments()
    assert _rel(Wg, Wo) <= 1e-12
    if np.abs(ro).max() > 0:
        assert _rel(rg, ro) <= 1e-12
    assert _rel(g.macro_residual(), o.macro_residual()) <= 1e-12
    Wsg, dg = g.predict()
    Wso, do = o.predict()
    assert _rel(Wsg, Wso) <= 1e-12 and _rel(dg, do) <= 1e-12


@pytest.mark.parametrize("name", list(HYB))
def test_hybrid_implicit_and_explicit_step_parity(name):
    o, g = _pair(HYB[name](), seed=32)
    for k in range(4):
        ro, rg = o.implicit_step(1), g.step(wl.IMPLICIT, 1)
        d = _rel_species(g.get_state(), o.get_state())
        print(f"{name} implicit step {k}: res {ro:.6e} / {rg:.6e}, state {d:.2e}")
        assert d <= 1e-12
        assert abs(rg - ro) <= 1e-9 * abs(ro)
    for k in range(2):
        o.explicit_step(1)
        g.step(wl.EXPLICIT, 1)
        assert _rel_species(g.get_state(), o.get_state()) <= 1e-12
    assert _rel(g.moments()[:, :4], o.moments()[:, :4]) <= 1e-12


@pytest.mark.parametrize("name", ["hybrid_bgk", "hybrid_random_order"])
def test_hybrid_converged_fields(name):
    cfg = HYB[name]()
    o, g = Oracle(cfg), _solver(cfg)
    it_o, res_o, ok_o = o.solve(1e-8, 3000)
    it_g, res_g, ok_g = g.solve(1e-8, 3000)
    print(f"{name}: oracle {it_o} iterations, GPU {it_g}")
    assert ok_o and ok_g and it_g == it_o
    mo, mg = o.moments(), g.moments()
    for q in range(4):
        assert np.max(np.abs(mg[:, q] - mo[:, q])) <= 1e-10 * max(1.0, np.abs(mo[:, q]).max())


@pytest.mark.parametrize("name", ["hybrid_bgk", "hybrid_shakhov_nc_limiter"])
def test_hybrid_fp32_mixed_steps(name):
    cfg = dict(HYB[name](), precision=wl.FP32_MIXED)
    o, g = _pair(dict(cfg, precision=wl.FP64), seed=33)
    g = _solver(cfg)
    g.set_state(o.get_state())
    for k in range(4):
        o.implicit_step(1)
        g.step(wl.IMPLICIT, 1)
        d = _rel_species(g.get_state(), o.get_state())
        print(f"{name} FP32 step {k}: state {d:.2e}")
        assert d <= 1e-5


def test_hybrid_free_stream_is_kept():
    c = wl.hybrid_cavity(n=12, nq=2, nv=12, jitter=0.2, seed=4, Kn=0.2)
    c.update(bc=[wl.BC_FARFIELD] * 4, far_rho=1.1, far_u=0.3, far_v=-0.2, far_T=1.2,
             init_rho=1.1, init_u=0.3, init_v=-0.2, init_T=1.2, limiter=1)
    g = _solver(c)
    f0 = g.get_state()
    g.step(wl.IMPLICIT, 3)
    g.step(wl.EXPLICIT, 2)
    assert _rel_species(g.get_state(), f0) <= 1e-14


# ------------------------------------------------------------ 3. full size
def test_hybrid_kn10_full_size_fp32_step():
    """The Kn 10 cavity (128^2 nodes, 101^2 Newton-Cotes velocities, Shakhov) on the
    28928-cell hybrid mesh in its FP32-mixed form: about 3e8 cell-velocity pairs, two
    velocity chunks in the flux, 160 velocity slices in the sweeps.  One implicit
    iteration from a seeded perturbation against the FP64 oracle."""
    cfg = wl.case("cavity_kn10_hybrid")
    assert cfg["precision"] == wl.FP32_MIXED
    o = Oracle(dict(cfg, precision=wl.FP64))
    g = _solver(cfg)
    f = _seeded(o.get_state(), 12, 0.02)
    o.set_state(f)
    g.set_state(f)
    o.implicit_step(1)
    g.step(wl.IMPLICIT, 1)
    fo, fg = o.get_state(), g.get_state()
    for s in range(2):
        assert _rel(fg[s], fo[s]) <= 2e-6
