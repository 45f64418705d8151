"""The continuum lid-driven cavity at Re = 1000 (the paper's Section 3.2 and Table 1), on
the HIP path (needs an MI355X).

- Parity at the full size (256^2 cells, 25^2 velocities): one implicit iteration from a
  seeded perturbation of the initial state, the whole state element by element against
  the oracle (1e-12 of the largest magnitude per species, as the other FP64 parity
  cases).  This exercises the sweeps at 511 hyperplanes and the macro sweep at the
  largest row staging this mesh takes.
- Accuracy: the steady flow on the paper's 256^2 mesh, solved to Res < 1e-8 with the
  point-relaxation predictor (64 sweeps), against the IDUGKS row of Table 1
  (tests/golden/cavity_re1000_table1.txt): the primary vortex within 2 % (stream function
  and vorticity) and 0.01 (centre), the secondary vortices within 10 % (stream function)
  and 0.02 (centres).
"""
import os

import numpy as np
import pytest

import workloads as wl
from cavity_vortex import load_golden, vortex_metrics
from oracle import Oracle

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def test_full_size_step_parity():
    from paper_1709_01819_amd import Solver
    cfg = wl.case("cavity_re1000")
    o, g = Oracle(cfg), Solver(cfg)
    f = o.get_state()
    f = f * wl.perturbation(f.shape, 17, 0.05)
    o.set_state(f)
    g.set_state(f)
    ro = o.implicit_step(1)
    rg = g.step(wl.IMPLICIT, 1)
    fo, fg = o.get_state(), g.get_state()
    for s in range(2):
        assert _rel(fg[s], fo[s]) <= 1e-12
    assert rg == pytest.approx(ro, rel=1e-9)


def test_steady_vortices_match_table1():
    from paper_1709_01819_amd import Solver
    cfg = dict(wl.case("cavity_re1000"), predictor=1, relax_sweeps=64)
    assert (cfg["ni"], cfg["nvx"]) == (256, 25)
    g = Solver(cfg)
    iters, res, ok = g.solve(1e-8, 20000)
    assert ok, (iters, res)
    m = g.moments()
    vm = vortex_metrics(m[:, 1], m[:, 2], cfg["ni"], cfg["nj"], cfg["wall_u"][3])
    gold = load_golden(os.path.join(HERE, "golden", "cavity_re1000_table1.txt"))
    print({k: round(v, 5) for k, v in vm.items()}, iters)
    assert vm["primary_psi"] == pytest.approx(gold["primary_psi"], rel=0.02)
    assert vm["primary_omega"] == pytest.approx(gold["primary_omega"], rel=0.02)
    for k in ("primary_x", "primary_y"):
        assert abs(vm[k] - gold[k]) < 0.01
    for k in ("left_psi_e4", "right_psi_e3"):
        assert vm[k] == pytest.approx(gold[k], rel=0.10)
    for k in ("left_x", "left_y", "right_x", "right_y"):
        assert abs(vm[k] - gold[k]) < 0.02
