"""Run-to-run reproducibility of the HIP path (needs an MI355X).

Every reduction (raw moments, face moments, the macroscopic residual, the wall ghost
density, the mass and the residual) sums in a fixed order, and no kernel uses atomics, so
the same state stepped the same way gives the same bits.  Two runs from one perturbed
state are compared bit for bit, with sizes that use several blocks, chunked velocity sets
and both precisions.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

CASES = {
    "cavity_tanh": lambda: wl.cavity(n=24, nj=20, stretch=1.5, nv=12, Kn=0.075),
    "cavity_shakhov_chunked": lambda: wl.cavity(n=6, stretch=None, nv=91, quad=wl.NEWTON_COTES,
                                                vmax=4.0, Kn=1.0, model=wl.SHAKHOV, Pr=2 / 3, K=1),
    "cylinder_limiter_fp32": lambda: wl.cylinder(ni=8, nj=12, rmax=6.0, nv=16, vmax=12.0, Kn=0.1,
                                                 precision=wl.FP32_MIXED),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_implicit_steps_are_bit_reproducible(name):
    from paper_1709_01819_amd import Solver
    g = Solver(CASES[name]())
    f0 = g.get_state()
    f0 = f0 * wl.perturbation(f0.shape, 11, 0.05)
    runs = []
    for _ in range(2):
        g.set_state(f0)
        res = [g.step(wl.IMPLICIT, 1) for _ in range(3)]
        runs.append((g.get_state(), np.array(res), g.residual()))
    (fa, ra, ma), (fb, rb, mb) = runs
    assert np.array_equal(fa, fb)
    assert np.array_equal(ra, rb)
    assert np.array_equal(ma, mb)
