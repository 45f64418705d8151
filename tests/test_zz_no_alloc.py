"""The allocation-free entry point (idugks_init_noalloc: the workspace is the library's
static scratch array) against the same calls on a caller-allocated workspace."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _run(cfg, static, seed):
    from paper_1709_01819_amd import Solver
    g = Solver(cfg, static_workspace=static)
    f = g.get_state()
    g.set_state(f * wl.perturbation(f.shape, seed, 0.05))
    r = g.step(wl.IMPLICIT, 3)
    out = (g.get_state(), g.moments(), r, g.flux())
    g.close()
    return out


def _check(cfg, seed):
    a = _run(cfg, False, seed)
    b = _run(cfg, True, seed)
    # same kernels on the same inputs: identical results
    for x, y in zip(a[:2], b[:2]):
        assert np.array_equal(x, y)
    assert a[2] == b[2]
    assert np.array_equal(a[3], b[3])


def test_noalloc_matches_allocated_workspace_twice():
    # a larger problem first, then a smaller one: the second must not see the first's data
    big = wl.cavity(n=20, nj=16, stretch=1.5, nv=12, Kn=0.2)
    small = dict(wl.couette(nj=16, nv=8), precision=wl.FP32_MIXED)
    _check(big, 41)
    _check(small, 42)


def test_noalloc_rejects_oversize_and_second_context():
    from paper_1709_01819_amd import Solver
    from paper_1709_01819_amd.abi import IdugksError
    with pytest.raises(IdugksError) as e:
        Solver(wl.case("cavity_kn0.075"), static_workspace=True)  # about 230 MB of workspace
    assert e.value.code == 2
    g = Solver(wl.couette(nj=8, nv=6), static_workspace=True)
    with pytest.raises(IdugksError) as e:
        Solver(wl.couette(nj=8, nv=6), static_workspace=True)
    assert e.value.code == 6
    g.close()
    h = Solver(wl.couette(nj=8, nv=6), static_workspace=True)  # released by destroy
    h.close()
