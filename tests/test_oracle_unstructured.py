"""Pins of the oracle on unstructured meshes of quadrilaterals and triangles.

The finite-volume form (Section 2.1) sums each cell's fluxes over its faces, whatever the
cell's shape; the implicit sweeps (Eq. 24-26, 29-31) take the cells in index order.  On
hybrid meshes with jittered nodes the oracle must keep what the mathematics fixes:

  same mesh, two descriptions   a structured mesh given as an unstructured one gives the
                                same iterations (only the side order of the sums differs)
  geometry / least squares      closed cell boundaries, total area, neighbour symmetry, the
                                least-squares gradient exact for linear fields (Eq. 15)
  fixed points                  gas at rest in a closed box; a uniform free stream
  conservation                  explicit DUGKS keeps the total mass of a closed cavity
  LU-SGS                        the micro sweeps equal the dense (D+L)^-1 D (D+U)^-1 of
                                the upwind operator, in any cell order
  steady state                  the implicit fixed point is the explicit steady state and
                                does not depend on the cell order of the sweeps
  discretisation                the hybrid-mesh cavity flow is close to the structured one
"""
import numpy as np
import pytest

import workloads as wl
from oracle import Oracle


def _perturbed(o, seed, amp=0.1):
    f = o.get_state()
    return f * wl.perturbation(f.shape, seed, amp)


def _hybrid(n=6, nq=1, nv=6, jitter=0.15, seed=0, **kw):
    return wl.hybrid_cavity(n=n, nq=nq, nv=nv, jitter=jitter, seed=seed, **kw)


def _farfield(cfg, rho=1.1, U=0.3, V=-0.2, T=1.2):
    c = dict(cfg)
    c.update(bc=[wl.BC_FARFIELD] * 4, far_rho=rho, far_u=U, far_v=V, far_T=T,
             init_rho=rho, init_u=U, init_v=V, init_T=T)
    return c


# ------------------------------------------------------------ the same mesh, two descriptions
@pytest.mark.parametrize("name", ["bgk_stretched", "shakhov_nc_limiter"])
def test_structured_mesh_as_unstructured_gives_the_same_iterations(name):
    if name == "bgk_stretched":
        cfg = wl.cavity(n=7, nj=6, stretch=1.5, nv=8, Kn=0.1)
    else:
        cfg = dict(wl.shrink(wl.case("cavity_kn10"), ni=7, nj=6, nv=9), precision=wl.FP64, limiter=1)
    a = Oracle(cfg)
    b = Oracle(wl.with_mesh(cfg, wl.mesh_of(cfg)))
    assert (a.nc, a.nv, a.dt) == (b.nc, b.nv, b.dt)
    f0 = _perturbed(a, 11, 0.05)
    a.set_state(f0)
    b.set_state(f0)
    scale = np.abs(f0).max()
    for mode in ("implicit", "implicit", "explicit", "implicit"):
        ra = getattr(a, mode + "_step")(1)
        rb = getattr(b, mode + "_step")(1)
        assert abs(ra - rb) <= 1e-12 * abs(ra)
        assert np.max(np.abs(a.get_state() - b.get_state())) <= 1e-13 * scale


# ------------------------------------------------------------ geometry and Eq. 15
@pytest.mark.parametrize("order", ["rows", "random"])
def test_hybrid_geometry_and_least_squares(order):
    cfg = _hybrid(n=8, nq=2, nv=4, jitter=0.2, seed=2)
    if order == "random":
        cfg = wl.with_mesh(cfg, wl.renumbered(cfg["mesh"], 5))
    o = Oracle(cfg)
    cn = cfg["mesh"]["cell_nodes"]
    ntri = int((cn[:, 3] < 0).sum())
    assert ntri == 2 * (8 - 4) ** 2 and o.nc == 8 * 8 - (8 - 4) ** 2 + ntri
    a, xc, yc = o.cells()
    sd = o.cell_sides()
    assert abs(a.sum() - 1.0) <= 1e-14
    cl = np.stack([(sd["S"] * sd["nx"]).sum(1), (sd["S"] * sd["ny"]).sum(1)])
    assert np.abs(cl).max() <= 1e-15
    assert np.all(sd["S"][cn[:, 3] < 0, 3] == 0.0)  # the absent side of a triangle
    for c in range(o.nc):
        for s in range(4):
            j = sd["nb"][c, s]
            if j >= 0:  # the neighbour sees this cell through a side of opposite normal
                t = list(sd["nb"][j]).index(c)
                assert sd["nx"][j, t] == -sd["nx"][c, s] and sd["ny"][j, t] == -sd["ny"][c, s]
                assert sd["S"][j, t] == sd["S"][c, s]
    nbdx = np.where(sd["nb"] >= 0, xc[sd["nb"]] - xc[:, None], 0.0)
    nbdy = np.where(sd["nb"] >= 0, yc[sd["nb"]] - yc[:, None], 0.0)
    I11, I12 = (sd["ax"] * nbdx).sum(1), (sd["ax"] * nbdy).sum(1)
    I21, I22 = (sd["ay"] * nbdx).sum(1), (sd["ay"] * nbdy).sum(1)
    assert np.abs(I11 - 1).max() <= 1e-12 and np.abs(I22 - 1).max() <= 1e-12
    assert np.abs(I12).max() <= 1e-12 and np.abs(I21).max() <= 1e-12
    # the oracle's own gradient of a linear field on the jittered hybrid mesh
    phi = 0.3 + 1.7 * xc - 0.9 * yc
    gx, gy = o.lsq_gradient(phi, 0)
    assert np.abs(gx - 1.7).max() <= 1e-12 and np.abs(gy + 0.9).max() <= 1e-12


# ------------------------------------------------------------ fixed points
@pytest.mark.parametrize("model", [wl.BGK, wl.SHAKHOV])
def test_hybrid_gas_at_rest_is_a_fixed_point(model):
    kw = dict(model=model, K=1, Pr=2.0 / 3.0) if model == wl.SHAKHOV else {}
    cfg = _hybrid(n=6, nq=1, nv=8, U=0.0, Kn=0.2, **kw)
    cfg["wall_T"] = [1.3] * 4
    cfg["init_T"] = 1.3
    o = Oracle(cfg)
    f0 = o.get_state()
    scale = np.abs(f0).max()
    assert np.max(np.abs(o.flux())) <= 1e-14 * scale
    o.explicit_step(1)
    assert np.max(np.abs(o.get_state() - f0)) <= 1e-14 * scale
    o.implicit_step(2)
    assert np.max(np.abs(o.get_state() - f0)) <= 1e-14 * scale


@pytest.mark.parametrize("limiter", [0, 1])
def test_hybrid_uniform_free_stream_is_a_fixed_point(limiter):
    o = Oracle(dict(_farfield(_hybrid(n=6, nq=1, nv=8, jitter=0.2)), limiter=limiter))
    f0 = o.get_state()
    scale = np.abs(f0).max()
    assert np.max(np.abs(o.flux())) <= 1e-14 * scale
    o.implicit_step(3)
    assert np.max(np.abs(o.get_state() - f0)) <= 1e-14 * scale
    o.explicit_step(2)
    assert np.max(np.abs(o.get_state() - f0)) <= 1e-14 * scale


def test_hybrid_explicit_dugks_conserves_mass_in_closed_cavity():
    o = Oracle(_hybrid(n=8, nq=2, nv=8, jitter=0.2, Kn=0.05))
    o.set_state(_perturbed(o, 7))
    a, _, _ = o.cells()
    m0 = (a * o.moments()[:, 0]).sum()
    for _ in range(5):
        o.explicit_step(1)
        assert abs((a * o.moments()[:, 0]).sum() - m0) <= 1e-14 * m0


# ------------------------------------------------------------ LU-SGS (Eq. 26)
@pytest.mark.parametrize("order", ["rows", "random"])
def test_hybrid_lusgs_equals_dense_factorisation(order):
    cfg = _hybrid(n=5, nq=1, nv=6, jitter=0.2, Kn=0.1)
    if order == "random":
        cfg = wl.with_mesh(cfg, wl.renumbered(cfg["mesh"], 1))
    o = Oracle(cfg)
    o.set_state(_perturbed(o, 1, 0.02))
    o.predict()
    sd = o.cell_sides()
    rng = np.random.default_rng(1709)
    for v in range(0, o.nv, 5):
        D, Cc = o.micro_operator(v)
        Lm = np.diag(D)
        Um = np.diag(D)
        for c in range(o.nc):
            for s in range(4):
                j = sd["nb"][c, s]
                if j < 0:
                    continue
                (Lm if j < c else Um)[c, j] -= Cc[c, s]
        r = rng.standard_normal(o.nc)
        ref = np.linalg.solve(Um, np.diag(D) @ np.linalg.solve(Lm, r))
        out = o.micro_sweep(v, r)
        assert np.max(np.abs(out - ref)) <= 1e-13 * np.abs(ref).max()


# ------------------------------------------------------------ steady states
def test_hybrid_implicit_fixed_point_is_the_explicit_steady_state():
    cfg = _hybrid(n=5, nq=1, nv=6, jitter=0.15, Kn=0.1)
    a, b = Oracle(cfg), Oracle(cfg)
    it, r, ok = a.solve(1e-14, 5000)
    assert ok
    for _ in range(400):
        if b.explicit_step(500) < 1e-15:
            break
    else:
        raise AssertionError("explicit DUGKS did not converge")
    assert np.max(np.abs(a.get_state() - b.get_state())) <= 1e-10 * np.abs(b.get_state()).max()


def test_hybrid_steady_state_does_not_depend_on_the_sweep_order():
    cfg = _hybrid(n=8, nq=2, nv=8, jitter=0.15, Kn=0.1)
    m = cfg["mesh"]
    rng = np.random.default_rng(1709 + 4)
    perm = rng.permutation(len(m["cell_nodes"]))
    cr = wl.with_mesh(cfg, dict(xn=m["xn"], yn=m["yn"], cell_nodes=m["cell_nodes"][perm],
                                side_tag=m["side_tag"][perm]))
    a, b = Oracle(cfg), Oracle(cr)
    ia, _, oka = a.solve(1e-13, 5000)
    ib, _, okb = b.solve(1e-13, 5000)
    assert oka and okb
    assert ia != ib  # the orders differ, so do the iterations on the way
    ma, mb = a.moments()[perm], b.moments()
    assert np.max(np.abs(ma[:, :4] - mb[:, :4])) <= 1e-9


def test_hybrid_cavity_flow_is_close_to_the_structured_one():
    """The same cavity (Kn 0.075, lid speed 0.16) on a uniform 16^2 mesh and on the hybrid
    mesh of the same nodes with triangles inside: the discretisations differ by a few
    percent of the lid speed at most."""
    kw = dict(n=16, nv=12, Kn=0.075, U=0.16)
    s = Oracle(wl.cavity(stretch=None, **kw))
    h = Oracle(wl.hybrid_cavity(nq=3, **kw))
    assert s.solve(1e-9, 5000)[2] and h.solve(1e-9, 5000)[2]
    _, xs, ys = s.cells()
    _, xh, yh = h.cells()
    ms, mh = s.moments(), h.moments()
    # velocity at the cavity's centre from the cells nearest to it (linear fit)
    def centre(x, y, m):
        k = np.argsort((x - 0.5) ** 2 + (y - 0.5) ** 2)[:8]
        A = np.stack([np.ones(8), x[k] - 0.5, y[k] - 0.5], 1)
        return [np.linalg.lstsq(A, m[k, q], rcond=None)[0][0] for q in (1, 2)]
    us, uh = centre(xs, ys, ms), centre(xh, yh, mh)
    assert abs(us[0]) > 0.01  # the vortex is there
    assert max(abs(us[0] - uh[0]), abs(us[1] - uh[1])) <= 0.05 * 0.16
