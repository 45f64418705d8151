"""Pins of the oracle's scheme: explicit DUGKS (Section 2.1), IDUGKS (Section 2.2),
boundaries (Section 2.3) and the Couette results of Section 3.1.

Each test checks the oracle against something the paper or mathematics fixes,
never against a retyped copy of the oracle's own formula:
  transforms      phi-bar-plus equals the composition of the Eq. 10 and Eq. 12 definitions
  fixed point     a uniform equilibrium (periodic box; closed cavity at rest) has zero flux
                  residual and is left unchanged by explicit and implicit steps
  geometry/LSQ    closed cell boundaries, total area, least squares exact for linear fields
  LU-SGS          the sweeps equal dense (D+L)^-1 D (D+U)^-1; upwind couplings point upstream
  steady states   implicit = explicit DUGKS on tiny grids, and both = a dense Newton root
  conservation    explicit DUGKS keeps the total mass of a closed cavity
  Couette         symmetry, constant shear stress, mu = tau p in the bulk, linear profile
                  with second-order convergence of its slope (Section 3.1)
"""
import numpy as np
import pytest

import workloads as wl
from oracle import Oracle


def _W(rho, U, V, T, K):
    return np.array([rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V + (K + 2) * 0.5 * T)])


def _perturbed(o, seed, amp=0.1):
    f = o.get_state()
    return f * wl.perturbation(f.shape, seed, amp)


# ---------------------------------------------------------------- transforms (Eq. 10, 12)
def test_barplus_is_composition_of_eq10_and_eq12():
    o = Oracle(wl.cavity(n=5, stretch=1.5, nv=8, Kn=0.05))
    o.set_state(_perturbed(o, 3))
    f = o.get_state()
    mo = o.moments()
    dt, h = o.dt, 0.5 * o.dt
    bp = o.barplus()
    for c in range(o.nc):
        rho, U, V, T, _, _, _, tau = mo[c]
        Ge, He = o.equilibrium(_W(rho, U, V, T, 3))
        for s, fe in ((0, Ge), (1, He)):
            phi = (2 * tau * f[s, c] + dt * fe) / (2 * tau + dt)      # Eq. 10 inverted
            ref = phi + 0.5 * h * (fe - phi) / tau                      # Eq. 12, vartheta=(feq-phi)/tau
            assert np.max(np.abs(bp[s, c] - ref)) <= 1e-14 * np.abs(ref).max()


# ---------------------------------------------------------------- fixed points
@pytest.mark.parametrize("model", [wl.BGK, wl.SHAKHOV])
def test_uniform_flow_in_periodic_box_is_fixed_point(model):
    # Shakhov: the discrete heat flux of a moving Maxwellian is a small quadrature error, so
    # the uniform Shakhov fixed point is only a BGK Maxwellian for a gas at rest (q = 0 by
    # symmetry of the velocity set)
    if model == wl.SHAKHOV:
        cfg = wl.periodic_box(n=5, nv=8, model=model, K=1, U=0.0, V=0.0)
    else:
        cfg = wl.periodic_box(n=5, nv=8, model=model, K=3)
    o = Oracle(cfg)
    f0 = o.get_state()
    scale = np.abs(f0).max()
    M = o.flux()
    assert np.max(np.abs(M)) <= 1e-14 * scale
    o.explicit_step(1)
    assert np.max(np.abs(o.get_state() - f0)) <= 1e-14 * scale
    o.implicit_step(2)
    assert np.max(np.abs(o.get_state() - f0)) <= 1e-14 * scale


@pytest.mark.parametrize("T", [1.0, 1.4])
def test_gas_at_rest_in_closed_cavity_is_fixed_point(T):
    cfg = wl.cavity(n=6, stretch=1.5, nv=10, U=0.0, Kn=0.2)
    cfg["wall_T"] = [T] * 4
    cfg["init_T"] = T
    o = Oracle(cfg)
    f0 = o.get_state()
    scale = np.abs(f0).max()
    assert np.max(np.abs(o.flux())) <= 1e-14 * scale
    o.explicit_step(1)
    assert np.max(np.abs(o.get_state() - f0)) <= 1e-14 * scale
    o.implicit_step(2)
    assert np.max(np.abs(o.get_state() - f0)) <= 1e-14 * scale


# ---------------------------------------------------------------- geometry and Eq. 15
@pytest.mark.parametrize("name", ["cavity", "ogrid", "couette"])
def test_geometry_and_least_squares(name):
    if name == "cavity":
        cfg, area = wl.cavity(n=9, stretch=1.5, nv=4), 1.0
    elif name == "ogrid":
        cfg = wl.cylinder(ni=6, nj=12, rmax=4.0, nv=4, vmax=4.0)
        area = None
    else:
        cfg, area = wl.couette(nj=8, nv=4), 1.0 / 8
    o = Oracle(cfg)
    a, xc, yc = o.cells()
    sd = o.cell_sides()
    # every cell boundary closes: sum_s S n = 0
    cl = np.stack([(sd["S"] * sd["nx"]).sum(1), (sd["S"] * sd["ny"]).sum(1)])
    assert np.abs(cl).max() <= 1e-14
    if area is not None:
        assert abs(a.sum() - area) <= 1e-14
    else:  # O-grid: area between the inscribed polygons of the two boundary circles
        nj, r1 = cfg["nj"], 4.0
        poly = 0.5 * nj * np.sin(2 * np.pi / nj)
        assert abs(a.sum() - poly * (r1 ** 2 - 1.0)) <= 1e-12
    # least squares is exact for linear fields: sum_j a_j d_j^T = I
    nbdx = np.zeros_like(sd["dx"])
    nbdy = np.zeros_like(sd["dy"])
    for c in range(o.nc):
        for s in range(4):
            j = sd["nb"][c, s]
            if j < 0:
                continue
            # neighbour image offset: centroid difference (periodic wrap adds the period)
            dxc, dyc = xc[j] - xc[c], yc[j] - yc[c]
            if name == "couette" and s < 2:
                dxc += (1.0 / 8) * (1 if s == 1 else -1)
            nbdx[c, s], nbdy[c, s] = dxc, dyc
    mask = sd["nb"] >= 0
    I11 = (sd["ax"] * nbdx * mask).sum(1)
    I12 = (sd["ax"] * nbdy * mask).sum(1)
    I21 = (sd["ay"] * nbdx * mask).sum(1)
    I22 = (sd["ay"] * nbdy * mask).sum(1)
    assert np.abs(I11 - 1).max() <= 1e-12 and np.abs(I22 - 1).max() <= 1e-12
    assert np.abs(I12).max() <= 1e-12 and np.abs(I21).max() <= 1e-12


# ---------------------------------------------------------------- LU-SGS (Eq. 26)
@pytest.mark.parametrize("name", ["cavity", "ogrid"])
def test_lusgs_equals_dense_factorisation(name):
    if name == "cavity":
        cfg = wl.cavity(n=4, nj=5, stretch=None, nv=6, Kn=0.1)
    else:
        cfg = wl.cylinder(ni=4, nj=6, rmax=3.0, nv=6, vmax=4.0)
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
                if j < 0 or j == c:
                    continue
                (Lm if j < c else Um)[c, j] -= Cc[c, s]
        r = rng.standard_normal(o.nc)
        ref = np.linalg.solve(Um, np.diag(D) @ np.linalg.solve(Lm, r))
        out = o.micro_sweep(v, r)
        assert np.max(np.abs(out - ref)) <= 1e-13 * np.abs(ref).max()


def test_upwind_couplings_point_upstream():
    o = Oracle(wl.cavity(n=4, stretch=None, nv=6, Kn=0.1))
    o.predict()
    xi, eta, _ = o.velocities()
    sd = o.cell_sides()
    for v in range(o.nv):
        D, Cc = o.micro_operator(v)
        if xi[v] > 0 and eta[v] > 0:
            # all information comes from lower-index (i-1, j-1) cells: the upper sweep is inert
            assert np.all(Cc[:, 1] == 0) and np.all(Cc[:, 3] == 0)
            inner = sd["nb"][:, 0] >= 0
            assert np.allclose(Cc[inner, 0], xi[v] * sd["S"][inner, 0], rtol=1e-15)
            r = np.arange(1.0, o.nc + 1)
            d = r.copy()
            for c in range(o.nc):  # forward substitution by hand
                for s in (0, 2):
                    j = sd["nb"][c, s]
                    if j >= 0:
                        d[c] += Cc[c, s] * d[j]
                d[c] /= D[c]
            assert np.allclose(o.micro_sweep(v, r), d, rtol=1e-14, atol=0)


# ---------------------------------------------------------------- steady states
def _explicit_to_steady(o, max_blocks=400):
    for _ in range(max_blocks):
        if o.explicit_step(500) < 1e-15:
            return
    raise AssertionError("explicit DUGKS did not converge")


@pytest.mark.parametrize("cfg", [wl.cavity(n=6, stretch=None, nv=6, Kn=0.1),
                                 wl.couette(nj=8, nv=8, Kn=0.1)], ids=["cavity", "couette"])
def test_implicit_and_explicit_reach_same_steady_state(cfg):
    a, b = Oracle(cfg), Oracle(cfg)
    it, r, ok = a.solve(1e-14, 5000)
    assert ok
    _explicit_to_steady(b)
    ma, mb = a.moments(), b.moments()
    assert np.max(np.abs(ma[:, :4] - mb[:, :4])) <= 1e-10
    assert np.max(np.abs(a.get_state() - b.get_state())) <= 1e-10 * np.abs(b.get_state()).max()


def test_steady_state_is_newton_root_of_explicit_residual():
    cfg = wl.cavity(n=3, stretch=None, nv=4, Kn=0.1)
    o, imp = Oracle(cfg), Oracle(cfg)
    f0 = o.get_state().ravel().copy()
    a, _, _ = o.cells()
    _, _, w = o.velocities()
    ell = np.zeros_like(f0).reshape(2, o.nc, o.nv)
    ell[0] = a[:, None] * w[None, :]
    ell = ell.ravel()
    M0 = ell @ f0

    def R(f):  # explicit residual up to the positive factor dt/area: step(f) - f
        o.set_state(f)
        o.explicit_step(1)
        return o.get_state().ravel() - f

    f = f0.copy()
    for _ in range(12):
        r = R(f)
        J = np.empty((f.size, f.size))
        for k in range(f.size):
            hk = 1e-7 * max(abs(f[k]), 1e-3)
            e = f.copy()
            e[k] += hk
            J[:, k] = (R(e) - r) / hk
        A = np.vstack([J, ell[None, :]])
        b = np.concatenate([-r, [M0 - ell @ f]])
        f = f + np.linalg.lstsq(A, b, rcond=None)[0]
        if np.abs(R(f)).max() < 1e-16:
            break
    assert np.abs(R(f)).max() < 1e-15
    it, res, ok = imp.solve(1e-14, 5000)
    assert ok
    assert np.max(np.abs(imp.get_state().ravel() - f)) <= 1e-11 * np.abs(f).max()


def test_explicit_dugks_conserves_mass_in_closed_cavity():
    o = Oracle(wl.cavity(n=8, stretch=1.5, nv=8, Kn=0.05))
    o.set_state(_perturbed(o, 7))
    a, _, _ = o.cells()
    m0 = (a * o.moments()[:, 0]).sum()
    for _ in range(5):
        o.explicit_step(1)
        assert abs((a * o.moments()[:, 0]).sum() - m0) <= 1e-14 * m0


# ---------------------------------------------------------------- Couette (Section 3.1)
def _stress(o):
    mo = o.moments()
    f = o.get_state()
    xi, eta, w = o.velocities()
    tau, U, V = mo[:, 7], mo[:, 1], mo[:, 2]
    pxy_t = (w[None, :] * (xi[None, :] - U[:, None]) * (eta[None, :] - V[:, None]) * f[0]).sum(1)
    return mo, 2 * tau / (2 * tau + o.dt) * pxy_t   # stress of phi from that of phi~ (Eq. 10)


def test_couette_symmetry_and_viscosity():
    o = Oracle(wl.case("couette"))
    it, r, ok = o.solve(1e-14, 5000)
    assert ok
    mo, pxy = _stress(o)
    U0 = 0.16 * np.sqrt(0.5)
    rho, U, V, T = mo[:, 0], mo[:, 1], mo[:, 2], mo[:, 3]
    # the sweeps run bottom to top, so only the converged state is symmetric
    assert np.max(np.abs(U + U[::-1])) <= 1e-9 * U0           # u(1-y) = -u(y)
    assert np.max(np.abs(rho - rho[::-1])) <= 1e-10
    assert np.max(np.abs(T - T[::-1])) <= 1e-10
    assert np.max(np.abs(V)) <= 2e-5 * U0                       # no wall-normal flow (cell moments)
    assert np.ptp(pxy[8:-8]) <= 1e-3 * abs(pxy.mean())          # constant shear in the bulk
    _, xc, yc = o.cells()
    dudy = np.gradient(U, yc)
    mu = mo[:, 7] * mo[:, 4]                                     # mu = tau p
    ratio = -pxy / dudy / mu
    assert np.all(np.abs(ratio[16:-16] - 1.0) <= 0.02)


def test_couette_near_continuum_linear_profile_second_order():
    U0 = 0.16 * np.sqrt(0.5)
    slopes = []
    for n in (16, 32, 64, 128):
        o = Oracle(wl.couette(nj=n, nv=8, Kn=0.01, cfl_imp=1000.0))
        it, r, ok = o.solve(1e-12, 20000)
        assert ok
        mo = o.moments()
        _, _, yc = o.cells()
        U = mo[:, 1]
        mid = (yc > 0.25) & (yc < 0.75)
        A = np.vstack([yc[mid] - 0.5, np.ones(mid.sum())]).T
        coef = np.linalg.lstsq(A, U[mid], rcond=None)[0]
        assert np.max(np.abs(U[mid] - A @ coef)) <= 1e-4 * U0    # linear bulk profile
        assert abs(coef[1]) <= 1e-6 * U0                         # centred on u = 0
        # slope within the wall-slip correction of the analytic 2U (slip ~ Kn)
        assert abs(coef[0] / (2 * U0) - 1.0) <= 3 * 0.01 * 2
        slopes.append(coef[0])
    s = np.array(slopes)
    order = np.log2((s[:-2] - s[1:-1]) / (s[1:-1] - s[2:]))
    assert np.all(order > 1.7) and np.all(order < 2.3)


def test_cfl_ramp_scales_the_implicit_time_step():
    """Start-up ramp of the implicit CFL: implicit iteration n takes min(cfl_imp,
    cfl_start g^n).  The implicit time step (Eq. 30) is proportional to the CFL, so on one
    state the ramped and the plain problem's dt_imp differ by exactly that ratio; the ramp
    saturates at cfl_imp, and set_state restarts it.  A ramp that is off, or that starts at
    cfl_imp, leaves the iteration unchanged."""
    base = wl.cavity(n=6, stretch=1.5, nv=6, Kn=0.075)
    cfl = base["cfl_imp"]
    a, b = Oracle(dict(base, cfl_start=2.0, cfl_growth=3.0)), Oracle(base)
    f = a.get_state()
    f = f * wl.perturbation(f.shape, 21, 0.05)
    a.set_state(f)
    done = 0
    for n, expect in ((0, 2.0), (2, 18.0), (5, 486.0), (7, cfl)):
        a.implicit_step(n - done) if n > done else None
        done = n
        b.set_state(a.get_state())
        ratio = a.predict()[1] / b.predict()[1]
        np.testing.assert_allclose(ratio, expect / cfl, rtol=1e-14)
    a.set_state(a.get_state())
    np.testing.assert_allclose(a.predict()[1] / b.predict()[1], 2.0 / cfl, rtol=1e-14)
    # saturated from the start: the same iterates as no ramp
    c = Oracle(dict(base, cfl_start=cfl, cfl_growth=1.0))
    c.set_state(f)
    b.set_state(f)
    assert c.implicit_step(3) == b.implicit_step(3)
    assert np.array_equal(c.get_state(), b.get_state())
