"""Workload definitions: structured meshes and physical parameters of the test cases.

Every case is a plain dict whose keys mirror the fields of the solver
configuration (``idugks_config`` in ``include/idugks.h``; the oracle has its own
struct with the same meaning).  Node coordinates are float64 arrays of length
``(ni+1)*(nj+1)`` with node ``(i, j)`` stored at ``i + j*(ni+1)``.

Units (the paper fixes none): gas constant R = 1/2, reference temperature 1 and
reference density 1, so the most probable speed sqrt(2RT) is 1 at the
reference state and temperature T equals 2RT.

The case shapes follow the paper's workloads (Couette flow, lid-driven cavity
at several Knudsen numbers, hypersonic cylinder; Section 3) at the sizes the
benchmark and the tests use.  Nothing here evaluates the method.
"""
import math

import numpy as np

BC_WALL, BC_FARFIELD, BC_PERIODIC = 0, 1, 2
GAUSS_HERMITE, NEWTON_COTES = 0, 1
BGK, SHAKHOV = 0, 1
FP64, FP32_MIXED = 0, 1
EXPLICIT, IMPLICIT = 0, 1
SWEEPS_AUTO, SWEEPS_LEVELS, SWEEPS_HYPERPLANES = 0, 1, 2

OMEGA_VHS = 0.81        # viscosity exponent mu ~ T^omega used by every case


def uniform_nodes(n, a=0.0, b=1.0):
    return np.linspace(a, b, n + 1)


def tanh_nodes(n, beta):
    """Wall-clustered nodes on [0, 1]: x_i = (1 + tanh(beta(2i/n - 1))/tanh(beta))/2."""
    s = 2.0 * np.arange(n + 1) / n - 1.0
    x = 0.5 * (1.0 + np.tanh(beta * s) / math.tanh(beta))
    x[0], x[-1] = 0.0, 1.0
    return x


def cartesian_mesh(xs, ys):
    """Tensor-product nodes; returns (ni, nj, xn, yn)."""
    ni, nj = len(xs) - 1, len(ys) - 1
    X, Y = np.meshgrid(np.asarray(xs, float), np.asarray(ys, float), indexing="xy")
    return ni, nj, np.ascontiguousarray(X.ravel()), np.ascontiguousarray(Y.ravel())


def ogrid_mesh(ni, nj, rmax):
    """O-grid around the unit circle: r_i = rmax^(i/ni), theta_j = 2 pi j / nj.

    i runs radially outward, j counter-clockwise; the j = nj ring of nodes
    repeats j = 0 exactly so that the mesh closes on itself.
    """
    r = rmax ** (np.arange(ni + 1) / ni)
    r[0], r[-1] = 1.0, float(rmax)
    th = 2.0 * math.pi * np.arange(nj + 1) / nj
    c, s = np.cos(th), np.sin(th)
    c[-1], s[-1] = c[0], s[0]
    X = c[:, None] * r[None, :]
    Y = s[:, None] * r[None, :]
    return ni, nj, np.ascontiguousarray(X.ravel()), np.ascontiguousarray(Y.ravel())


def _base(ni, nj, xn, yn, bc):
    return dict(
        ni=ni, nj=nj, xn=xn, yn=yn, bc=list(bc),
        wall_u=[0.0] * 4, wall_v=[0.0] * 4, wall_T=[1.0] * 4,
        far_rho=1.0, far_u=0.0, far_v=0.0, far_T=1.0,
        quad=GAUSS_HERMITE, nvx=16, nvy=16, vmax=0.0,
        model=BGK, Kn=0.1, Pr=1.0, omega=OMEGA_VHS, K=3,
        cfl_phys=0.5, cfl_imp=100.0, limiter=0, precision=FP64,
        init_rho=1.0, init_u=0.0, init_v=0.0, init_T=1.0,
    )


def couette(nj=64, nv=16, Kn=0.1, U=0.16 * math.sqrt(0.5), cfl_imp=100.0, model=BGK,
            Pr=1.0, K=3, quad=GAUSS_HERMITE, vmax=0.0):
    """Planar Couette flow: one cell across x (periodic), walls at y = 0 and y = 1.

    The bottom wall moves with -U, the top wall with +U, both at T = 1.
    """
    ni, nj_, xn, yn = cartesian_mesh([0.0, 1.0 / nj], uniform_nodes(nj))
    c = _base(ni, nj_, xn, yn, [BC_PERIODIC, BC_PERIODIC, BC_WALL, BC_WALL])
    c["wall_u"][2], c["wall_u"][3] = -U, U
    c.update(nvx=nv, nvy=nv, Kn=Kn, cfl_imp=cfl_imp, model=model, Pr=Pr, K=K, quad=quad,
             vmax=vmax)
    return c


def cavity(n=64, stretch=1.5, nv=28, quad=GAUSS_HERMITE, vmax=0.0, Kn=0.075, U=0.16,
           model=BGK, Pr=1.0, K=3, cfl_imp=1000.0, precision=FP64, nj=None):
    """Lid-driven square cavity [0,1]^2; the lid (j+ side) moves with +U, all walls at T = 1.

    ``stretch`` is the tanh clustering parameter (None for a uniform mesh).
    """
    nj = n if nj is None else nj
    xs = uniform_nodes(n) if stretch is None else tanh_nodes(n, stretch)
    ys = uniform_nodes(nj) if stretch is None else tanh_nodes(nj, stretch)
    ni, nj_, xn, yn = cartesian_mesh(xs, ys)
    c = _base(ni, nj_, xn, yn, [BC_WALL] * 4)
    c["wall_u"][3] = U
    c.update(nvx=nv, nvy=nv, quad=quad, vmax=vmax, Kn=Kn, model=model, Pr=Pr, K=K,
             cfl_imp=cfl_imp, precision=precision)
    return c


VMAX_RE = 2.5 * math.sqrt(1.5)   # [-2.5, 2.5] at RT = 1/3, rescaled to RT = 1/2


def cavity_re(Re=1000.0, n=256, nv=25, vmax=VMAX_RE, Ma=0.1 * math.sqrt(3.0), K=3,
              cfl_imp=1000.0, precision=FP64):
    """The continuum lid-driven cavity of the paper's Section 3.2: a uniform n^2 mesh and
    nv^2 velocities spaced uniformly on [-vmax, vmax]^2 (Newton-Cotes).

    The lid speed is U = Ma sqrt(gamma R T) at T = 1 (gamma = (K+4)/(K+2)) and the
    Reynolds number is U L / mu with mu = Kn / sqrt(pi) at T = 1, the solvers' reading of
    Eq. 37 (rho = L = 2RT = 1), so Kn = U sqrt(pi) / Re.  The paper's velocity range
    [-2.5, 2.5] is read at RT = 1/3 (the usual unit of its continuum examples) and mapped to
    this module's RT = 1/2 at the same extent in thermal speeds; its 9 points per direction
    do not resolve the viscous stress here, and on the 256^2 mesh 17 points leave the
    primary vortex's vorticity 5% low while 25 points meet Table 1 (measured).
    """
    gam = (K + 4.0) / (K + 2.0)
    U = Ma * math.sqrt(gam * 0.5)
    Kn = U * math.sqrt(math.pi) / Re
    return cavity(n=n, stretch=None, nv=nv, quad=NEWTON_COTES, vmax=vmax, Kn=Kn, U=U, K=K,
                  cfl_imp=cfl_imp, precision=precision)


def cylinder(ni=96, nj=160, rmax=15.0, nv=100, vmax=15.0, Kn=0.1, Ma=5.0, cfl_imp=50.0,
             precision=FP32_MIXED, limiter=1):
    """Monatomic (K = 1) Shakhov flow past the unit-radius cylinder, free stream along +x.

    The sound speed is sqrt(gamma R T) with gamma = 5/3 and RT = 1/2 at T = 1.
    """
    ni_, nj_, xn, yn = ogrid_mesh(ni, nj, rmax)
    c = _base(ni_, nj_, xn, yn, [BC_WALL, BC_FARFIELD, BC_PERIODIC, BC_PERIODIC])
    u_inf = Ma * math.sqrt(5.0 / 3.0 * 0.5)
    c.update(far_rho=1.0, far_u=u_inf, far_v=0.0, far_T=1.0,
             init_rho=1.0, init_u=u_inf, init_v=0.0, init_T=1.0,
             quad=NEWTON_COTES, nvx=nv, nvy=nv, vmax=vmax, model=SHAKHOV, Pr=2.0 / 3.0, K=1,
             Kn=Kn, cfl_imp=cfl_imp, precision=precision, limiter=limiter)
    return c


def periodic_box(n=6, nv=6, U=0.1, V=-0.05, T=1.2, rho=1.1, Kn=0.1, model=BGK, K=3):
    """Fully periodic square box holding a uniform (moving) gas; used for fixed-point checks."""
    ni, nj, xn, yn = cartesian_mesh(uniform_nodes(n), uniform_nodes(n))
    c = _base(ni, nj, xn, yn, [BC_PERIODIC] * 4)
    Pr = 2.0 / 3.0 if model == SHAKHOV else 1.0
    c.update(nvx=nv, nvy=nv, Kn=Kn, model=model, Pr=Pr, K=K,
             init_rho=rho, init_u=U, init_v=V, init_T=T)
    return c


def _c1():
    return couette(nj=64, nv=16, Kn=0.1, cfl_imp=100.0)


def _c2(precision=FP64):
    return cavity(n=64, stretch=1.5, nv=28, Kn=0.075, cfl_imp=1000.0, precision=precision)


def _c3(precision=FP32_MIXED):
    # the paper's CFL of 1000 is stable for this case up to a 64^2 mesh (its own has 60^2
    # cells); on 96^2 and 128^2 the second-order residual against the first-order implicit
    # operator diverges there, so the 128^2 workload runs at 100
    return cavity(n=128, stretch=None, nv=101, quad=NEWTON_COTES, vmax=4.0, Kn=10.0,
                  model=SHAKHOV, Pr=2.0 / 3.0, K=1, cfl_imp=100.0, precision=precision)


def _c4(precision=FP32_MIXED):
    # started impulsively at CFL 50 the wake goes to negative densities within two
    # iterations; the CFL ramps up from 0.5 by 2% per implicit iteration (reaching 50
    # after 233)
    return dict(cylinder(precision=precision), cfl_start=0.5, cfl_growth=1.02)


def _c5():
    return cavity(n=64, stretch=1.5, nv=28, Kn=1.0, cfl_imp=1000.0)


def _c6(precision=FP64):
    return cavity_re(Re=1000.0, n=256, nv=25, vmax=VMAX_RE, precision=precision)


def _c7(precision=FP32_MIXED):
    # the Kn 10 cavity on a hybrid mesh of the same 129^2 nodes: quadrilaterals in a band of
    # 8 cells along the walls, two triangles in every other grid cell (28928 cells).  On
    # this mesh the implicit iteration is stable only up to an implicit CFL of about 5 (at
    # 10 and above it diverges within a few hundred iterations, with the second-order
    # residual; with the first-order one it converges at 100)
    from .meshes import hybrid_square, with_mesh
    return dict(with_mesh(_c3(precision), hybrid_square(128, 8)), cfl_imp=5.0)


_CASES = {
    "couette": _c1,           # Couette flow, 64 cells, GH 16x16, Kn = 0.1
    "cavity_kn0.075": _c2,    # cavity 64^2 tanh, GH 28x28, Kn = 0.075
    "cavity_kn10": _c3,       # cavity 128^2, NC 101x101 on [-4,4]^2, Shakhov, Kn = 10, CFL 100
    "cylinder_ma5": _c4,      # O-grid 96x160, NC 100x100 on [-15,15]^2, Shakhov, Ma = 5
    "cavity_kn1": _c5,        # cavity 64^2 tanh, GH 28x28, Kn = 1 (sensitivities)
    "cavity_re1000": _c6,     # cavity 256^2 uniform, NC 25x25 on +-2.5 sqrt(3/2), Re = 1000
    "cavity_kn10_hybrid": _c7,  # cavity_kn10 on a hybrid quad/triangle mesh, 28928 cells, CFL 5
}
CASE_NAMES = tuple(_CASES)


def case(name, **kw):
    """Return the configuration dict of a named workload."""
    return _CASES[name](**kw)


def shrink(cfg, ni=None, nj=None, nv=None):
    """A smaller copy of a case with the same physics (same mesh family and boundaries).

    The mesh is rebuilt with the requested cell counts; the velocity grid keeps its
    quadrature family and range with ``nv`` points per direction.
    """
    c = dict(cfg)
    c["bc"] = list(cfg["bc"])
    for k in ("wall_u", "wall_v", "wall_T"):
        c[k] = list(cfg[k])
    ni = cfg["ni"] if ni is None else ni
    nj = cfg["nj"] if nj is None else nj
    if cfg["bc"][2] == BC_PERIODIC and cfg["bc"][0] == BC_WALL and cfg["bc"][1] == BC_FARFIELD:
        rmax = float(np.hypot(cfg["xn"][cfg["ni"]], cfg["yn"][cfg["ni"]]))
        _, _, xn, yn = ogrid_mesh(ni, nj, rmax)
    elif cfg["ni"] == 1 and cfg["bc"][0] == BC_PERIODIC:
        _, _, xn, yn = cartesian_mesh([0.0, 1.0 / nj], uniform_nodes(nj))
        ni = 1
    else:
        xs_old = cfg["xn"][: cfg["ni"] + 1]
        stretched = not np.allclose(np.diff(xs_old), np.diff(xs_old)[0])
        if stretched:
            beta = 1.5
            _, _, xn, yn = cartesian_mesh(tanh_nodes(ni, beta), tanh_nodes(nj, beta))
        else:
            _, _, xn, yn = cartesian_mesh(uniform_nodes(ni), uniform_nodes(nj))
    c.update(ni=ni, nj=nj, xn=xn, yn=yn)
    if nv is not None:
        c.update(nvx=nv, nvy=nv)
    return c


def perturbation(shape, seed, amp=0.1):
    """Seeded multiplicative noise 1 + amp*U(-1, 1) (numpy default_rng(1709 + seed))."""
    rng = np.random.default_rng(1709 + seed)
    return 1.0 + amp * rng.uniform(-1.0, 1.0, size=shape)
