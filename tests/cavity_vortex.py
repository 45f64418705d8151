"""Vortex centres of a lid-driven cavity solution (test helper, not part of the solver).

The quantities of the paper's Table 1 (Section 3.2): the stream function psi at the centre
of the primary vortex and of the two bottom-corner secondary vortices, the centres' x and
y, and the vorticity at the primary centre, all in units of the lid speed and the cavity
side.  Velocities are cell averages on a uniform ni x nj mesh of [0, 1]^2.

psi follows u = d psi / dy with psi = 0 on the bottom wall: at a cell centre it is the
midpoint-rule integral of u from the wall up the cell's column.  A centre is the
extremum of psi over the cells of a region, refined by the stationary point of the
quadratic through its 3 x 3 neighbourhood; the vorticity dv/dx - du/dy (central
differences at the cell centres) is interpolated bilinearly to it.
"""
import numpy as np


def stream_function(u, h):
    """psi[j, i] at the cell centres from u[j, i] (rows j bottom to top), cell height h."""
    return h * (np.cumsum(u, axis=0) - 0.5 * u)


def vorticity(u, v, h):
    """dv/dx - du/dy at the interior cell centres (NaN on the border rows and columns)."""
    w = np.full(u.shape, np.nan)
    w[1:-1, 1:-1] = ((v[1:-1, 2:] - v[1:-1, :-2]) - (u[2:, 1:-1] - u[:-2, 1:-1])) / (2.0 * h)
    return w


def refine(f, j, i, h):
    """Stationary point of the quadratic through f[j-1:j+2, i-1:i+2] (centre cell (j, i)):
    returns (x offset, y offset, value) in units of length."""
    fx = (f[j, i + 1] - f[j, i - 1]) / (2 * h)
    fy = (f[j + 1, i] - f[j - 1, i]) / (2 * h)
    fxx = (f[j, i + 1] - 2 * f[j, i] + f[j, i - 1]) / h ** 2
    fyy = (f[j + 1, i] - 2 * f[j, i] + f[j - 1, i]) / h ** 2
    fxy = (f[j + 1, i + 1] - f[j - 1, i + 1] - f[j + 1, i - 1] + f[j - 1, i - 1]) / (4 * h ** 2)
    H = np.array([[fxx, fxy], [fxy, fyy]])
    d = -np.linalg.solve(H, np.array([fx, fy]))
    d = np.clip(d, -h, h)
    return d[0], d[1], f[j, i] + 0.5 * (fx * d[0] + fy * d[1])


def bilinear(f, x, y, h):
    """f at (x, y) from its values at the cell centres ((i + 1/2) h, (j + 1/2) h)."""
    gx, gy = x / h - 0.5, y / h - 0.5
    i0, j0 = int(np.floor(gx)), int(np.floor(gy))
    tx, ty = gx - i0, gy - j0
    return ((1 - tx) * (1 - ty) * f[j0, i0] + tx * (1 - ty) * f[j0, i0 + 1] +
            (1 - tx) * ty * f[j0 + 1, i0] + tx * ty * f[j0 + 1, i0 + 1])


def centre(psi, h, sign, xr, yr):
    """Extremum (sign -1: minimum, +1: maximum) of psi over the cells whose centres lie in
    xr x yr, refined: returns (psi, x, y)."""
    n_j, n_i = psi.shape
    xc = (np.arange(n_i) + 0.5) * h
    yc = (np.arange(n_j) + 0.5) * h
    mi = (xc >= xr[0]) & (xc <= xr[1])
    mj = (yc >= yr[0]) & (yc <= yr[1])
    sub = np.where(mj[:, None] & mi[None, :], sign * psi, -np.inf)
    j, i = np.unravel_index(np.argmax(sub), sub.shape)
    j = min(max(j, 1), n_j - 2)
    i = min(max(i, 1), n_i - 2)
    dx, dy, val = refine(sign * psi, j, i, h)
    return sign * val, xc[i] + dx, yc[j] + dy


def vortex_metrics(U, V, ni, nj, u_lid):
    """Table 1 quantities from cell velocities U, V (arrays of ni * nj, cell i + j ni) of a
    uniform mesh of [0, 1]^2 with ni = nj."""
    assert ni == nj
    h = 1.0 / ni
    u = np.asarray(U, float).reshape(nj, ni) / u_lid
    v = np.asarray(V, float).reshape(nj, ni) / u_lid
    psi = stream_function(u, h)
    w = vorticity(u, v, h)
    p_psi, p_x, p_y = centre(psi, h, -1, (0.2, 0.8), (0.2, 0.8))
    l_psi, l_x, l_y = centre(psi, h, +1, (0.0, 0.3), (0.0, 0.3))
    r_psi, r_x, r_y = centre(psi, h, +1, (0.6, 1.0), (0.0, 0.4))
    return {
        "primary_omega": abs(bilinear(w, p_x, p_y, h)), "primary_psi": p_psi,
        "primary_x": p_x, "primary_y": p_y,
        "left_psi_e4": 1e4 * l_psi, "left_x": l_x, "left_y": l_y,
        "right_psi_e3": 1e3 * r_psi, "right_x": r_x, "right_y": r_y,
    }


def load_golden(path):
    """name -> value from a whitespace table with # comments."""
    out = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            out[k] = float(v)
    return out
