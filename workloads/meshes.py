"""Unstructured mesh descriptions (quadrilaterals and triangles) for the workloads.

A mesh is a dict ``{"xn", "yn", "cell_nodes", "side_tag"}`` stored under the key
``"mesh"`` of a case: node coordinates (float64, any count), per cell its four node
indices counter-clockwise with -1 in the fourth slot of a triangle (int32 [nc, 4]),
and per cell side, for sides on the boundary, which of the case's four boundary
conditions applies (0..3, -1 elsewhere; int32 [nc, 4]).  Side s of a cell is the edge
from its node s to the next.  Nothing here evaluates the method.
"""
import numpy as np

from .cases import BC_PERIODIC, cavity

# boundary-condition slot of each wall of a rectangle (the structured side order i-, i+, j-, j+)
_LEFT, _RIGHT, _BOTTOM, _TOP = 0, 1, 2, 3


def _tags(cell_nodes, on_side):
    """side_tag from a function on_side(a, b) -> slot or -1 for the edge between nodes a, b."""
    nc = cell_nodes.shape[0]
    tag = np.full((nc, 4), -1, np.int32)
    for c in range(nc):
        nn = 3 if cell_nodes[c, 3] < 0 else 4
        for s in range(nn):
            tag[c, s] = on_side(cell_nodes[c, s], cell_nodes[c, (s + 1) % nn])
    return tag


def mesh_of(cfg):
    """The structured mesh of a case without periodic sides as an unstructured description
    with the same cells in the same order (cell i + j ni) and the same nodes."""
    if BC_PERIODIC in cfg["bc"]:
        raise ValueError("periodic sides have no unstructured description")
    ni, nj = cfg["ni"], cfg["nj"]
    I, J = np.meshgrid(np.arange(ni), np.arange(nj), indexing="xy")
    I, J = I.ravel(), J.ravel()
    node = lambda i, j: i + j * (ni + 1)  # noqa: E731
    cn = np.stack([node(I, J), node(I + 1, J), node(I + 1, J + 1), node(I, J + 1)], axis=1).astype(np.int32)

    def on_side(a, b):
        ia, ja, ib, jb = a % (ni + 1), a // (ni + 1), b % (ni + 1), b // (ni + 1)
        if ja == jb == 0:
            return _BOTTOM
        if ja == jb == nj:
            return _TOP
        if ia == ib == 0:
            return _LEFT
        if ia == ib == ni:
            return _RIGHT
        return -1

    return dict(xn=np.asarray(cfg["xn"], float).copy(), yn=np.asarray(cfg["yn"], float).copy(),
                cell_nodes=cn, side_tag=_tags(cn, on_side))


def with_mesh(cfg, mesh):
    """A copy of a case on an unstructured mesh."""
    c = dict(cfg)
    for k in ("bc", "wall_u", "wall_v", "wall_T"):
        c[k] = list(cfg[k])
    c["mesh"] = mesh
    return c


def hybrid_square(n, nq, nodes=None, jitter=0.0, seed=0):
    """Hybrid mesh of the unit square: an n x n grid of nodes (uniform, or the given 1D
    node positions), quadrilaterals in the band of nq cells along the four walls and two
    triangles in every other grid cell, split along alternating diagonals.  Cells are
    numbered row by row (a split cell's two triangles consecutively).  jitter > 0 moves
    every node off the boundary by up to jitter times the local spacing in x and y
    (numpy default_rng(1709 + seed)); keep it below 0.25 for valid cells."""
    xs = np.linspace(0.0, 1.0, n + 1) if nodes is None else np.asarray(nodes, float)
    if len(xs) != n + 1:
        raise ValueError("need n + 1 node positions")
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    xn, yn = X.ravel().copy(), Y.ravel().copy()
    if jitter > 0:
        rng = np.random.default_rng(1709 + seed)
        h = np.diff(xs)
        hl = np.minimum(np.r_[h[0], h], np.r_[h, h[-1]])  # smaller adjacent spacing per node
        for j in range(1, n):
            for i in range(1, n):
                k = i + j * (n + 1)
                xn[k] += jitter * hl[i] * rng.uniform(-1.0, 1.0)
                yn[k] += jitter * hl[j] * rng.uniform(-1.0, 1.0)
    node = lambda i, j: i + j * (n + 1)  # noqa: E731
    cells = []
    for j in range(n):
        for i in range(n):
            a, b, c, d = node(i, j), node(i + 1, j), node(i + 1, j + 1), node(i, j + 1)
            if i < nq or j < nq or i >= n - nq or j >= n - nq:
                cells.append((a, b, c, d))
            elif (i + j) % 2 == 0:
                cells.append((a, b, c, -1))
                cells.append((a, c, d, -1))
            else:
                cells.append((a, b, d, -1))
                cells.append((b, c, d, -1))
    cn = np.array(cells, np.int32)

    def on_side(p, q):
        ip, jp, iq, jq = p % (n + 1), p // (n + 1), q % (n + 1), q // (n + 1)
        if jp == jq == 0:
            return _BOTTOM
        if jp == jq == n:
            return _TOP
        if ip == iq == 0:
            return _LEFT
        if ip == iq == n:
            return _RIGHT
        return -1

    return dict(xn=xn, yn=yn, cell_nodes=cn, side_tag=_tags(cn, on_side))


def renumbered(mesh, seed):
    """The same mesh with its cells in a seeded random order (numpy default_rng(1709 +
    seed)); the implicit sweeps then follow that order."""
    rng = np.random.default_rng(1709 + seed)
    perm = rng.permutation(mesh["cell_nodes"].shape[0])
    return dict(xn=mesh["xn"], yn=mesh["yn"], cell_nodes=np.ascontiguousarray(mesh["cell_nodes"][perm]),
                side_tag=np.ascontiguousarray(mesh["side_tag"][perm]))


def hybrid_cavity(n=64, nq=4, nv=28, jitter=0.0, seed=0, **kw):
    """The lid-driven cavity of ``cases.cavity`` (lid on the top wall) on a hybrid
    quadrilateral/triangle mesh of the unit square (``hybrid_square``, uniform nodes)."""
    base = cavity(n=n, stretch=None, nv=nv, **kw)
    return with_mesh(base, hybrid_square(n, nq, jitter=jitter, seed=seed))
