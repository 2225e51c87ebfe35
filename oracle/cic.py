"""Cloud-in-cell mass assignment and interpolation (test infrastructure only).

The particle-mesh solver of the paper (JaxPM / FastPM, section 2.2.1 item 2)
paints particles to a mesh with the CIC kernel and reads the force back with
the same kernel; the likelihood bins galaxies with CIC as well (section
2.2.2).  The paper gives no node convention; the reading used here puts mesh
node c at position c * cell (no half-cell offset), with periodic wrapping.

For a particle at position x (never wrapped; the wrap happens on the node
index) and u = x / cell, each axis has i0 = floor(u), t = u - i0 and weights
(1 - t) on node i0 mod n and t on node (i0 + 1) mod n.  W(x - c) is the
product of the three axis weights.  Its gradient along axis a is
(+-1 / cell) times the other two weights (+ for the upper node).

Positions are (3, P) arrays; meshes are (n, n, n) arrays.
"""
import itertools

import numpy as np

__all__ = ["paint", "readout", "readout_gradient", "paint_jvp", "readout_jvp"]

_CORNERS = list(itertools.product((0, 1), repeat=3))


def _stencil(pos, n, cell):
    u = np.asarray(pos, dtype=np.float64) / cell
    i0 = np.floor(u).astype(np.int64)
    return i0, u - i0


def _corner(i0, t, n, offs):
    """Flat node index and per-axis weights and weight slopes of one corner."""
    idx = np.zeros(i0.shape[1], dtype=np.int64)
    w, dw = [], []
    for a, o in enumerate(offs):
        idx = idx * n + (i0[a] + o) % n
        w.append(t[a] if o else 1.0 - t[a])
        dw.append(1.0 if o else -1.0)
    return idx, w, dw


def paint(pos, n, cell, weight=None):
    """rho(c) = sum_n weight_n W(x_n - c)  (weight 1 if None)."""
    i0, t = _stencil(pos, n, cell)
    rho = np.zeros(n ** 3)
    for offs in _CORNERS:
        idx, w, _ = _corner(i0, t, n, offs)
        wt = w[0] * w[1] * w[2]
        if weight is not None:
            wt = wt * weight
        rho += np.bincount(idx, weights=wt, minlength=n ** 3)
    return rho.reshape(n, n, n)


def readout(pos, mesh, cell):
    """value_n = sum_c W(x_n - c) mesh(c)."""
    n = mesh.shape[0]
    i0, t = _stencil(pos, n, cell)
    flat = mesh.reshape(-1)
    out = np.zeros(i0.shape[1])
    for offs in _CORNERS:
        idx, w, _ = _corner(i0, t, n, offs)
        out += w[0] * w[1] * w[2] * flat[idx]
    return out


def readout_gradient(pos, mesh, cell):
    """(3, P) gradient wrt x_n of sum_c W(x_n - c) mesh(c).

    Equal to the transpose of painting with respect to positions:
    x_bar_n = sum_c rho_bar(c) grad W(x_n - c)."""
    n = mesh.shape[0]
    i0, t = _stencil(pos, n, cell)
    flat = mesh.reshape(-1)
    out = np.zeros((3, i0.shape[1]))
    for offs in _CORNERS:
        idx, w, dw = _corner(i0, t, n, offs)
        m = flat[idx]
        out[0] += dw[0] * w[1] * w[2] * m
        out[1] += w[0] * dw[1] * w[2] * m
        out[2] += w[0] * w[1] * dw[2] * m
    return out / cell


def paint_jvp(pos, dpos, n, cell):
    """Tangent of paint(pos) along position tangent dpos (3, P)."""
    i0, t = _stencil(pos, n, cell)
    dpos = np.asarray(dpos, dtype=np.float64)
    rho = np.zeros(n ** 3)
    for offs in _CORNERS:
        idx, w, dw = _corner(i0, t, n, offs)
        s = (dw[0] * w[1] * w[2] * dpos[0] + w[0] * dw[1] * w[2] * dpos[1]
             + w[0] * w[1] * dw[2] * dpos[2]) / cell
        rho += np.bincount(idx, weights=s, minlength=n ** 3)
    return rho.reshape(n, n, n)


def readout_jvp(pos, dpos, mesh, dmesh, cell):
    """Tangent of readout(pos, mesh) along (dpos, dmesh)."""
    g = readout_gradient(pos, mesh, cell)
    return readout(pos, dmesh, cell) + np.sum(g * dpos, axis=0)
