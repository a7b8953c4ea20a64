"""Primary-vortex centre of a lid-driven cavity from its velocity field (test
infrastructure): the stream function psi with d psi / d y = u_x, integrated
up each column from the bottom wall, has its interior minimum at the centre
of the primary vortex (lid moving in +x on the top face).  The minimum is
refined by a quadratic fit over the 3 x 3 nodes around the discrete minimum.

Coordinates are normalised by the cavity size: node (i, j) of an nx x ny
lattice with half-way walls sits at x* = (i + 1/2) / nx, y* = (j + 1/2) / ny,
the convention of the paper's vortex tables (Sec. 5.4, primary-vortex table).
"""
import numpy as np


def stream_function(ux, a):
    """psi[j, i] = integral of u_x dy from the bottom wall (half a node below
    row 0) to node j, trapezoidal; a = dy."""
    c = np.cumsum(ux, axis=0)
    return a * (c - 0.5 * ux)


def primary_vortex(ux, uy, a):
    """(x*, y*) of the primary vortex centre and psi there."""
    psi = stream_function(ux, a)
    ny, nx = psi.shape
    j, i = np.unravel_index(np.argmin(psi[1:-1, 1:-1]), (ny - 2, nx - 2))
    j, i = j + 1, i + 1
    w = psi[j - 1:j + 2, i - 1:i + 2]
    # quadratic model psi = c0 + cx X + cy Y + cxx X^2 + cyy Y^2 + cxy X Y
    X, Y = np.meshgrid([-1.0, 0.0, 1.0], [-1.0, 0.0, 1.0])
    A = np.stack([np.ones(9), X.ravel(), Y.ravel(), X.ravel() ** 2, Y.ravel() ** 2,
                  (X * Y).ravel()], 1)
    c = np.linalg.lstsq(A, w.ravel(), rcond=None)[0]
    H = np.array([[2 * c[3], c[5]], [c[5], 2 * c[4]]])
    dx, dy = np.linalg.solve(H, -c[1:3])
    dx, dy = float(np.clip(dx, -1, 1)), float(np.clip(dy, -1, 1))
    return (i + dx + 0.5) / nx, (j + dy + 0.5) / ny, float(psi[j, i])
