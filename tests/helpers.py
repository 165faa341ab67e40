"""Independent textbook implementations used to pin the oracle.

These are written from the mathematics, not from the oracle: numpy loops for
cloud-in-cell weights, a linear solve for the rotation's defining equation,
and dense brute-force assembly on tiny grids.
"""
import numpy as np


def cic_nodes_weights(x, n, h):
    """For each particle: 8 (node index, weight) pairs of trilinear interpolation."""
    x = np.asarray(x, dtype=np.float64)
    np_ = x.shape[1]
    nodes = np.zeros((np_, 8), dtype=np.int64)
    w = np.ones((np_, 8))
    i = [np.floor(x[d] / h[d]).astype(np.int64) for d in range(3)]
    f = [x[d] / h[d] - i[d] for d in range(3)]
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        gx = (i[0] + ax) % n[0]
        gy = (i[1] + ay) % n[1]
        gz = (i[2] + az) % n[2]
        nodes[:, a] = gx + n[0] * (gy + n[1] * gz)
        for d, ad in enumerate((ax, ay, az)):
            w[:, a] *= f[d] if ad else (1.0 - f[d])
    return nodes, w


def cross_matrix(B):
    """[B x] with [B x] u = B x u."""
    return np.array([[0.0, -B[2], B[1]], [B[2], 0.0, -B[0]], [-B[1], B[0], 0.0]])


def alpha_by_solve(B, beta):
    """alpha as the inverse of (I + beta [B x]): vbar - beta vbar x B = u  <=>  (I + beta[Bx]) vbar = u."""
    A = np.eye(3) + beta * cross_matrix(B)
    return np.linalg.inv(A)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    if den == 0.0:
        return float(np.max(np.abs(a)))
    return float(np.max(np.abs(a - b)) / den)


def periodic_relerr(a, b, L):
    """Relative max-norm of position differences taken modulo the box."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    worst = 0.0
    for d in range(3):
        diff = a[d] - b[d]
        diff = diff - L[d] * np.round(diff / L[d])
        worst = max(worst, float(np.max(np.abs(diff))) / L[d] if diff.size else 0.0)
    return worst
