"""Independent closed forms and textbook references used to pin the oracle.

Nothing here is imported by the GPU library or by the oracle. The kernels are
written from their textbook definitions (radius-h support) so that the pins
do not re-use the oracle's own code.
"""
import math

import numpy as np

PI = math.pi


def cubic_w(q):
    q = np.asarray(q, dtype=np.float64)
    return np.where(q <= 0.5, 1 - 6 * q ** 2 + 6 * q ** 3, np.where(q < 1, 2 * (1 - q) ** 3, 0.0))


def cubic_dw(q):
    q = np.asarray(q, dtype=np.float64)
    return np.where(q <= 0.5, -12 * q + 18 * q ** 2, np.where(q < 1, -6 * (1 - q) ** 2, 0.0))


CUBIC_NORM = 8.0 / PI


def W(r, h):
    return CUBIC_NORM / h ** 3 * cubic_w(r / h)


def dWdr(r, h):
    return CUBIC_NORM / h ** 4 * cubic_dw(r / h)


def min_image(xi, xj, box):
    d = xi - xj
    return d - box * np.round(d / box)


def pair_table(x, lists, box):
    """Flattened (i, j, x_ij) over neighbour lists."""
    ii = np.concatenate([np.full(len(l), i) for i, l in enumerate(lists)])
    jj = np.concatenate(lists)
    d = min_image(x[:, ii], x[:, jj], box)
    return ii, jj, d


def lattice_corr_closed_form(n_side, h, box=1.0):
    """Perfect lattice: B = 0, grad A = 0, grad B = -(c1/c2) I (cubic symmetry).

    With m1 = 0, m2 = c2 I, d_g m1^a = c1 delta_ag and d m2 odd => 0:
    c2 = 1/3 sum_j V r^2 W, c1 = m0 + 1/3 sum_j V r W'.
    """
    dx = box / n_side
    k = int(math.ceil(h / dx)) + 1
    g = np.arange(-k, k + 1) * dx
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2).ravel()
    r = r[r < h]
    # V = m / rho_SPH with equal masses: V = 1 / sum W
    V = 1.0 / W(r, h).sum()
    m0 = V * W(r, h).sum()
    c2 = V * (r ** 2 * W(r, h)).sum() / 3.0
    c1 = m0 + V * (r * dWdr(r, h)).sum() / 3.0
    return -c1 / c2, V


def textbook_sph_accel(x, m, V, P, h, box, sym_lists):
    """Kernel-averaged SPH pressure force, F_ij = -V_i V_j (P_i+P_j) 1/2 (gW(h_i)+gW(h_j))."""
    n = m.size
    a = np.zeros((3, n))
    for i in range(n):
        js = sym_lists[i]
        if len(js) == 0:
            continue
        d = min_image(x[:, [i]], x[:, js], box)
        r = np.sqrt((d ** 2).sum(0))
        g = 0.5 * (dWdr(r, h[i]) + dWdr(r, h[js])) * d / r
        F = -V[i] * V[js] * (P[i] + P[js]) * g
        a[:, i] = F.sum(1) / m[i]
    return a
