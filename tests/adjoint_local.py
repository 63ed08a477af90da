"""The transposed streaming operator and the BGK Jacobian at single nodes of
a jittered-lattice cloud, from the oracle's own routines on a disc of nodes
around each node (the reference of the full-size reversed-step test).

For a node q, entry k of the transposed streaming operator gathers
W_k[m][j] lam_k(m) over every node m whose departure owner's stencil holds q
in slot j (Sec. 2, eq. shape_vector; the adjoint of the streaming sum).

Locality. With every coordinate jittered by at most 0.3 h, any point is
within 0.8 sqrt(2) h < 1.14 h of a node, and the 37 lattice points within
sqrt(10) h of a node's lattice point give it at least 30 nodes within
sqrt(10) h + 0.6 sqrt(2) h < 4.02 h: every stencil radius (K <= 30) is below
4.02 h (asserted for each stencil formed). So an m that reaches q lies within
sqrt(2) h + 1.14 h + 4.02 h < 8 h of q (the candidates), and every nearest-node
and stencil search around it stays within 9.42 h + 1.14 h + 4.02 h < 16 h of q:
the oracle's routines run on that disc of nodes give their global answers."""
import numpy as np

import oracle

R_CAND, R_DISC = 8.0, 16.0   # candidate and search-disc radii in spacings h


def _min_image(d, L):
    return (d + 0.5 * L) % L - 0.5 * L


def transposed_row(c, K, m_deg, lam_u, q):
    """(S^T lam)(q) for k = 0..8 (paper stencil rule, dx = h) and the
    magnitude sum over the gathered terms of |W lam| per k."""
    assert K <= 30
    L = c.period[0]
    h = c.h
    ex, ey, _, _ = oracle.tables()
    dxq = _min_image(c.x - c.x[q], L)
    dyq = _min_image(c.y - c.y[q], L)
    r2 = dxq * dxq + dyq * dyq
    disc = np.nonzero(r2 < (R_DISC * h) ** 2)[0]          # ascending user indices
    xd, yd = c.x[disc], c.y[disc]
    cand = disc[r2[disc] < (R_CAND * h) ** 2]
    stencils = {}
    out = np.zeros(9)
    mag = np.zeros(9)
    out[0] = lam_u[q, 0]
    mag[0] = abs(lam_u[q, 0])
    for m in cand:
        for k in range(1, 9):
            px, py = c.x[m] - ex[k] * h, c.y[m] - ey[k] * h
            s = int(disc[oracle.nearest(xd, yd, c.period, px, py)])
            if s not in stencils:
                sl = int(np.searchsorted(disc, s))
                st = disc[oracle.knn_one(xd, yd, c.period, K, sl)]
                rx = _min_image(c.x[st] - c.x[s], L)
                ry = _min_image(c.y[st] - c.y[s], L)
                # the radius bound the candidate and disc radii rest on
                assert float(np.sqrt(rx * rx + ry * ry).max()) < 4.02 * h
                stencils[s] = (st, rx, ry)
            st, rx, ry = stencils[s]
            hit = np.nonzero(st == q)[0]
            if hit.size == 0:
                continue
            qx = _min_image(px - c.x[s], L)
            qy = _min_image(py - c.y[s], L)
            w = oracle.shape_vector(rx, ry, qx, qy, m_deg)
            t = w[hit[0]] * lam_u[m, k]
            out[k] += t
            mag[k] += abs(t)
    return out, mag


def collision_jacobian(f, tau):
    """J[a][b] = d C_a / d f_b at the populations f of one node, central
    differences of the oracle's collision."""
    J = np.empty((9, 9))
    for b in range(9):
        e = 1e-6 * max(1.0, abs(f[b]))
        fp, fm = f.copy(), f.copy()
        fp[b] += e
        fm[b] -= e
        J[:, b] = (oracle.collide(fp[None, :], tau)[0] - oracle.collide(fm[None, :], tau)[0]) / (2 * e)
    return J
