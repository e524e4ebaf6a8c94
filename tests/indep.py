"""Independent helpers for the oracle pins: tensor Lagrange interpolation
through numpy's Legendre Vandermonde (a library routine), so that checks of
the oracle do not reuse the oracle's own basis code."""
import numpy as np
from numpy.polynomial import legendre as L

from paper_2501_12349_amd.workloads import gll_points


def lag(N, r, der=0):
    """phi_i^(der)(r) for GLL nodes, shape [len(r)][N]."""
    z = gll_points(N)
    V = L.legvander(z, N - 1)
    C = np.linalg.inv(V)                      # column i: Legendre coeffs of phi_i
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    out = np.empty((r.size, N))
    for i in range(N):
        c = C[:, i]
        for _ in range(der):
            c = L.legder(c)
        out[:, i] = L.legval(r, c)
    return out


def map_points(nodes, N, R, e, r, der=None):
    """x_e(r) for element ids e[n] and reference points r[R][n]; der is an
    optional tuple of derivative orders per reference direction."""
    der = der or (0,) * R
    e = np.asarray(e)
    r = np.asarray(r, dtype=np.float64)
    ph = [lag(N, r[a], der[a]) for a in range(R)]
    X = nodes[e]                               # [n][D][NP]
    n, D = X.shape[0], X.shape[1]
    if R == 2:
        X = X.reshape(n, D, N, N)              # [n][D][j][i]
        return np.einsum("ndji,ni,nj->dn", X, ph[0], ph[1])
    X = X.reshape(n, D, N, N, N)               # [n][D][k][j][i]
    return np.einsum("ndkji,ni,nj,nk->dn", X, ph[0], ph[1], ph[2])


def surface_normal(nodes, N, e, r):
    t1 = map_points(nodes, N, 2, e, r, (1, 0))
    t2 = map_points(nodes, N, 2, e, r, (0, 1))
    n = np.cross(t1.T, t2.T).T
    return n / np.linalg.norm(n, axis=0)
