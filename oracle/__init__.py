"""findpts oracle -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``findpts_oracle.c``: a plain, slow FP64 CPU
implementation of the processor-local findpts path of arXiv 2501.12349
(Setup: Section 3.1 and 4.1-4.3; Find: Section 3.2, 3.2.1 and 4.4;
Interpolate: Section 3.3).  Only ``tests/``, the package smoke check and the
CPU-baseline leg of the benchmark may import it; the product library never
does, and this module imports nothing from the product package.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "findpts_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

INTERIOR, BORDER, NOT_FOUND = 0, 1, 2


def build(force=False):
    """Compile the oracle with gcc (OpenMP); a no-op when it is up to date."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
           "-fopenmp", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int32)
        L.orc_gll.argtypes = [ctypes.c_int, D, D]
        L.orc_lagrange.argtypes = [ctypes.c_int, D, ctypes.c_double, D, D, D]
        L.orc_cheb_points.argtypes = [ctypes.c_int, D]
        L.orc_basis_bounds.argtypes = [ctypes.c_int, ctypes.c_int, D, D]
        L.orc_bound_1d.argtypes = [ctypes.c_int, ctypes.c_int, D, D, D]
        L.orc_bound_2d.argtypes = [ctypes.c_int, ctypes.c_int, D, D, D]
        L.orc_setup.restype = P
        L.orc_setup.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_longlong, D, ctypes.c_double,
                                ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                ctypes.c_double]
        L.orc_free.argtypes = [P]
        L.orc_get_boxes.argtypes = [P, D, D, D, I]
        L.orc_get_hash.restype = ctypes.c_int
        L.orc_get_hash.argtypes = [P, D, ctypes.POINTER(ctypes.c_longlong)]
        L.orc_get_cells.argtypes = [P, ctypes.POINTER(ctypes.c_longlong), I]
        L.orc_map.argtypes = [P, ctypes.c_longlong, D, D, D, D]
        L.orc_newton.argtypes = [P, ctypes.c_longlong, D, D, D, I, I]
        L.orc_find.argtypes = [P, ctypes.c_longlong, D, ctypes.c_int, I, I, D, D,
                               D, I, I, ctypes.c_int]
        L.orc_eval.argtypes = [P, ctypes.c_longlong, I, I, D, ctypes.c_int, D, D,
                               ctypes.c_int]
        L.orc_eval_order.restype = ctypes.c_int
        L.orc_eval_order.argtypes = [P, ctypes.c_longlong, I, I, D, ctypes.c_int, ctypes.c_int,
                                     D, D, ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def max_threads():
    """OpenMP threads the oracle uses."""
    return int(lib().orc_max_threads())


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def gll(N):
    """GLL nodes and weights with N points (Section 2)."""
    z = np.zeros(N)
    w = np.zeros(N)
    if lib().orc_gll(N, _d(z), _d(w)) != 0:
        raise ValueError("N out of range")
    return z, w


def lagrange(N, r, deriv=2):
    """phi_i(r), phi_i'(r), phi_i''(r) at the GLL nodes (product form)."""
    z, _ = gll(N)
    ph, d1, d2 = np.zeros(N), np.zeros(N), np.zeros(N)
    nul = ctypes.POINTER(ctypes.c_double)()
    lib().orc_lagrange(N, _d(z), float(r), _d(ph), _d(d1) if deriv >= 1 else nul,
                       _d(d2) if deriv >= 2 else nul)
    return ph, d1, d2


def cheb_points(M):
    eta = np.zeros(M)
    lib().orc_cheb_points(M, _d(eta))
    return eta


def basis_bounds(N, M):
    """(lo, hi) arrays [N][M] of the piecewise-linear basis bounds."""
    lo = np.zeros((N, M))
    hi = np.zeros((N, M))
    if lib().orc_basis_bounds(N, M, _d(lo), _d(hi)) != 0:
        raise ValueError("bad N/M")
    return lo, hi


def bound_1d(u, M):
    u = np.ascontiguousarray(u, dtype=np.float64)
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_bound_1d(len(u), M, _d(u), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def bound_2d(u, M):
    """u[j][i] (i fastest) -> (min, max) bound."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    N = u.shape[0]
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_bound_2d(N, M, _d(u.reshape(-1)), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


class Mesh:
    """Oracle mesh: setup (boxes + local map) over host nodes
    [nel][D][N^R] (i fastest)."""

    def __init__(self, nodes, dim, ref_dim, nodes_1d, bbox_tol=0.1, hash_n=0,
                 eps_d=1e-10, max_iter=50, newton_tol=1e-10):
        self.nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self.D, self.R, self.N = dim, ref_dim, nodes_1d
        self.nel = self.nodes.shape[0]
        self.NP = nodes_1d ** ref_dim
        assert self.nodes.shape == (self.nel, dim, self.NP), self.nodes.shape
        h = lib().orc_setup(dim, ref_dim, nodes_1d, self.nel, _d(self.nodes),
                            bbox_tol, hash_n, eps_d, max_iter, newton_tol)
        if not h:
            raise ValueError("oracle setup rejected the arguments")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def boxes(self):
        D, n = self.D, self.nel
        aabb = np.zeros((n, D, 2))
        A = np.zeros((n, D, D))
        c = np.zeros((n, D))
        ok = np.zeros(n, dtype=np.int32)
        lib().orc_get_boxes(self._h, _d(aabb), _d(A), _d(c), _i(ok))
        return aabb, A, c, ok

    def hash_info(self):
        out = np.zeros(9)
        nnz = ctypes.c_longlong()
        NL = lib().orc_get_hash(self._h, _d(out), ctypes.byref(nnz))
        D = self.D
        return dict(NL=NL, lo=out[:D].copy(), hi=out[3:3 + D].copy(),
                    delta=out[6:6 + D].copy(), nnz=nnz.value)

    def cells(self):
        """Cell lists of the local map: offsets [N_L^D + 1], element ids."""
        h = self.hash_info()
        off = np.zeros(h["NL"] ** self.D + 1, dtype=np.int64)
        el = np.zeros(max(h["nnz"], 1), dtype=np.int32)
        lib().orc_get_cells(self._h, off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                            _i(el))
        return off, el[:h["nnz"]]

    def map(self, e, r):
        """x(r), G (D x R), H2 (D x R x R) of element e."""
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1))
        x = np.zeros(self.D)
        G = np.zeros((self.D, self.R))
        H2 = np.zeros((self.D, self.R, self.R))
        lib().orc_map(self._h, int(e), _d(r), _d(x), _d(G), _d(H2))
        return x, G, H2

    def newton(self, e, x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
        r = np.zeros(3)
        d = ctypes.c_double()
        it = np.zeros(1, dtype=np.int32)
        cv = np.zeros(1, dtype=np.int32)
        lib().orc_newton(self._h, int(e), _d(x), _d(r), ctypes.byref(d), _i(it), _i(cv))
        return r[:self.R].copy(), d.value, int(it[0]), bool(cv[0])

    def find(self, pts, mode=0, nthreads=0):
        """pts: [D][n] -> dict(code, elem, r [R][n], dist, margin [5][n],
        iters, ncand).  mode 0: local map; 1: all boxes; 2: all elements."""
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        n = pts.shape[1]
        code = np.zeros(n, np.int32)
        elem = np.zeros(n, np.int32)
        r = np.zeros((self.R, n))
        dist = np.zeros(n)
        margin = np.zeros((5, n))
        iters = np.zeros(n, np.int32)
        ncand = np.zeros(n, np.int32)
        lib().orc_find(self._h, n, _d(pts), mode, _i(code), _i(elem), _d(r), _d(dist),
                       _d(margin), _i(iters), _i(ncand), nthreads)
        return dict(code=code, elem=elem, r=r, dist=dist, margin=margin,
                    iters=iters, ncand=ncand)

    def eval(self, res, field, nthreads=0, field_nodes_1d=None):
        """field: [nf][nel][Nf^R] -> [nf][n] (NaN where NOT_FOUND).  Nf
        (field_nodes_1d) defaults to the geometry's N."""
        field = np.ascontiguousarray(field, dtype=np.float64)
        if field.ndim == 2:
            field = field[None]
        nf = field.shape[0]
        Nf = self.N if field_nodes_1d is None else int(field_nodes_1d)
        assert field.shape[1:] == (self.nel, Nf ** self.R), field.shape
        code = np.ascontiguousarray(res["code"], dtype=np.int32)
        elem = np.ascontiguousarray(res["elem"], dtype=np.int32)
        r = np.ascontiguousarray(res["r"], dtype=np.float64)
        n = code.shape[0]
        out = np.zeros((nf, n))
        if lib().orc_eval_order(self._h, n, _i(code), _i(elem), _d(r), nf, Nf, _d(field),
                                _d(out), nthreads) != 0:
            raise ValueError("field order out of range")
        return out
