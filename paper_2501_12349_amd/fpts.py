"""Python binding of the fpts C-ABI (include/fpts.h): argument marshalling
only.  Device memory and streams come from PyTorch; every step of Find and
Interpolate runs in the HIP kernels of libfpts.so.  There is no CPU path:
without the library or a HIP device the calls raise."""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfpts.so")

INTERIOR, BORDER, NOT_FOUND = 0, 1, 2
FP64, MIXED = 0, 1
_PREC = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}

# Entry points declared in include/fpts.h.
EXPORTS = ("fpts_params_default", "fpts_setup", "fpts_destroy", "fpts_update_nodes",
           "fpts_find_workspace_size", "fpts_find", "fpts_eval_workspace_size",
           "fpts_eval", "fpts_eval_order", "fpts_find_eval_workspace_size", "fpts_find_eval",
           "fpts_find_stats_get", "fpts_profile", "fpts_profile_read",
           "fpts_get_boxes", "fpts_get_hash", "fpts_get_cells", "fpts_status_string",
           "fpts_find_eval_noalloc")

# Entry points declared in include/fpts_lpt.h.
LPT_EXPORTS = ("fpts_lpt_workspace_size", "fpts_lpt_step")

# Entry points declared in include/fpts_serve.h.
SERVE_EXPORTS = ("fpts_server_create", "fpts_server_destroy", "fpts_server_add_mesh",
                 "fpts_server_submit", "fpts_server_poll", "fpts_server_wait",
                 "fpts_server_drain", "fpts_server_stats_get")


class FptsError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("ref_dim", ctypes.c_int),
                ("nodes_1d", ctypes.c_int), ("hash_n", ctypes.c_int),
                ("n_elem", ctypes.c_int64), ("bbox_tol", ctypes.c_double),
                ("surf_eps_d", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("newton_tol", ctypes.c_double), ("mixed_max_iter", ctypes.c_int),
                ("mixed_tol", ctypes.c_double)]


class FindStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("passes", ctypes.c_int64),
                ("evals", ctypes.c_int64), ("evals_h2", ctypes.c_int64),
                ("passes_fp32", ctypes.c_int64), ("evals_fp32", ctypes.c_int64),
                ("evals_h2_exec", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("sweeps_h2", ctypes.c_int64), ("sweeps_fp32", ctypes.c_int64),
                ("overflow_points", ctypes.c_int64), ("evals_fp32_node", ctypes.c_int64),
                ("parked_pairs", ctypes.c_int64), ("listed_points", ctypes.c_int64)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("locate_ms", ctypes.c_double), ("nearest_ms", ctypes.c_double),
                ("newton_ms", ctypes.c_double),
                ("select_ms", ctypes.c_double), ("eval_bin_ms", ctypes.c_double),
                ("eval_ms", ctypes.c_double), ("advance_ms", ctypes.c_double),
                ("face_ms", ctypes.c_double), ("find_calls", ctypes.c_int64), ("eval_calls", ctypes.c_int64),
                ("lpt_calls", ctypes.c_int64)]


class LptParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("periodic", ctypes.c_int * 3), ("hint", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("points", ctypes.c_int64), ("max_in_flight", ctypes.c_int64),
                ("max_batch_requests", ctypes.c_int64), ("peak_bytes", ctypes.c_size_t),
                ("budget_bytes", ctypes.c_size_t)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libfpts.so (built by build.py); raises when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch's HIP runtime is loaded first, so that the library binds to the
    # same runtime and shares its device memory and streams
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise FptsError("libfpts.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    L.fpts_params_default.argtypes = [ctypes.POINTER(Params), i32, i32, i32, i64]
    L.fpts_params_default.restype = None
    L.fpts_setup.argtypes = [ctypes.POINTER(Params), vp, vp, ctypes.POINTER(vp)]
    L.fpts_destroy.argtypes = [vp]
    L.fpts_update_nodes.argtypes = [vp, vp, vp]
    L.fpts_find_workspace_size.argtypes = [vp, i64]
    L.fpts_find_workspace_size.restype = ctypes.c_size_t
    L.fpts_find.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, vp, ctypes.c_size_t, vp]
    L.fpts_eval_workspace_size.argtypes = [vp, i64]
    L.fpts_eval_workspace_size.restype = ctypes.c_size_t
    L.fpts_eval.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]
    L.fpts_eval_order.argtypes = [vp, i64, vp, vp, vp, i32, i32, vp, vp, vp, ctypes.c_size_t,
                                  vp]
    L.fpts_find_eval_workspace_size.argtypes = [vp, i64]
    L.fpts_find_eval_workspace_size.restype = ctypes.c_size_t
    L.fpts_find_eval.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, i32, i32, vp, vp, vp,
                                 ctypes.c_size_t, vp]
    L.fpts_find_eval_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, i32, i32, vp, vp, vp]
    L.fpts_find_stats_get.argtypes = [vp, i64, vp, i32, ctypes.POINTER(FindStats), vp]
    L.fpts_profile.argtypes = [vp, i32]
    L.fpts_profile_read.argtypes = [vp, ctypes.POINTER(KernelTimes)]
    L.fpts_get_boxes.argtypes = [vp, vp, vp, vp]
    L.fpts_get_hash.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i32),
                                ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.fpts_get_cells.argtypes = [vp, vp, vp]
    L.fpts_lpt_workspace_size.argtypes = [vp, i64]
    L.fpts_lpt_workspace_size.restype = ctypes.c_size_t
    L.fpts_lpt_step.argtypes = [vp, ctypes.POINTER(LptParams), i64, i32, vp, vp, vp, vp, vp,
                                vp, vp, vp, i32, vp, ctypes.c_size_t, vp]
    L.fpts_status_string.argtypes = [i32]
    L.fpts_status_string.restype = ctypes.c_char_p
    L.fpts_server_create.argtypes = [ctypes.c_size_t, i32, i64, ctypes.POINTER(vp)]
    L.fpts_server_destroy.argtypes = [vp]
    L.fpts_server_add_mesh.argtypes = [vp, vp, i32, vp, ctypes.POINTER(i32)]
    L.fpts_server_submit.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, i32, vp,
                                     ctypes.POINTER(i64)]
    L.fpts_server_poll.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(dbl),
                                   ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.fpts_server_wait.argtypes = [vp, i64]
    L.fpts_server_drain.argtypes = [vp]
    L.fpts_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise FptsError("fpts error %d: %s" % (
            status, load_library().fpts_status_string(status).decode()))


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Mesh:
    """A mesh resident on the current HIP device (fpts_setup).

    nodes: host array [n_elem][dim][nodes_1d^ref_dim] (first reference
    index fastest).  dim/ref_dim default to the volume case of nodes'
    shape; pass ref_dim=2 with dim=3 for surface quads."""

    def __init__(self, nodes, nodes_1d, dim=None, ref_dim=None, bbox_tol=0.1, hash_n=0,
                 surf_eps_d=1e-10, max_iter=50, newton_tol=1e-10, mixed_tol=None,
                 mixed_max_iter=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise FptsError("no HIP device visible")
        L = load_library()
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        nel, D, NP = nodes.shape
        dim = D if dim is None else dim
        if ref_dim is None:
            ref_dim = next((k for k in (dim, dim - 1, 1) if NP == nodes_1d ** k), dim)
        p = Params()
        L.fpts_params_default(ctypes.byref(p), dim, ref_dim, nodes_1d, nel)
        p.bbox_tol, p.hash_n, p.surf_eps_d = bbox_tol, hash_n, surf_eps_d
        p.max_iter, p.newton_tol = max_iter, newton_tol
        if mixed_tol is not None:
            p.mixed_tol = mixed_tol
        if mixed_max_iter is not None:
            p.mixed_max_iter = mixed_max_iter
        if NP != nodes_1d ** ref_dim or D != dim:
            raise FptsError("nodes shape %s does not match dim/ref_dim/nodes_1d" %
                            (nodes.shape,))
        h = ctypes.c_void_p()
        _check(L.fpts_setup(ctypes.byref(p), nodes.ctypes.data_as(ctypes.c_void_p),
                            _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.dim, self.ref_dim, self.N, self.n_elem, self.NP = dim, ref_dim, nodes_1d, nel, NP
        self._ws = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().fpts_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- workspaces
    def update_nodes(self, nodes, stream=None):
        """Move the mesh (fpts_update_nodes): nodes [n_elem][dim][NP] float64,
        a device tensor or a host array (copied to the device first); boxes,
        centres and the local map are recomputed on the device."""
        import torch
        if not isinstance(nodes, torch.Tensor):
            nodes = torch.from_numpy(np.ascontiguousarray(nodes, dtype=np.float64)).cuda()
        if nodes.dtype != torch.float64 or not nodes.is_cuda or \
                tuple(nodes.shape) != (self.n_elem, self.dim, self.NP):
            raise FptsError("nodes must be a float64 device tensor [%d][%d][%d]" % (
                self.n_elem, self.dim, self.NP))
        nodes = nodes.contiguous()
        _check(load_library().fpts_update_nodes(self._h, _dptr(nodes), _stream_ptr(stream)))
        self._ws = None

    def find_workspace_bytes(self, n):
        return load_library().fpts_find_workspace_size(self._h, n)

    def eval_workspace_bytes(self, n):
        return load_library().fpts_eval_workspace_size(self._h, n)

    def workspace(self, nbytes):
        """A cached uint8 device buffer of at least nbytes (256-aligned)."""
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        return self._ws

    # -- Find
    def find(self, pts, precision="fp64", out=None, ws=None, stream=None):
        """pts: float64 device tensor [dim][n] -> dict(code, elem, r, dist)."""
        import torch
        L = load_library()
        if pts.dtype != torch.float64 or not pts.is_cuda or pts.dim() != 2 or \
                pts.shape[0] != self.dim:
            raise FptsError("pts must be a float64 device tensor [dim][n]")
        pts = pts.contiguous()
        n = pts.shape[1]
        if out is None:
            out = dict(code=torch.empty(n, dtype=torch.int32, device=pts.device),
                       elem=torch.empty(n, dtype=torch.int32, device=pts.device),
                       r=torch.empty((self.ref_dim, n), dtype=torch.float64, device=pts.device),
                       dist=torch.empty(n, dtype=torch.float64, device=pts.device))
        need = self.find_workspace_bytes(n)
        if need == 0:
            raise FptsError("too many points for one find call")
        wsb = ws if ws is not None else self.workspace(need)
        _check(L.fpts_find(self._h, n, _dptr(pts), _dptr(out["code"]), _dptr(out["elem"]),
                           _dptr(out["r"]), _dptr(out["dist"]), _PREC[precision],
                           _dptr(wsb), wsb.numel(), _stream_ptr(stream)))
        self._last_find_ws = (wsb, n)
        return out

    def find_stats(self, stream=None, newton_pass=0):
        """Counters of the last find (synchronises the stream); newton_pass 1 =
        primary candidates, 2 = other candidates, 3 = face passes of primary
        pairs, 0 = all."""
        wsb, n = self._last_find_ws
        st = FindStats()
        _check(load_library().fpts_find_stats_get(self._h, n, _dptr(wsb), int(newton_pass),
                                                  ctypes.byref(st), _stream_ptr(stream)))
        return {k: getattr(st, k) for k, _ in FindStats._fields_}

    # -- Interpolate
    def eval(self, res, field, out=None, ws=None, stream=None, field_nodes_1d=None):
        """field: float64 device tensor [n_fields][n_elem][Nf^ref_dim] (or
        [n_elem][Nf^ref_dim]) -> [n_fields][n].  Nf = field_nodes_1d, the
        field's own GLL nodes per direction, defaults to the geometry's."""
        import torch
        L = load_library()
        Nf = self.N if field_nodes_1d is None else int(field_nodes_1d)
        if field.dim() == 2:
            field = field.unsqueeze(0)
        if field.dtype != torch.float64 or not field.is_cuda or \
                tuple(field.shape[1:]) != (self.n_elem, Nf ** self.ref_dim):
            raise FptsError("field must be float64 [n_fields][n_elem][Nf^ref_dim] on the device")
        field = field.contiguous()
        n = res["code"].shape[0]
        nf = field.shape[0]
        if out is None:
            out = torch.empty((nf, n), dtype=torch.float64, device=field.device)
        need = self.eval_workspace_bytes(n)
        wsb = ws if ws is not None else self.workspace(need)
        _check(L.fpts_eval_order(self._h, n, _dptr(res["code"]), _dptr(res["elem"]),
                                 _dptr(res["r"].contiguous()), nf, Nf, _dptr(field), _dptr(out),
                                 _dptr(wsb), wsb.numel(), _stream_ptr(stream)))
        return out

    # -- particle transport (include/fpts_lpt.h)
    def lpt_workspace_bytes(self, n):
        return load_library().fpts_lpt_workspace_size(self._h, n)

    def lpt_step(self, particles, field, first=False, precision="fp64", ws=None, stream=None):
        """One time step of a Particles set through this mesh's fluid
        velocity ``field`` [dim][n_elem][NP] (float64, device)."""
        import torch
        P = particles
        if field.dtype != torch.float64 or not field.is_cuda or \
                tuple(field.shape) != (self.dim, self.n_elem, self.NP):
            raise FptsError("field must be float64 [dim][n_elem][NP] on the device")
        need = self.lpt_workspace_bytes(P.n)
        if need == 0:
            raise FptsError("too many particles for one step")
        wsb = ws if ws is not None else self.workspace(need)
        f = P.find
        _check(load_library().fpts_lpt_step(
            self._h, ctypes.byref(P.params), P.n, 1 if first else 0, _dptr(P.x), _dptr(P.v),
            _dptr(P.hist), _dptr(field.contiguous()), _dptr(f["code"]), _dptr(f["elem"]),
            _dptr(f["r"]), _dptr(f["dist"]), _PREC[precision], _dptr(wsb), wsb.numel(),
            _stream_ptr(stream)))

    # -- Find and Interpolate in one call
    def find_eval_workspace_bytes(self, n):
        return load_library().fpts_find_eval_workspace_size(self._h, n)

    def find_eval(self, pts, field, precision="fp64", out=None, u=None, ws=None, stream=None,
                  field_nodes_1d=None):
        """fpts_find_eval: (dict(code, elem, r, dist), u [n_fields][n])."""
        import torch
        L = load_library()
        if pts.dtype != torch.float64 or not pts.is_cuda or pts.dim() != 2 or \
                pts.shape[0] != self.dim:
            raise FptsError("pts must be a float64 device tensor [dim][n]")
        Nf = self.N if field_nodes_1d is None else int(field_nodes_1d)
        if field.dim() == 2:
            field = field.unsqueeze(0)
        if field.dtype != torch.float64 or not field.is_cuda or \
                tuple(field.shape[1:]) != (self.n_elem, Nf ** self.ref_dim):
            raise FptsError("field must be float64 [n_fields][n_elem][Nf^ref_dim] on the device")
        pts = pts.contiguous()
        field = field.contiguous()
        n = pts.shape[1]
        nf = field.shape[0]
        if out is None:
            out = dict(code=torch.empty(n, dtype=torch.int32, device=pts.device),
                       elem=torch.empty(n, dtype=torch.int32, device=pts.device),
                       r=torch.empty((self.ref_dim, n), dtype=torch.float64, device=pts.device),
                       dist=torch.empty(n, dtype=torch.float64, device=pts.device))
        if u is None:
            u = torch.empty((nf, n), dtype=torch.float64, device=pts.device)
        need = self.find_eval_workspace_bytes(n)
        if need == 0:
            raise FptsError("too many points for one call")
        wsb = ws if ws is not None else self.workspace(need)
        _check(L.fpts_find_eval(self._h, n, _dptr(pts), _dptr(out["code"]), _dptr(out["elem"]),
                                _dptr(out["r"]), _dptr(out["dist"]), _PREC[precision], nf, Nf,
                                _dptr(field), _dptr(u), _dptr(wsb), wsb.numel(),
                                _stream_ptr(stream)))
        self._last_find_ws = (wsb, n)
        return out, u

    # -- kernel timing (HIP events on the call's stream)
    def profile(self, enable=True):
        _check(load_library().fpts_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        kt = KernelTimes()
        _check(load_library().fpts_profile_read(self._h, ctypes.byref(kt)))
        return {k: getattr(kt, k) for k, _ in KernelTimes._fields_}

    # -- setup products
    def boxes(self):
        D = self.dim
        aabb = np.zeros((self.n_elem, D, 2))
        A = np.zeros((self.n_elem, D, D))
        c = np.zeros((self.n_elem, D))
        _check(load_library().fpts_get_boxes(self._h, aabb.ctypes.data, A.ctypes.data,
                                             c.ctypes.data))
        return aabb, A, c

    def hash_info(self):
        D = self.dim
        lo, hi, de = np.zeros(D), np.zeros(D), np.zeros(D)
        nl, mc = ctypes.c_int(), ctypes.c_int()
        nnz = ctypes.c_int64()
        _check(load_library().fpts_get_hash(self._h, lo.ctypes.data, hi.ctypes.data,
                                            de.ctypes.data, ctypes.byref(nl),
                                            ctypes.byref(nnz), ctypes.byref(mc)))
        return dict(NL=nl.value, lo=lo, hi=hi, delta=de, nnz=nnz.value, max_cell=mc.value)

    def cells(self):
        """Cell lists of the local map: offsets [N_L^dim + 1], element ids."""
        h = self.hash_info()
        off = np.zeros(h["NL"] ** self.dim + 1, dtype=np.int32)
        el = np.zeros(max(h["nnz"], 1), dtype=np.int32)
        _check(load_library().fpts_get_cells(self._h, off.ctypes.data, el.ctypes.data))
        return off, el[:h["nnz"]]


class Particles:
    """Device state of n particles for Mesh.lpt_step: positions x and
    velocities v [dim][n], the Adams-Bashforth history [2][dim][n] and the
    Find result of x.  ``start(mesh)`` runs the initial Find.  hint=True
    searches each particle's previous element first (fpts_lpt.h)."""

    def __init__(self, x, v, tau, dt, lo, hi, periodic, hint=False):
        import torch
        if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 2 or \
                tuple(v.shape) != tuple(x.shape) or v.dtype != torch.float64 or not v.is_cuda:
            raise FptsError("x and v must be float64 device tensors [dim][n]")
        D, n = x.shape
        self.x = x.contiguous().clone()
        self.v = v.contiguous().clone()
        self.hist = torch.zeros((2, D, n), dtype=torch.float64, device=x.device)
        self.n = n
        self.params = LptParams()
        self.params.tau, self.params.dt = float(tau), float(dt)
        self.params.hint = 1 if hint else 0
        for d in range(3):
            self.params.lo[d] = float(lo[d]) if d < D else 0.0
            self.params.hi[d] = float(hi[d]) if d < D else 1.0
            self.params.periodic[d] = int(periodic[d]) if d < D else 0
        self.find = None

    def start(self, mesh, precision="fp64", stream=None):
        self.find = mesh.find(self.x, precision=precision, stream=stream)
        return self


class Server:
    """Request loop over resident meshes (include/fpts_serve.h): requests
    are admitted by device memory, same-mesh requests batched into one
    find + eval launch set, batches overlapped on n_streams streams."""

    def __init__(self, budget_bytes, n_streams=4, max_batch_points=1 << 22):
        import torch
        if not torch.cuda.is_available():
            raise FptsError("no HIP device visible")
        L = load_library()
        h = ctypes.c_void_p()
        _check(L.fpts_server_create(int(budget_bytes), n_streams, max_batch_points,
                                    ctypes.byref(h)))
        self._h = h
        self._meshes = []
        self._live = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().fpts_server_destroy(self._h)
        self._h = None
        self._live = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_mesh(self, mesh, field=None):
        """Register a resident Mesh with its fields ([n_fields][n_elem][NP]
        float64 on the device, or None); returns the mesh id."""
        nf = 0
        fp = ctypes.c_void_p()
        if field is not None:
            if field.dim() == 2:
                field = field.unsqueeze(0)
            field = field.contiguous()
            nf = field.shape[0]
            fp = _dptr(field)
        mid = ctypes.c_int()
        _check(load_library().fpts_server_add_mesh(self._h, mesh._h, nf, fp, ctypes.byref(mid)))
        self._meshes.append((mesh, field, nf))
        return mid.value

    def outputs(self, mesh_id, n, device="cuda"):
        """Output tensors for a request of n points against mesh_id."""
        import torch
        mesh, field, nf = self._meshes[mesh_id]
        return dict(code=torch.empty(n, dtype=torch.int32, device=device),
                    elem=torch.empty(n, dtype=torch.int32, device=device),
                    r=torch.empty((mesh.ref_dim, n), dtype=torch.float64, device=device),
                    dist=torch.empty(n, dtype=torch.float64, device=device),
                    u=torch.empty((max(nf, 1), n), dtype=torch.float64, device=device))

    def submit(self, mesh_id, pts, precision="fp64", out=None, stream=None):
        """Queue find + eval of pts ([dim][n] float64 on the device) into out
        (from outputs(); allocated here when None); returns (request id,
        output dict).  The request waits for the work queued on ``stream``
        (default: torch's current stream) before it reads the points, so a
        non-contiguous input copied here, or points still being produced,
        are safe."""
        mesh, field, nf = self._meshes[mesh_id]
        pts = pts.contiguous()
        n = pts.shape[1]
        if out is None:
            out = self.outputs(mesh_id, n, pts.device)
        rid = ctypes.c_int64()
        _check(load_library().fpts_server_submit(
            self._h, mesh_id, n, _dptr(pts), _dptr(out["code"]), _dptr(out["elem"]),
            _dptr(out["r"]), _dptr(out["dist"]), _dptr(out["u"]) if nf else ctypes.c_void_p(),
            _PREC[precision], _stream_ptr(stream), ctypes.byref(rid)))
        self._live[rid.value] = (pts, out)
        return rid.value, out

    def poll(self, rid):
        st = ctypes.c_int()
        t = [ctypes.c_double() for _ in range(3)]
        _check(load_library().fpts_server_poll(self._h, rid, ctypes.byref(st),
                                               *[ctypes.byref(x) for x in t]))
        return st.value, t[0].value, t[1].value, t[2].value

    def wait(self, rid):
        _check(load_library().fpts_server_wait(self._h, rid))

    def drain(self):
        _check(load_library().fpts_server_drain(self._h))

    def release(self, rid):
        self._live.pop(rid, None)

    def stats(self):
        st = ServerStats()
        _check(load_library().fpts_server_stats_get(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}
