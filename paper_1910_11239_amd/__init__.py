"""Fast tensor-product Schwarz smoothers for SIPG on MI355X (gfx950).

Thin ctypes binding of ``libfts.so`` (C ABI in ``include/fts.h``): argument
marshalling only.  Vectors are torch float64 CUDA tensors (cell-major,
lexicographic, x fastest); every call is enqueued on the current torch
stream.  There is no CPU fallback: if the library is not built the first call
raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfts.so")

FTS_CELL, FTS_VERTEX_PATCH = 0, 1
PREC = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
KIND = {"cell": FTS_CELL, "vertex": FTS_VERTEX_PATCH}

_lib = None


class FtsError(RuntimeError):
    pass


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("degree", ctypes.c_int32), ("ncells", ctypes.c_int32 * 3),
                ("h", ctypes.c_void_p * 3), ("penalty_factor", ctypes.c_double)]


_VP, _I32, _I64, _D, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_SIGS = {
    "fts_set_allocator": (_I32, [_ALLOC_T, _FREE_T, _VP]),
    "fts_version": (ctypes.c_char_p, []),
    "fts_last_error": (_I32, [ctypes.c_char_p, _SZ]),
    "fts_level_create": (_I32, [_VP, _VP]),
    "fts_level_destroy": (_I32, [_VP]),
    "fts_level_ndofs": (_I64, [_VP]),
    "fts_setup_1d_eigs": (_I32, [_VP, _I32, _VP]),
    "fts_eigs_destroy": (_I32, [_VP]),
    "fts_eigs_get": (_I32, [_VP, _I32, _I32, _VP, _VP, _VP, _VP]),
    "fts_eigs_n": (_I32, [_VP]),
    "fts_eigs_set_schedule": (_I32, [_VP, _I32]),
    "fts_apply_operator": (_I32, [_VP, _VP, _VP, _VP]),
    "fts_residual": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "fts_smooth_ws_bytes": (_SZ, [_VP]),
    "fts_schwarz_smooth": (_I32, [_VP, _VP, _D, _I32, _VP, _VP, _I32, _VP, _SZ, _VP]),
    "fts_schwarz_smooth_mult": (_I32, [_VP, _VP, _D, _I32, _VP, _VP, _I32, _VP, _SZ, _VP]),
    "fts_schwarz_smooth_noalloc": (_I32, [_VP, _VP, _D, _I32, _VP, _VP, _I32, _VP]),
    "fts_schwarz_apply": (_I32, [_VP, _VP, _D, _I32, _VP, _VP, _VP]),
    "fts_restrict": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "fts_prolongate_add": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "fts_hierarchy_create": (_I32, [_VP, _I32, _I32, _VP, _VP, _I32, _I32, _VP]),
    "fts_hierarchy_destroy": (_I32, [_VP]),
    "fts_hierarchy_level": (_VP, [_VP, _I32]),
    "fts_hierarchy_eigs": (_VP, [_VP, _I32]),
    "fts_vcycle": (_I32, [_VP, _I32, _VP, _VP, _VP]),
    "fts_coarse_solve": (_I32, [_VP, _VP, _VP, _VP]),
    "fts_pcg_ws_bytes": (_SZ, [_VP]),
    "fts_hierarchy_set_omega": (_I32, [_VP, _VP]),
    "fts_hierarchy_set_smoother": (_I32, [_VP, _I32]),
    "fts_gmres_ws_bytes": (_SZ, [_VP, _I32]),
    "fts_gmres": (_I32, [_VP, _I32, _VP, _VP, _D, _I32, _I32, _VP, _SZ, _VP, _VP, _VP, _VP]),
    "fts_hierarchy_enable_adjoint": (_I32, [_VP]),
    "fts_vcycle_adjoint": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "fts_batch_create": (_I32, [_VP, _I32, _VP]),
    "fts_batch_destroy": (_I32, [_VP]),
    "fts_batch_ndofs": (_I64, [_VP]),
    "fts_batch_mesh_offset": (_I32, [_VP, _I32, _VP, _VP]),
    "fts_batch_residual": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "fts_batch_apply": (_I32, [_VP, _D, _I32, _VP, _VP, _VP]),
    "fts_batch_ws_bytes": (_SZ, [_VP]),
    "fts_batch_smooth": (_I32, [_VP, _D, _I32, _VP, _VP, _I32, _VP, _SZ, _VP]),
    "fts_batch_set_launch": (_I32, [_VP, _I32, _I32, _I32]),
    "fts_batch_get_launch": (_I32, [_VP, _VP, _VP, _VP]),
    "fts_batch_autotune": (_I32, [_VP, _I32, _VP, _VP, ctypes.c_char_p, _SZ]),
    "fts_pcg": (_I32, [_VP, _I32, _VP, _VP, _D, _I32, _VP, _SZ, _VP, _VP, _VP, _VP]),
    "fts_mapped_level_create": (_I32, [_VP, _VP]),
    "fts_mapped_level_destroy": (_I32, [_VP]),
    "fts_mapped_level_ndofs": (_I64, [_VP]),
    "fts_mapped_surrogate_widths": (_I32, [_VP, _VP]),
    "fts_mapped_apply_operator": (_I32, [_VP, _VP, _VP, _VP]),
    "fts_mapped_residual": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "fts_mapped_schwarz_apply": (_I32, [_VP, _D, _VP, _VP, _VP]),
    "fts_mapped_smooth_ws_bytes": (_SZ, [_VP]),
    "fts_mapped_schwarz_smooth": (_I32, [_VP, _D, _VP, _VP, _I32, _VP, _SZ, _VP]),
    "fts_mapped_hierarchy_create": (_I32, [_VP, _I32, _VP, _I32, _I32, _VP]),
    "fts_mapped_hierarchy_destroy": (_I32, [_VP]),
    "fts_mapped_hierarchy_ndofs": (_I64, [_VP]),
    "fts_mapped_hierarchy_set_smoother": (_I32, [_VP, _I32]),
    "fts_mapped_hierarchy_set_local_solver": (_I32, [_VP, _I32]),
    "fts_mapped_vcycle": (_I32, [_VP, _VP, _VP, _VP]),
    "fts_mapped_pcg_ws_bytes": (_SZ, [_VP]),
    "fts_mapped_pcg": (_I32, [_VP, _VP, _VP, _D, _I32, _VP, _SZ, _VP, _VP, _VP, _VP]),
}


# Device memory of the library's handles is torch memory: the library asks the
# allocator registered here (fts_set_allocator), which keeps each block as a
# torch uint8 tensor until the library releases it.
_live = {}


def _torch_alloc(nbytes, ctx):
    try:
        import torch
        t = torch.empty(int(nbytes), dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))
    except Exception:  # reported to the caller of the library as an allocation failure
        return None
    _live[t.data_ptr()] = t
    return t.data_ptr()


def _torch_free(ptr, ctx):
    if ptr is not None and _live is not None:
        _live.pop(ptr, None)


_ALLOC_CB = _ALLOC_T(_torch_alloc)
_FREE_CB = _FREE_T(_torch_free)


def device_bytes_held():
    """Bytes of torch memory the library's handles hold."""
    return sum(t.numel() for t in _live.values())


def lib():
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FtsError(f"{LIB_PATH} is not built: run `python -m paper_1910_11239_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(handle, name)
            f.restype = res
            f.argtypes = args
        if handle.fts_set_allocator(_ALLOC_CB, _FREE_CB, None) != 0:
            raise FtsError("fts_set_allocator failed")
        _lib = handle
    return _lib


def last_error():
    buf = ctypes.create_string_buffer(1024)
    lib().fts_last_error(buf, 1024)
    return buf.value.decode()


def _check(status, what):
    if status != 0:
        raise FtsError(f"{what} failed with status {status}: {last_error()}")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _desc(dim, k, widths, gamma_hat):
    ws = [np.ascontiguousarray(np.asarray(w, dtype=np.float64)) for w in widths]
    if len(ws) != dim:
        raise ValueError("need one width array per axis")
    d = MeshDesc()
    d.dim, d.degree, d.penalty_factor = dim, k, float(gamma_hat)
    for a in range(3):
        d.ncells[a] = len(ws[a]) if a < dim else 1
        d.h[a] = ws[a].ctypes.data if a < dim else None
    return d, ws


class Level:
    """One mesh with its operator tables (fts_level)."""

    def __init__(self, dim, k, widths, gamma_hat=1.0, _handle=None, _owner=None):
        self.dim, self.k = dim, k
        self.widths = tuple(np.asarray(w, dtype=np.float64) for w in widths)
        self.gamma_hat = gamma_hat
        self._owner = _owner
        if _handle is not None:
            self._h = ctypes.c_void_p(_handle)
        else:
            d, keep = _desc(dim, k, self.widths, gamma_hat)
            h = ctypes.c_void_p()
            _check(lib().fts_level_create(ctypes.byref(d), ctypes.byref(h)), "fts_level_create")
            self._h = h
        self.ndofs = int(lib().fts_level_ndofs(self._h))

    def __del__(self):
        if getattr(self, "_owner", None) is None and getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fts_level_destroy(self._h)
            self._h = None

    def apply(self, x, y):
        _check(lib().fts_apply_operator(self._h, _ptr(x, self.ndofs, "x"), _ptr(y, self.ndofs, "y"), _stream()),
               "fts_apply_operator")
        return y

    def residual(self, b, x, r):
        _check(lib().fts_residual(self._h, _ptr(b, self.ndofs, "b"), _ptr(x, self.ndofs, "x"),
                                  _ptr(r, self.ndofs, "r"), _stream()), "fts_residual")
        return r


class Eigs:
    """1-D eigen-data of all subdomains of a level (fts_setup_1d_eigs)."""

    def __init__(self, level, kind="vertex", _handle=None, _owner=None):
        self.level, self.kind = level, kind
        self._owner = _owner
        if _handle is not None:
            self._h = ctypes.c_void_p(_handle)
        else:
            h = ctypes.c_void_p()
            _check(lib().fts_setup_1d_eigs(level._h, KIND[kind], ctypes.byref(h)), "fts_setup_1d_eigs")
            self._h = h
        self.n = int(lib().fts_eigs_n(self._h))

    def __del__(self):
        if getattr(self, "_owner", None) is None and getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fts_eigs_destroy(self._h)
            self._h = None

    def set_schedule(self, schedule):
        """'auto' (default: 'owner' on levels of at least 4,096 cells, 'staged'
        below), 'owner' (owner-computes tiles for 16-bit 3-D vertex patches,
        staged otherwise), 'staged' (deterministic staging buffer + gather) or
        'colored' (2^d parquet colors)."""
        _check(lib().fts_eigs_set_schedule(self._h, {"staged": 0, "colored": 1, "owner": 2, "auto": 3}[schedule]),
               "fts_eigs_set_schedule")

    def get(self, axis, index):
        n = self.n
        A, M, S = (np.zeros((n, n)) for _ in range(3))
        lam = np.zeros(n)
        _check(lib().fts_eigs_get(self._h, axis, index, A.ctypes.data, M.ctypes.data, S.ctypes.data,
                                  lam.ctypes.data), "fts_eigs_get")
        return A, M, S, lam


def smooth_ws_bytes(level):
    return int(lib().fts_smooth_ws_bytes(level._h))


def schwarz_smooth(level, eigs, omega, b, x, nsweeps=1, prec="f64", ws=None):
    import torch
    if ws is None:
        ws = torch.empty(level.ndofs, dtype=torch.float64, device=x.device)
    _check(lib().fts_schwarz_smooth(level._h, eigs._h, float(omega), PREC[prec], _ptr(b, level.ndofs, "b"),
                                    _ptr(x, level.ndofs, "x"), int(nsweeps), _ptr(ws, None, "ws"),
                                    ws.numel() * 8, _stream()), "fts_schwarz_smooth")
    return x


def schwarz_smooth_noalloc(level, eigs, omega, b, x, nsweeps=1, prec="f64"):
    """fts_schwarz_smooth without a workspace argument: the residual lives in
    the library's static device array (levels of up to 4,194,304 DoFs); the
    call allocates nothing."""
    _check(lib().fts_schwarz_smooth_noalloc(level._h, eigs._h, float(omega), PREC[prec], _ptr(b, level.ndofs, "b"),
                                            _ptr(x, level.ndofs, "x"), int(nsweeps), _stream()),
           "fts_schwarz_smooth_noalloc")
    return x


def schwarz_smooth_mult(level, eigs, omega, b, x, nsweeps=1, prec="f64", ws=None):
    """Multiplicative smoother (Alg. multsmoother): a residual before each color."""
    import torch
    if ws is None:
        ws = torch.empty(level.ndofs, dtype=torch.float64, device=x.device)
    _check(lib().fts_schwarz_smooth_mult(level._h, eigs._h, float(omega), PREC[prec], _ptr(b, level.ndofs, "b"),
                                         _ptr(x, level.ndofs, "x"), int(nsweeps), _ptr(ws, None, "ws"),
                                         ws.numel() * 8, _stream()), "fts_schwarz_smooth_mult")
    return x


def schwarz_apply(level, eigs, omega, r, x, prec="f64"):
    _check(lib().fts_schwarz_apply(level._h, eigs._h, float(omega), PREC[prec], _ptr(r, level.ndofs, "r"),
                                   _ptr(x, level.ndofs, "x"), _stream()), "fts_schwarz_apply")
    return x


def restrict(coarse, fine, rf, bc):
    _check(lib().fts_restrict(coarse._h, fine._h, _ptr(rf, fine.ndofs, "rf"), _ptr(bc, coarse.ndofs, "bc"),
                              _stream()), "fts_restrict")
    return bc


def prolongate_add(coarse, fine, ec, xf):
    _check(lib().fts_prolongate_add(coarse._h, fine._h, _ptr(ec, coarse.ndofs, "ec"),
                                    _ptr(xf, fine.ndofs, "xf"), _stream()), "fts_prolongate_add")
    return xf


class Hierarchy:
    """Multigrid hierarchy (fts_hierarchy_create); level 0 is the coarsest."""

    def __init__(self, dim, k, widths, nlevels, kind="vertex", omegas=0.5, gamma_hats=1.0, m_pre=2, m_post=2):
        om = np.full(nlevels, float(omegas)) if np.isscalar(omegas) else np.asarray(omegas, dtype=np.float64)
        gh = np.full(nlevels, float(gamma_hats)) if np.isscalar(gamma_hats) else np.asarray(gamma_hats, np.float64)
        om, gh = np.ascontiguousarray(om), np.ascontiguousarray(gh)
        d, keep = _desc(dim, k, widths, gh[-1])
        h = ctypes.c_void_p()
        _check(lib().fts_hierarchy_create(ctypes.byref(d), nlevels, KIND[kind], om.ctypes.data, gh.ctypes.data,
                                          m_pre, m_post, ctypes.byref(h)), "fts_hierarchy_create")
        self._h = h
        self.dim, self.k, self.nlevels, self.kind = dim, k, nlevels, kind
        self.levels = []
        for l in range(nlevels):
            lh = lib().fts_hierarchy_level(self._h, l)
            self.levels.append(Level(dim, k, [np.zeros(1)] * dim, gh[l], _handle=lh, _owner=self))
        self.eigs = [None] + [Eigs(self.levels[l], kind, _handle=lib().fts_hierarchy_eigs(self._h, l), _owner=self)
                              for l in range(1, nlevels)]
        self.ndofs = self.levels[-1].ndofs

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fts_hierarchy_destroy(self._h)
            self._h = None

    def vcycle(self, b, x, prec="f64"):
        _check(lib().fts_vcycle(self._h, PREC[prec], _ptr(b, self.ndofs, "b"), _ptr(x, self.ndofs, "x"),
                                _stream()), "fts_vcycle")
        return x

    def pcg(self, b, x, rtol=1e-10, maxit=200, prec="f64", ws=None):
        """Flexible PCG with one V-cycle as preconditioner; x: initial guess, updated.
        Returns (iterations, final relative residual, history of relative residuals)."""
        import torch
        nbytes = int(lib().fts_pcg_ws_bytes(self._h))
        if ws is None:
            ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=x.device)
        hist = np.zeros(maxit + 1)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        _check(lib().fts_pcg(self._h, PREC[prec], _ptr(b, self.ndofs, "b"), _ptr(x, self.ndofs, "x"),
                             float(rtol), int(maxit), _ptr(ws, None, "ws"), ws.numel() * 8, ctypes.byref(it),
                             ctypes.byref(rel), hist.ctypes.data, _stream()), "fts_pcg")
        return it.value, rel.value, hist[:it.value + 1]

    def set_smoother(self, smoother):
        """'additive' (default), 'multiplicative' (colors in the same order
        before and after the coarse correction) or 'multiplicative_symmetric'
        (reversed after it) on every smoothed level."""
        code = {"additive": 0, "multiplicative": 1, "multiplicative_symmetric": 2}[smoother]
        _check(lib().fts_hierarchy_set_smoother(self._h, code), "fts_hierarchy_set_smoother")

    def gmres(self, b, x, rtol=1e-10, restart=30, maxit=200, prec="f64", ws=None):
        """Flexible restarted GMRES with one V-cycle as right preconditioner; x:
        initial guess, updated.  Returns (iterations, final relative residual,
        history of relative residuals)."""
        import torch
        nbytes = int(lib().fts_gmres_ws_bytes(self._h, int(restart)))
        if ws is None:
            ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=x.device)
        hist = np.zeros(maxit + 1)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        _check(lib().fts_gmres(self._h, PREC[prec], _ptr(b, self.ndofs, "b"), _ptr(x, self.ndofs, "x"),
                               float(rtol), int(restart), int(maxit), _ptr(ws, None, "ws"), ws.numel() * 8,
                               ctypes.byref(it), ctypes.byref(rel), hist.ctypes.data, _stream()), "fts_gmres")
        return it.value, rel.value, hist[:it.value + 1]

    def set_omega(self, omegas):
        om = np.ascontiguousarray(np.broadcast_to(np.asarray(omegas, dtype=np.float64), (self.nlevels,)))
        _check(lib().fts_hierarchy_set_omega(self._h, om.ctypes.data), "fts_hierarchy_set_omega")

    def vcycle_adjoint(self, b, x_in, lam_out, lam_b=None, lam_x=None):
        """Reverse mode of x_out = MG(x_in, b).  lam_b (+=) and lam_x (=) are CUDA
        tensors or None; returns (d_omega, d_penalty) per level (numpy, level 0 first)."""
        _check(lib().fts_hierarchy_enable_adjoint(self._h), "fts_hierarchy_enable_adjoint")
        dom, dpen = np.zeros(self.nlevels), np.zeros(self.nlevels)
        n = self.ndofs
        _check(lib().fts_vcycle_adjoint(self._h, _ptr(b, n, "b"), _ptr(x_in, n, "x_in"), _ptr(lam_out, n, "lam_out"),
                                        None if lam_b is None else _ptr(lam_b, n, "lam_b"),
                                        None if lam_x is None else _ptr(lam_x, n, "lam_x"),
                                        dom.ctypes.data, dpen.ctypes.data, _stream()), "fts_vcycle_adjoint")
        return dom, dpen

    def coarse_solve(self, b0, x0):
        n0 = self.levels[0].ndofs
        _check(lib().fts_coarse_solve(self._h, _ptr(b0, n0, "b0"), _ptr(x0, n0, "x0"), _stream()),
               "fts_coarse_solve")
        return x0


class MappedDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("degree", ctypes.c_int32), ("ncells", ctypes.c_int32 * 3),
                ("vertices", ctypes.c_void_p), ("penalty_factor", ctypes.c_double)]


class MappedLevel:
    """Mesh of multilinearly mapped cells with Cartesian surrogate local solvers
    (fts_mapped_*).  verts: (prod(ncells + 1), dim) array, x fastest."""

    def __init__(self, dim, k, ncells, verts, gamma_hat=1.0):
        self.dim, self.k = dim, k
        self.ncells = tuple(int(m) for m in ncells)
        self._verts = np.ascontiguousarray(np.asarray(verts, dtype=np.float64))
        d = MappedDesc()
        d.dim, d.degree, d.penalty_factor = dim, k, float(gamma_hat)
        for a in range(3):
            d.ncells[a] = self.ncells[a] if a < dim else 1
        d.vertices = self._verts.ctypes.data
        h = ctypes.c_void_p()
        _check(lib().fts_mapped_level_create(ctypes.byref(d), ctypes.byref(h)), "fts_mapped_level_create")
        self._h = h
        self.ndofs = int(lib().fts_mapped_level_ndofs(self._h))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fts_mapped_level_destroy(self._h)
            self._h = None

    def surrogate_widths(self):
        out = np.zeros((int(np.prod(self.ncells)), self.dim))
        _check(lib().fts_mapped_surrogate_widths(self._h, out.ctypes.data), "fts_mapped_surrogate_widths")
        return out

    def apply(self, x, y):
        _check(lib().fts_mapped_apply_operator(self._h, _ptr(x, self.ndofs, "x"), _ptr(y, self.ndofs, "y"),
                                               _stream()), "fts_mapped_apply_operator")
        return y

    def residual(self, b, x, r):
        _check(lib().fts_mapped_residual(self._h, _ptr(b, self.ndofs, "b"), _ptr(x, self.ndofs, "x"),
                                         _ptr(r, self.ndofs, "r"), _stream()), "fts_mapped_residual")
        return r

    def schwarz_apply(self, omega, r, x):
        _check(lib().fts_mapped_schwarz_apply(self._h, float(omega), _ptr(r, self.ndofs, "r"),
                                              _ptr(x, self.ndofs, "x"), _stream()), "fts_mapped_schwarz_apply")
        return x

    def schwarz_smooth(self, omega, b, x, nsweeps=1, ws=None):
        import torch
        if ws is None:
            ws = torch.empty(self.ndofs, dtype=torch.float64, device=x.device)
        _check(lib().fts_mapped_schwarz_smooth(self._h, float(omega), _ptr(b, self.ndofs, "b"),
                                               _ptr(x, self.ndofs, "x"), int(nsweeps), _ptr(ws, None, "ws"),
                                               ws.numel() * 8, _stream()), "fts_mapped_schwarz_smooth")
        return x


class MappedHierarchy:
    """Multigrid on mapped meshes (fts_mapped_hierarchy_*): vertex arrays of
    every level, coarsest first (each level the uniform refinement of the
    previous one on its cell maps); additive cell smoother with Cartesian
    surrogate solvers, omega per level (omegas[0] unused)."""

    def __init__(self, dim, k, coarse_ncells, level_verts, gamma_hat, omegas, m_pre=1, m_post=1):
        n = len(level_verts)
        self._verts = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in level_verts]
        descs = (MappedDesc * n)()
        for l in range(n):
            d = descs[l]
            d.dim, d.degree, d.penalty_factor = dim, k, float(gamma_hat)
            for a in range(3):
                d.ncells[a] = int(coarse_ncells[a]) * 2 ** l if a < dim else 1
            d.vertices = self._verts[l].ctypes.data
        om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
        if om.size != n:
            raise ValueError("one omega per level")
        h = ctypes.c_void_p()
        _check(lib().fts_mapped_hierarchy_create(descs, n, om.ctypes.data, int(m_pre), int(m_post),
                                                 ctypes.byref(h)), "fts_mapped_hierarchy_create")
        self._h = h
        self.ndofs = int(lib().fts_mapped_hierarchy_ndofs(self._h))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fts_mapped_hierarchy_destroy(self._h)
            self._h = None

    def set_smoother(self, smoother):
        """'additive' or 'multiplicative' (red-black cells, reversed in post-smoothing)."""
        code = {"additive": 0, "multiplicative": 1}[smoother]
        _check(lib().fts_mapped_hierarchy_set_smoother(self._h, code), "fts_mapped_hierarchy_set_smoother")

    def set_local_solver(self, local):
        """'surrogate' (fast diagonalisation of the Cartesian surrogate) or
        'exact' (inverses of the mapped cell blocks)."""
        code = {"surrogate": 0, "exact": 1}[local]
        _check(lib().fts_mapped_hierarchy_set_local_solver(self._h, code), "fts_mapped_hierarchy_set_local_solver")

    def vcycle(self, b, x):
        _check(lib().fts_mapped_vcycle(self._h, _ptr(b, self.ndofs, "b"), _ptr(x, self.ndofs, "x"), _stream()),
               "fts_mapped_vcycle")
        return x

    def pcg(self, b, x, rtol=1e-8, maxit=200, ws=None):
        """CG with one V-cycle as preconditioner; x: initial guess, updated.
        Returns (iterations, final relative residual, history)."""
        import torch
        nbytes = int(lib().fts_mapped_pcg_ws_bytes(self._h))
        if ws is None:
            ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=x.device)
        hist = np.zeros(maxit + 1)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        _check(lib().fts_mapped_pcg(self._h, _ptr(b, self.ndofs, "b"), _ptr(x, self.ndofs, "x"), float(rtol),
                                    int(maxit), _ptr(ws, None, "ws"), ws.numel() * 8, ctypes.byref(it),
                                    ctypes.byref(rel), hist.ctypes.data, _stream()), "fts_mapped_pcg")
        return it.value, rel.value, hist[:it.value + 1]


class Batch:
    """Many independent 3-D meshes smoothed together (fts_batch_*).
    meshes: list of (k, widths, gamma_hat)."""

    def __init__(self, meshes):
        descs = (MeshDesc * len(meshes))()
        self._keep = []
        for i, (k, widths, gh) in enumerate(meshes):
            d, ws = _desc(3, k, widths, gh)
            descs[i] = d
            self._keep.append(ws)
        h = ctypes.c_void_p()
        _check(lib().fts_batch_create(descs, len(meshes), ctypes.byref(h)), "fts_batch_create")
        self._h = h
        self.nmesh = len(meshes)
        self.ndofs = int(lib().fts_batch_ndofs(self._h))
        self.offsets = []
        for i in range(self.nmesh):
            off, n = ctypes.c_int64(), ctypes.c_int64()
            _check(lib().fts_batch_mesh_offset(self._h, i, ctypes.byref(off), ctypes.byref(n)), "fts_batch_mesh_offset")
            self.offsets.append((off.value, n.value))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fts_batch_destroy(self._h)
            self._h = None

    def residual(self, b, x, r):
        n = self.ndofs
        _check(lib().fts_batch_residual(self._h, _ptr(b, n, "b"), _ptr(x, n, "x"), _ptr(r, n, "r"), _stream()),
               "fts_batch_residual")
        return r

    def apply(self, omega, r, x, prec="f32"):
        n = self.ndofs
        _check(lib().fts_batch_apply(self._h, float(omega), PREC[prec], _ptr(r, n, "r"), _ptr(x, n, "x"),
                                     _stream()), "fts_batch_apply")
        return x

    def smooth(self, omega, b, x, nsweeps=1, prec="f32", ws=None):
        import torch
        n = self.ndofs
        if ws is None:
            ws = torch.empty(n, dtype=torch.float64, device=x.device)
        _check(lib().fts_batch_smooth(self._h, float(omega), PREC[prec], _ptr(b, n, "b"), _ptr(x, n, "x"),
                                      int(nsweeps), _ptr(ws, None, "ws"), ws.numel() * 8, _stream()),
               "fts_batch_smooth")
        return x

    def set_launch(self, threads, grid, chunk):
        _check(lib().fts_batch_set_launch(self._h, threads, grid, chunk), "fts_batch_set_launch")

    def get_launch(self):
        t, g, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fts_batch_get_launch(self._h, ctypes.byref(t), ctypes.byref(g), ctypes.byref(c)),
               "fts_batch_get_launch")
        return t.value, g.value, c.value

    def autotune(self, r, prec="f32"):
        buf = ctypes.create_string_buffer(8192)
        _check(lib().fts_batch_autotune(self._h, PREC[prec], _ptr(r, self.ndofs, "r"), _stream(), buf, 8192),
               "fts_batch_autotune")
        return buf.value.decode()


class VCycleIterations:
    """u_{i+1} = MG_L(u_i, b), u_0 = 0, for ``ncycles`` V-cycles, differentiable
    with respect to b, the per-level damping omega_l and the per-level penalty
    factor gamma_hat_l through a hand-written adjoint (fts_vcycle_adjoint),
    which recomputes each cycle's sweeps from the stored cycle inputs.  The
    hierarchy of a penalty vector is built once and cached (the 1-D eigen-data
    and the coarse factor depend on it; omega is set per call)."""

    def __init__(self, dim, k, widths, nlevels, kind="vertex", m_pre=2, m_post=2, ncycles=4):
        self.args = (dim, k, widths, nlevels, kind, m_pre, m_post)
        self.ncycles = ncycles
        self._cache = {}

    def hierarchy(self, gammas):
        key = tuple(float(g) for g in gammas)
        if key not in self._cache:
            dim, k, widths, nlevels, kind, m_pre, m_post = self.args
            self._cache[key] = Hierarchy(dim, k, widths, nlevels, kind, 0.5, np.asarray(key), m_pre, m_post)
        return self._cache[key]

    def __call__(self, b, omegas, gammas):
        return _VCycleFn.apply(b, omegas, gammas, self)


def _vcycle_fn():
    import torch

    class VCycleFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, b, omegas, gammas, solver):
            h = solver.hierarchy(gammas.detach().cpu().numpy())
            om = np.array(omegas.detach().cpu().numpy(), dtype=np.float64)
            h.set_omega(om)
            u = torch.zeros_like(b)
            inputs = []
            for _ in range(solver.ncycles):
                inputs.append(u.clone())
                h.vcycle(b, u)
            # the hierarchy is shared by every call with these penalties: keep
            # this call's damping so that backward recomputes the same sweeps
            ctx.h, ctx.inputs, ctx.omegas = h, inputs, om
            ctx.param_like = ((omegas.device, omegas.dtype), (gammas.device, gammas.dtype))
            ctx.save_for_backward(b)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            (b,) = ctx.saved_tensors
            h = ctx.h
            h.set_omega(ctx.omegas)
            lam = grad_u.contiguous().clone()
            lam_b = torch.zeros_like(b)
            lam_x = torch.empty_like(b)
            dom = np.zeros(h.nlevels)
            dpen = np.zeros(h.nlevels)
            for x_in in reversed(ctx.inputs):
                o, pnl = h.vcycle_adjoint(b, x_in, lam, lam_b, lam_x)
                dom += o
                dpen += pnl
                lam, lam_x = lam_x, lam
            (om_dev, om_dt), (g_dev, g_dt) = ctx.param_like
            return (lam_b, torch.as_tensor(dom).to(device=om_dev, dtype=om_dt),
                    torch.as_tensor(dpen).to(device=g_dev, dtype=g_dt), None)

    return VCycleFn


class _LazyFn:
    _fn = None

    def apply(self, *args):
        if _LazyFn._fn is None:
            _LazyFn._fn = _vcycle_fn()
        return _LazyFn._fn.apply(*args)


_VCycleFn = _LazyFn()
