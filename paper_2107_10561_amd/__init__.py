"""MI355X space-time Vanka multigrid: Python binding of the C ABI in include/stv.h.

Argument marshalling only: every step of the solver runs in the HIP library
(_lib/libstv.so).  Device vectors are torch float64 CUDA tensors; the library
launches on the stream current when the Solver is created.  Importing this
module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libstv.so")

STV_OK, STV_EINVAL, STV_ENOMEM, STV_EHIP, STV_ESTATE, STV_ESINGULAR, STV_ENOCONV, STV_ENUMERIC = \
    0, -1, -2, -3, -4, -5, -6, -7
STV_F64, STV_F32, STV_STORE_FULL = 0, 1, 2
STV_LAST_WRITER, STV_POU, STV_ADDITIVE = 0, 1, 2
KERNEL_CLASSES = {"sweep": 0, "residual": 1, "transfer": 2, "coarse": 3, "krylov": 4,
                  "inverse": 5, "coarse_factor": 6, "graph": 7}
_ERRNAMES = {STV_EINVAL: "STV_EINVAL", STV_ENOMEM: "STV_ENOMEM", STV_EHIP: "STV_EHIP",
             STV_ESTATE: "STV_ESTATE", STV_ESINGULAR: "STV_ESINGULAR",
             STV_ENOCONV: "STV_ENOCONV", STV_ENUMERIC: "STV_ENUMERIC"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                      "(run paper_2107_10561_amd/build.py or __graft_entry__.build())")


class StvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class _Level(ctypes.Structure):
    _fields_ = [("n_sdofs", ctypes.c_int32), ("bsr_rowptr", ctypes.c_void_p),
                ("bsr_col", ctypes.c_void_p), ("bsr_val", ctypes.c_void_p),
                ("nnzb", ctypes.c_int64), ("n_cells", ctypes.c_int32), ("n_ls", ctypes.c_int32),
                ("cell_sdofs", ctypes.c_void_p), ("P_rowptr", ctypes.c_void_p),
                ("P_col", ctypes.c_void_p), ("P_val", ctypes.c_void_p), ("P_nnz", ctypes.c_int64)]


class _MG(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("omega", ctypes.c_double),
                ("mode", ctypes.c_int32)]


class _GP(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_it", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("use_x0", ctypes.c_int32), ("fixed_iters", ctypes.c_int32), ("mg", _MG)]


class _GI(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("true_relres", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int32),
                ("history_len", ctypes.c_int32)]


def _load():
    # torch first: the library then binds to the HIP runtime torch already
    # loaded (same soname), so one runtime owns the device, streams and memory
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    I64P = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "stv_create": (I, [ctypes.POINTER(P), I, P]),
        "stv_destroy": (None, [P]),
        "stv_last_error": (ctypes.c_char_p, [P]),
        "stv_validate_hierarchy": (I, [I, I, I, ctypes.POINTER(_Level), ctypes.c_char_p, ctypes.c_size_t]),
        "stv_set_hierarchy": (I, [P, I, I, I, ctypes.POINTER(_Level)]),
        "stv_build_cell_inverses": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "stv_residual": (I, [P, I, P, P, P]),
        "stv_vanka_sweep": (I, [P, I, P, P, I, D, I]),
        "stv_restrict": (I, [P, I, P, P]),
        "stv_prolongate_add": (I, [P, I, P, P]),
        "stv_coarse_solve": (I, [P, P, P]),
        "stv_vcycle": (I, [P, P, P, ctypes.POINTER(_MG)]),
        "stv_vcycle_noalloc": (I, [P, P, P, ctypes.POINTER(_MG)]),
        "stv_gmres_solve": (I, [P, P, P, ctypes.POINTER(_GP), ctypes.POINTER(_GI)]),
        "stv_get_cell_inverse": (I, [P, I, I, P]),
        "stv_level_info": (I, [P, I, I64P, I64P, I64P, I64P]),
        "stv_set_timing": (I, [P, I]),
        "stv_set_timing_filter": (I, [P, ctypes.c_uint, ctypes.c_uint]),
        "stv_set_option": (I, [P, I, ctypes.c_int64]),
        "stv_set_batch": (I, [P, I, I, I, ctypes.POINTER(I), ctypes.POINTER(ctypes.POINTER(_Level))]),
        "stv_instance_layout": (I, [P, I, ctypes.POINTER(I), I64P, I64P]),
        "stv_instance_info": (I, [P, I, ctypes.POINTER(_GI)]),
        "stv_set_launch": (I, [P, I, I, I]),
        "stv_vcycle_transposed": (I, [P, P, P, ctypes.POINTER(_MG)]),
        "stv_gmres_solve_transposed": (I, [P, P, P, ctypes.POINTER(_GP), ctypes.POINTER(_GI)]),
        "stv_cell_contract": (I, [P, I, P, P, I, P, P, P, P, P, P]),
        "stv_cell_dot": (I, [P, I, P, I, P, P, P]),
        "stv_cell_gradient": (I, [P, I, P, P, I, P, P, P, P, P, D, I, P, P, D, P]),
        "stv_cell_scatter": (I, [P, I, I, P, P, P, P]),
        "stv_dot": (I, [P, P, P, P]),
        "stv_set_kron_factors": (I, [P, I, P, P, P, P]),
        "stv_autotune": (I, [P, ctypes.POINTER(I), I]),
        "stv_transfer_shapes": (I, [P, I, I, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "stv_kernel_stats": (I, [P, I, I, I64P, ctypes.POINTER(D)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = _load()
EXPORTED = ("stv_create", "stv_destroy", "stv_last_error", "stv_validate_hierarchy",
            "stv_set_hierarchy", "stv_build_cell_inverses", "stv_residual", "stv_vanka_sweep",
            "stv_restrict", "stv_prolongate_add", "stv_coarse_solve", "stv_vcycle",
            "stv_gmres_solve", "stv_get_cell_inverse", "stv_level_info", "stv_set_timing",
            "stv_kernel_stats", "stv_set_option", "stv_set_batch", "stv_instance_layout",
            "stv_instance_info", "stv_set_launch", "stv_autotune", "stv_vcycle_transposed",
            "stv_gmres_solve_transposed", "stv_cell_contract", "stv_cell_dot", "stv_dot",
            "stv_set_kron_factors", "stv_set_timing_filter", "stv_vcycle_noalloc",
            "stv_cell_gradient", "stv_cell_scatter", "stv_transfer_shapes")

COARSE_ALGOS = {"auto": 0, "panels": 1, "slabs": 2, "tournament": 3}


def library():
    return _lib


def _get(L, key):
    return L[key] if isinstance(L, dict) else getattr(L, key)


def _marshal_levels(levels):
    """ABI level structs from generator levels (dicts or objects with n_sdofs,
    rowptr, col, val, cell_sdofs, P); returns (array, keepalive)."""
    keep = []
    arr = (_Level * len(levels))()
    for g, L in enumerate(levels):
        rp = np.ascontiguousarray(_get(L, "rowptr"), dtype=np.int32)
        col = np.ascontiguousarray(_get(L, "col"), dtype=np.int32)
        val = np.ascontiguousarray(_get(L, "val"), dtype=np.float64).reshape(-1)
        csd = np.ascontiguousarray(_get(L, "cell_sdofs"), dtype=np.int32)
        keep += [rp, col, val, csd]
        s = arr[g]
        s.n_sdofs = int(_get(L, "n_sdofs"))
        s.bsr_rowptr, s.bsr_col, s.bsr_val = rp.ctypes.data, col.ctypes.data, val.ctypes.data
        s.nnzb = int(col.shape[0])
        s.n_cells = int(csd.shape[0])
        s.n_ls = int(csd.shape[1]) if csd.ndim == 2 else 0
        s.cell_sdofs = csd.ctypes.data
        Pt = _get(L, "P")
        if Pt is not None:
            prp = np.ascontiguousarray(Pt[0], dtype=np.int32)
            pcol = np.ascontiguousarray(Pt[1], dtype=np.int32)
            pval = np.ascontiguousarray(Pt[2], dtype=np.float64)
            keep += [prp, pcol, pval]
            s.P_rowptr, s.P_col, s.P_val = prp.ctypes.data, pcol.ctypes.data, pval.ctypes.data
            s.P_nnz = int(pcol.shape[0])
        else:
            s.P_rowptr = s.P_col = s.P_val = None
            s.P_nnz = 0
    return arr, keep


def validate_hierarchy(levels, dim: int, k: int):
    """Host-only validation (no device needed).  Returns (status, message)."""
    arr, keep = _marshal_levels(levels)
    buf = ctypes.create_string_buffer(512)
    rc = _lib.stv_validate_hierarchy(len(levels), dim, k, arr, buf, 512)
    return rc, buf.value.decode()


class Solver:
    """One library context on one device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = ctypes.c_void_p()
        rc = _lib.stv_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != STV_OK:
            raise StvError(rc, _lib.stv_last_error(None).decode())
        self._h = h
        self.dim = self.k = self.b = None
        self.n_st = []

    def close(self):
        if getattr(self, "_h", None):
            _lib.stv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != STV_OK:
            raise StvError(rc, _lib.stv_last_error(self._h).decode())
        return rc

    def _vec(self, t, level, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise ValueError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != self.n_st[level]:
            raise ValueError(f"{name} has {t.numel()} entries, level {level} needs {self.n_st[level]}")
        return ctypes.c_void_p(t.data_ptr())

    def set_hierarchy(self, levels, dim: int, k: int):
        arr, keep = _marshal_levels(levels)
        self._check(_lib.stv_set_hierarchy(self._h, len(levels), dim, k, arr))
        self.n_inst = 1
        self.dim, self.k, self.b = dim, k, k + 1
        self.n_st = [int(_get(L, "n_sdofs")) * (k + 1) for L in levels]
        self.n_levels = len(levels)

    def set_batch(self, hierarchies, dim: int, k: int):
        """Upload many independent hierarchies (a list of level lists, each
        coarsest first) as one batch; finest-level vectors are then the
        instances' vectors concatenated (see instance_layout)."""
        n = len(hierarchies)
        marsh = [_marshal_levels(levels) for levels in hierarchies]
        nlev = (ctypes.c_int * n)(*[len(levels) for levels in hierarchies])
        ptrs = (ctypes.POINTER(_Level) * n)(*[ctypes.cast(a, ctypes.POINTER(_Level)) for a, _ in marsh])
        self._check(_lib.stv_set_batch(self._h, n, dim, k, nlev, ptrs))
        self.dim, self.k, self.b = dim, k, k + 1
        D = max(len(levels) for levels in hierarchies)
        self.n_levels = D
        self.n_st = []
        for g in range(D):
            tot = 0
            for levels in hierarchies:
                l = g - (D - len(levels))
                if l >= 0:
                    tot += int(_get(levels[l], "n_sdofs"))
            self.n_st.append(tot * (k + 1))
        self.n_inst = n

    def instance_layout(self, inst: int):
        """(levels, first vector element, vector length) of an instance on the
        packed finest level."""
        nl, off, rows = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.stv_instance_layout(self._h, inst, ctypes.byref(nl), ctypes.byref(off),
                                             ctypes.byref(rows)))
        return nl.value, off.value * self.b, rows.value * self.b

    def instance_info(self, inst: int):
        gi = _GI()
        self._check(_lib.stv_instance_info(self._h, inst, ctypes.byref(gi)))
        return dict(iters=gi.iters, restarts=gi.restarts, converged=bool(gi.converged),
                    true_relres=gi.true_relres)

    def build_cell_inverses(self, fp32: bool = False, full: bool = False):
        bl, bc = ctypes.c_int(-1), ctypes.c_int(-1)
        storage = (STV_F32 if fp32 else STV_F64) | (STV_STORE_FULL if full else 0)
        rc = _lib.stv_build_cell_inverses(self._h, storage, ctypes.byref(bl), ctypes.byref(bc))
        if rc == STV_ESINGULAR:
            err = StvError(rc, _lib.stv_last_error(self._h).decode())
            err.level, err.cell = bl.value, bc.value
            raise err
        self._check(rc)

    def residual(self, level, r, d, out):
        rp = self._vec(r, level, "r") if r is not None else None
        self._check(_lib.stv_residual(self._h, level, rp, self._vec(d, level, "d"),
                                      self._vec(out, level, "out")))

    def vanka_sweep(self, level, r, d, n_sweeps=1, omega=0.7, mode=STV_LAST_WRITER):
        self._check(_lib.stv_vanka_sweep(self._h, level, self._vec(r, level, "r"),
                                         self._vec(d, level, "d"), n_sweeps, omega, mode))

    def restrict(self, level, rho, r_c):
        self._check(_lib.stv_restrict(self._h, level, self._vec(rho, level, "rho"),
                                      self._vec(r_c, level - 1, "r_c")))

    def prolongate_add(self, level, d_c, d):
        self._check(_lib.stv_prolongate_add(self._h, level, self._vec(d_c, level - 1, "d_c"),
                                            self._vec(d, level, "d")))

    def coarse_solve(self, r, d):
        self._check(_lib.stv_coarse_solve(self._h, self._vec(r, 0, "r"), self._vec(d, 0, "d")))

    def vcycle(self, r, d, nu1=2, nu2=2, omega=0.7, mode=STV_LAST_WRITER):
        top = self.n_levels - 1
        mg = _MG(nu1, nu2, omega, mode)
        self._check(_lib.stv_vcycle(self._h, self._vec(r, top, "r"), self._vec(d, top, "d"),
                                    ctypes.byref(mg)))

    def vcycle_noalloc(self, r, d, nu1=2, nu2=2, omega=0.7, mode=STV_LAST_WRITER):
        """The same V-cycle with its work vectors in the library's fixed device
        workspace: the call allocates no device memory."""
        top = self.n_levels - 1
        mg = _MG(nu1, nu2, omega, mode)
        self._check(_lib.stv_vcycle_noalloc(self._h, self._vec(r, top, "r"),
                                            self._vec(d, top, "d"), ctypes.byref(mg)))

    def gmres_solve(self, b, x, restart=30, max_it=1000, rtol=1e-8, use_x0=False,
                    fixed_iters=0, nu1=2, nu2=2, omega=0.7, mode=STV_LAST_WRITER,
                    raise_on_noconv=True):
        top = self.n_levels - 1
        gp = _GP(restart, max_it, rtol, int(use_x0), fixed_iters, _MG(nu1, nu2, omega, mode))
        cap = max_it + 2 if fixed_iters == 0 else fixed_iters + 2
        hist = (ctypes.c_double * cap)()
        gi = _GI(0, 0, 0, 0.0, hist, cap, 0)
        rc = _lib.stv_gmres_solve(self._h, self._vec(b, top, "b"), self._vec(x, top, "x"),
                                  ctypes.byref(gp), ctypes.byref(gi))
        info = dict(iters=gi.iters, restarts=gi.restarts, converged=bool(gi.converged),
                    true_relres=gi.true_relres, history=list(hist[:gi.history_len]), status=rc)
        if rc != STV_OK and (rc != STV_ENOCONV or raise_on_noconv):
            self._check(rc)
        return info

    def vcycle_transposed(self, r, d, nu1=2, nu2=2, omega=0.7):
        top = self.n_levels - 1
        mg = _MG(nu1, nu2, omega, STV_LAST_WRITER)
        self._check(_lib.stv_vcycle_transposed(self._h, self._vec(r, top, "r"),
                                               self._vec(d, top, "d"), ctypes.byref(mg)))

    def gmres_solve_transposed(self, b, x, restart=30, max_it=1000, rtol=1e-8, use_x0=False,
                               fixed_iters=0, nu1=2, nu2=2, omega=0.7, raise_on_noconv=True):
        """Solve J^T x = b (inverses built with full=True)."""
        top = self.n_levels - 1
        gp = _GP(restart, max_it, rtol, int(use_x0), fixed_iters,
                 _MG(nu1, nu2, omega, STV_LAST_WRITER))
        gi = _GI(0, 0, 0, 0.0, None, 0, 0)
        rc = _lib.stv_gmres_solve_transposed(self._h, self._vec(b, top, "b"),
                                             self._vec(x, top, "x"), ctypes.byref(gp),
                                             ctypes.byref(gi))
        info = dict(iters=gi.iters, restarts=gi.restarts, converged=bool(gi.converged),
                    true_relres=gi.true_relres, status=rc)
        if rc != STV_OK and (rc != STV_ENOCONV or raise_on_noconv):
            self._check(rc)
        return info

    def _out(self, t, n, name):
        """A device output array of exactly n float64 entries."""
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise ValueError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries, {n} needed")
        return ctypes.c_void_p(t.data_ptr())

    def cell_contract(self, level, lam, x, refs, kptr, kidx, kw, tw, out):
        """out[T] = sum_l tw[l] lam_T,l . K_T x_T,l, K_T = sum kw refs[kidx] (device out)."""
        refs = np.ascontiguousarray(refs, dtype=np.float64)
        kptr = np.ascontiguousarray(kptr, dtype=np.int32)
        kidx = np.ascontiguousarray(kidx, dtype=np.int32)
        kw = np.ascontiguousarray(kw, dtype=np.float64)
        tw = np.ascontiguousarray(tw, dtype=np.float64)
        n_cells = self.level_info(level)["n_cells"]
        if kptr.shape != (n_cells + 1,):
            raise ValueError(f"kptr needs {n_cells + 1} entries")
        if kidx.size != kw.size or (kptr.size and kptr[-1] > kidx.size):
            raise ValueError("kidx and kw must have kptr[-1] entries")
        if refs.ndim != 3 or tw.size != self.b:
            raise ValueError("refs must be (n_ref, n_ls, n_ls) and tw have k+1 entries")
        optr = self._out(out, n_cells, "out")
        self._check(_lib.stv_cell_contract(
            self._h, level, self._vec(lam, level, "lam"), self._vec(x, level, "x"),
            int(refs.shape[0]), refs.ctypes.data, kptr.ctypes.data, kidx.ctypes.data,
            kw.ctypes.data, tw.ctypes.data, optr))

    def cell_dot(self, level, lam, cells, f, out):
        """out[j] = sum over cell cells[j]'s DoFs of lam times f[j] (device out)."""
        cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1)
        f = np.ascontiguousarray(f, dtype=np.float64)
        n_loc = self.level_info(level)["n_loc"]
        if f.size != cells.size * n_loc:
            raise ValueError(f"f must hold {cells.size} x {n_loc} values")
        optr = self._out(out, int(cells.size), "out")
        self._check(_lib.stv_cell_dot(self._h, level, self._vec(lam, level, "lam"),
                                      int(cells.size), cells.ctypes.data, f.ctypes.data, optr))

    def cell_gradient(self, level, lam, x, refs, kptr, kidx, kw, tw, sc, cells, f, sf, out):
        """out[T] = sc * (cell_contract form of T) + sf * lam_T . f[k] for T = cells[k]
        (device out, one value per cell)."""
        refs = np.ascontiguousarray(refs, dtype=np.float64)
        kptr = np.ascontiguousarray(kptr, dtype=np.int32)
        kidx = np.ascontiguousarray(kidx, dtype=np.int32)
        kw = np.ascontiguousarray(kw, dtype=np.float64)
        tw = np.ascontiguousarray(tw, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1)
        f = np.ascontiguousarray(f, dtype=np.float64)
        info = self.level_info(level)
        n_cells = info["n_cells"]
        if kptr.shape != (n_cells + 1,):
            raise ValueError(f"kptr needs {n_cells + 1} entries")
        if kidx.size != kw.size or (kptr.size and kptr[-1] > kidx.size):
            raise ValueError("kidx and kw must have kptr[-1] entries")
        if refs.ndim != 3 or tw.size != self.b:
            raise ValueError("refs must be (n_ref, n_ls, n_ls) and tw have k+1 entries")
        if f.size != cells.size * info["n_loc"]:
            raise ValueError(f"f must hold {cells.size} x {info['n_loc']} values")
        optr = self._out(out, n_cells, "out")
        self._check(_lib.stv_cell_gradient(
            self._h, level, self._vec(lam, level, "lam"), self._vec(x, level, "x"),
            int(refs.shape[0]), refs.ctypes.data, kptr.ctypes.data, kidx.ctypes.data,
            kw.ctypes.data, tw.ctypes.data, float(sc), int(cells.size), cells.ctypes.data,
            f.ctypes.data, float(sf), optr))

    def cell_scatter(self, level, cells, coef, f, y):
        """y[DoF j of cell cells[k]] += coef[k] * f[k][j] (y: device vector of the level)."""
        cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1)
        coef = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1)
        f = np.ascontiguousarray(f, dtype=np.float64)
        n_loc = self.level_info(level)["n_loc"]
        if coef.size != cells.size or f.size != cells.size * n_loc:
            raise ValueError(f"coef must hold {cells.size} values and f {cells.size} x {n_loc}")
        self._check(_lib.stv_cell_scatter(self._h, level, int(cells.size), cells.ctypes.data,
                                          coef.ctypes.data, f.ctypes.data,
                                          self._vec(y, level, "y")))

    def dot(self, a, b):
        """Per-instance dot products of two finest-level vectors (host list)."""
        top = self.n_levels - 1
        out = (ctypes.c_double * self.n_inst)()
        self._check(_lib.stv_dot(self._h, self._vec(a, top, "a"), self._vec(b, top, "b"), out))
        return list(out)

    def get_cell_inverse(self, level, cell):
        info = self.level_info(level)
        n = info["n_loc"]
        out = np.empty((n, n), dtype=np.float64)
        self._check(_lib.stv_get_cell_inverse(self._h, level, cell, out.ctypes.data))
        return out

    def level_info(self, level):
        a, b, c, d = (ctypes.c_int64() for _ in range(4))
        self._check(_lib.stv_level_info(self._h, level, ctypes.byref(a), ctypes.byref(b),
                                        ctypes.byref(c), ctypes.byref(d)))
        return dict(n_sdofs=a.value, n_cells=b.value, n_loc=c.value, inverse_bytes=d.value)

    def set_coarse_algorithm(self, name: str):
        """Dense inversion of the coarsest matrix: "auto", "panels", "slabs" or
        "tournament"."""
        self._check(_lib.stv_set_option(self._h, 1, COARSE_ALGOS[name]))

    def set_kron_factors(self, level: int, mval, aval, C, tw):
        """Residual of `level` from its spatial factors (blocks = C[i,l] M +
        delta_il tw[i] A); mval = aval = None drops them."""
        if mval is None and aval is None:
            self._check(_lib.stv_set_kron_factors(self._h, level, None, None, None, None))
            return
        mval = np.ascontiguousarray(mval, dtype=np.float64)
        aval = np.ascontiguousarray(aval, dtype=np.float64)
        C = np.ascontiguousarray(C, dtype=np.float64)
        tw = np.ascontiguousarray(tw, dtype=np.float64)
        self._check(_lib.stv_set_kron_factors(self._h, level, mval.ctypes.data, aval.ctypes.data,
                                              C.ctypes.data, tw.ctypes.data))

    def set_launch(self, level: int, spmv_rows: int, sweep_wgs: int):
        """Launch shapes of one level's residual and sweep kernels."""
        self._check(_lib.stv_set_launch(self._h, level, spmv_rows, sweep_wgs))

    def transfer_shapes(self, level: int, p_shape: int = 0, pt_shape: int = 0):
        """Set (when > 0) and return the transfer shapes (P, P^T) between
        `level` and level-1: shape t takes 2^(t-1) lanes per row."""
        cp, ct = ctypes.c_int(0), ctypes.c_int(0)
        self._check(_lib.stv_transfer_shapes(self._h, level, p_shape, pt_shape,
                                             ctypes.byref(cp), ctypes.byref(ct)))
        return cp.value, ct.value

    def autotune(self):
        """Time the launch shapes on the device and keep the fastest; returns
        {level: (residual shape, sweep workgroups)}."""
        cap = 2 * self.n_levels
        ch = (ctypes.c_int * cap)()
        self._check(_lib.stv_autotune(self._h, ch, cap))
        return {g: (ch[2 * g], ch[2 * g + 1]) for g in range(self.n_levels)}

    def set_coarse_overlap(self, on: bool):
        """Coarse factorisation concurrent with the cell inverses (default) or before them."""
        self._check(_lib.stv_set_option(self._h, 3, int(bool(on))))

    def set_inverse_cus(self, n: int):
        """Compute units the 3d complex cell-inverse kernel may hold while the
        coarse factorisation runs beside it (0: no cap, the default; -1: five
        eighths of the device's)."""
        self._check(_lib.stv_set_option(self._h, 4, int(n)))

    def set_coarse_lookahead(self, on: bool):
        """Look-ahead updates in the complex-pivot coarse chain (default on)."""
        self._check(_lib.stv_set_option(self._h, 5, int(bool(on))))

    def set_graph(self, on: bool):
        """Replay the V-cycle from a captured HIP graph (identical results)."""
        self._check(_lib.stv_set_option(self._h, 2, int(bool(on))))

    def set_timing(self, on: bool, classes=None, levels=None):
        """Per-kernel timing on or off; classes (names of KERNEL_CLASSES) and
        levels (indices) restrict what is recorded (None: all)."""
        cmask = (1 << len(KERNEL_CLASSES)) - 1 if classes is None else \
            sum(1 << KERNEL_CLASSES[c] for c in classes)
        lmask = 0xFFFFFFFF if levels is None else sum(1 << g for g in levels)
        self._check(_lib.stv_set_timing_filter(self._h, cmask, lmask))
        self._check(_lib.stv_set_timing(self._h, int(on)))

    def kernel_stats(self, name: str, level: int = -1):
        """(launches, total ms) of one kernel class on one level (-1: all levels)."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        self._check(_lib.stv_kernel_stats(self._h, KERNEL_CLASSES[name], level, ctypes.byref(n),
                                          ctypes.byref(ms)))
        return n.value, ms.value
