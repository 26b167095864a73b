"""MI355X (gfx950) GAP regression hot path: thin Python binding of libgap.

Argument marshalling only: every step runs in the HIP kernels of libgap.so
(built in-tree by ``paper_2310_03921_amd.build``).  PyTorch provides device
memory and the stream.  There is no CPU fallback: without the library or a
gfx950 device every call raises.

Column-major matrices (K_MM, K_NM, the least-squares matrix A) are held in
torch tensors of shape (columns, ld): element (row r, column c) is t[c, r].
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgap.so")

GAP_OK, GAP_E_INVALID, GAP_E_NOT_PD, GAP_E_RANK = 0, -1, -2, -3
GAP_E_NOMEM, GAP_E_HIP, GAP_E_UNSUPPORTED = -4, -5, -6
_STATUS = {0: "GAP_OK", -1: "GAP_E_INVALID", -2: "GAP_E_NOT_PD", -3: "GAP_E_RANK",
           -4: "GAP_E_NOMEM", -5: "GAP_E_HIP", -6: "GAP_E_UNSUPPORTED"}
PRECISION = {"fp64": 0, "bf16x3": 1}
_DT = {torch.float32: 0, torch.float64: 1}


class GapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class gap_atoms(ctypes.Structure):
    _fields_ = [("n_cfg", ctypes.c_int64), ("n_atoms", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("D", ctypes.c_int64),
                ("cfg_ptr", ctypes.c_void_p), ("desc", ctypes.c_void_p),
                ("desc_dt", ctypes.c_int), ("ld_desc", ctypes.c_int64),
                ("pair_ptr", ctypes.c_void_p), ("pair_j", ctypes.c_void_p),
                ("jac", ctypes.c_void_p), ("jac_dt", ctypes.c_int), ("ld_jac", ctypes.c_int64)]


class gap_sparse(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("D", ctypes.c_int64), ("ld_x", ctypes.c_int64),
                ("X", ctypes.c_void_p), ("zeta", ctypes.c_int), ("delta", ctypes.c_double)]


class gap_fit_info(ctypes.Structure):
    _fields_ = [("resid_norm", ctypes.c_double * 8), ("min_abs_rdiag", ctypes.c_double),
                ("max_abs_rdiag", ctypes.c_double), ("refine_done", ctypes.c_int)]


_lib = None


def lib():
    """Load libgap.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2310_03921_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        S = ctypes.c_int
        sigs = {
            "gap_create": ([ctypes.POINTER(P), I32, P], S),
            "gap_destroy": ([P], S),
            "gap_last_error": ([P], ctypes.c_char_p),
            "gap_sync": ([P], S),
            "gap_workspace_query": ([P, P, P, ctypes.POINTER(ctypes.c_size_t)], S),
            "gap_pair_transpose": ([P, P, P, P], S),
            "gap_build_kmm": ([P, P, P, I64], S),
            "gap_build_knm": ([P, P, P, I32, P, I64], S),
            "gap_build_knm_species": ([P, P, P, I32, P, I32, P, I64], S),
            "gap_predict_species": ([P, P, P, P, I32, P, I32, P, P, P, P], S),
            "gap_lstsq": ([P, P, I64, I64, I64, P, P], S),
            "gap_fit": ([P, P, I64, I64, P, P, P, ctypes.c_double, P, P, I32, P, P], S),
            "gap_build_local_rows": ([P, P, P, P, I64, P, I64], S),
            "gap_build_virial_rows": ([P, P, P, P, P, I64], S),
            "gap_predict_variance": ([P, P, P, P, ctypes.c_double, P, I64, P], S),
            "gap_select_cur": ([P, P, I64, ctypes.c_double, P, P, P], S),
            "gap_build_2b_rows": ([P, P, P, P, P, I64], S),
            "gap_build_kmm_2b": ([P, P, P, I64], S),
            "gap_predict_2b": ([P, P, P, P, P, P, P], S),
            "gap_fold_init": ([P, P, I64, I64, P, ctypes.c_double], S),
            "gap_fold_rows": ([P, P, I64, I64, I64, P, P], S),
            "gap_fold_solve": ([P, P, I64, I64, P, P, P], S),
            "gap_refine_rows": ([P, P, P, P, P, P, P, P], S),
            "gap_refine_weights": ([P, P, P, P, I64], S),
            "gap_refine_rows_s": ([P, P, P, P, I64, P, P, P, P, P], S),
            "gap_refine_solve": ([P, P, I64, I64, P, ctypes.c_double, P, P], S),
            "gap_predict": ([P, P, P, P, I32, P, P, P, P], S),
            "gap_predict_backward": ([P, P, P, P, I32, P, P, P, P], S),
            "gap_forces": ([P, P, P, P], S),
            "gap_forces_noalloc": ([P, P, P, P], S),
            "gap_split_bf16x3": ([P, P, I32, I64, I64, I64, P, P, P, P], S),
            "gap_set_workspace_limit": ([P, ctypes.c_size_t], S),
            "gap_set_fit_report": ([P, I32], S),
            "gap_timing": ([P, I32], S),
            "gap_timing_read": ([P, P, P, I32], S),
            "gap_timing_name": ([I32], ctypes.c_char_p),
            "gap_timing_count": ([], I32),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _f64(t: torch.Tensor) -> torch.Tensor:
    """FP64 contiguous view or copy of a device tensor (the ABI takes double*)."""
    return t.to(torch.float64).contiguous()


def _round4(n: int) -> int:
    return (n + 3) // 4 * 4


def _aligned(t: torch.Tensor) -> bool:
    """The ABI's vector loads need 32-byte aligned base pointers."""
    return t.data_ptr() % 32 == 0


def padded_rows(x: torch.Tensor, D: int, dtype=None, device=None) -> torch.Tensor:
    """A (..., D) array as a contiguous, 32-byte aligned device tensor of rows
    zero-padded to round4(D) (the input itself when it already is one)."""
    x = torch.as_tensor(x)
    dtype = dtype or x.dtype
    if D % 4 == 0:
        y = x.to(device=device, dtype=dtype).contiguous()
        return y if _aligned(y) else y.clone()
    out = torch.zeros(*x.shape[:-1], _round4(D), dtype=dtype, device=device)
    out[..., :D] = x.to(device=device, dtype=dtype)
    return out


def _aligned_view(t: torch.Tensor | None) -> torch.Tensor | None:
    """t itself when its base is 32-byte aligned, else an aligned copy (a row
    range of an FP32 array with an odd row offset starts 16 bytes off)."""
    if t is None or t.numel() == 0 or _aligned(t):
        return t
    return t.clone()


@dataclass
class Atoms:
    """Device arrays of a batch of configurations (see gap_atoms in gap.h)."""
    cfg_ptr: torch.Tensor      # int64 [n_cfg+1]
    desc: torch.Tensor         # f32/f64 [n_atoms, ld]
    pair_ptr: torch.Tensor     # int64 [n_atoms+1]
    pair_j: torch.Tensor       # int32 [n_pairs]
    jac: torch.Tensor | None   # f32/f64 [n_pairs, 3, ld]
    D: int

    @classmethod
    def from_host(cls, cfg_ptr, desc, pair_ptr, pair_j, jac, device="cuda", desc_dtype=None,
                  jac_dtype=None):
        desc = torch.as_tensor(desc)
        D = int(desc.shape[1])
        j = None
        if jac is not None:
            jt = torch.as_tensor(jac)
            j = padded_rows(jt, D, dtype=jac_dtype or jt.dtype, device=device)
        return cls(torch.as_tensor(cfg_ptr, dtype=torch.int64).to(device),
                   padded_rows(desc, D, dtype=desc_dtype or desc.dtype, device=device),
                   torch.as_tensor(pair_ptr, dtype=torch.int64).to(device),
                   torch.as_tensor(pair_j, dtype=torch.int32).to(device), j, D)

    def configs(self, c0: int, c1: int) -> "Atoms":
        """Configurations [c0, c1) of this batch: descriptors and Jacobians are
        views (no copy) when their first row is 32-byte aligned, else aligned
        copies; the three index arrays are rebased copies."""
        cp = self.cfg_ptr[c0:c1 + 1]
        a0, a1 = int(cp[0]), int(cp[-1])
        pp = self.pair_ptr[a0:a1 + 1]
        p0, p1 = int(pp[0]), int(pp[-1])
        return Atoms(cp - a0, _aligned_view(self.desc[a0:a1]), pp - p0,
                     self.pair_j[p0:p1] - a0,
                     None if self.jac is None else _aligned_view(self.jac[p0:p1]), self.D)

    @property
    def n_cfg(self):
        return self.cfg_ptr.numel() - 1

    @property
    def n_atoms(self):
        return self.desc.shape[0]

    @property
    def n_pairs(self):
        return self.pair_j.numel()

    @property
    def n_rows(self):
        return self.n_cfg + 3 * self.n_atoms

    def struct(self) -> gap_atoms:
        s = gap_atoms()
        s.n_cfg, s.n_atoms, s.n_pairs, s.D = self.n_cfg, self.n_atoms, self.n_pairs, self.D
        s.cfg_ptr = self.cfg_ptr.data_ptr()
        s.desc = self.desc.data_ptr()
        s.desc_dt = _DT[self.desc.dtype]
        s.ld_desc = self.desc.shape[1]
        s.pair_ptr = self.pair_ptr.data_ptr()
        s.pair_j = self.pair_j.data_ptr() if self.n_pairs else 0
        if self.jac is not None:
            s.jac = self.jac.data_ptr()
            s.jac_dt = _DT[self.jac.dtype]
            s.ld_jac = self.jac.shape[-1]
        else:
            s.jac, s.jac_dt, s.ld_jac = 0, 1, _round4(self.D)
        return s


@dataclass
class Sparse:
    """Sparse points X (FP64 [M, ld]) and the kernel hyperparameters zeta, delta."""
    X: torch.Tensor
    D: int
    zeta: int = 4
    delta: float = 1.0

    @classmethod
    def from_host(cls, X, zeta=4, delta=1.0, device="cuda"):
        X = torch.as_tensor(X, dtype=torch.float64)
        return cls(padded_rows(X, X.shape[1], dtype=torch.float64, device=device),
                   int(X.shape[1]), int(zeta), float(delta))

    @property
    def M(self):
        return self.X.shape[0]

    def struct(self) -> gap_sparse:
        s = gap_sparse()
        s.M, s.D, s.ld_x = self.M, self.D, self.X.shape[1]
        s.X = self.X.data_ptr()
        s.zeta, s.delta = self.zeta, self.delta
        return s


class gap_se2b(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("x", ctypes.c_void_p), ("delta", ctypes.c_double),
                ("theta", ctypes.c_double), ("r_cut", ctypes.c_double),
                ("cut_width", ctypes.c_double)]


@dataclass
class SE2b:
    """Two-body squared-exponential descriptor: sparse distances x (FP64 [M]) and
    the kernel parameters (see gap_se2b in gap.h)."""
    x: torch.Tensor
    delta: float = 1.0
    theta: float = 0.5
    r_cut: float = 4.5
    cut_width: float = 1.0

    @classmethod
    def from_host(cls, x, device="cuda", **kw):
        return cls(torch.as_tensor(x, dtype=torch.float64).to(device).contiguous(), **kw)

    @property
    def M(self):
        return self.x.numel()

    def struct(self) -> gap_se2b:
        s = gap_se2b()
        s.M, s.x = self.M, self.x.data_ptr()
        s.delta, s.theta, s.r_cut, s.cut_width = self.delta, self.theta, self.r_cut, self.cut_width
        return s


def colmajor(rows: int, cols: int, ld: int | None = None, device="cuda") -> torch.Tensor:
    """A zeroed column-major FP64 buffer: tensor (cols, ld), element (r, c) at t[c, r]."""
    ld = _round4(rows) if ld is None else ld
    return torch.zeros(cols, ld, dtype=torch.float64, device=device)


# Handles still open when the interpreter exits are closed by an atexit hook,
# while the HIP runtime is still up, rather than by __del__ during teardown
# (after the runtime, or a profiler attached to it, may have finalised).
_open_handles: "weakref.WeakSet[Gap]" = weakref.WeakSet()


@atexit.register
def _close_open_handles():
    for g in list(_open_handles):
        try:
            g.close()
        except Exception:
            pass


class Gap:
    """A libgap handle bound to one device and the current torch stream."""

    def __init__(self, device: int | None = None, stream: torch.cuda.Stream | None = None):
        L = lib()
        if not torch.cuda.is_available():
            raise RuntimeError("libgap needs a gfx950 GPU; none is visible")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        self._fit_report = True
        st = L.gap_create(ctypes.byref(self._h), self.device, ctypes.c_void_p(self.stream.cuda_stream))
        if st != GAP_OK:
            raise GapError(st, f"gap_create failed on device {self.device}")
        _open_handles.add(self)

    def close(self):
        if self._h:
            lib().gap_destroy(self._h)
            self._h = ctypes.c_void_p()
        _open_handles.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != GAP_OK:
            raise GapError(st, lib().gap_last_error(self._h).decode())

    def sync(self):
        self._check(lib().gap_sync(self._h))

    def set_workspace_limit(self, nbytes: int):
        """Cap the optional workspace (pre-split Jacobians); 0 removes the cap."""
        self._check(lib().gap_set_workspace_limit(self._h, int(nbytes)))

    def set_fit_report(self, final_residual: bool):
        """Whether fit() computes the residual after its last refinement step (default True)."""
        self._check(lib().gap_set_fit_report(self._h, 1 if final_residual else 0))
        self._fit_report = bool(final_residual)

    def timing(self, enable: bool = True):
        """Record HIP events around each library stage on this handle's stream."""
        self._check(lib().gap_timing(self._h, 1 if enable else 0))

    def timing_read(self, reset: bool = True) -> dict:
        """{stage: (total_ms, intervals)} accumulated since the last reset (waits for the events)."""
        L = lib()
        n = L.gap_timing_count()
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        self._check(L.gap_timing_read(self._h, ms, cnt, 1 if reset else 0))
        return {L.gap_timing_name(i).decode(): (ms[i], cnt[i]) for i in range(n)}

    def workspace_bytes(self, atoms: Atoms, sparse: Sparse) -> int:
        a, s, n = atoms.struct(), sparse.struct(), ctypes.c_size_t()
        self._check(lib().gap_workspace_query(self._h, ctypes.byref(a), ctypes.byref(s),
                                              ctypes.byref(n)))
        return n.value

    def pair_transpose(self, atoms: Atoms):
        a = atoms.struct()
        dev = atoms.desc.device
        tptr = torch.empty(atoms.n_atoms + 1, dtype=torch.int64, device=dev)
        tpair = torch.empty(max(atoms.n_pairs, 1), dtype=torch.int32, device=dev)
        self._check(lib().gap_pair_transpose(self._h, ctypes.byref(a), _ptr(tptr), _ptr(tpair)))
        return tptr, tpair[:atoms.n_pairs]

    def build_kmm(self, sparse: Sparse, out: torch.Tensor | None = None) -> torch.Tensor:
        M = sparse.M
        out = colmajor(M, M, M, sparse.X.device) if out is None else out
        s = sparse.struct()
        self._check(lib().gap_build_kmm(self._h, ctypes.byref(s), _ptr(out), out.shape[1]))
        return out

    def design_buffer(self, atoms: Atoms, sparse: Sparse) -> torch.Tensor:
        """Column-major buffer sized for gap_fit: ld = round4(n_rows + M), M + 1 columns."""
        return colmajor(atoms.n_rows + sparse.M, sparse.M + 1, device=sparse.X.device)

    def build_knm(self, atoms: Atoms, sparse: Sparse, precision: str = "fp64",
                  out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.design_buffer(atoms, sparse) if out is None else out
        a, s = atoms.struct(), sparse.struct()
        self._check(lib().gap_build_knm(self._h, ctypes.byref(a), ctypes.byref(s),
                                        PRECISION[precision], _ptr(out), out.shape[1]))
        return out

    def build_knm_species(self, atoms: Atoms, sparse: Sparse, species: torch.Tensor, z: int,
                          precision: str = "fp64", out: torch.Tensor | None = None,
                          col0: int = 0, row0: int = 0) -> torch.Tensor:
        """Rows of the per-species GP block of species z (only atoms with
        species == z are centres) written at (row0, col0) of the column-major
        buffer `out` (default: a new design buffer)."""
        out = self.design_buffer(atoms, sparse) if out is None else out
        a, s = atoms.struct(), sparse.struct()
        sp_ = species.to(torch.int32).contiguous()
        self._check(lib().gap_build_knm_species(
            self._h, ctypes.byref(a), ctypes.byref(s), PRECISION[precision], _ptr(sp_), int(z),
            ctypes.c_void_p(out.data_ptr() + 8 * (row0 + col0 * out.shape[1])), out.shape[1]))
        self._keep_species = sp_
        return out

    def predict_species(self, atoms: Atoms, sparse: Sparse, c: torch.Tensor,
                        species: torch.Tensor, z: int, precision: str = "fp64", e_atom=True,
                        e_cfg=True, dEdd=False, forces=False):
        """gap_predict of the per-species block of species z (other atoms: 0)."""
        dev = sparse.X.device
        N, D = atoms.n_atoms, atoms.D
        out = {
            "e_atom": torch.empty(N, dtype=torch.float64, device=dev) if e_atom else None,
            "e_cfg": torch.empty(atoms.n_cfg, dtype=torch.float64, device=dev) if e_cfg else None,
            "dEdd": torch.empty(N, D, dtype=torch.float64, device=dev) if dEdd else None,
            "forces": torch.empty(N, 3, dtype=torch.float64, device=dev) if forces else None,
        }
        a, s = atoms.struct(), sparse.struct()
        c = _f64(c)
        sp_ = species.to(torch.int32).contiguous()
        self._check(lib().gap_predict_species(self._h, ctypes.byref(a), ctypes.byref(s), _ptr(c),
                                              PRECISION[precision], _ptr(sp_), int(z),
                                              _ptr(out["e_atom"]), _ptr(out["e_cfg"]),
                                              _ptr(out["dEdd"]), _ptr(out["forces"])))
        self._keep_species = (sp_, c)
        return out

    def build_local_rows(self, atoms: Atoms, sparse: Sparse, atom_idx: torch.Tensor,
                         out: torch.Tensor | None = None, row0: int = 0) -> torch.Tensor:
        """Local-property rows of the atoms atom_idx (int32, device) written at
        rows [row0, row0 + n) of the column-major buffer `out` (default: a new
        n x M buffer)."""
        n = int(atom_idx.numel())
        M = sparse.M
        out = colmajor(n, M, device=sparse.X.device) if out is None else out
        a, s = atoms.struct(), sparse.struct()
        idx = atom_idx.to(torch.int32).contiguous()
        self._check(lib().gap_build_local_rows(
            self._h, ctypes.byref(a), ctypes.byref(s), _ptr(idx) if n else None, n,
            ctypes.c_void_p(out.data_ptr() + 8 * row0), out.shape[1]))
        self._keep_idx = idx
        return out

    def build_virial_rows(self, atoms: Atoms, sparse: Sparse, pair_r: torch.Tensor,
                          out: torch.Tensor | None = None, row0: int = 0) -> torch.Tensor:
        """Virial rows (9 per configuration) written at rows [row0, row0 + 9 n_cfg)
        of the column-major buffer `out` (default: a new 9 n_cfg x M buffer).
        pair_r: FP64 [n_pairs, 3] displacement vectors of the pairs."""
        M, n = sparse.M, 9 * atoms.n_cfg
        out = colmajor(n, M, device=sparse.X.device) if out is None else out
        a, s = atoms.struct(), sparse.struct()
        r = _f64(pair_r)
        self._check(lib().gap_build_virial_rows(
            self._h, ctypes.byref(a), ctypes.byref(s), _ptr(r),
            ctypes.c_void_p(out.data_ptr() + 8 * row0), out.shape[1]))
        self._keep_r = r
        return out

    def lstsq(self, A: torch.Tensor, m: int, n: int):
        x = torch.empty(n, dtype=torch.float64, device=A.device)
        rd = (ctypes.c_double * 2)()
        self._check(lib().gap_lstsq(self._h, _ptr(A), A.shape[1], m, n, _ptr(x), rd))
        return x, (rd[0], rd[1])

    def fit(self, A: torch.Tensor, n_rows: int, Kmm: torch.Tensor, y: torch.Tensor,
            sigma: torch.Tensor, jitter: float, sparse: Sparse, train: Atoms | None = None,
            refine_steps: int = 0):
        c = torch.empty(sparse.M, dtype=torch.float64, device=A.device)
        s = sparse.struct()
        info = gap_fit_info()
        tr = ctypes.byref(train.struct()) if train is not None else None
        y, sigma, Kmm = _f64(y), _f64(sigma), _f64(Kmm)
        self._check(lib().gap_fit(self._h, _ptr(A), A.shape[1], n_rows, _ptr(Kmm),
                                  _ptr(y), _ptr(sigma), float(jitter),
                                  tr, ctypes.byref(s), int(refine_steps), _ptr(c),
                                  ctypes.byref(info)))
        n_rn = info.refine_done + (1 if self._fit_report else 0)
        return c, {"resid_norm": list(info.resid_norm)[:n_rn],
                   "min_abs_rdiag": info.min_abs_rdiag, "max_abs_rdiag": info.max_abs_rdiag,
                   "refine_done": info.refine_done}

    # ------------------------------------------------------- streamed fit
    def fold_buffer(self, M: int, max_rows: int, device="cuda") -> torch.Tensor:
        """State of a streamed fit: column-major, M + 1 columns, ld = round4(M + 1 + max_rows)."""
        return colmajor(M + 1 + max_rows, M + 1, device=device)

    def fold_block(self, T: torch.Tensor, M: int, col0: int = 0) -> int:
        """Device address of the block area (row M + 1) of a fold state, column col0."""
        return T.data_ptr() + 8 * (M + 1 + col0 * T.shape[1])

    def build_knm_block(self, atoms: Atoms, sparse: Sparse, T: torch.Tensor,
                        precision: str = "fp64", M: int | None = None, col0: int = 0):
        """L-hat K_NM of `atoms` written into the block area of the fold state T
        (of M columns, default sparse.M), from column col0 on."""
        a, s = atoms.struct(), sparse.struct()
        M = sparse.M if M is None else M
        self._check(lib().gap_build_knm(self._h, ctypes.byref(a), ctypes.byref(s),
                                        PRECISION[precision],
                                        ctypes.c_void_p(self.fold_block(T, M, col0)),
                                        T.shape[1]))

    # ------------------------------------------------ two-body SE descriptor
    def build_2b_rows(self, atoms: Atoms, k2: SE2b, pair_r: torch.Tensor,
                      out: torch.Tensor | None = None, row0: int = 0, col0: int = 0):
        """Two-body rows (n_cfg + 3 n_atoms) x k2.M written at (row0, col0) of the
        column-major buffer `out` (default: a new buffer)."""
        n = atoms.n_rows
        out = colmajor(n, k2.M, device=k2.x.device) if out is None else out
        a, s = atoms.struct(), k2.struct()
        r = _f64(pair_r)
        self._check(lib().gap_build_2b_rows(
            self._h, ctypes.byref(a), _ptr(r), ctypes.byref(s),
            ctypes.c_void_p(out.data_ptr() + 8 * (row0 + col0 * out.shape[1])), out.shape[1]))
        self._keep_r = r
        return out

    def build_2b_block(self, atoms: Atoms, k2: SE2b, pair_r: torch.Tensor, T: torch.Tensor,
                       M: int, col0: int):
        """Two-body rows written into the block area of a fold state of M columns."""
        return self.build_2b_rows(atoms, k2, pair_r, out=T, row0=M + 1, col0=col0)

    def build_kmm_2b(self, k2: SE2b, out: torch.Tensor | None = None, row0: int = 0,
                     col0: int = 0) -> torch.Tensor:
        out = colmajor(k2.M, k2.M, k2.M, k2.x.device) if out is None else out
        s = k2.struct()
        self._check(lib().gap_build_kmm_2b(
            self._h, ctypes.byref(s),
            ctypes.c_void_p(out.data_ptr() + 8 * (row0 + col0 * out.shape[1])), out.shape[1]))
        return out

    def predict_2b(self, atoms: Atoms, k2: SE2b, pair_r: torch.Tensor, c: torch.Tensor,
                   e_cfg=True, forces=True):
        dev = k2.x.device
        out = {"e_cfg": torch.empty(atoms.n_cfg, dtype=torch.float64, device=dev) if e_cfg else None,
               "forces": torch.empty(atoms.n_atoms, 3, dtype=torch.float64, device=dev)
               if forces else None}
        a, s = atoms.struct(), k2.struct()
        r, c = _f64(pair_r), _f64(c)
        self._check(lib().gap_predict_2b(self._h, ctypes.byref(a), _ptr(r), ctypes.byref(s),
                                         _ptr(c), _ptr(out["e_cfg"]), _ptr(out["forces"])))
        self._keep_r = (r, c)
        return out

    def fold_init(self, T: torch.Tensor, M: int, Kmm: torch.Tensor, jitter: float):
        self._check(lib().gap_fold_init(self._h, _ptr(T), T.shape[1], M, _ptr(_f64(Kmm)),
                                        float(jitter)))

    def fold_rows(self, T: torch.Tensor, M: int, n_rows: int, y: torch.Tensor,
                  sigma: torch.Tensor):
        y, sigma = _f64(y), _f64(sigma)
        self._check(lib().gap_fold_rows(self._h, _ptr(T), T.shape[1], M, n_rows, _ptr(y),
                                        _ptr(sigma)))
        # the call is asynchronous: keep the inputs alive until the stream passes it
        self._keep = (y, sigma)

    def fold_solve(self, T: torch.Tensor, M: int):
        c = torch.empty(M, dtype=torch.float64, device=T.device)
        res = ctypes.c_double()
        rd = (ctypes.c_double * 2)()
        self._check(lib().gap_fold_solve(self._h, _ptr(T), T.shape[1], M, _ptr(c),
                                         ctypes.byref(res), rd))
        self._keep = None
        return c, res.value, (rd[0], rd[1])

    @staticmethod
    def _inplace_f64(t: torch.Tensor, name: str) -> torch.Tensor:
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise GapError(GAP_E_INVALID, f"{name} must be a contiguous float64 tensor (updated in place)")
        return t

    def refine_rows(self, atoms: Atoms, sparse: Sparse, c: torch.Tensor, y: torch.Tensor,
                    sigma: torch.Tensor, g: torch.Tensor, rr: torch.Tensor | None = None):
        """g += K^T Sigma^-1/2 r (and rr += r . r) over the batch's rows, with
        r = Sigma^-1/2 (y - K c) and K the exact FP64 rows; y and sigma in the
        batch's row order (energies of its configurations, then forces)."""
        c, y, sigma = _f64(c), _f64(y), _f64(sigma)
        self._inplace_f64(g, "g")
        if rr is not None:
            self._inplace_f64(rr, "rr")
        a, s = atoms.struct(), sparse.struct()
        self._check(lib().gap_refine_rows(self._h, ctypes.byref(a), ctypes.byref(s), _ptr(c),
                                          _ptr(y), _ptr(sigma), _ptr(g), _ptr(rr)))
        # the call is asynchronous: keep the inputs alive until the stream passes it
        self._keep = (c, y, sigma)

    def refine_weights(self, atoms: Atoms, sparse: Sparse, out: torch.Tensor | None = None):
        """The batch's exact FP64 kernel-gradient scale S [n_atoms, round4(M)],
        kept between refinement passes (gap_refine_rows_s)."""
        M = sparse.M
        if out is None:
            out = torch.empty(max(atoms.n_atoms, 1), _round4(M), dtype=torch.float64,
                              device=sparse.X.device)
        a, s = atoms.struct(), sparse.struct()
        self._check(lib().gap_refine_weights(self._h, ctypes.byref(a), ctypes.byref(s), _ptr(out),
                                             out.shape[1]))
        return out

    def refine_rows_s(self, atoms: Atoms, sparse: Sparse, S: torch.Tensor, c: torch.Tensor,
                      y: torch.Tensor, sigma: torch.Tensor, g: torch.Tensor,
                      rr: torch.Tensor | None = None):
        """refine_rows with the batch's S from refine_weights."""
        c, y, sigma = _f64(c), _f64(y), _f64(sigma)
        self._inplace_f64(g, "g")
        if rr is not None:
            self._inplace_f64(rr, "rr")
        a, s = atoms.struct(), sparse.struct()
        self._check(lib().gap_refine_rows_s(self._h, ctypes.byref(a), ctypes.byref(s), _ptr(S),
                                            S.shape[1], _ptr(c), _ptr(y), _ptr(sigma), _ptr(g),
                                            _ptr(rr)))
        self._keep = (c, y, sigma)

    def refine_solve(self, R: torch.Tensor, M: int, Kmm: torch.Tensor, jitter: float,
                     g: torch.Tensor, c: torch.Tensor):
        """c += (R^T R)^-1 (g - (K_MM + jitter I) c); g is overwritten by the step.
        R: a column-major factor (A after fit, or a fold state)."""
        self._inplace_f64(g, "g")
        self._inplace_f64(c, "c")
        self._check(lib().gap_refine_solve(self._h, _ptr(R), R.shape[1], M, _ptr(_f64(Kmm)),
                                           float(jitter), _ptr(g), _ptr(c)))
        self._keep = None

    def predict(self, atoms: Atoms, sparse: Sparse, c: torch.Tensor, precision: str = "fp64",
                e_atom=True, e_cfg=True, dEdd=False, forces=False):
        dev = sparse.X.device
        N, D = atoms.n_atoms, atoms.D
        out = {
            "e_atom": torch.empty(N, dtype=torch.float64, device=dev) if e_atom else None,
            "e_cfg": torch.empty(atoms.n_cfg, dtype=torch.float64, device=dev) if e_cfg else None,
            "dEdd": torch.empty(N, D, dtype=torch.float64, device=dev) if dEdd else None,
            "forces": torch.empty(N, 3, dtype=torch.float64, device=dev) if forces else None,
        }
        a, s = atoms.struct(), sparse.struct()
        c = _f64(c)
        self._check(lib().gap_predict(self._h, ctypes.byref(a), ctypes.byref(s), _ptr(c),
                                      PRECISION[precision], _ptr(out["e_atom"]),
                                      _ptr(out["e_cfg"]), _ptr(out["dEdd"]), _ptr(out["forces"])))
        return out

    def predict_variance(self, atoms: Atoms, sparse: Sparse, Kmm: torch.Tensor, jitter: float,
                         R: torch.Tensor) -> torch.Tensor:
        """Predictive variance of each atom's local energy.  R: the column-major
        buffer whose leading M x M upper triangle is the fit's triangular factor
        (A after gap.fit, or a fold state)."""
        var = torch.empty(atoms.n_atoms, dtype=torch.float64, device=sparse.X.device)
        a, s = atoms.struct(), sparse.struct()
        self._check(lib().gap_predict_variance(self._h, ctypes.byref(a), ctypes.byref(s),
                                               _ptr(_f64(Kmm)), float(jitter), _ptr(R),
                                               R.shape[1], _ptr(var)))
        return var

    def select_cur(self, atoms: Atoms, n_sparse: int, jitter: float = 0.0,
                   u: torch.Tensor | None = None):
        """CUR sparse-point selection: (indices [n_sparse] int32 in decreasing
        key order, leverage [n_atoms])."""
        dev = atoms.desc.device
        idx = torch.empty(max(n_sparse, 1), dtype=torch.int32, device=dev)
        lev = torch.empty(atoms.n_atoms, dtype=torch.float64, device=dev)
        a = atoms.struct()
        uu = None if u is None else _f64(u)
        self._check(lib().gap_select_cur(self._h, ctypes.byref(a), int(n_sparse), float(jitter),
                                         _ptr(uu), _ptr(idx), _ptr(lev)))
        return idx[:n_sparse], lev

    def predict_backward(self, atoms: Atoms, sparse: Sparse, c: torch.Tensor, g_e: torch.Tensor,
                         precision: str = "fp64", d_desc=True, d_c=True, d_X=True):
        dev = sparse.X.device
        N, M, D = atoms.n_atoms, sparse.M, atoms.D
        dd = torch.empty(N, D, dtype=torch.float64, device=dev) if d_desc else None
        dc = torch.empty(M, dtype=torch.float64, device=dev) if d_c else None
        dX = torch.empty(M, D, dtype=torch.float64, device=dev) if d_X else None
        a, s = atoms.struct(), sparse.struct()
        c, g_e = _f64(c), _f64(g_e)
        self._check(lib().gap_predict_backward(self._h, ctypes.byref(a), ctypes.byref(s), _ptr(c),
                                               PRECISION[precision], _ptr(g_e),
                                               _ptr(dd), _ptr(dc), _ptr(dX)))
        return dd, dc, dX

    def forces(self, atoms: Atoms, dEdd: torch.Tensor) -> torch.Tensor:
        F = torch.empty(atoms.n_atoms, 3, dtype=torch.float64, device=dEdd.device)
        a = atoms.struct()
        dEdd = _f64(dEdd)
        self._check(lib().gap_forces(self._h, ctypes.byref(a), _ptr(dEdd), _ptr(F)))
        return F

    def split_bf16x3(self, x: torch.Tensor, cols: int, transposed: bool = False):
        """The BF16X3 split of a row-major device array x [rows, ld] (f32 or f64,
        ld % 4 == 0): raw bf16 bits of hi and lo as int16 tensors [rows,
        round32(cols)], and with transposed=True (FP64 only) also the transposed
        halves [cols, round32(rows)]."""
        rows = x.shape[0]
        ldp, ldm = (cols + 31) // 32 * 32, (rows + 31) // 32 * 32
        dev = x.device
        hi = torch.empty(max(rows, 1), ldp, dtype=torch.int16, device=dev)
        lo = torch.empty_like(hi)
        ht = torch.empty(cols, ldm, dtype=torch.int16, device=dev) if transposed else None
        lt = torch.empty_like(ht) if transposed else None
        self._check(lib().gap_split_bf16x3(self._h, _ptr(x), _DT[x.dtype], rows, cols, x.shape[1],
                                           _ptr(hi), _ptr(lo), _ptr(ht), _ptr(lt)))
        return hi[:rows], lo[:rows], ht, lt

    def forces_noalloc(self, atoms: Atoms, dEdd: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """gap_forces with no device allocation inside the library: `out`
        (FP64 [n_atoms, 3]) is the caller's, the scratch is the library's static
        array.  dEdd must already be a contiguous FP64 device tensor."""
        if dEdd.dtype != torch.float64 or not dEdd.is_contiguous():
            raise GapError(GAP_E_INVALID, "dEdd must be a contiguous float64 tensor")
        a = atoms.struct()
        self._check(lib().gap_forces_noalloc(self._h, ctypes.byref(a), _ptr(dEdd), _ptr(out)))
        return out


_default = {}


def default_handle() -> Gap:
    dev = torch.cuda.current_device()
    key = (dev, torch.cuda.current_stream(dev).cuda_stream)
    if key not in _default:
        _default[key] = Gap(dev)
    return _default[key]


class GapPredict(torch.autograd.Function):
    """Per-atom energies eps_i = sum_m c_m delta^2 (d_i . x_m)^zeta with a hand-written backward.

    forward(desc [N, D], X [M, D], c [M], cfg_ptr, zeta, delta, precision) -> e_atom [N] (FP64).
    backward gives dE/d desc, dE/d X and dE/d c from gap_predict_backward, which
    recomputes (d . x)^(zeta-1) instead of keeping it from the forward pass.
    """

    @staticmethod
    def forward(ctx, desc, X, c, zeta=4, delta=1.0, precision="fp64"):
        gap = default_handle()
        D = desc.shape[1]
        dev = desc.device
        desc_p = padded_rows(desc.detach(), D, device=dev)
        atoms = Atoms(torch.tensor([0, desc.shape[0]], dtype=torch.int64, device=dev), desc_p.detach(),
                      torch.zeros(desc.shape[0] + 1, dtype=torch.int64, device=dev),
                      torch.zeros(0, dtype=torch.int32, device=dev), None, D)
        sp = Sparse(padded_rows(X.detach(), D, dtype=torch.float64, device=dev), D, int(zeta),
                    float(delta))
        c64 = c.detach().to(torch.float64).contiguous()
        out = gap.predict(atoms, sp, c64, precision, e_atom=True, e_cfg=False)["e_atom"]
        ctx.save_for_backward(desc, X, c)
        ctx.meta = (int(zeta), float(delta), precision)
        return out

    @staticmethod
    def backward(ctx, g_e):
        desc, X, c = ctx.saved_tensors
        zeta, delta, precision = ctx.meta
        gap = default_handle()
        D = desc.shape[1]
        dev = desc.device
        desc_p = padded_rows(desc.detach(), D, device=dev)
        atoms = Atoms(torch.tensor([0, desc.shape[0]], dtype=torch.int64, device=dev), desc_p.detach(),
                      torch.zeros(desc.shape[0] + 1, dtype=torch.int64, device=dev),
                      torch.zeros(0, dtype=torch.int32, device=dev), None, D)
        sp = Sparse(padded_rows(X.detach(), D, dtype=torch.float64, device=dev), D, zeta, delta)
        dd, dc, dX = gap.predict_backward(atoms, sp, c.detach().to(torch.float64).contiguous(),
                                          g_e.detach().to(torch.float64).contiguous(), precision,
                                          ctx.needs_input_grad[0], ctx.needs_input_grad[2],
                                          ctx.needs_input_grad[1])
        return (dd.to(desc.dtype) if dd is not None else None,
                dX.to(X.dtype) if dX is not None else None,
                dc.to(c.dtype) if dc is not None else None, None, None, None)


def gap_energy(desc, X, c, zeta=4, delta=1.0, precision="fp64"):
    """Differentiable per-atom GAP energies (see GapPredict)."""
    return GapPredict.apply(desc, X, c, zeta, delta, precision)
