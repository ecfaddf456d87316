"""Python binding of libghsvd.so (argument marshalling only).

Every step of the solve runs in the HIP library; PyTorch provides device
memory and the current stream.  Matrices are torch complex128 CUDA tensors in
column-major (Fortran) order, i.e. stride(0) == 1; `fortran_empty` and
`to_device_fortran` make such tensors.  Importing this module fails loudly
when the built library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# GHSVD_LIB selects another build of the same library (e.g. an instrumented one).
LIB_PATH = os.environ.get("GHSVD_LIB") or os.path.join(_PKG, "libghsvd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "(hipcc, gfx950). The solver has no CPU fallback.")

_lib = ctypes.CDLL(LIB_PATH)

FP64, MIXED = 0, 1
POINTWISE, BLOCKED = 0, 1
STATUS = {0: "ok", 1: "not converged", -1: "invalid argument", -2: "rank deficient",
          -3: "non-finite", -4: "workspace too small", -5: "device error"}


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("variant", ctypes.c_int), ("reduce", ctypes.c_int),
                ("block_width", ctypes.c_int), ("waves_per_pair", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("sort", ctypes.c_int),
                ("crit_literal", ctypes.c_int), ("inner_order", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("sweeps_fp32", ctypes.c_int),
                ("sweeps_fp64", ctypes.c_int), ("sweeps_blocked", ctypes.c_int),
                ("n2x2", ctypes.c_int), ("m_r", ctypes.c_int), ("p_r", ctypes.c_int),
                ("n_plus", ctypes.c_int), ("pairs_visited", ctypes.c_longlong),
                ("pairs_transformed", ctypes.c_longlong), ("pairs_big", ctypes.c_longlong),
                ("pw_visited", ctypes.c_longlong), ("pw_transformed", ctypes.c_longlong)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class FastInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("path", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("pad", ctypes.c_int), ("cond_est", ctypes.c_double),
                ("rotations", ctypes.c_longlong), ("hz", Info)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("pad", "hz")}
        d["path"] = "fast" if self.path == 0 else "hz"
        d["hz"] = self.hz.as_dict()
        return d


_p = ctypes.c_void_p
_i = ctypes.c_int
_sz = ctypes.c_size_t

_lib.ghsvd_default_options.argtypes = [ctypes.POINTER(Options)]
_lib.ghsvd_default_options.restype = None
_lib.ghsvd_workspace_size.argtypes = [_i, _i, _i, ctypes.POINTER(Options)]
_lib.ghsvd_workspace_size.restype = _sz
_lib.ghsvd_solve.argtypes = [_i, _i, _i, _p, _i, _p, _p, _i, _p, _p, _i, _p, _sz,
                             ctypes.POINTER(Options), ctypes.POINTER(Info), _p]
_lib.ghsvd_solve.restype = _i
_lib.ghsvd_workspace_size_batched.argtypes = [_i, _p, _p, _p, ctypes.POINTER(Options)]
_lib.ghsvd_workspace_size_batched.restype = _sz
_lib.ghsvd_solve_batched.argtypes = [_i, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _sz,
                                     ctypes.POINTER(Options), _p, _p]
_lib.ghsvd_solve_batched.restype = _i
_lib.ghsvd_reduce.argtypes = [_i, _i, _i, _p, _i, _p, _p, _i, _p, _i, _p, _p, _i, _p,
                              ctypes.POINTER(_i), _p]
_lib.ghsvd_reduce.restype = _i
_lib.ghsvd_pair_params.argtypes = [_i, _p, _p, _p, _p, _p, _p, ctypes.c_double, _i, _p, _p, _p]
_lib.ghsvd_pair_params.restype = _i
_lib.ghsvd_sweeps.argtypes = [_i, _i, _i, _p, _i, _i, _p, _i, _p, _i, _i, _i, _i, _p,
                              ctypes.POINTER(_i), _p]
_lib.ghsvd_sweeps.restype = _i
_lib.ghsvd_block_sweeps.argtypes = [_i, _i, _i, _p, _i, _i, _p, _i, _p, _i, _i, _i, _i, _i, _p,
                                    ctypes.POINTER(_i), _p]
_lib.ghsvd_block_sweeps.restype = _i
_lib.ghsvd_block_sweeps_noalloc.argtypes = _lib.ghsvd_block_sweeps.argtypes
_lib.ghsvd_block_sweeps_noalloc.restype = _i
NOALLOC_SCRATCH_BYTES = 32 << 20  # GHSVD_NOALLOC_SCRATCH_BYTES
_lib.ghsvd_round_robin.argtypes = [_i, _p, _p]
_lib.ghsvd_round_robin.restype = _i
_lib.ghsvd_profile_enable.argtypes = [_i]
_lib.ghsvd_profile_enable.restype = None
_lib.ghsvd_profile_read.argtypes = [_i, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
_lib.ghsvd_profile_read.restype = _i
_lib.ghsvd_autotune.argtypes = [_i, _p, _p, _p, _p, _p, _p, _p, _p, _p, _sz, ctypes.POINTER(Options),
                                ctypes.POINTER(_i), ctypes.POINTER(_i), _p, _p]
_lib.ghsvd_autotune.restype = _i
_lib.ghsvd_autotune_clear.argtypes = []
_lib.ghsvd_autotune_clear.restype = None
_lib.ghsvd_full.argtypes = [_i, _i, _i, _p, _i, _i, _p, _i, _p, _i, _p, _i, _p, _i, _p, _p, _p, _i,
                            _p, _sz, _p]
_lib.ghsvd_full.restype = _i
_lib.ghsvd_full_workspace_size.argtypes = [_i]
_lib.ghsvd_full_workspace_size.restype = _sz
_lib.ghsvd_fast_workspace_size.argtypes = [_i, _i, _i, ctypes.POINTER(Options)]
_lib.ghsvd_fast_workspace_size.restype = _sz
_lib.ghsvd_solve_fast.argtypes = [_i, _i, _i, _p, _i, _p, _p, _i, _p, _p, _i, ctypes.c_double, _i,
                                  _p, _sz, ctypes.POINTER(Options), ctypes.POINTER(FastInfo), _p]
_lib.ghsvd_solve_fast.restype = _i
_lib.ghsvd_hebpj_workspace_size.argtypes = [_i, _i]
_lib.ghsvd_hebpj_workspace_size.restype = _sz
_lib.ghsvd_hebpj_batched.argtypes = [_i, _i, _p, _p, _p, _p, _p, _p, _sz, _p]
_lib.ghsvd_hebpj_batched.restype = _i
_lib.ghsvd_phase1_workspace_size.argtypes = [_i, _i]
_lib.ghsvd_phase1_workspace_size.restype = _sz
_lib.ghsvd_phase1.argtypes = [_i, _i, _i, _p, _p, _i, _p, _p, _i, _p, _p, _i, _p, _p, _sz, _p]
_lib.ghsvd_phase1.restype = _i
_lib.ghsvd_status_string.argtypes = [_i]
_lib.ghsvd_status_string.restype = ctypes.c_char_p

EXPORTED = ["ghsvd_default_options", "ghsvd_workspace_size", "ghsvd_solve",
            "ghsvd_workspace_size_batched", "ghsvd_solve_batched", "ghsvd_reduce",
            "ghsvd_pair_params", "ghsvd_sweeps", "ghsvd_round_robin", "ghsvd_status_string",
            "ghsvd_profile_enable", "ghsvd_profile_read", "ghsvd_block_sweeps",
            "ghsvd_autotune", "ghsvd_autotune_clear", "ghsvd_full", "ghsvd_full_workspace_size",
            "ghsvd_block_sweeps_noalloc", "ghsvd_hebpj_workspace_size", "ghsvd_hebpj_batched",
            "ghsvd_phase1_workspace_size", "ghsvd_phase1", "ghsvd_fast_workspace_size",
            "ghsvd_solve_fast"]


class GhsvdError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status} ({_lib.ghsvd_status_string(status).decode()})")
        self.status = status


# --- tensor helpers ---------------------------------------------------------------

def fortran_empty(rows: int, cols: int, dtype=torch.complex128, device="cuda") -> torch.Tensor:
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def to_device_fortran(a: np.ndarray, device="cuda") -> torch.Tensor:
    a = np.asarray(a)
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to(device)
    return t.t()


def _check_fortran(t: torch.Tensor, name: str) -> int:
    if t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    return max(t.stride(1), t.shape[0], 1)


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


INNER = {"full": 0, "cross": 1, "fb": 2, "full_jqr": 3, "fb_jqr": 4, "ml_bo": 5, "ml_fb": 6}


def options(precision="fp64", variant="pointwise", reduce=True, block_width=0,
            waves_per_pair=0, max_sweeps=0, sort=True, crit_literal=False,
            inner_order="cross") -> Options:
    o = Options()
    _lib.ghsvd_default_options(ctypes.byref(o))
    o.precision = {"fp64": FP64, "mixed": MIXED}[precision]
    o.variant = {"pointwise": POINTWISE, "blocked": BLOCKED}[variant]
    o.reduce = int(bool(reduce))
    o.block_width = int(block_width)
    o.waves_per_pair = int(waves_per_pair)
    if int(max_sweeps) > 0:
        o.max_sweeps = int(max_sweeps)
    o.sort = int(bool(sort))
    o.crit_literal = int(bool(crit_literal))
    o.inner_order = INNER[inner_order]
    return o


def workspace_size(m: int, n: int, p: int, opt: Options | None = None) -> int:
    return int(_lib.ghsvd_workspace_size(m, n, p, ctypes.byref(opt) if opt else None))


def solve(F: torch.Tensor, J: torch.Tensor, G: torch.Tensor, *, work: torch.Tensor | None = None,
          stream=None, check=True, out=None, **kw):
    """lambda (n,) float64, X (n, n) complex128 column-major, info dict."""
    opt = options(**kw)
    m, n = F.shape
    p = G.shape[0]
    ldf = _check_fortran(F, "F")
    ldg = _check_fortran(G, "G")
    if J.dtype != torch.int8 or not J.is_cuda or J.numel() != m:
        raise TypeError("J must be an int8 CUDA tensor with m entries")
    if out is None:
        lam = torch.empty(n, dtype=torch.float64, device=F.device)
        X = fortran_empty(n, n, device=F.device)
    else:
        lam, X = out
    if work is None:
        need = workspace_size(m, n, p, opt)
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=F.device)
    info = Info()
    rc = _lib.ghsvd_solve(m, n, p, F.data_ptr(), ldf, J.data_ptr(), G.data_ptr(), ldg,
                          lam.data_ptr(), X.data_ptr(), max(X.stride(1), n), work.data_ptr(),
                          work.numel(), ctypes.byref(opt), ctypes.byref(info), _stream_ptr(stream))
    if check and rc < 0:
        raise GhsvdError(rc, "ghsvd_solve")
    return lam, X, info.as_dict()


def solve_fast(F: torch.Tensor, J: torch.Tensor, G: torch.Tensor, *, cond_max: float = 1e4,
               max_sweeps: int = 0, fallback: dict | None = None, work=None, stream=None,
               check=True):
    """The explicit-formation route (ghsvd_solve_fast): lambda, X, info dict.
    fallback: ghsvd_solve options (keyword dict) for the implicit HZ path
    taken when S is too ill-conditioned, or None to get GHSVD_ERANK instead."""
    m, n = F.shape
    p = G.shape[0]
    ldf = _check_fortran(F, "F")
    ldg = _check_fortran(G, "G")
    if J.dtype != torch.int8 or not J.is_cuda or J.numel() != m:
        raise TypeError("J must be an int8 CUDA tensor with m entries")
    fb = options(**fallback) if fallback is not None else None
    fbp = ctypes.byref(fb) if fb is not None else None
    lam = torch.empty(n, dtype=torch.float64, device=F.device)
    X = fortran_empty(n, n, device=F.device)
    if work is None:
        need = int(_lib.ghsvd_fast_workspace_size(m, n, p, fbp))
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=F.device)
    info = FastInfo()
    rc = _lib.ghsvd_solve_fast(m, n, p, F.data_ptr(), ldf, J.data_ptr(), G.data_ptr(), ldg,
                               lam.data_ptr(), X.data_ptr(), n, float(cond_max), int(max_sweeps),
                               work.data_ptr(), work.numel(), fbp, ctypes.byref(info),
                               _stream_ptr(stream))
    if check and rc < 0:
        raise GhsvdError(rc, "ghsvd_solve_fast")
    return lam, X, info.as_dict()


def solve_batched(Fs, Js, Gs, *, stream=None, check=True, **kw):
    """Lists of per-pencil tensors -> (list of lambda, list of X, list of info dicts, status)."""
    opt = options(**kw)
    b = len(Fs)
    m = np.array([F.shape[0] for F in Fs], dtype=np.int32)
    n = np.array([F.shape[1] for F in Fs], dtype=np.int32)
    p = np.array([G.shape[0] for G in Gs], dtype=np.int32)
    ldf = np.array([_check_fortran(F, "F") for F in Fs], dtype=np.int32)
    ldg = np.array([_check_fortran(G, "G") for G in Gs], dtype=np.int32)
    lams = [torch.empty(int(k), dtype=torch.float64, device=Fs[0].device) for k in n]
    Xs = [fortran_empty(int(k), int(k), device=Fs[0].device) for k in n]
    ldx = np.array([int(k) for k in n], dtype=np.int32)
    fp = np.array([F.data_ptr() for F in Fs], dtype=np.uint64)
    jp = np.array([J.data_ptr() for J in Js], dtype=np.uint64)
    gp = np.array([G.data_ptr() for G in Gs], dtype=np.uint64)
    lp = np.array([t.data_ptr() for t in lams], dtype=np.uint64)
    xp = np.array([t.data_ptr() for t in Xs], dtype=np.uint64)
    need = int(_lib.ghsvd_workspace_size_batched(b, m.ctypes.data, n.ctypes.data, p.ctypes.data,
                                                  ctypes.byref(opt)))
    work = torch.empty(max(need, 1), dtype=torch.uint8, device=Fs[0].device)
    infos = (Info * b)()
    rc = _lib.ghsvd_solve_batched(b, m.ctypes.data, n.ctypes.data, p.ctypes.data, fp.ctypes.data,
                                  ldf.ctypes.data, jp.ctypes.data, gp.ctypes.data, ldg.ctypes.data,
                                  lp.ctypes.data, xp.ctypes.data, ldx.ctypes.data, work.data_ptr(),
                                  work.numel(), ctypes.byref(opt), ctypes.cast(infos, _p),
                                  _stream_ptr(stream))
    if check and rc < 0:
        raise GhsvdError(rc, "ghsvd_solve_batched")
    return lams, Xs, [infos[k].as_dict() for k in range(b)], rc


def reduce(F: torch.Tensor, J: torch.Tensor, G: torch.Tensor, stream=None):
    """(Fsq, Jsq, Gsq, perm, n2x2) of the one-time reduction."""
    m, n = F.shape
    p = G.shape[0]
    ldf = _check_fortran(F, "F")
    ldg = _check_fortran(G, "G")
    Fsq = fortran_empty(n, n, device=F.device)
    Gsq = fortran_empty(n, n, device=F.device)
    Jsq = torch.empty(n, dtype=torch.int8, device=F.device)
    perm = torch.empty(n, dtype=torch.int32, device=F.device)
    n2 = ctypes.c_int(0)
    rc = _lib.ghsvd_reduce(m, n, p, F.data_ptr(), ldf, J.data_ptr(), G.data_ptr(), ldg,
                           Fsq.data_ptr(), n, Jsq.data_ptr(), Gsq.data_ptr(), n, perm.data_ptr(),
                           ctypes.byref(n2), _stream_ptr(stream))
    if rc < 0:
        raise GhsvdError(rc, "ghsvd_reduce")
    return Fsq, Jsq, Gsq, perm, n2.value


def pair_params(a, b, c, sa, sb, sc, tol, crit_literal=0, stream=None):
    """Batched 2x2 step on device tensors; returns (Z (count, 4) complex128, kind int32)."""
    count = a.numel()
    Z = torch.empty((count, 4), dtype=torch.complex128, device=a.device)
    kind = torch.empty(count, dtype=torch.int32, device=a.device)
    rc = _lib.ghsvd_pair_params(count, a.data_ptr(), b.data_ptr(), c.data_ptr(), sa.data_ptr(),
                                sb.data_ptr(), sc.data_ptr(), float(tol), int(crit_literal),
                                Z.data_ptr(), kind.data_ptr(), _stream_ptr(stream))
    if rc < 0:
        raise GhsvdError(rc, "ghsvd_pair_params")
    return Z, kind


def sweeps(F, n_plus: int, G, Z, nsweeps: int, waves_per_pair=0, crit_literal=0, stream=None):
    """In-place pointwise FP64 sweeps; returns (status, sweeps_done, counters (nsweeps, 3))."""
    m, n = F.shape
    p = G.shape[0]
    cnt = np.zeros(3 * nsweeps, dtype=np.int64)
    done = ctypes.c_int(0)
    rc = _lib.ghsvd_sweeps(m, n, p, F.data_ptr(), _check_fortran(F, "F"), int(n_plus),
                           G.data_ptr(), _check_fortran(G, "G"), Z.data_ptr(),
                           _check_fortran(Z, "Z"), int(nsweeps), int(waves_per_pair),
                           int(crit_literal), cnt.ctypes.data, ctypes.byref(done),
                           _stream_ptr(stream))
    return rc, done.value, cnt.reshape(nsweeps, 3)


def block_sweeps(F, n_plus: int, G, Z, nsweeps: int, block_width=0, crit_literal=0,
                 inner_order="cross", stream=None, noalloc=False):
    """In-place Level-2 blocked FP64 sweeps; returns (status, sweeps_done, counters (nsweeps, 3)).
    noalloc=True calls ghsvd_block_sweeps_noalloc (scratch in the library's static array)."""
    m, n = F.shape
    p = G.shape[0]
    cnt = np.zeros(3 * nsweeps, dtype=np.int64)
    done = ctypes.c_int(0)
    fn = _lib.ghsvd_block_sweeps_noalloc if noalloc else _lib.ghsvd_block_sweeps
    rc = fn(m, n, p, F.data_ptr(), _check_fortran(F, "F"), int(n_plus),
            G.data_ptr(), _check_fortran(G, "G"), Z.data_ptr(),
            _check_fortran(Z, "Z"), int(block_width), INNER[inner_order],
            int(nsweeps),
            int(crit_literal), cnt.ctypes.data, ctypes.byref(done),
            _stream_ptr(stream))
    return rc, done.value, cnt.reshape(nsweeps, 3)


def full_workspace_size(n: int) -> int:
    return int(_lib.ghsvd_full_workspace_size(int(n)))


def full(F, n_plus: int, G, Z, work=None, stream=None):
    """Full GHSVD from swept factors (ghsvd_full): (U, V, sigma_f, sigma_g, X).
    work: a uint8 CUDA tensor of at least full_workspace_size(n) bytes (None:
    one is allocated here, through torch)."""
    m, n = F.shape
    p = G.shape[0]
    U = fortran_empty(m, n, device=F.device)
    V = fortran_empty(p, n, device=F.device)
    X = fortran_empty(n, n, device=F.device)
    sf = torch.empty(n, dtype=torch.float64, device=F.device)
    sg = torch.empty(n, dtype=torch.float64, device=F.device)
    if work is None:
        nbytes = full_workspace_size(n)
        work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=F.device)
    rc = _lib.ghsvd_full(m, n, p, F.data_ptr(), _check_fortran(F, "F"), int(n_plus), G.data_ptr(),
                         _check_fortran(G, "G"), Z.data_ptr(), _check_fortran(Z, "Z"),
                         U.data_ptr(), m, V.data_ptr(), p, sf.data_ptr(), sg.data_ptr(),
                         X.data_ptr(), n, work.data_ptr(), work.numel(), _stream_ptr(stream))
    if rc < 0:
        raise GhsvdError(rc, "ghsvd_full")
    return U, V, sf, sg, X


def hebpj_batched(T, work=None, stream=None):
    """ZHEBPJ of every atom block (ghsvd_hebpj_batched).  T: complex128 CUDA
    tensor of shape (n_atoms, r, r) whose [a] is T_a transposed in memory, i.e.
    T_a column-major (`atoms_to_device` builds it).  Returns (Mt, Jt, piv,
    stats) with Mt of the same layout, Jt (n_atoms, r) int8, piv (n_atoms, r)
    int32, stats (n_atoms, 2) int32."""
    na, r, r2 = T.shape
    if r != r2 or T.dtype != torch.complex128 or not T.is_cuda or not T.is_contiguous():
        raise ValueError("T must be a contiguous complex128 CUDA tensor (n_atoms, r, r)")
    Mt = torch.empty_like(T)
    Jt = torch.empty((na, r), dtype=torch.int8, device=T.device)
    piv = torch.empty((na, r), dtype=torch.int32, device=T.device)
    stats = torch.empty((na, 2), dtype=torch.int32, device=T.device)
    if work is None:
        work = torch.empty(max(int(_lib.ghsvd_hebpj_workspace_size(na, r)), 1),
                           dtype=torch.uint8, device=T.device)
    rc = _lib.ghsvd_hebpj_batched(na, r, T.data_ptr(), Mt.data_ptr(), Jt.data_ptr(),
                                  piv.data_ptr(), stats.data_ptr(), work.data_ptr(),
                                  work.numel(), _stream_ptr(stream))
    if rc < 0:
        raise GhsvdError(rc, "ghsvd_hebpj_batched")
    return Mt, Jt, piv, stats


def atoms_to_device(T: np.ndarray, device="cuda") -> torch.Tensor:
    """(r, r, n_atoms) column-major numpy blocks -> (n_atoms, r, r) tensor whose
    [a] holds T_a column-major (memory order i + r j + r^2 a)."""
    return torch.from_numpy(np.ascontiguousarray(np.transpose(T, (2, 1, 0)))).to(device)


def phase1(T, H, U, work=None, stream=None):
    """Phase 1 (ghsvd_phase1): (F, J, G, stats).  T as for `hebpj_batched`,
    H a column-major complex128 CUDA tensor (2 nl n_atoms, n), U a float64
    CUDA tensor (n_atoms, nl) (row a = the diagonal of U_a)."""
    na, r, _ = T.shape
    nl = r // 2
    m, n = H.shape
    if U.dtype != torch.float64 or tuple(U.shape) != (na, nl) or not U.is_contiguous():
        raise ValueError("U must be a contiguous float64 tensor (n_atoms, nl)")
    F = fortran_empty(m, n, device=H.device)
    G = fortran_empty(m, n, device=H.device)
    J = torch.empty(m, dtype=torch.int8, device=H.device)
    stats = torch.empty((na, 2), dtype=torch.int32, device=H.device)
    if work is None:
        work = torch.empty(max(int(_lib.ghsvd_phase1_workspace_size(na, nl)), 1),
                           dtype=torch.uint8, device=H.device)
    rc = _lib.ghsvd_phase1(na, nl, n, T.data_ptr(), H.data_ptr(), _check_fortran(H, "H"),
                           U.data_ptr(), F.data_ptr(), m, J.data_ptr(), G.data_ptr(), m,
                           stats.data_ptr(), work.data_ptr(), work.numel(), _stream_ptr(stream))
    if rc < 0:
        raise GhsvdError(rc, "ghsvd_phase1")
    return F, J, G, stats


def round_robin(n: int):
    N = n + (n % 2)
    slots = N // 2
    pp = np.zeros(max(1, (N - 1) * slots), dtype=np.int32)
    qq = np.zeros_like(pp)
    steps = _lib.ghsvd_round_robin(n, pp.ctypes.data, qq.ctypes.data)
    return steps, pp[: steps * slots].reshape(steps, slots), qq[: steps * slots].reshape(steps, slots)


PROF_KINDS = {"pair64": 0, "pair32": 1, "gram": 2, "inner": 3, "update": 4, "gram32": 5,
              "inner32": 6, "update32": 7, "reduce": 8}


def profile_enable(every: int) -> None:
    """Time every `every`-th launch of each sweep-kernel kind with HIP events (0 disables)."""
    _lib.ghsvd_profile_enable(int(every))


def profile_read(kind: str = "pair64"):
    """(kernel milliseconds of the timed launches, timed launches, all launches) of one kind."""
    ms = ctypes.c_double(0.0)
    timed = ctypes.c_longlong(0)
    total = ctypes.c_longlong(0)
    rc = _lib.ghsvd_profile_read(PROF_KINDS[kind], ctypes.byref(ms), ctypes.byref(timed),
                                 ctypes.byref(total))
    if rc < 0:
        raise GhsvdError(rc, "ghsvd_profile_read")
    return ms.value, timed.value, total.value


def autotune(Fs, Js, Gs, *, stream=None, **kw):
    """Times trial sweeps on these pencils and stores the fastest launch
    parameters for their shape class; returns (block_width, waves_per_pair,
    trial_ms dict)."""
    opt = options(**kw)
    b = len(Fs)
    m = np.array([F.shape[0] for F in Fs], dtype=np.int32)
    n = np.array([F.shape[1] for F in Fs], dtype=np.int32)
    p = np.array([G.shape[0] for G in Gs], dtype=np.int32)
    ldf = np.array([_check_fortran(F, "F") for F in Fs], dtype=np.int32)
    ldg = np.array([_check_fortran(G, "G") for G in Gs], dtype=np.int32)
    fp = np.array([F.data_ptr() for F in Fs], dtype=np.uint64)
    jp = np.array([J.data_ptr() for J in Js], dtype=np.uint64)
    gp = np.array([G.data_ptr() for G in Gs], dtype=np.uint64)
    aopt = options(**{**kw, "block_width": 0})
    need = int(_lib.ghsvd_workspace_size_batched(b, m.ctypes.data, n.ctypes.data, p.ctypes.data,
                                                  ctypes.byref(aopt)))
    work = torch.empty(max(need, 1), dtype=torch.uint8, device=Fs[0].device)
    w = ctypes.c_int(0)
    wpp = ctypes.c_int(0)
    t = np.zeros(7, dtype=np.float32)
    rc = _lib.ghsvd_autotune(b, m.ctypes.data, n.ctypes.data, p.ctypes.data, fp.ctypes.data,
                             ldf.ctypes.data, jp.ctypes.data, gp.ctypes.data, ldg.ctypes.data,
                             work.data_ptr(), work.numel(), ctypes.byref(opt), ctypes.byref(w),
                             ctypes.byref(wpp), t.ctypes.data, _stream_ptr(stream))
    if rc < 0:
        raise GhsvdError(rc, "ghsvd_autotune")
    trials = {f"pointwise_wpp{k}": float(t[i]) for i, k in enumerate((1, 2, 4, 8))}
    trials.update({f"blocked_w{k}": float(t[4 + i]) for i, k in enumerate((8, 16, 32))})
    return w.value, wpp.value, trials


def autotune_clear() -> None:
    _lib.ghsvd_autotune_clear()
