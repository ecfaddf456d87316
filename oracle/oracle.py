"""ctypes front end of the CPU oracle (hz_oracle.c) -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this module.  The solver never does.  `build()` compiles the C file
with gcc -O2 -ffp-contract=off into oracle/liboracle.so; `build(mutant=k)`
compiles a copy with the planted mistake number k (for the pin tests).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hz_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23

_c_int = ctypes.c_int
_c_dbl = ctypes.c_double
_p = ctypes.c_void_p


def build(mutant: int = 0, out: str | None = None) -> str:
    """Compile the oracle; returns the path of the shared library."""
    if out is None:
        out = LIB if mutant == 0 else os.path.join(
            tempfile.gettempdir(), f"liboracle_mut{mutant}_{os.getpid()}.so")
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
           f"-DORA_MUTANT={int(mutant)}", SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class Oracle:
    def __init__(self, path: str | None = None):
        path = path or LIB
        if not os.path.exists(path):
            path = build()
        self.lib = ctypes.CDLL(path)
        L = self.lib
        L.ora_pair_params.argtypes = [_c_dbl] * 9 + [_c_int, _p]
        L.ora_pair_params.restype = _c_int
        L.ora_round_robin.argtypes = [_c_int, _p, _p]
        L.ora_round_robin.restype = _c_int
        L.ora_hz_run.argtypes = [_c_int, _c_int, _c_int, _p, _c_int, _p, _p, _c_int, _p,
                                 _c_int, _c_int, _c_int, _c_dbl, _c_int, _c_int, _p]
        L.ora_hz_run.restype = _c_int
        L.ora_hz_post.argtypes = [_c_int, _c_int, _c_int, _p, _c_int, _p, _p, _c_int, _p,
                                  _c_int, _c_int, _p, _p, _c_int]
        L.ora_hz_post.restype = _c_int
        L.ora_qr.argtypes = [_c_int, _c_int, _p, _c_int]
        L.ora_qr.restype = _c_int
        L.ora_jqr.argtypes = [_c_int, _c_int, _p, _c_int, _p, _p, _p]
        L.ora_jqr.restype = _c_int
        L.ora_ghsvd.argtypes = [_c_int, _c_int, _c_int, _p, _c_int, _p, _p, _c_int,
                                _c_int, _c_int, _c_int, _c_dbl, _c_int, _c_int, _p, _p,
                                _c_int, _p]
        L.ora_ghsvd.restype = _c_int
        L.ora_hz_block_run.argtypes = [_c_int, _c_int, _c_int, _p, _c_int, _p, _p, _c_int, _p,
                                       _c_int, _c_int, _c_int, _c_dbl, _c_int, _c_int, _p]
        L.ora_hz_block_run.restype = _c_int
        L.ora_hz_block_run_ex.argtypes = L.ora_hz_block_run.argtypes[:-1] + [_c_int, _p]
        L.ora_hz_block_run_ex.restype = _c_int

    # -- 2x2 step -------------------------------------------------------------
    def pair_params(self, a, b, c, sa, sb, sc, tol, crit_literal=0):
        """Returns (kind, Z') with Z' a 2x2 complex array (kind: 0 skip,
        1 small, 2 big, < 0 error)."""
        z = np.zeros(8)
        kind = self.lib.ora_pair_params(float(a), float(b), float(np.real(c)),
                                        float(np.imag(c)), float(sa), float(sb),
                                        float(np.real(sc)), float(np.imag(sc)),
                                        float(tol), int(crit_literal),
                                        z.ctypes.data)
        Z = np.array([[z[0] + 1j * z[1], z[4] + 1j * z[5]],
                      [z[2] + 1j * z[3], z[6] + 1j * z[7]]])
        return kind, Z

    def round_robin(self, n: int):
        N = n + (n % 2)
        slots = N // 2
        pp = np.zeros(max(1, (N - 1) * slots), dtype=np.int32)
        qq = np.zeros_like(pp)
        steps = self.lib.ora_round_robin(n, pp.ctypes.data, qq.ctypes.data)
        return steps, pp[: steps * slots].reshape(steps, slots), qq[: steps * slots].reshape(steps, slots)

    # -- sweeps ---------------------------------------------------------------
    def hz_run(self, F, J, G, Z=None, order=0, max_sweeps=30, eps=EPS64,
               crit_literal=0, stop_rule=0):
        """Runs sweeps in place on copies; returns (status, F, G, Z, stats)."""
        F = np.array(F, dtype=np.complex128, order="F", copy=True)
        G = np.array(G, dtype=np.complex128, order="F", copy=True)
        m, n = F.shape
        p = G.shape[0]
        Z = (np.eye(n, dtype=np.complex128, order="F") if Z is None
             else np.array(Z, dtype=np.complex128, order="F", copy=True))
        J8 = np.ascontiguousarray(J, dtype=np.int8)
        stats = np.zeros(6, dtype=np.int64)
        st = self.lib.ora_hz_run(m, n, p, F.ctypes.data, m, J8.ctypes.data, G.ctypes.data,
                                 p, Z.ctypes.data, n, int(order), int(max_sweeps),
                                 float(eps), int(crit_literal), int(stop_rule),
                                 stats.ctypes.data)
        return st, F, G, Z, stats

    def hz_block_run(self, F, J, G, Z=None, w=8, max_sweeps=30, eps=EPS64, crit_literal=0,
                     inner_order=0, stop_all=None):
        """Level-2 block sweeps in place on copies; returns (status, F, G, Z, stats).
        inner_order 0: BO, one round-robin inner sweep per block pivot; 1: BO with
        cross-block inner pairs after the first block step of a sweep; 2: FB, inner
        sweeps until one applies no transformation, at most 30; 3, 4: the shortened
        pivot swept by a nested Level-2 run of width 8 (one blocked sweep, or
        blocked sweeps until one applies no transformation, at most 30).
        stop_all: the run's own stopping test (None or False: a sweep with no big
        transformation; True: one with no transformation at all)."""
        F = np.array(F, dtype=np.complex128, order="F", copy=True)
        G = np.array(G, dtype=np.complex128, order="F", copy=True)
        m, n = F.shape
        p = G.shape[0]
        Z = (np.eye(n, dtype=np.complex128, order="F") if Z is None
             else np.array(Z, dtype=np.complex128, order="F", copy=True))
        J8 = np.ascontiguousarray(J, dtype=np.int8)
        stats = np.zeros(6, dtype=np.int64)
        st = self.lib.ora_hz_block_run_ex(m, n, p, F.ctypes.data, m, J8.ctypes.data,
                                          G.ctypes.data, p, Z.ctypes.data, n, int(w),
                                          int(max_sweeps), float(eps), int(crit_literal),
                                          int(inner_order), int(bool(stop_all)),
                                          stats.ctypes.data)
        return st, F, G, Z, stats

    def hz_post(self, F, J, G, Z, sort=1):
        F = np.asfortranarray(F, dtype=np.complex128)
        G = np.asfortranarray(G, dtype=np.complex128)
        Z = np.asfortranarray(Z, dtype=np.complex128)
        m, n = F.shape
        p = G.shape[0]
        J8 = np.ascontiguousarray(J, dtype=np.int8)
        lam = np.zeros(n)
        X = np.zeros((n, n), dtype=np.complex128, order="F")
        st = self.lib.ora_hz_post(m, n, p, F.ctypes.data, m, J8.ctypes.data, G.ctypes.data,
                                  p, Z.ctypes.data, n, int(sort), lam.ctypes.data,
                                  X.ctypes.data, n)
        return st, lam, X

    # -- reduction ------------------------------------------------------------
    def qr(self, A):
        R = np.array(A, dtype=np.complex128, order="F", copy=True)
        p, n = R.shape
        st = self.lib.ora_qr(p, n, R.ctypes.data, p)
        return st, R[:n, :].copy(order="F")

    def jqr(self, F, J):
        A = np.array(F, dtype=np.complex128, order="F", copy=True)
        m, n = A.shape
        Jw = np.array(J, dtype=np.int8, copy=True)
        perm = np.zeros(n, dtype=np.int32)
        n2 = np.zeros(1, dtype=np.int32)
        st = self.lib.ora_jqr(m, n, A.ctypes.data, m, Jw.ctypes.data, perm.ctypes.data,
                              n2.ctypes.data)
        return st, A[:n, :].copy(order="F"), Jw[:n].copy(), perm, int(n2[0]), A

    def reduce(self, F, J, G):
        """JQR of F, P2 applied to G, QR of G P2: (status, Fsq, Jsq, Gsq, perm, n2x2)."""
        st, Fsq, Jsq, perm, n2, _ = self.jqr(F, J)
        if st != 0:
            return st, None, None, None, perm, n2
        st2, Gsq = self.qr(np.asfortranarray(G[:, perm]))
        return st2, Fsq, Jsq, Gsq, perm, n2

    # -- whole path -----------------------------------------------------------
    def ghsvd(self, F, J, G, reduce=False, order=0, max_sweeps=30, eps=EPS64,
              crit_literal=0, sort=1):
        """Returns (status, lambda, X, stats) for the pencil (F^* J F, G^* G)."""
        F = np.asfortranarray(F, dtype=np.complex128)
        G = np.asfortranarray(G, dtype=np.complex128)
        m, n = F.shape
        p = G.shape[0]
        J8 = np.ascontiguousarray(J, dtype=np.int8)
        lam = np.zeros(n)
        X = np.zeros((n, n), dtype=np.complex128, order="F")
        stats = np.zeros(6, dtype=np.int64)
        st = self.lib.ora_ghsvd(m, n, p, F.ctypes.data, m, J8.ctypes.data, G.ctypes.data,
                                p, int(bool(reduce)), int(order), int(max_sweeps),
                                float(eps), int(crit_literal), int(sort), lam.ctypes.data,
                                X.ctypes.data, n, stats.ctypes.data)
        return st, lam, X, stats


_default = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
