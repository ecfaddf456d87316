"""Seeded synthetic pencils (F, J, G) of the shapes the solver is benchmarked on.

This module only draws inputs: it holds none of the solver's arithmetic, and
both the HIP path and the CPU oracle consume what it returns.

Recipe (one pencil of order n):
  * F: m x n, entries i.i.d. (N(0,1) + i N(0,1)) / sqrt(2), m = ceil(ratio_f * n).
  * J: +1 on the first m_plus rows, -1 on the rest (int8).
  * G: p x n, G = U diag(s) W^*, with U the first n columns of a p x p Haar
    unitary, W an n x n Haar unitary (Q of a complex Gaussian matrix with the
    phases of diag(R) moved into Q, Mezzadri's construction), and
    s_j = 10**Uniform(log10(s_lo), 0) i.i.d., unsorted.  cond(G^*G) is then
    at most s_lo**-2.
  * Draw order inside one pencil: F, s, U, W; all from one numpy PCG64 stream.
All arrays are complex128 in Fortran (column-major) order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Pencil:
    F: np.ndarray   # m x n complex128, Fortran order
    J: np.ndarray   # m int8, entries +1 / -1
    G: np.ndarray   # p x n complex128, Fortran order
    s: np.ndarray   # the singular values used to build G (unsorted)
    seed: int
    index: int

    @property
    def m(self) -> int:
        return self.F.shape[0]

    @property
    def n(self) -> int:
        return self.F.shape[1]

    @property
    def p(self) -> int:
        return self.G.shape[0]

    @property
    def m_plus(self) -> int:
        return int((self.J > 0).sum())


def _gauss(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    re = rng.standard_normal((rows, cols))
    im = rng.standard_normal((rows, cols))
    return (re + 1j * im) / math.sqrt(2.0)


def haar_frame(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """First `cols` columns of a Haar-distributed rows x rows unitary matrix."""
    a = _gauss(rng, rows, cols)
    q, r = np.linalg.qr(a)
    d = np.diagonal(r)
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1.0), 1.0)
    return q * ph[None, :]


def make_pencil(rng: np.random.Generator, n: int, m: int, m_plus: int, p: int,
                s_lo: float, seed: int = -1, index: int = 0,
                j_identity: bool = False) -> Pencil:
    F = _gauss(rng, m, n)
    if j_identity:
        m_plus = m
    J = np.where(np.arange(m) < m_plus, 1, -1).astype(np.int8)
    s = 10.0 ** rng.uniform(math.log10(s_lo), 0.0, size=n)
    U = haar_frame(rng, p, n)
    W = haar_frame(rng, n, n)
    G = (U * s[None, :]) @ W.conj().T
    return Pencil(np.asfortranarray(F), J, np.asfortranarray(G), s, seed, index)


def make_pencil_device(rng: np.random.Generator, n: int, m: int, m_plus: int, p: int,
                       s_lo: float, device, j_identity: bool = False):
    """The recipe of `make_pencil` with the same draws in the same order, but
    the two Haar QRs and the product G = U diag(s) W^* run on `device` (torch),
    which keeps large batches cheap to build.  The Gaussian draws and s are
    identical; U, W and G differ from `make_pencil`'s by rounding only.
    Returns (F, J, G, s): column-major complex128 / int8 device tensors, s numpy."""
    import torch

    def frame(a):
        q, r = torch.linalg.qr(torch.from_numpy(a).to(device))
        d = torch.diagonal(r)
        ad = d.abs()
        ph = torch.where(ad > 0, d / torch.where(ad > 0, ad, torch.ones_like(ad)),
                         torch.ones_like(d))
        return q * ph[None, :]

    def fortran(t):
        return t.t().contiguous().t()

    F = _gauss(rng, m, n)
    if j_identity:
        m_plus = m
    J = np.where(np.arange(m) < m_plus, 1, -1).astype(np.int8)
    s = 10.0 ** rng.uniform(math.log10(s_lo), 0.0, size=n)
    U = frame(_gauss(rng, p, n))
    W = frame(_gauss(rng, n, n))
    st = torch.from_numpy(s).to(device=device, dtype=torch.complex128)
    G = (U * st[None, :]) @ W.conj().t().contiguous()
    Fd = fortran(torch.from_numpy(F).to(device))
    return Fd, torch.from_numpy(J).to(device), fortran(G), s


def workload_pencil_device(number: int, k: int, device, j_identity: bool = False):
    """Pencil k of a workload, built by `make_pencil_device`."""
    w = WORKLOADS[number]
    seed = 1000 + number
    n = workload_sizes(number)[k]
    m = rows_for(n, w["f_ratio"])
    p = rows_for(n, w["g_ratio"])
    m_plus = int(round(w["plus_frac"] * m))
    return make_pencil_device(pencil_rng(seed, w["batch"], k), n, m, m_plus, p, w["s_lo"],
                              device, j_identity=j_identity)


def pencil_rng(seed: int, batch: int, k: int) -> np.random.Generator:
    """Generator of pencil k of a batch: SeedSequence(seed).spawn(batch)[k]."""
    if batch == 1:
        return np.random.Generator(np.random.PCG64(seed))
    child = np.random.SeedSequence(seed).spawn(batch)[k]
    return np.random.Generator(np.random.PCG64(child))


def rows_for(n: int, ratio: float) -> int:
    return int(math.ceil(ratio * n))


# The five workloads, seed = 1000 + workload number.
#   1: n=64, F 96x64, J 72+/24-, G 128x64, s in [1e-4, 1]
#   2: n=1024, F 1536x1024, J 1152+/384-, G 2048x1024, s in [1e-8, 1]
#   3: n=4096, F 6144x4096, J 3:1, G 8192x4096, s in [1e-5, 1] (and a J = I run)
#   4: 64 pencils, n_k ~ U{300..900}, F 1.5n x n, J 3:1, G 2n x n, s in [1e-6, 1]
#   5: 16 pencils, n_k ~ U{2000..6000}, F 1.5n x n, J 4:1, G 2n x n, s in [1e-6, 1]
WORKLOADS = {
    1: dict(batch=1, n=(64, 64), f_ratio=1.5, plus_frac=0.75, g_ratio=2.0, s_lo=1e-4),
    2: dict(batch=1, n=(1024, 1024), f_ratio=1.5, plus_frac=0.75, g_ratio=2.0, s_lo=1e-8),
    3: dict(batch=1, n=(4096, 4096), f_ratio=1.5, plus_frac=0.75, g_ratio=2.0, s_lo=1e-5),
    4: dict(batch=64, n=(300, 900), f_ratio=1.5, plus_frac=0.75, g_ratio=2.0, s_lo=1e-6),
    5: dict(batch=16, n=(2000, 6000), f_ratio=1.5, plus_frac=0.8, g_ratio=2.0, s_lo=1e-6),
}


def workload_sizes(number: int) -> list[int]:
    """Pencil orders n_k of a workload (drawn from the workload's own seed)."""
    w = WORKLOADS[number]
    lo, hi = w["n"]
    if lo == hi:
        return [lo] * w["batch"]
    rng = np.random.Generator(np.random.PCG64(1000 + number))
    return [int(v) for v in rng.integers(lo, hi + 1, size=w["batch"])]


def workload_pencil(number: int, k: int = 0, j_identity: bool = False,
                    n_override: int | None = None) -> Pencil:
    """Pencil k of a workload.  `n_override` shrinks the order (same recipe)."""
    w = WORKLOADS[number]
    seed = 1000 + number
    n = workload_sizes(number)[k] if n_override is None else n_override
    m = rows_for(n, w["f_ratio"])
    p = rows_for(n, w["g_ratio"])
    m_plus = int(round(w["plus_frac"] * m))
    rng = pencil_rng(seed, w["batch"], k)
    return make_pencil(rng, n, m, m_plus, p, w["s_lo"], seed=seed, index=k,
                       j_identity=j_identity)


def random_pencil(seed: int, n: int, m: int, m_plus: int, p: int, s_lo: float,
                  j_identity: bool = False) -> Pencil:
    """A one-off pencil for tests (same recipe, free sizes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_pencil(rng, n, m, m_plus, p, s_lo, seed=seed, j_identity=j_identity)


def random_pairs(seed: int, count: int) -> dict:
    """Random 2x2 pivot data: a Hermitian [[a, c], [conj(c), b]] and a Hermitian
    positive definite [[s_a, s_c], [conj(s_c), s_b]], entries over 12 decades.

    s_c = sqrt(s_a s_b) * x * exp(i theta) with x in [0, 1) (one tenth of the
    draws have x within 1e-6 of 1, one tenth have x = 0); a, b of either sign.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sa = 10.0 ** rng.uniform(-6, 6, size=count)
    sb = 10.0 ** rng.uniform(-6, 6, size=count)
    x = rng.uniform(0.0, 1.0, size=count)
    kind = rng.integers(0, 10, size=count)
    x = np.where(kind == 0, 1.0 - 10.0 ** rng.uniform(-12, -6, size=count), x)
    x = np.where(kind == 1, 0.0, x)
    th = rng.uniform(-math.pi, math.pi, size=count)
    sc = np.sqrt(sa * sb) * x * np.exp(1j * th)
    scale_h = 10.0 ** rng.uniform(-6, 6, size=count)
    a = scale_h * sa * rng.standard_normal(count)
    b = scale_h * sb * rng.standard_normal(count) * 10.0 ** rng.uniform(-2, 2, size=count)
    c = scale_h * np.sqrt(sa * sb) * (rng.standard_normal(count)
                                       + 1j * rng.standard_normal(count))
    return dict(a=a, b=b, c=c, sa=sa, sb=sb, sc=sc)


# ----------------------------------------------------------------------------
# Phase 1 inputs (Section 4.1): atom blocks T_a, H_a = [A_a; B_a], U_a.
#
# Recipe for atom a of a set (seed, kind, N_L, n), all from the generator
# pencil_rng(seed, N_A, a), in this order:
#   * T_a = Q diag(l) Q^*, r = 2 N_L, Q an r x r Haar unitary, |l_i| =
#     10**Uniform(-2, 0) i.i.d.; kind "A": 3 positive and r - 3 negative l_i
#     (the sign pattern the paper reports for its datasets A), kind "B": atoms
#     of even index positive definite, odd index negative definite (datasets
#     B); the signs are then shuffled, so the pivoting has work to do.
#   * H_a: r x n, entries i.i.d. (N(0,1) + i N(0,1)) / sqrt(2).
#   * u_a: N_L doubles, Uniform(0.5, 2) (the diagonal of U_a).
# The paper's shapes: A1 (N_L = 121, N_A = 108, n = 3275) and B1 (N_L = 49,
# N_A = 512, n = 2256).
# ----------------------------------------------------------------------------
PHASE1_SETS = {
    "A1": dict(kind="A", nl=121, atoms=108, n=3275, seed=2001),
    "B1": dict(kind="B", nl=49, atoms=512, n=2256, seed=2002),
}


def phase1_atom(seed: int, atoms: int, a: int, kind: str, nl: int, n: int):
    """(T_a, H_a, u_a) of atom a: T_a r x r and H_a r x n complex128 (Fortran
    order), u_a N_L doubles."""
    rng = pencil_rng(seed, atoms, a)
    r = 2 * nl
    Q = haar_frame(rng, r, r)
    mag = 10.0 ** rng.uniform(-2.0, 0.0, size=r)
    if kind == "A":
        sign = np.where(np.arange(r) < min(3, r), 1.0, -1.0)
    else:
        sign = np.full(r, 1.0 if a % 2 == 0 else -1.0)
    sign = sign[rng.permutation(r)]
    T = (Q * (sign * mag)[None, :]) @ Q.conj().T
    T = 0.5 * (T + T.conj().T)
    H = _gauss(rng, r, n)
    u = rng.uniform(0.5, 2.0, size=nl)
    return np.asfortranarray(T), np.asfortranarray(H), u


def phase1_set(seed: int, atoms: int, kind: str, nl: int, n: int):
    """All atoms: T (r, r, N_A) Fortran, H (r N_A, n) Fortran, U (N_L, N_A)."""
    r = 2 * nl
    T = np.zeros((r, r, atoms), dtype=np.complex128, order="F")
    H = np.zeros((r * atoms, n), dtype=np.complex128, order="F")
    U = np.zeros((nl, atoms), order="F")
    for a in range(atoms):
        Ta, Ha, ua = phase1_atom(seed, atoms, a, kind, nl, n)
        T[:, :, a] = Ta
        H[a * r:(a + 1) * r, :] = Ha
        U[:, a] = ua
    return T, H, U
