"""Helpers shared by the GPU parity tests (inputs to the device, comparisons)."""
import numpy as np
import torch

from paper_1907_08560_amd import ghsvd

EPS = 2.0 ** -52


def to_dev(P, dev="cuda"):
    F = ghsvd.to_device_fortran(P.F, dev)
    G = ghsvd.to_device_fortran(P.G, dev)
    J = torch.from_numpy(np.ascontiguousarray(P.J, dtype=np.int8)).to(dev)
    return F, J, G


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def factor_invariants(F, J, G, lam, X):
    """(||(GX)^*(GX) - I||_max, max |off(X^* H X)| / sqrt(|l_i l_j|), max |diag - l| / |l|)
    evaluated on the factors (never on a formed S)."""
    n = X.shape[1]
    GX = G @ X
    FX = F @ X
    e_s = np.abs(GX.conj().T @ GX - np.eye(n)).max()
    Hx = FX.conj().T @ (J[:, None].astype(np.float64) * FX)
    off = Hx - np.diag(np.diag(Hx))
    scale = np.sqrt(np.outer(np.abs(lam), np.abs(lam)))
    e_h = float(np.max(np.abs(off) / np.maximum(scale, np.abs(lam).max() * 1e-16)))
    e_d = float(np.max(np.abs(np.real(np.diag(Hx)) - lam) / np.abs(lam)))
    return float(e_s), e_h, e_d
