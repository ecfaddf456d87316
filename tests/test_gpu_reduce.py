"""GPU parity of the one-time reduction (Section 5) against the oracle.

The pivot decisions (P2, the row swaps behind J_sq, the 2x2 pivot count) are
integer results and must match exactly; the square factors element by
element within a tolerance scaled by the column norms of the oracle's
factors (the hyperbolic reflectors are not norm preserving).
"""
import numpy as np
import pytest
import torch

from paper_1907_08560_amd import ghsvd, synth
from gpu_util import host, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("number,n_override", [(1, None), (2, 160), (4, 257), (5, 96)])
def test_reduce_elementwise(oracle, number, n_override):
    P = synth.workload_pencil(number, n_override=n_override)
    F, J, G = to_dev(P)
    Fsq, Jsq, Gsq, perm, n2 = ghsvd.reduce(F, J, G)
    st, Fo, Jo, Go, perm_o, n2o = oracle.reduce(P.F, P.J, P.G)
    assert st == 0
    assert np.array_equal(host(perm), perm_o)
    assert np.array_equal(host(Jsq), Jo)
    assert n2 == n2o
    # G's factor: the oracle's Householder QR of G (unpivoted), columns
    # permuted by P2; its Gram equals that of the oracle's QR of G P2.
    st_g, Rg = oracle.qr(np.asfortranarray(P.G))
    assert st_g == 0
    for A, B in ((host(Fsq), Fo), (host(Gsq), Rg[:, perm_o])):
        colscale = np.linalg.norm(B, axis=0)
        err = np.max(np.abs(A - B) / colscale[None, :])
        assert err < 1e-10, err
    Gs = host(Gsq)
    SG = Go.conj().T @ Go
    assert np.abs(Gs.conj().T @ Gs - SG).max() < 1e-12 * np.abs(SG).max()
    # invariants of the square factors against the tall ones
    Fs = host(Fsq)
    H = P.F.conj().T @ (P.J[:, None] * P.F)
    Hp = H[np.ix_(perm_o, perm_o)]
    assert np.abs(Fs.conj().T @ (host(Jsq)[:, None] * Fs) - Hp).max() < 1e-11 * np.abs(H).max()
    inv = np.argsort(perm_o)
    assert np.array_equal(np.tril(Gs[:, inv], -1), np.zeros((P.n, P.n)))


def test_reduce_isotropic_2x2():
    # Columns of zero J-norm with a large J-product: one 2x2 pivot.
    F = np.zeros((6, 2), dtype=complex)
    J = np.array([1, 1, 1, -1, -1, -1], dtype=np.int8)
    F[0, 0] = F[3, 0] = 1.0
    F[1, 1] = F[4, 1] = 1.0
    F[0, 1], F[3, 1] = 2.0, -2.0
    G = np.eye(3, 2, dtype=complex) + 0.1
    Fd = ghsvd.to_device_fortran(F)
    Gd = ghsvd.to_device_fortran(G)
    Jd = torch.from_numpy(J).cuda()
    Fsq, Jsq, Gsq, perm, n2 = ghsvd.reduce(Fd, Jd, Gd)
    assert n2 == 1
    Fs = host(Fsq)
    H = F.conj().T @ (J[:, None] * F)
    pm = host(perm)
    assert np.abs(Fs.conj().T @ (host(Jsq)[:, None] * Fs) - H[np.ix_(pm, pm)]).max() < 1e-14


@pytest.mark.parametrize("n,m,m_plus,p", [(300, 1300, 975, 2100), (600, 900, 675, 1200),
                                           (301, 1900, 1425, 1500), (257, 2300, 1725, 600)])
def test_reduce_register_and_streaming_columns(oracle, n, m, m_plus, p):
    """Shapes whose trailing columns are longer than the register-resident
    step holds (1024 or 2048 rows) at the first steps and fit later, so
    both forms of the column step run in one factorization.  The last two
    take F's columns through 8 rows per thread (one column per step
    workgroup) and, for m = 2300, from the streaming loops through 8, 6 and
    4 rows per thread, where the step workgroups switch to two columns each
    (odd column counts included).

    The pivot decisions must match exactly.  The hyperbolic factor's
    elementwise bar is set by its own forward sensitivity: the oracle is run
    again on F with relative noise of 1e-16 (a rounding-level change of the
    input, with the same pivots), and the GPU factor, whose sums round in a
    different order, may differ from the oracle's by 20 times that change
    (at least 1e-10).  The J-Gram of the factor must reproduce P2^T F^* J F P2
    to 1e-11 of its largest entry."""
    P = synth.random_pencil(900 + n, n, m, m_plus, p, 1e-4)
    F, J, G = to_dev(P)
    Fsq, Jsq, Gsq, perm, n2 = ghsvd.reduce(F, J, G)
    st, Fo, Jo, Go, perm_o, n2o = oracle.reduce(P.F, P.J, P.G)
    assert st == 0
    assert np.array_equal(host(perm), perm_o)
    assert np.array_equal(host(Jsq), Jo)
    assert n2 == n2o
    colscale = np.linalg.norm(Fo, axis=0)
    rng = np.random.default_rng(n)
    Fn = P.F * (1.0 + 1e-16 * rng.standard_normal(P.F.shape))
    st_n, Fo_n, _, _, perm_n, _ = oracle.reduce(Fn, P.J, P.G)
    assert st_n == 0 and np.array_equal(perm_n, perm_o)
    sens = np.max(np.abs(Fo_n - Fo) / colscale[None, :])
    err = np.max(np.abs(host(Fsq) - Fo) / colscale[None, :])
    assert err < max(1e-10, 20.0 * sens), (err, sens)
    H = P.F.conj().T @ (P.J[:, None] * P.F)
    Hp = H[np.ix_(perm_o, perm_o)]
    Fs = host(Fsq)
    assert np.abs(Fs.conj().T @ (host(Jsq)[:, None] * Fs) - Hp).max() < 1e-11 * np.abs(H).max()
    st_g, Rg = oracle.qr(np.asfortranarray(P.G))
    assert st_g == 0
    B = Rg[:, perm_o]
    err_g = np.max(np.abs(host(Gsq) - B) / np.linalg.norm(B, axis=0)[None, :])
    assert err_g < 1e-10, err_g
