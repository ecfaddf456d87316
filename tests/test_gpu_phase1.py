"""GPU parity of Phase 1 (Section 4: ZHEBPJ of the atom blocks, the assembly of
F~, J~, G~) against the oracle.

Pivots and signs are integers decided in FP64 on both sides: the pivot
sequence (piv, with order-2 pivots marked) and J~ must be identical.  The
factor M~ and F~ are compared element by element: the GPU folds the
transformation of each pivot block into the elimination step (rows [W, J^Y],
Schur update Y^* J^ Y) while the oracle factors first and transforms
afterwards, so entries differ by rounding, amplified by the pivot growth; the
gate is 1e-11 of the largest entry of the atom's factor, and of the largest
entry of F~_a for the product.  G~ is a scaled copy and
must be exact.  The full A1-shaped set (108 atoms, N_L = 121, n = 3275) runs in
the same launch configuration the benchmark times, with three atoms checked
against the oracle.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

from oracle import phase1 as P1
from paper_1907_08560_amd import ghsvd, synth
from gpu_util import host

pytestmark = pytest.mark.gpu


def expected_piv(perm, blocks):
    piv = np.array(perm, dtype=np.int64)
    for k, s in blocks:
        if s == 2:
            piv[k] = -(perm[k] + 1)
            piv[k + 1] = -(perm[k + 1] + 1)
    return piv


def check_atoms(T, Mt, Jt, piv, stats, tag, atoms=None):
    r, _, na = T.shape
    Mt, Jt, piv, stats = host(Mt), host(Jt), host(piv), host(stats)
    for a in (range(na) if atoms is None else atoms):
        Mo, Jo, perm, ex = P1.hebpj(T[:, :, a])
        assert np.array_equal(piv[a], expected_piv(perm, ex["blocks"])), (tag, a)
        assert np.array_equal(Jt[a], Jo), (tag, a)
        assert stats[a, 0] == sum(1 for _, s in ex["blocks"] if s == 2), (tag, a)
        assert stats[a, 1] == int((Jo == 0).sum()), (tag, a)
        Mg = Mt[a].T  # [a] holds M~_a column-major
        scale = max(np.abs(Mo).max(), 1e-300)
        err = np.abs(Mg - Mo).max() / scale
        assert err <= 1e-11, (tag, a, err)
        rec = Mg.conj().T @ (Jo.astype(float)[:, None] * Mg)
        assert np.abs(rec - T[:, :, a]).max() <= 1e-12 * np.abs(T[:, :, a]).max() + 1e-300


@pytest.mark.parametrize("kind,nl,atoms", [("A", 1, 3), ("A", 4, 5), ("B", 7, 6), ("A", 20, 4),
                                           ("B", 49, 3), ("A", 121, 2), ("A", 256, 1)])
def test_hebpj_matches_oracle(kind, nl, atoms):
    T, _, _ = synth.phase1_set(31 + nl, atoms, kind, nl, 1)
    Mt, Jt, piv, stats = ghsvd.hebpj_batched(ghsvd.atoms_to_device(T))
    check_atoms(T, Mt, Jt, piv, stats, f"{kind} nl={nl}")


def test_hebpj_edge_cases():
    r = 8
    rng = np.random.default_rng(9)
    X = rng.standard_normal((r, r)) + 1j * rng.standard_normal((r, r))
    zero_diag = X + X.conj().T
    np.fill_diagonal(zero_diag, 0.0)  # order-2 pivots
    # zero rows and columns stay exactly zero under any elimination order, so
    # the Schur complement ends exactly zero on both sides
    Y = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    live = [0, 2, 3, 5, 7]
    singular = np.zeros((r, r), dtype=complex)
    singular[np.ix_(live, live)] = Y + Y.conj().T
    T = np.zeros((r, r, 4), dtype=np.complex128, order="F")
    T[:, :, 0] = zero_diag
    T[:, :, 1] = singular
    T[:, :, 2] = 0.0  # all signs 0
    T[:, :, 3] = np.diag(np.arange(1, r + 1) * (-1.0) ** np.arange(r))
    Mt, Jt, piv, stats = ghsvd.hebpj_batched(ghsvd.atoms_to_device(T))
    check_atoms(T, Mt, Jt, piv, stats, "edge")
    assert int(host(stats)[2, 1]) == r
    # a NaN is reported per atom; the other atoms are unaffected
    T2 = T.copy(order="F")
    T2[1, 2, 1] = np.nan
    Mt, Jt, piv, stats = ghsvd.hebpj_batched(ghsvd.atoms_to_device(T2))
    s = host(stats)
    assert s[1, 0] == -3 and np.all(host(Jt)[1] == 0)
    check_atoms(T, Mt, Jt, piv, stats, "edge-nan", atoms=[0, 2, 3])


def test_hebpj_rejects_bad_sizes():
    T = torch.zeros((1, 513, 513), dtype=torch.complex128, device="cuda")
    with pytest.raises(ghsvd.GhsvdError):
        ghsvd.hebpj_batched(T)


def check_phase1(T, H, U, F, J, G, atoms, tag):
    r = T.shape[0]
    nl = r // 2
    for a in atoms:
        Mo, Jo, _, _ = P1.hebpj(T[:, :, a])
        Ha = H[a * r:(a + 1) * r]
        Fo = Mo @ Ha
        Fg = host(F[a * r:(a + 1) * r])
        err = np.abs(Fg - Fo).max() / np.abs(Fo).max()
        assert err <= 1e-11, (tag, a, err)
        assert np.array_equal(host(J[a * r:(a + 1) * r]), Jo), (tag, a)
        Go = np.vstack([Ha[:nl], U[:, a][:, None] * Ha[nl:]])
        assert np.array_equal(host(G[a * r:(a + 1) * r]), Go), (tag, a)


@pytest.mark.parametrize("kind,nl,atoms,n", [("A", 20, 5, 130), ("B", 9, 7, 64), ("A", 1, 2, 1),
                                             ("A", 33, 3, 65)])
def test_phase1_matches_oracle(kind, nl, atoms, n):
    T, H, U = synth.phase1_set(41 + n, atoms, kind, nl, n)
    F, J, G, stats = ghsvd.phase1(ghsvd.atoms_to_device(T), ghsvd.to_device_fortran(H),
                                  torch.from_numpy(np.ascontiguousarray(U.T)).cuda())
    assert np.all(host(stats)[:, 0] >= 0)
    check_phase1(T, H, U, F, J, G, range(atoms), f"{kind} nl={nl} n={n}")


def test_phase1_a1_shape_sampled():
    """The A1-shaped set at full size, three atoms against the oracle."""
    cfg = synth.PHASE1_SETS["A1"]
    T, H, U = synth.phase1_set(cfg["seed"], cfg["atoms"], cfg["kind"], cfg["nl"], cfg["n"])
    print(f"A1 set: m = {H.shape[0]}, n = {H.shape[1]}", flush=True)
    F, J, G, stats = ghsvd.phase1(ghsvd.atoms_to_device(T), ghsvd.to_device_fortran(H),
                                  torch.from_numpy(np.ascontiguousarray(U.T)).cuda())
    s = host(stats)
    assert np.all(s[:, 0] >= 0) and np.all(s[:, 1] == 0)
    Jh = host(J).reshape(cfg["atoms"], -1)
    assert np.all((Jh > 0).sum(axis=1) == 3)  # inertia of every T_a
    check_phase1(T, H, U, F, J, G, [0, 57, cfg["atoms"] - 1], "A1")


def test_phase1_then_solve_gives_pencil_eigenvalues():
    """Phase 1 on the GPU, then the GHSVD solve, against the eigenvalues of
    H = sum_a H_a^* T_a H_a, S = sum_a S_a^* S_a formed on the host."""
    T, H, U = synth.phase1_set(51, 4, "A", 10, 60)
    F, J, G, stats = ghsvd.phase1(ghsvd.atoms_to_device(T), ghsvd.to_device_fortran(H),
                                  torch.from_numpy(np.ascontiguousarray(U.T)).cuda())
    lam, X, info = ghsvd.solve(F, J, G)
    r, nl = T.shape[0], T.shape[0] // 2
    Hm = sum(H[a * r:(a + 1) * r].conj().T @ T[:, :, a] @ H[a * r:(a + 1) * r] for a in range(4))
    Sm = 0
    for a in range(4):
        Ha = H[a * r:(a + 1) * r]
        Sa = np.vstack([Ha[:nl], U[:, a][:, None] * Ha[nl:]])
        Sm = Sm + Sa.conj().T @ Sa
    ref = np.sort(sla.eigh(Hm, Sm, eigvals_only=True))
    np.testing.assert_allclose(np.sort(host(lam)), ref, rtol=1e-10, atol=0)
