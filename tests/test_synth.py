"""The seeded input generator: determinism and the stated recipe."""
import numpy as np

from paper_1907_08560_amd import synth


def test_deterministic():
    a = synth.workload_pencil(1)
    b = synth.workload_pencil(1)
    assert np.array_equal(a.F, b.F) and np.array_equal(a.G, b.G) and np.array_equal(a.J, b.J)


def test_workload_one_shape():
    P = synth.workload_pencil(1)
    assert P.F.shape == (96, 64) and P.G.shape == (128, 64)
    assert P.m_plus == 72 and np.all(P.J[:72] == 1) and np.all(P.J[72:] == -1)
    assert P.F.flags.f_contiguous and P.G.flags.f_contiguous
    sv = np.linalg.svd(P.G, compute_uv=False)
    assert np.allclose(np.sort(sv), np.sort(P.s), rtol=1e-10)
    assert sv.min() >= 1e-4 * (1 - 1e-9) and sv.max() <= 1.0 + 1e-9


def test_batched_sizes():
    n4 = synth.workload_sizes(4)
    assert len(n4) == 64 and min(n4) >= 300 and max(n4) <= 900
    n5 = synth.workload_sizes(5)
    assert len(n5) == 16 and min(n5) >= 2000 and max(n5) <= 6000
    P = synth.workload_pencil(4, 3, n_override=50)
    assert P.F.shape == (75, 50) and P.G.shape == (100, 50) and P.m_plus == 56


def test_j_identity():
    P = synth.workload_pencil(3, j_identity=True, n_override=40)
    assert np.all(P.J == 1)
