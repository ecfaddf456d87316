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


def test_device_builder_matches_host_recipe():
    """The torch-side builder draws the same numbers in the same order; its QRs
    and product only change G by rounding."""
    import torch
    P = synth.random_pencil(7, 40, 60, 45, 80, 1e-6)
    rng = np.random.Generator(np.random.PCG64(7))
    F, J, G, s = synth.make_pencil_device(rng, 40, 60, 45, 80, 1e-6, "cpu")
    assert F.stride(0) == 1 and G.stride(0) == 1
    assert np.array_equal(F.numpy(), P.F)
    assert np.array_equal(J.numpy(), P.J)
    assert np.array_equal(s, P.s)
    assert np.abs(G.numpy() - P.G).max() <= 1e-13 * np.abs(P.G).max()
    sv = np.linalg.svd(G.numpy(), compute_uv=False)
    assert np.allclose(np.sort(sv), np.sort(P.s), rtol=1e-10, atol=0)
    assert torch.is_tensor(G) and G.dtype == torch.complex128
