"""The allocation-free blocked sweeps (ghsvd_block_sweeps_noalloc) against
ghsvd_block_sweeps, through the C ABI.

Both run the same kernels in the same launch geometry; only where the scratch
lives differs (a library-owned static device array instead of an allocation
per call).  The swept F, G, Z, the per-sweep counters, the sweep count and
the status must agree bit for bit, on two calls in a row (the second with a
smaller pencil, so it runs over what the first left in the array), and a
pencil whose scratch exceeds the array is rejected before any work.
"""
import math

import numpy as np
import pytest
import torch

from paper_1907_08560_amd import ghsvd, synth
from gpu_util import host, to_dev

pytestmark = pytest.mark.gpu


def pencil(seed, n, s_lo):
    m = int(math.ceil(1.5 * n))
    p = 2 * n
    return synth.random_pencil(seed, n, m, int(round(0.75 * m)), p, s_lo)


def sweep_both(P, w, inner, nsweeps):
    F, J, G = to_dev(P)
    Z = ghsvd.to_device_fortran(np.eye(P.n, dtype=np.complex128))
    outs = []
    for noalloc in (False, True):
        Fw = F.t().clone().t()
        Gw = G.t().clone().t()
        Zw = Z.t().clone().t()
        rc, done, cnt = ghsvd.block_sweeps(Fw, P.m_plus, Gw, Zw, nsweeps, block_width=w,
                                           inner_order=inner, noalloc=noalloc)
        torch.cuda.synchronize()
        outs.append((rc, done, cnt, host(Fw), host(Gw), host(Zw)))
    return outs


def assert_same(a, b):
    assert a[0] == b[0] and a[1] == b[1], (a[:2], b[:2])
    assert np.array_equal(a[2], b[2])
    for x, y in zip(a[3:], b[3:]):
        assert np.array_equal(np.ascontiguousarray(x).view(np.float64),
                              np.ascontiguousarray(y).view(np.float64))


@pytest.mark.parametrize("w,inner", [(16, "cross"), (32, "full"), (8, "fb")])
def test_noalloc_matches_block_sweeps_two_calls(w, inner):
    big = pencil(911, 300, 1e-4)
    first = sweep_both(big, w, inner, 60)
    assert first[0][0] == 0 and first[0][1] > 3
    assert_same(*first)
    small = pencil(912, 70, 1e-3)
    second = sweep_both(small, w, inner, 60)
    assert second[0][0] == 0
    assert_same(*second)


def test_noalloc_rejects_oversized_pencil():
    n = 2048
    F = ghsvd.fortran_empty(n, n, device="cuda")
    G = ghsvd.fortran_empty(n, n, device="cuda")
    Z = ghsvd.fortran_empty(n, n, device="cuda")
    F.zero_()
    rc, done, cnt = ghsvd.block_sweeps(F, n, G, Z, 1, block_width=32, noalloc=True)
    assert rc == -4 and done == 0
    torch.cuda.synchronize()
    assert not bool(F.abs().amax() > 0)
