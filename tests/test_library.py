"""Host-side checks of the C interface (no GPU needed): the library loads,
exports every symbol include/ghsvd.h declares, and its host-only helpers
agree with the independent oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1907_08560_amd", "libghsvd.so")
HEADER = os.path.join(ROOT, "include", "ghsvd.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ghsvd_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libghsvd.so not built")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_1907_08560_amd import ghsvd
    assert sorted(ghsvd.EXPORTED) == declared_functions()


def test_round_robin_matches_oracle(oracle):
    from paper_1907_08560_amd import ghsvd
    for n in (1, 2, 3, 10, 11, 64, 101):
        s1, p1, q1 = ghsvd.round_robin(n)
        s2, p2, q2 = oracle.round_robin(n)
        assert s1 == s2
        assert np.array_equal(p1, p2) and np.array_equal(q1, q2)


def test_workspace_and_defaults(lib):
    from paper_1907_08560_amd import ghsvd
    o = ghsvd.options()
    assert o.reduce == 1 and o.max_sweeps == 60 and o.sort == 1
    assert ghsvd.workspace_size(96, 64, 128, o) > 3 * 64 * 64 * 16
    assert ghsvd.workspace_size(10, 20, 30, o) == 0      # m < n
    assert ghsvd.workspace_size(30, 20, 10, o) == 0      # p < n
    assert ghsvd.workspace_size(30, 0, 30, o) == 0


def test_status_strings(lib):
    from paper_1907_08560_amd import ghsvd
    for s in (0, 1, -1, -2, -3, -4, -5):
        assert ghsvd._lib.ghsvd_status_string(s)


def test_full_workspace_size(lib):
    from paper_1907_08560_amd import ghsvd
    assert ghsvd.full_workspace_size(1024) >= 4 * 1024 * 1024 * 16
    assert ghsvd.full_workspace_size(64) < ghsvd.full_workspace_size(65)
    assert ghsvd.full_workspace_size(0) == 0
    assert ghsvd.full_workspace_size(4097) == 0
