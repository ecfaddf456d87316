"""GPU parity of ghsvd_solve_batched: many pencils of uneven order in one call
(the batched workload's recipe, downsized so the oracle finishes in seconds).

Each pencil's eigenvalues match the oracle; with the launch geometry fixed
(waves per pair, block width) each pencil's result is bitwise identical to
its own single-pencil solve, since no reduction crosses pencils; a pencil with
bad input fails alone.
"""
import numpy as np
import pytest
import torch

from paper_1907_08560_amd import ghsvd, synth
from gpu_util import host, rel_err, to_dev

pytestmark = pytest.mark.gpu

SIZES = [37, 64, 90, 51, 120, 8, 77, 101]


def pencils():
    return [synth.workload_pencil(4, k, n_override=n) for k, n in enumerate(SIZES)]


@pytest.fixture(scope="module")
def oracle_lams(oracle):
    out = []
    for P in pencils():
        st, lam, X, stats = oracle.ghsvd(P.F, P.J, P.G, max_sweeps=80)
        assert st == 0
        out.append(lam)
    return out


@pytest.mark.parametrize("precision,variant", [("fp64", "pointwise"), ("fp64", "blocked"),
                                               ("mixed", "blocked"), ("mixed", "pointwise")])
def test_batched_matches_oracle_and_single(oracle_lams, precision, variant):
    Ps = pencils()
    dev = [to_dev(P) for P in Ps]
    kw = dict(precision=precision, variant=variant, waves_per_pair=4, block_width=8)
    lams, Xs, infos, rc = ghsvd.solve_batched([d[0] for d in dev], [d[1] for d in dev],
                                              [d[2] for d in dev], **kw)
    assert rc == 0, infos
    for k, P in enumerate(Ps):
        assert infos[k]["status"] == 0
        lam = host(lams[k])
        assert rel_err(lam, oracle_lams[k]) <= 1e-10, (k, rel_err(lam, oracle_lams[k]))
        lam1, X1, info1 = ghsvd.solve(*dev[k], **kw)
        assert torch.equal(lam1, lams[k]) and torch.equal(X1, Xs[k]), k
        assert info1["sweeps_fp64"] == infos[k]["sweeps_fp64"]


def test_batched_isolates_failures(oracle_lams):
    Ps = pencils()[:4]
    dev = [list(to_dev(P)) for P in Ps]
    F1 = dev[1][0].clone()
    F1[2, 2] = float("nan")
    dev[1][0] = F1
    J3 = dev[3][1].clone()
    J3[0] = 3
    dev[3][1] = J3
    lams, Xs, infos, rc = ghsvd.solve_batched([d[0] for d in dev], [d[1] for d in dev],
                                              [d[2] for d in dev], check=False)
    assert [i["status"] for i in infos] == [0, -3, 0, -1]
    assert rc == -3
    for k in (0, 2):
        assert rel_err(host(lams[k]), oracle_lams[k]) <= 1e-10


def test_batched_square_and_tall_mixed(oracle):
    # a square pencil (no reduction) next to tall ones
    Ps = pencils()[:3]
    Q = synth.random_pencil(77, 30, 30, 20, 30, 1e-2)
    Ps.append(Q)
    dev = [to_dev(P) for P in Ps]
    lams, Xs, infos, rc = ghsvd.solve_batched([d[0] for d in dev], [d[1] for d in dev],
                                              [d[2] for d in dev], variant="blocked")
    assert rc == 0
    assert infos[3]["m_r"] == 30 and infos[0]["m_r"] == Ps[0].n
    for k, P in enumerate(Ps):
        st, lam_o, _, _ = oracle.ghsvd(P.F, P.J, P.G, max_sweeps=80)
        assert rel_err(host(lams[k]), lam_o) <= 1e-10


@pytest.mark.parametrize("count", [70, 1030])
def test_batched_many_pencils(count):
    """More pencils than one 64-lane lookup chunk (70), and more than the
    ballot lookup covers (1030, binary search): every workgroup must find
    its pencil, so each pencil's result equals its own single solve."""
    sizes = [4 + (k * 7) % 9 for k in range(count)]
    Ps = [synth.random_pencil(5000 + k, n, 2 * n, n + 1, 2 * n, 1e-2) for k, n in enumerate(sizes)]
    dev = [to_dev(P) for P in Ps]
    kw = dict(precision="fp64", variant="blocked", waves_per_pair=1, block_width=8)
    lams, Xs, infos, rc = ghsvd.solve_batched([d[0] for d in dev], [d[1] for d in dev],
                                              [d[2] for d in dev], **kw)
    assert rc == 0
    for k in sorted({0, 1, 63, 64, 65, count // 2, count - 1}):
        assert infos[k]["status"] == 0, (k, infos[k])
        lam1, X1, info1 = ghsvd.solve(*dev[k], **kw)
        assert torch.equal(lam1, lams[k]) and torch.equal(X1, Xs[k]), k


@pytest.mark.parametrize("precision,inner", [("fp64", "cross"), ("mixed", "cross"),
                                             ("fp64", "full"), ("fp64", "fb")])
def test_large_batch_every_inner_order(oracle_lams, precision, inner):
    # 112 pencils (14 copies of the batch, 532 block pairs per launch at w = 8)
    # in every inner ordering: each pencil matches the oracle and equals its
    # own single solve bit for bit
    Ps = pencils()
    dev = [to_dev(P) for P in Ps] * 14
    kw = dict(precision=precision, variant="blocked", waves_per_pair=4, block_width=8,
              inner_order=inner)
    lams, Xs, infos, rc = ghsvd.solve_batched([d[0] for d in dev], [d[1] for d in dev],
                                              [d[2] for d in dev], **kw)
    assert rc == 0, infos
    for k in range(len(Ps)):
        assert rel_err(host(lams[k]), oracle_lams[k]) <= 1e-10
    for k in (0, 4, len(Ps) * 13 + 1):
        lam1, X1, info1 = ghsvd.solve(*dev[k], **kw)
        assert torch.equal(lam1, lams[k]) and torch.equal(X1, Xs[k]), k
        assert info1["sweeps_fp64"] == infos[k]["sweeps_fp64"]


def test_batched_reduction_windows_match_single_solves():
    # one pencil whose F columns need the streaming loops at first beside
    # small ones: in the batch every pencil's column steps run one column per
    # step workgroup in those windows, in its single solve two; the
    # arithmetic per column is the same, so the results are bitwise equal
    shapes = [(150, 2200, 1650, 300), (120, 400, 300, 240), (91, 300, 225, 182),
              (64, 1700, 1275, 128)]
    Ps = [synth.random_pencil(950 + k, n, m, mp, p, 1e-3) for k, (n, m, mp, p) in enumerate(shapes)]
    devs = [to_dev(P) for P in Ps]
    kw = dict(precision="fp64", variant="blocked", block_width=16)
    lam, X, infos, rc = ghsvd.solve_batched([d[0] for d in devs], [d[1] for d in devs],
                                            [d[2] for d in devs], **kw)
    assert rc == 0
    for k, (F, J, G) in enumerate(devs):
        l1, X1, info1 = ghsvd.solve(F, J, G, **kw)
        assert info1["status"] == 0
        assert torch.equal(lam[k], l1) and torch.equal(X[k], X1), k
