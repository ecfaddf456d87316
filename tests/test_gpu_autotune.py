"""GPU checks of the launch tuner (ghsvd_autotune): it returns candidates it
timed, a later solve with automatic launch parameters gives the same result,
bit for bit, as a solve with those parameters set explicitly, and both match
the oracle.
"""
import numpy as np
import pytest
import torch

from paper_1907_08560_amd import ghsvd, synth
from gpu_util import host, rel_err, to_dev

pytestmark = pytest.mark.gpu

SIZES = [120, 77, 96]


@pytest.mark.parametrize("variant", ["pointwise", "blocked"])
def test_autotune_then_solve(oracle, variant):
    ghsvd.autotune_clear()
    Ps = [synth.workload_pencil(4, k, n_override=n) for k, n in enumerate(SIZES)]
    dev = [to_dev(P) for P in Ps]
    Fs, Js, Gs = [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev]
    w, wpp, trials = ghsvd.autotune(Fs, Js, Gs, variant=variant)
    assert wpp in (1, 2, 4, 8)
    assert all(trials[f"pointwise_wpp{k}"] > 0 for k in (1, 2, 4, 8))
    if variant == "blocked":
        assert w in (8, 16)
        assert trials["blocked_w8"] > 0 and trials["blocked_w16"] > 0 and trials["blocked_w32"] > 0
    lam_a, X_a, inf_a, rc = ghsvd.solve_batched(Fs, Js, Gs, variant=variant)
    assert rc == 0
    lam_e, X_e, inf_e, rc = ghsvd.solve_batched(Fs, Js, Gs, variant=variant, block_width=w,
                                                waves_per_pair=wpp)
    assert rc == 0
    for k, P in enumerate(Ps):
        assert torch.equal(lam_a[k], lam_e[k]) and torch.equal(X_a[k], X_e[k])
        st, lam_o, _, _ = oracle.ghsvd(P.F, P.J, P.G, max_sweeps=80)
        assert rel_err(host(lam_a[k]), lam_o) <= 1e-10
    ghsvd.autotune_clear()
