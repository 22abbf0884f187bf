"""Kernel-choice autotuner: the threshold rule on synthetic timings (CPU),
and one tuning run on the GPU that must pick a bound among the one-wave
variants' stage blocks and leave the results unchanged."""
import numpy as np
import pytest

from paper_2003_02547_amd import autotune as A


def test_choose_bound_threshold_rule():
    t = {(4, 4, 0): (1.0, 2.0), (8, 4, 0): (1.0, 2.0), (8, 8, 0): (1.0, 1.5), (16, 8, 0): (3.0, 2.0),
         (8, 16, 0): (1.0, 2.0)}
    # (16, 8) and (8, 16) both have nz = 24; (16, 8) loses, so the bound stops below 24
    assert A.choose_bound(t) == 16
    assert A.choose_bound({(4, 4, 0): (2.0, 1.0)}) == 0
    assert A.choose_bound({(4, 4, 0): (1.0, 2.0), (16, 8, 0): (1.0, 2.0)}) == 24
    assert A.choose_bound({}) == 0


@pytest.mark.gpu
def test_tune_on_device_sets_a_valid_bound():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2003_02547_amd import binding as B
    from paper_2003_02547_amd import workloads as W
    old = B.lib().oqp_get_wave_max()
    try:
        out = A.tune(count=32, N=8, reps=1, apply=True)
        nzs = {0} | {nx + nu for nx, nu, ng in B.variants()}
        assert out["bound"] in nzs
        assert B.lib().oqp_get_wave_max() == out["bound"]
        assert len(out["timings"]) == len(B.variants())
        qps = [W.mass_spring_chain4(s) for s in range(1, 4)]
        for r in B.solve(qps):
            assert r.status == B.SUCCESS
    finally:
        B.set_wave_max(old)
