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


def test_schedule_decision_rules():
    # a variant keeps its bit only where the one-wave kernel is faster
    assert A.choose_variant_mask({0: (1.0, 2.0), 3: (2.0, 1.0), 5: (1.0, 1.0)}, 0xFF) == 0xFF & ~(1 << 3) & ~(1 << 5)
    assert A.choose_variant_mask({}, 0x7) == 0x7
    # fastest launch schedule; ties: fewer streams, then the LDS split
    t = {(0, 1): 3.0, (1, 1): 2.0, (3, 1): 2.0, (0, 0): 3.0, (1, 0): 2.0, (3, 0): 1.5}
    assert A.choose_launch(t) == (3, 0)
    t[(3, 0)] = 2.0
    assert A.choose_launch(t) == (1, 1)
    with pytest.raises(ValueError):
        A.choose_launch({})


@pytest.mark.gpu
def test_tune_schedule_on_device():
    """A tuned schedule for a small uneven batch: a valid mask and launch
    choice, applied process wide, cached by the batch's kernel groups, and
    results that meet the KKT tolerance under it."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2003_02547_amd import binding as B
    from paper_2003_02547_amd import workloads as W
    L = B.lib()
    old_mask, old_split = L.oqp_get_variant_mask(), L.oqp_get_lds_split()
    try:
        qps = [W.random_uneven(i) for i in range(48)]
        out = A.tune_schedule(qps, reps=1, stream_options=(0, 1))
        assert out["streams"] in (0, 1) and out["lds_split"] in (0, 1)
        assert L.oqp_get_variant_mask() == out["variant_mask"] and L.oqp_get_lds_split() == out["lds_split"]
        assert set(out["launch"]) == {"0x1", "1x1", "0x0", "1x0"}
        nv = L.oqp_variant_count()
        b = B.Batch(qps, streams=out["streams"]).load().solve().fetch().sync()
        for i in range(len(qps)):
            g = b.variant(i)[0]
            if g < nv:
                assert (out["variant_mask"] >> g) & 1
            r = b.result(i)
            assert r.status == B.SUCCESS and max(r.res) <= 1e-8
        L.oqp_set_variant_mask(old_mask)
        again = A.tune_schedule(qps, reps=1, stream_options=(0, 1))
        assert again is out  # cached by the batch signature
    finally:
        L.oqp_set_variant_mask(old_mask)
        L.oqp_set_lds_split(old_split)
