"""The autotuner's decision rule (host only) and, on the GPU, that its choice
meets the gate and is the fastest candidate that does."""
import pytest

from paper_2209_13121_amd import autotune as T


def R(ms, e, f, kind="F16X2", leaf=64):
    return T.Result(tree={"leaf_max": leaf}, kind=kind, ms=ms, energy_err=e, force_err=f)


def test_select_fastest_within_gate():
    rs = [R(5.0, 1e-7, 1e-6, "F32"), R(3.0, 2e-6, 1e-6, "F16X2"), R(4.0, 1e-8, 2e-6, "BF16X3"),
          R(2.0, 1e-9, 3e-5, "F16X2", 32)]
    best = T.select(rs)
    assert best.kind == "BF16X3" and best.ms == 4.0


def test_select_ties_and_none():
    rs = [R(3.0, 1e-7, 1e-6, "F32"), R(3.0, 1e-7, 1e-6, "F16X2")]
    assert T.select(rs).kind == "F32"
    assert T.select([R(1.0, 1e-3, 1e-6)]) is None
    assert T.select([]) is None
    # the gate is inclusive
    assert T.select([R(1.0, 1e-6, 1e-5)]) is not None


@pytest.mark.gpu
def test_tune_on_clusters():
    import torch
    from paper_2209_13121_amd import workloads as W
    pos, q, _ = W.molecular_clusters(50_000, 61)
    dev = torch.device("cuda:0")
    tp, tq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
    best, results = T.tune(tp, tq, 8, [{"depth": 7, "leaf_max": 32}, {"depth": 7, "leaf_max": 64}],
                           side=0.0, reps=3)
    assert len(results) == 6
    assert best is not None and best.meets(1e-6, 1e-5)
    assert all(best.ms <= r.ms for r in results if r.meets(1e-6, 1e-5))
