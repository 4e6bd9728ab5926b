"""Learning-rate schedule of the training driver (host logic only): linear warm-up, cosine decay to the final
rate, the first rate before the schedule starts and the final one after it ends."""
import math

import pytest

train = pytest.importorskip("paper_2409_02912_amd.train")


def _trainer(lr):
    t = train.Trainer.__new__(train.Trainer)   # the schedule needs no device state
    t.lr = lr
    return t


def test_constant_without_schedule():
    t = _trainer(1e-3)
    assert t.lr_at(0) == 1e-3 and t.lr_at(10 ** 6) == 1e-3


def test_warmup_then_cosine():
    t = _trainer(1e-3)
    t.set_schedule(100, 1100, warmup=100, lr_final=1e-5)
    assert t.lr_at(100) == pytest.approx(1e-3 / 100)
    assert t.lr_at(199) == pytest.approx(1e-3)
    assert t.lr_at(200) == pytest.approx(1e-3)                       # cosine at its start
    mid = 200 + (1100 - 100 - 100) // 2
    assert t.lr_at(mid) == pytest.approx(1e-5 + 0.5 * (1e-3 - 1e-5))
    assert t.lr_at(1100) == pytest.approx(1e-5)
    assert t.lr_at(5000) == pytest.approx(1e-5)
    lrs = [t.lr_at(s) for s in range(200, 1101, 50)]
    assert all(a >= b for a, b in zip(lrs, lrs[1:]))


def test_steps_before_the_start_take_the_first_rate():
    # resuming a checkpoint whose step is below the schedule's start (a warm restart set ahead of it)
    t = _trainer(1.5e-4)
    t.set_schedule(250000, 400000, warmup=0, lr_final=1e-6)
    assert t.lr_at(245589) == pytest.approx(1.5e-4)
    t.set_schedule(250000, 400000, warmup=10, lr_final=1e-6)
    assert t.lr_at(245589) == pytest.approx(1.5e-4 / 10)
    assert math.isfinite(t.lr_at(0))
