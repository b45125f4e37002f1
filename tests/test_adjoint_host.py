"""Host logic of the reverse-pass driver: the checkpoint interval it picks so
that the checkpoints and the tape fit in device memory (CPU only)."""

import pytest

from paper_2507_14282_amd.adjoint import checkpoint_interval


def test_requested_interval_when_it_fits():
    assert checkpoint_interval(400, 20, 1e9, 100e9) == 20
    assert checkpoint_interval(40, 20, 9e9, 288e9) == 20        # (2 + 20) states of 9 GB
    assert checkpoint_interval(7, 20, 1e6, 1e12) == 7           # never more than the steps


def test_smaller_interval_when_memory_is_short():
    # 40 steps, 9 GB states, 120 GB usable: (ceil(40/k) + k) * 9 <= 120 first holds at k = 8
    k = checkpoint_interval(40, 20, 9e9, 150e9)
    assert k == 8
    assert (-(-40 // k) + k) * 9e9 <= 0.8 * 150e9
    assert (-(-40 // 9) + 9) * 9e9 > 0.8 * 150e9


def test_no_interval_fits():
    # 400 steps need at least 40 states; 40 x 9 GB > 0.8 x 288 GB
    with pytest.raises(MemoryError):
        checkpoint_interval(400, 20, 9e9, 288e9)
