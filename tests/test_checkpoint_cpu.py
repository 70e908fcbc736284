"""Checkpoint interval of the differentiable solve (host logic, CPU)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2603_15964_amd.autograd import checkpoint_interval  # noqa: E402

GB = 1 << 30


def test_every_state_kept_when_it_fits():
    # 100 steps of 64 x 262144 doubles (13.4 GB) on a GPU with 250 GB free
    assert checkpoint_interval(100, 64 * 262144 * 8, 250 * GB) == 1


def test_sqrt_interval_when_it_does_not_fit():
    # the same run with 20 GB free: ceil(sqrt(100)) = 10
    assert checkpoint_interval(100, 64 * 262144 * 8, 20 * GB) == 10
    assert checkpoint_interval(101, 64 * 262144 * 8, 20 * GB) == 11
    assert checkpoint_interval(1, 10 * GB, 1 * GB) == 1


def test_budget_boundary():
    # exactly half the free memory still fits
    assert checkpoint_interval(10, GB, 20 * GB) == 1
    assert checkpoint_interval(11, GB, 20 * GB) == 4
