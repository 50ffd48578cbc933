"""Host logic of the request loop: the plateau test that retires a run
stalled at its rounding floor."""
import numpy as np

from paper_1109_6672_amd.serving import Plateau


def _first_plateau(seq):
    pl = Plateau()
    for i, r in enumerate(seq):
        if pl.update(r):
            return i
    return None


def test_onset_and_decaying_oscillation_are_not_a_plateau():
    t = np.arange(400)
    onset = 1e-9 * np.exp(0.5 * np.arange(30))                  # growing from a quiescent start
    decay = onset[-1] * np.exp(-0.03 * t) * (1.5 + np.cos(0.7 * t))  # oscillating, decaying envelope
    assert _first_plateau(np.concatenate([onset, decay])) is None


def test_a_noise_floor_is_a_plateau():
    rng = np.random.default_rng(7)
    decay = 1e-3 * np.exp(-0.1 * np.arange(100))
    floor = 1e-7 * (1 + 0.2 * rng.random(400))
    i = _first_plateau(np.concatenate([decay, floor]))
    assert i is not None and 100 < i < 400


def test_a_late_hump_of_the_transient_is_not_a_plateau():
    # a second, lower hump lasting longer than ten checks
    seq = list(np.linspace(1e-6, 1e-3, 10)) + list(np.linspace(1e-3, 2e-4, 8)) + list(np.linspace(2e-4, 5e-4, 15)) \
        + list(5e-4 * np.exp(-0.1 * np.arange(40)))
    assert _first_plateau(seq) is None


def test_a_transient_stall_far_above_the_floor_is_not_a_plateau():
    # an impulsive start, then a stall at 2 % of the peak for 20 checks
    seq = [5e-2] + list(np.linspace(7e-3, 1e-3, 20)) + [1.2e-3, 1.1e-3] * 10 + list(1e-3 * np.exp(-0.05 * np.arange(60)))
    assert _first_plateau(seq) is None


def test_minimum_is_counted_from_the_last_maximum():
    # a quiet start sets a tiny early minimum; without the reset the rising
    # residual would be taken for a stall after 10 checks
    seq = [1e-12] + list(np.linspace(1e-8, 1e-4, 40)) + list(1e-4 * np.exp(-0.2 * np.arange(60)))
    assert _first_plateau(seq) is None


def test_a_floor_near_a_thousandth_of_the_peak_is_a_plateau():
    # 16-bit storage: the residual settles near 1e-4 after an onset peak of
    # about 0.1 and never reaches a tolerance of 1e-8
    rng = np.random.default_rng(3)
    seq = [0.1] + list(0.1 * np.exp(-0.15 * np.arange(1, 50))) + list(1e-4 * (1 + 0.3 * rng.random(300)))
    i = _first_plateau(seq)
    assert i is not None and 50 < i < 350
