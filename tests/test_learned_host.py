"""Host logic of the learned-initialiser experiment: the summary it reports
(the secondary benchmark figure) from per-target rows."""
import pytest

from paper_2211_03516_amd import learned


def _row(seed, plain_steps, learned_steps, reached, fallback, plain_s, learned_s, e_p, e_l):
    return {"target_seed": seed, "plain_steps": plain_steps, "learned_steps": learned_steps,
            "learned_reached": reached, "fallback": fallback, "plain_s": plain_s, "learned_s": learned_s,
            "dose_error_plain_start": e_p, "dose_error_learned_start": e_l}


def test_summary_means_and_counts():
    rows = [_row(1, 50, 30, True, False, 0.6, 0.4, 0.5, 0.3),
            _row(2, 50, 50, False, False, 0.7, 0.8, 0.9, 0.8),
            _row(3, 50, 40, True, True, 0.5, 0.45, 0.4, 0.6)]
    s = learned.summarise(rows)
    assert s["targets"] == 3
    assert s["mean_plain_steps"] == 50.0
    assert s["mean_learned_steps"] == pytest.approx(40.0)
    assert s["mean_plain_s"] == pytest.approx(0.6) and s["mean_learned_s"] == pytest.approx(0.55)
    assert s["reached"] == 2 and s["fallbacks"] == 1
    assert s["mean_dose_error_plain_start"] == pytest.approx(0.6)
    assert s["mean_dose_error_learned_start"] == pytest.approx(0.5666666666666667)
