"""The accuracy score of the multicanonical comparison (ln g = ln H - ln W
against the stored exact ln g): zero for a histogram that reproduces the
exact density of states, invariant under a constant shift of ln W, and equal
to the perturbation's half-spread for a known perturbation."""
import os

import numpy as np

from paper_1709_04394_amd import learned_muca as lm

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lng_L16.txt")


def _setup():
    ex = np.loadtxt(GOLD)
    rng = np.random.default_rng(3)
    H = rng.integers(1000, 5000, size=ex.size).astype(np.int64)
    m = np.isfinite(ex)
    H[~m] = 0
    lnW = np.zeros(ex.size)
    lnW[m] = np.log(H[m]) - ex[m] + 7.25  # ln H - ln W = ln g_exact - 7.25
    return ex, H, lnW, m


def test_exact_histogram_scores_zero():
    ex, H, lnW, _ = _setup()
    lse, best = lm.lng_errors(H, lnW, ex)
    assert lse < 1e-9 and best < 1e-9


def test_constant_shift_of_weights_is_invisible():
    ex, H, lnW, _ = _setup()
    assert np.allclose(lm.lng_errors(H, lnW + 123.0, ex), lm.lng_errors(H, lnW, ex), atol=1e-9)


def test_known_perturbation():
    ex, H, lnW, m = _setup()
    pert = np.zeros(ex.size)
    pert[m] = np.linspace(-0.02, 0.03, int(m.sum()))  # spread 0.05 -> best-constant error 0.025
    lse, best = lm.lng_errors(H, lnW - pert, ex)
    assert abs(best - 0.025) < 1e-9
    assert lse >= best - 1e-12


def test_empty_level_is_infinite():
    ex, H, lnW, m = _setup()
    H = H.copy()
    H[np.flatnonzero(m)[3]] = 0
    assert lm.lng_errors(H, lnW, ex) == (float("inf"), float("inf"))


def test_score_stage_end_to_end(tmp_path, capsys):
    # the command-line score stage on synthetic files: two runs of one arm whose
    # summed histogram reproduces the exact ln g up to a constant, one that
    # does not
    import json

    ex, H, lnW, m = _setup()
    np.savez(tmp_path / "weights.npz", lnW_plain=lnW, lnW_learned=lnW, lnW_init=lnW, L=16)
    conv = {arm: {"iterations": 1.0, "sweeps_per_walker": 10.0, "total_sweeps": 10.0, "seconds": 0.0,
                  "min_over_max": 1.0, "converged": True} for arm in ("plain", "learned")}
    (tmp_path / "converge.json").write_text(json.dumps(conv))
    np.save(tmp_path / "H_plain_1.npy", H)
    np.save(tmp_path / "H_plain_2.npy", 2 * H)
    Hb = H.copy()
    Hb[np.flatnonzero(m)[:10]] *= 2
    np.save(tmp_path / "H_learned_1.npy", Hb)
    lm.main(["score", "--dir", str(tmp_path), "--exact", GOLD])
    out = json.loads(capsys.readouterr().out)
    assert out["plain"]["max_abs_lng_error_best_constant"] < 1e-9
    assert set(out["plain"]["runs"]) == {"H_plain_1", "H_plain_2"}
    assert abs(out["learned"]["max_abs_lng_error_best_constant"] - np.log(2) / 2) < 1e-9
