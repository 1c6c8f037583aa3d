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
    # the command-line score stage on synthetic files: converged weights of
    # two seeds per arm, sweeps to flat per seed, and production checkpoints
    # whose histograms reproduce the exact ln g up to a constant (plain) or
    # only after the second checkpoint (learned: the first one has ten levels
    # doubled, an error of ln 2 / 2 after the best constant)
    import json

    ex, H, lnW, m = _setup()
    conv = {"L": 16, "seeds": [1, 2], "mlp_loss": [1.0, 0.1], "runs": {}}
    for sd, (fp, fl) in ((1, (900, 500)), (2, (1100, 700))):
        conv["runs"][str(sd)] = {
            "plain": {"sweeps_per_walker_incl_prep": fp}, "learned": {"sweeps_per_walker_incl_prep": fl}}
        for arm in ("plain", "learned"):
            np.save(tmp_path / ("lnW_%s_%d.npy" % (arm, sd)), lnW)
    (tmp_path / "converge.json").write_text(json.dumps(conv))
    Hb = H.copy()
    Hb[np.flatnonzero(m)[:10]] *= 2
    for arm, hs in (("plain", [H, 3 * H]), ("learned", [Hb, 2 * Hb + 2 * H])):
        base = tmp_path / ("prod_%s_1_7" % arm)
        np.save(str(base) + ".npy", np.stack(hs))
        (tmp_path / ("prod_%s_1_7.json" % arm)).write_text(json.dumps(
            {"arm": arm, "seed": 1, "pseed": 7, "walkers": 64, "burn": 0, "checkpoints": [10, 30]}))
    lm.main(["score", "--dir", str(tmp_path), "--exact", GOLD, "--target", "0.01"])
    out = json.loads(capsys.readouterr().out)
    pl, le = out["arms"]["plain"], out["arms"]["learned"]
    assert pl["sweeps_to_flat_incl_prep"] == [900, 1100] and pl["mean"] == 1000
    assert le["mean"] == 600 and abs(out["mean_sweeps_to_flat_ratio_learned_over_plain"] - 0.6) < 1e-12
    pp, lp = pl["production"]["prod_plain_1_7"], le["production"]["prod_learned_1_7"]
    assert max(pp["errors_best_constant"]) < 1e-9 and pp["walker_sweeps_to_target"] == 10 * 64
    assert abs(lp["errors_best_constant"][0] - np.log(2) / 2) < 1e-9
    assert lp["errors_best_constant"][1] > 1e-3 and lp["walker_sweeps_to_target"] is None
    # the same files as markdown: one table per arm and seed of the summed runs
    lm.main(["score", "--dir", str(tmp_path), "--exact", GOLD, "--target", "0.01", "--markdown"])
    md = capsys.readouterr().out
    assert "## plain arm (weights of seed 1; runs prod_plain_1_7)" in md
    assert "## learned arm (weights of seed 1; runs prod_learned_1_7)" in md
    assert md.count("| Production walker-sweeps |") == 2 and md.count("\n| 640 |") == 2
    # plain: within the target at the first checkpoint, 10 sweeps x 64 walkers
    # of production plus 900 x 4096 of the flat phase
    assert "Within 0.01 after 640 production walker-sweeps; with the 3.69e+06 walker-sweeps of the flat" in md
    assert "Not within 0.01 after 1.92e+03 production walker-sweeps" in md
