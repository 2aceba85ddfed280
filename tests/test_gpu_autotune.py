"""The autotuner on the GPU: every swept configuration computes the oracle's product, and the fit and the
model's pick come out of the sweep consistently (Section 4.1's procedure at a small scale)."""

import numpy as np
import pytest

from gen import laplacian, random_sparse
from gpu_util import check_forward, say
from oracle import spmv as OS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05096_amd import autotune as T  # noqa: E402


def _checker(A, seen, store):
    def on_trial(M, x, y, trial):
        perm = M.structure()["perm"]
        x_in = np.empty(A.n)
        x_in[perm] = x.double().cpu().numpy()
        yg = y.double().cpu().numpy()
        check_forward(yg, A, x_in, perm, store, False, label=f"{trial}")  # x_in: the values the GPU read
        seen.append(trial)
    return on_trial


@pytest.mark.parametrize("objective", ["forward", "step"])
def test_sweep_checks_every_candidate(objective):
    A = random_sparse(5000, 9.0, seed=11, empty_row_frac=0.03)
    seen = []
    say("autotune sweep", objective)
    res = T.sweep(A, "f64", srs_list=(16, 48), ssrs_list=(2, 4), lanes_list=(1, 2, 4), reps=3,
                  objective=objective, threads=2, name="rand5000", on_trial=_checker(A, seen, "f64"))
    assert len(res.trials) == 2 * 2 * 3 and len(seen) == len(res.trials)
    assert {(t.srs, t.ssrs, t.lanes) for t in res.trials} == {(a, b, c) for a in (16, 48) for b in (2, 4)
                                                             for c in (1, 2, 4)}
    assert all(t.waves == t.ssrs for t in res.trials)
    assert all(np.isfinite(t.us) and t.us > 0 for t in res.trials)
    assert res.best.us == min(t.us for t in res.trials)
    assert res.rdensity == pytest.approx(A.nnz / A.n)


def test_fit_and_model_pick_over_two_matrices():
    mats = [laplacian((40, 40), "2d5", 4.0), laplacian((14, 14, 14), "3d27", 26.0)]
    results = []
    for A in mats:
        seen = []
        say("autotune fit", A.n, A.nnz)
        results.append(T.sweep(A, "f32", srs_list=(16, 32, 64), ssrs_list=(2, 4), lanes_list=(1, 2), reps=3,
                               threads=2, on_trial=_checker(A, seen, "f32")))
        assert len(seen) == 12
    consts = T.fit(results)
    # two points: the log-regression passes through both optima
    for res in results:
        assert T.model_pick(consts["srs"], res.rdensity) == res.best.srs
        assert T.model_pick(consts["ssrs"], res.rdensity) == res.best.ssrs
    ev = T.evaluate(results, consts)
    for e, res in zip(ev, results):
        assert e["model_srs"] in (16, 32, 64) and e["model_ssrs"] in (2, 4)
        assert e["ratio"] >= 1.0
        assert e["best"]["us"] == res.best.us


def test_workload_grid_report(tmp_path, capsys):
    """The single-workload grid sweep: every cell timed, the optimum and the three models' picks reported."""
    out = tmp_path / "grid.md"
    say("autotune grid c1")
    T.main(["--workload", "c1", "--store", "f64", "--objective", "forward", "--srs", "8,16", "--ssrs", "2,4",
            "--lanes", "1,2", "--threads", "2", "--markdown", str(out)])
    text = out.read_text()
    assert "| 8 | " in text and "| 16 | " in text and "Optimum: SRS" in text
    for model in ("mi355x", "volta", "ampere"):
        assert f"| {model} | (" in text
