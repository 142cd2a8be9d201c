"""The user-level interface on the GPU: a fit from a JSON configuration finds
the clusters of the d = 2 configuration (N = 10 000), a run split into two
by a checkpoint repeats the uninterrupted run bit for bit (labels, K and
log-posterior traces; with and without the learned proposal's network
state), and the command-line tool gives the Python run's labels."""
import json
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _data(name="gauss_d2", n=None, seed=1):
    from paper_2204_08988_amd import datagen
    return datagen.workload(name, seed, n)


def test_fit_finds_clusters_and_writes_json(tmp_path):
    from paper_2204_08988_amd import fit
    x, lab = _data()
    res = fit.fit(x, {"alpha": 10.0, "iterations": 150, "burn_out": 5, "seed": 1}, gt=lab,
                  result_path=tmp_path / "r.json")
    assert 4 <= res["K"] <= 10 and res["nmi"] > 0.8
    assert len(res["labels"]) == x.shape[0] and len(res["weights"]) == res["K"]
    assert len(res["iter_time"]) == 150 and all(t > 0 for t in res["iter_time"])
    assert 0.0 < sum(res["weights"]) < 1.0  # the rest is the weight of a new cluster (the alpha slot)
    back = json.loads((tmp_path / "r.json").read_text())
    assert back["labels"] == res["labels"] and back["K"] == res["K"]


@pytest.mark.parametrize("cfg,name,n", [
    ({"iterations": 40, "burn_out": 3, "seed": 4}, "gauss_d2", None),
    ({"iterations": 40, "burn_out": 3, "seed": 5, "precision": "bf16"}, "gauss_d32", 40_000),
    ({"iterations": 30, "burn_out": 3, "seed": 6, "prior_type": "Multinomial"}, "mult_v100", 20_000),
    ({"iterations": 30, "burn_out": 3, "seed": 7, "learned": 3, "train_every": 4, "train_until": 30,
      "train_steps": 5, "train_batch": 1024}, "gauss_d64", 30_000),
])
def test_checkpoint_resume_repeats_the_run(tmp_path, cfg, name, n):
    from paper_2204_08988_amd import fit
    x, lab = _data(name, n, 2)
    full = fit.fit(x, cfg)
    half = dict(cfg, iterations=cfg["iterations"] // 2)
    a = fit.fit(x, half, checkpoint_path=tmp_path / "c.ckpt")
    b = fit.fit(x, half, resume_path=tmp_path / "c.ckpt")
    assert b["last_iteration"] == full["last_iteration"]
    assert a["K_trace"] + b["K_trace"] == full["K_trace"]
    assert a["logpost_trace"] + b["logpost_trace"] == full["logpost_trace"]
    assert b["labels"] == full["labels"] and b["weights"] == full["weights"]
    assert max(full["K_trace"]) > 1


def test_checkpoint_rejects_another_configuration(tmp_path):
    from paper_2204_08988_amd import fit
    from paper_2204_08988_amd._lib import DpmmError
    x, _ = _data()
    fit.fit(x, {"iterations": 3, "seed": 1}, checkpoint_path=tmp_path / "c.ckpt")
    with pytest.raises(DpmmError):
        fit.fit(x, {"iterations": 3, "seed": 2}, resume_path=tmp_path / "c.ckpt")
    with pytest.raises(DpmmError):
        fit.fit(x[:500], {"iterations": 3, "seed": 1}, resume_path=tmp_path / "c.ckpt")


def test_cli_matches_python_fit(tmp_path):
    from paper_2204_08988_amd import _lib, fit
    x, lab = _data()
    cfg = {"alpha": 10.0, "iterations": 60, "burn_out": 5, "seed": 3}
    res = fit.fit(x, cfg, gt=lab)
    np.save(tmp_path / "x.npy", x)
    np.save(tmp_path / "gt.npy", lab)
    (tmp_path / "p.json").write_text(json.dumps(cfg))
    cli = os.path.join(os.path.dirname(_lib.__file__), "dpmm_fit")
    r = subprocess.run([cli, f"--model_path={tmp_path / 'x.npy'}", f"--params_path={tmp_path / 'p.json'}",
                        f"--gt_path={tmp_path / 'gt.npy'}", f"--result_path={tmp_path / 'r.json'}",
                        f"--checkpoint_path={tmp_path / 'c.ckpt'}"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = json.loads((tmp_path / "r.json").read_text())
    assert got["labels"] == res["labels"] and got["K"] == res["K"]
    assert got["K_trace"] == res["K_trace"]
    assert np.isclose(got["nmi"], res["nmi"], rtol=1e-12)
    # the CLI's checkpoint resumes in Python
    cont = fit.fit(x, dict(cfg, iterations=10), resume_path=tmp_path / "c.ckpt")
    ref = fit.fit(x, dict(cfg, iterations=70))
    assert cont["labels"] == ref["labels"]
