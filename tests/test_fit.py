"""CPU tests of the user-level interface: the host NMI of the library
(dpmm_nmi) against the oracle's and scikit-learn's, the configuration
defaults and checks of fit.load_config, and the command-line tool's
configuration and .npy parsing (--check_config touches no device)."""
import json
import os
import subprocess

import numpy as np
import pytest

from oracle import nmi as oracle_nmi
from paper_2204_08988_amd import _lib, fit

CLI = os.path.join(os.path.dirname(_lib.__file__), "dpmm_fit")


@pytest.mark.parametrize("n,ka,kb", [(1000, 5, 7), (50_000, 40, 3), (7, 1, 1), (300, 1, 4), (1, 1, 1)])
def test_library_nmi_matches_oracle_and_sklearn(n, ka, kb):
    g = np.random.Generator(np.random.PCG64(n + ka))
    a = g.integers(0, ka, n) * 3 - 5          # arbitrary label values
    b = np.where(g.random(n) < 0.6, a, g.integers(0, kb, n))
    assert np.isclose(_lib.nmi(a, b), oracle_nmi.nmi(a, b), rtol=1e-12, atol=1e-15)
    skm = pytest.importorskip("sklearn.metrics")
    if len(np.unique(a)) > 1 or len(np.unique(b)) > 1:
        assert np.isclose(_lib.nmi(a, b), skm.normalized_mutual_info_score(a, b), rtol=1e-10, atol=1e-12)


def test_nmi_of_a_permuted_labelling_is_one():
    a = np.repeat(np.arange(6), 50)
    assert np.isclose(_lib.nmi(a, (a * 7 + 3) % 11), 1.0)


def test_load_config_defaults_and_checks(tmp_path):
    cfg = fit.load_config({"alpha": 3.0})
    assert cfg["alpha"] == 3.0 and cfg["iterations"] == 100 and cfg["prior_type"] == "Gaussian"
    p = tmp_path / "c.json"
    p.write_text(json.dumps({"prior_type": "Multinomial", "iterations": 7}))
    cfg = fit.load_config(str(p))
    assert cfg["prior_type"] == "Multinomial" and cfg["iterations"] == 7
    with pytest.raises(ValueError):
        fit.load_config({"alhpa": 1.0})
    with pytest.raises(ValueError):
        fit.load_config({"prior_type": "Poisson2"})


def _cli(*args):
    return subprocess.run([CLI, *args], capture_output=True, text=True)


def test_cli_check_config(tmp_path):
    x = np.zeros((123, 5), dtype=np.float32)
    np.save(tmp_path / "x.npy", x)
    (tmp_path / "p.json").write_text(json.dumps({"alpha": 2.5, "iterations": 9, "seed": 77, "burn_out": 3,
                                                 "hyper_params": {"kappa": 2.0, "m": [0, 0, 0, 0, 0]}}))
    r = _cli(f"--model_path={tmp_path / 'x.npy'}", f"--params_path={tmp_path / 'p.json'}", "--check_config")
    assert r.returncode == 0, r.stderr
    got = json.loads(r.stdout)
    assert got["alpha"] == 2.5 and got["iterations"] == 9 and got["seed"] == 77 and got["burn_out"] == 3
    assert got["n"] == 123 and got["d"] == 5 and got["prior_type"] == "Gaussian"
    r = _cli(f"--model_path={tmp_path / 'x.npy'}", "--prior_type=Multinomial", "--check_config")
    assert r.returncode == 0 and json.loads(r.stdout)["prior_type"] == "Multinomial"


@pytest.mark.parametrize("bad", ['{"alhpa": 1}', '{"alpha": "x"}', '{"alpha": 1,}', '[1, 2]',
                                 '{"prior_type": "Poisson2"}'])
def test_cli_rejects_bad_configuration(tmp_path, bad):
    np.save(tmp_path / "x.npy", np.zeros((4, 2), dtype=np.float32))
    (tmp_path / "p.json").write_text(bad)
    r = _cli(f"--model_path={tmp_path / 'x.npy'}", f"--params_path={tmp_path / 'p.json'}", "--check_config")
    assert r.returncode == 1 and "dpmm_fit:" in r.stderr


def test_cli_requires_data(tmp_path):
    r = _cli("--check_config")
    assert r.returncode == 1 and "model_path" in r.stderr
    (tmp_path / "x.npy").write_bytes(b"not an array")
    r = _cli(f"--model_path={tmp_path / 'x.npy'}", "--check_config")
    assert r.returncode == 1 and "npy" in r.stderr
