"""User-level fit (the paper's interface, Sec. 3.4): a JSON configuration in,
a JSON-ready result out (labels, weights, NMI against ground truth when
given, time per iteration), and checkpoint files to save and resume a run.

Argument marshalling over the C ABI only: the run is dpmm_fit, the final
parameter draw dpmm_sample_params, the NMI dpmm_nmi, the checkpoints
dpmm_save_checkpoint / dpmm_load_checkpoint.

Configuration keys (JSON object; every key optional except as noted):
  prior_type     "Gaussian" (default), "Multinomial" or "Poisson"
  alpha          DP concentration (default 10)
  iterations     iterations to run (default 100)
  burn_out       iterations a new cluster waits before it may split or merge (default 15)
  seed           Philox key (default 1)
  k_max          capacity in clusters (default 512)
  precision      "fp32" (default), "bf16", "bf16x3" (Gaussian d = 32, 64, 128)
  merge_form     "paper" (default) or "inverse_split"
  hyper_params   Gaussian: {"kappa": 1, "m": data mean, "nu": d + 3, "psi": identity};
                 Multinomial: {"alpha": [1, ...]} (the Dirichlet prior, length V);
                 Poisson: {"shape": [1, ...], "rate": [1, ...]} (the Gamma prior, length d)
  learned        principal axes of the learned split proposal (0 = off); with
                 train_every, train_until, train_steps, train_batch, train_lr
"""
import json
import os

import numpy as np

from . import _lib
from .sampler import Sampler

DEFAULTS = {"prior_type": "Gaussian", "alpha": 10.0, "iterations": 100, "burn_out": 15, "seed": 1, "k_max": 512,
            "precision": "fp32", "merge_form": "paper", "learned": 0, "train_every": 10, "train_until": 60,
            "train_steps": 20, "train_batch": 4096, "train_lr": 1e-3}


def load_config(config):
    """A configuration dict from a dict or the path of a JSON file, defaults filled in."""
    if isinstance(config, (str, os.PathLike)):
        with open(config) as f:
            config = json.load(f)
    cfg = dict(DEFAULTS)
    cfg.update(config or {})
    unknown = set(cfg) - set(DEFAULTS) - {"hyper_params"}
    if unknown:
        raise ValueError(f"unknown configuration keys: {sorted(unknown)}")
    if cfg["prior_type"] not in ("Gaussian", "Multinomial", "Poisson"):
        raise ValueError("prior_type must be Gaussian, Multinomial or Poisson")
    return cfg


def make_sampler(cfg, x):
    """The sampler context of a configuration for data x (numpy, N x d)."""
    d = x.shape[1]
    hp = dict(cfg.get("hyper_params") or {})
    if cfg["prior_type"] == "Gaussian":
        m = np.asarray(hp.get("m", np.asarray(x, dtype=np.float64).mean(0)), dtype=np.float64)
        psi = np.asarray(hp.get("psi", np.eye(d)), dtype=np.float64)
        return Sampler("gaussian", d, cfg["k_max"], cfg["alpha"], cfg["seed"], kappa=float(hp.get("kappa", 1.0)),
                       nu=float(hp.get("nu", d + 3.0)), m=m, psi=psi, burn_out=cfg["burn_out"],
                       merge_form=cfg["merge_form"], precision=cfg["precision"], learned=cfg["learned"])
    if cfg["prior_type"] == "Poisson":
        return Sampler("poisson", d, cfg["k_max"], cfg["alpha"], cfg["seed"],
                       gamma_shape=np.asarray(hp.get("shape", np.ones(d)), dtype=np.float64),
                       gamma_rate=np.asarray(hp.get("rate", np.ones(d)), dtype=np.float64), burn_out=cfg["burn_out"],
                       merge_form=cfg["merge_form"])
    beta = np.asarray(hp.get("alpha", np.ones(d)), dtype=np.float64)
    return Sampler("multinomial", d, cfg["k_max"], cfg["alpha"], cfg["seed"], beta=beta, burn_out=cfg["burn_out"],
                   merge_form=cfg["merge_form"])


def fit(x, config=None, gt=None, result_path=None, checkpoint_path=None, resume_path=None):
    """Fit a DPMM to x (numpy N x d float32 for Gaussian, N x V int32 counts
    for Multinomial and Poisson) on the current GPU.  resume_path: continue from a
    checkpoint (the configuration and data must match the run that wrote
    it); checkpoint_path: save the final state there.  Returns the result
    dict (also written as JSON to result_path when given)."""
    import torch
    cfg = load_config(config)
    gauss = cfg["prior_type"] == "Gaussian"
    x = np.ascontiguousarray(x, dtype=np.float32 if gauss else np.int32)
    S = make_sampler(cfg, x)
    try:
        xt = torch.from_numpy(x).cuda()
        n = x.shape[0]
        if resume_path:
            z = torch.empty(n, dtype=torch.int32, device="cuda")
            zs = torch.empty(n, dtype=torch.uint8, device="cuda")
            t_done = S.load_checkpoint(resume_path, z, zs)
        else:
            z, zs = S.init_labels(n)
            t_done = 0
        trace, secs = S.fit(xt, t_done + 1, cfg["iterations"], z, zs,
                            train_every=cfg["train_every"] if cfg["learned"] else 0,
                            train_until=cfg["train_until"], train_steps=cfg["train_steps"],
                            train_batch=cfg["train_batch"], train_lr=cfg["train_lr"])
        t_last = t_done + cfg["iterations"]
        if checkpoint_path:
            S.save_checkpoint(checkpoint_path, t_last, z, zs)
        # the parameters of the final clusters: the draw the next iteration would make
        S.sample_params(t_last + 1)
        log_pi, log_pisub, comp = S.get_params()
        labels = z.cpu().numpy()
        res = {"labels": labels.tolist(), "K": S.K, "weights": np.exp(log_pi).tolist(),
               "iter_time": [float(s) for s in secs], "K_trace": [r["K"] for r in trace],
               "logpost_trace": [r["logpost"] for r in trace], "splits": [r["splits"] for r in trace],
               "merges": [r["merges"] for r in trace], "last_iteration": t_last,
               "config": {k: v for k, v in cfg.items() if k != "hyper_params"}}
        if gauss:
            d = x.shape[1]
            res["means"] = comp[:, 0, :d].tolist()
            res["covariances"] = comp[:, 0, d:].reshape(-1, d, d).tolist()
        else:
            res["log_theta"] = comp[:, 0, :].tolist()
        if gt is not None:
            res["nmi"] = _lib.nmi(np.asarray(gt), labels)
        if result_path:
            with open(result_path, "w") as f:
                json.dump(res, f)
        return res
    finally:
        S.close()
