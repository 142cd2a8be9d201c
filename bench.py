"""Throughput of the DPMM sub-cluster sampler hot path on one MI355X.

A step is one full sampler iteration through the C ABI (dpmm_step: FP64
parameter draws, the label/sub-label kernel, the statistics kernel, split /
merge bookkeeping and relabelling) over the whole data set, resident in HBM.

Workload: the Gaussian precision-form configuration, N = 1e6 points, d = 32,
20 true clusters (means N(0, 25 I), covariances Wishart(d + 2, I/d), weights
Dirichlet(1)).  `value` is the BF16 matrix-core form by default; the FP32 and
bf16x3 forms are timed beside it.  Before the warm-up each chain is run until
its cluster count has settled, so the timed steps score the converged K.

Prints one JSON line: metric (point-cluster evaluations per second: N (K + 2)
scores per step), iterations per second, the label kernel's roofline figures
from HIP events recorded on the sampler's stream, and the FP64 oracle's rate
on a bounded sample on the host cores (rank 0, one GPU only).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "gauss_d32"
SEED = 1
ALPHA = 10.0
PEAK_FP32_VALU = 78.6e12   # 256 CU x 64 FMA lanes x 2 flop x 2.4 GHz (non-packed FP32)
PEAK_BF16_MFMA = 2.5e15    # dense BF16 matrix-core peak
PEAK_FP32_MFMA = 157.3e12  # dense FP32 matrix-core peak
PEAK_FP64_MFMA = 78.6e12   # dense FP64 matrix-core peak
# HBM bytes per step of the cluster-draw kernel and of the sub-label +
# statistics kernels at this workload, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# scaled by a device copy of known size (profiles/traffic_gauss_d32_n1e6.md);
# None once a kernel changes
MEASURED_TRAFFIC = {"k_label_gauss_mfma32<false,false>": 133.3e6,
                    "k_sub_labels_mfma<32>+k_sub_stats_w<32,false>": 304.7e6}


def flops_per_eval(d):
    # centring (d), triangular whitening d(d+1)/2 FMAs, squared norm d FMAs
    return d * (d + 1) + 2 * d


def cpu_baseline(x, z, zs, K, d, budget_s=12.0):
    """Time the FP64 oracle's full iteration on a bounded sample of the data."""
    from oracle import niw, sampler
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    n_s = 50_000
    xs = x[:n_s].astype(np.float64)
    model = sampler.Model("gaussian", ALPHA, niw.NIWPrior(1.0, x.mean(0).astype(np.float64), d + 3.0, np.eye(d)),
                          seed=SEED, burn_out=5)
    zz = z[:n_s].astype(np.int64)
    zzs = zs[:n_s].astype(np.int64)
    used = np.unique(zz)
    remap = np.full(K, -1)
    remap[used] = np.arange(used.size)
    state = sampler.State(int(used.size), remap[zz], zzs, np.full(used.size, 100, dtype=np.int64))
    evals = 0
    t0 = time.perf_counter()
    t = 10_000
    while True:
        k_now = state.K
        state, info = sampler.step(model, xs, state, t)
        evals += n_s * (k_now + 2)
        t += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": evals / el, "unit": "point-cluster evals/s", "cores": int(cores), "kind": "oracle",
            "sample": f"full FP64 oracle iterations on the first {n_s} points of the workload "
                      f"({t - 10_000} iterations, {el:.1f} s)"}


def run_form(torch, x, n, d, m, precision, steps, warmup, k_true):
    """Converge the chain, then time `steps` full iterations of one precision form."""
    from paper_2204_08988_amd.sampler import Sampler
    S = Sampler("gaussian", d, 128, ALPHA, SEED, kappa=1.0, nu=d + 3.0, m=m, psi=np.eye(d), burn_out=5,
                precision=precision)
    z, zs = S.init_labels(n)
    t = 1
    ks = []
    for _ in range(400):
        info = S.step(x, t, z, zs)
        t += 1
        ks.append(info["K"])
        if len(ks) > 30 and len(set(ks[-15:])) == 1 and info["K"] >= k_true // 2:
            break
    for _ in range(warmup):
        S.step(x, t, z, zs)
        t += 1
    torch.cuda.synchronize()
    evals = 0
    ms = {"params": 0.0, "labels": 0.0, "sort": 0.0, "stats": 0.0, "splitmerge": 0.0}
    kernel_ms = 0.0
    k_sum = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        info = S.step(x, t, z, zs)
        t += 1
        evals += n * (info["K"] + 2)
        k_sum += info["K"]
        for key in ms:
            ms[key] += info["ms_" + key]
        kernel_ms += info["ms_label_kernel"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_mean = k_sum / steps
    res = {
        "precision": precision,
        "value": evals / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "iters_per_s": steps / elapsed,
        "k_mean": k_mean,
        "phase_ms": {key: v / steps for key, v in ms.items()},
        "label_kernel_ms": kernel_ms / steps,
        "stats_kernel_ms": ms["stats"] / steps,
        "label_evals_per_s": n * k_mean / (ms["labels"] / steps / 1e3),
    }
    return S, z, zs, res


AB_WORKLOAD = "gauss_d64"


def label_step(args):
    """Label-step throughput at a workload's true mixture: the statistics come
    from the generating labels, nothing splits or merges (burn_out beyond the
    run), and each timed iteration redraws the parameters and the labels."""
    import torch
    from paper_2204_08988_amd import datagen
    from paper_2204_08988_amd.sampler import Sampler
    name = args.label_step
    spec = datagen.WORKLOADS[name]
    gauss = isinstance(spec, datagen.GaussianSpec)
    n = int(float(args.n)) if args.n else None
    x_np, labels = datagen.workload(name, 5, n)
    n, d = x_np.shape
    K = int(labels.max()) + 1
    x = torch.from_numpy(x_np).cuda()
    del x_np
    prec = args.precision if gauss and d in (32, 64, 128) else "fp32"  # matrix-core forms: d = 32, 64, 128
    if gauss:
        S = Sampler("gaussian", d, max(2 * K, 16), ALPHA, SEED, kappa=1.0, nu=d + 3.0, m=np.zeros(d), psi=np.eye(d),
                    burn_out=10 ** 9, precision=prec)
    else:
        S = Sampler("multinomial", d, max(2 * K, 16), ALPHA, SEED, beta=np.ones(d), burn_out=10 ** 9)
    z = torch.from_numpy(labels.astype(np.int32)).cuda()
    zs = torch.from_numpy((np.arange(n) % 2).astype(np.uint8)).cuda()
    S.set_state(K, [0] * K)
    S.suffstats(x, z, zs)
    ms = {"params": 0.0, "labels": 0.0, "sort": 0.0, "stats": 0.0, "splitmerge": 0.0}
    kernel_ms = 0.0
    for t in range(1, args.warmup + 1):
        S.step(x, t, z, zs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.warmup + 1, args.warmup + args.steps + 1):
        info = S.step(x, t, z, zs)
        for key in ms:
            ms[key] += info["ms_" + key]
        kernel_ms += info["ms_label_kernel"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = {k: v / args.steps for k, v in ms.items()}
    kernel_ms /= args.steps
    lab_s = ms["labels"] / 1e3
    evals = n * K / lab_s  # the whole cluster-draw phase
    # the roofline of the main cluster-draw kernel alone (events around its launch)
    ker_s = kernel_ms / 1e3
    fpe = flops_per_eval(d) if gauss else 2 * d  # multinomial: sum_v x_v log theta_kv
    flops = n * K * fpe / ker_s
    fused = d <= 4 or not gauss  # these label kernels also draw the sub-labels
    bpp = 4 * d + 4 + (1 if fused else 0)  # x read, z (and zsub) written
    hbm = bpp * n / ker_s
    if prec == "fp32":
        roof = {"bound": "alu", "achieved": flops / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                "frac": flops / PEAK_FP32_VALU}
    else:
        roof = {"bound": "mfma", "achieved": flops / 1e12, "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
                "frac": flops / PEAK_BF16_MFMA}
    roof.update({"kernel_ms": kernel_ms, "hbm_achieved_GBs": hbm / 1e9, "hbm_frac": hbm / 8e12,
                 "algorithmic_flops_per_eval": fpe, "hbm_bytes_per_point": bpp})
    out = {"metric": "point-cluster evals/s in label step", "value": evals, "unit": "point-cluster evals/s",
           "higher_is_better": True, "dtype": prec if gauss else "fp32 (int32 counts)",
           "data": "synthetic",
           "config": {"workload": f"{name}: N={n}, d={d}, {spec.k} true clusters at the generating mixture "
                                  "(statistics from the true labels, no split or merge)", "n": n, "d": d, "K": K},
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "phase_ms": ms,
           "label_kernel": roof}
    print(json.dumps(out), flush=True)


def run_chain(torch, x, n, d, m, iters, learned, train_every, train_until, train_steps, batch, lr, seed=SEED):
    """One chain from K = 1 with the BF16 form: per iteration (t, seconds since
    the start, K, log posterior).  The learned chain trains every `train_every`
    iterations up to iteration `train_until` (the growth phase, while clusters
    still hold several components and their sub-labels carry a signal); its
    training time is inside the clock."""
    from paper_2204_08988_amd.sampler import Sampler
    S = Sampler("gaussian", d, 512, ALPHA, seed, kappa=1.0, nu=d + 3.0, m=m, psi=np.eye(d), burn_out=5,
                precision="bf16", learned=learned)
    z, zs = S.init_labels(n)
    torch.cuda.synchronize()
    rec, tries, acc, t_train = [], 0, 0, 0.0
    t0 = time.perf_counter()
    for t in range(1, iters + 1):
        info = S.step(x, t, z, zs)
        if learned:
            tries += 1
            acc += info["learned_accepted"]
            if t % train_every == 0 and t <= train_until:
                a = time.perf_counter()
                S.mlp_train(x, z, zs, train_steps, batch, lr)
                t_train += time.perf_counter() - a
        rec.append((t, time.perf_counter() - t0, info["K"], info["logpost"]))
    return S, z, rec, {"learned_moves": tries, "learned_accepted": acc, "train_s": t_train}


def ab_one(args, torch, x, n, d, m, labels, seed):
    """Both chains under one seed; the plateau is that seed's plain chain's."""
    from oracle import nmi as nmi_mod
    chains = {}
    for form, learned in (("plain", 0), ("learned", args.ab_axes)):
        S, z, rec, extra = run_chain(torch, x, n, d, m, args.ab_iters, learned, args.ab_train_every,
                                     args.ab_train_until, args.ab_train_steps, args.ab_batch, args.ab_lr, seed)
        chains[form] = (rec, extra, nmi_mod.nmi(labels, z.cpu().numpy()), S.K)
        S.close()
    # the plateau: mean log posterior of the plain chain's last quarter; a chain
    # has reached it once within max(3 standard deviations of that tail, 1e-5 of
    # the level) -- converged chains can settle in modes a few hundred nats
    # apart (one cluster more or less), far below 1e-5 of the level
    tail = np.array([r[3] for r in chains["plain"][0][-max(1, args.ab_iters // 4):]])
    level = float(tail.mean())
    tol = max(3.0 * float(tail.std()), 1e-5 * abs(level))
    out = {"seed": seed, "plateau_logpost": level, "plateau_tol": tol}
    for form, (rec, extra, nmi, K) in chains.items():
        hit = next((r for r in rec if r[3] >= level - tol), None)
        out[form] = {"time_to_plateau_s": None if hit is None else hit[1],
                     "iters_to_plateau": None if hit is None else hit[0],
                     "total_s": rec[-1][1], "final_K": K, "final_logpost": rec[-1][3], "nmi": nmi,
                     "trace": [[r[0], round(r[1], 4), r[2], r[3]] for r in rec if r[0] % 5 == 0], **extra}
    p, l = out["plain"], out["learned"]
    out["speedup_wall"] = (p["time_to_plateau_s"] / l["time_to_plateau_s"]
                           if p["time_to_plateau_s"] and l["time_to_plateau_s"] else None)
    out["speedup_iters"] = (p["iters_to_plateau"] / l["iters_to_plateau"]
                            if p["iters_to_plateau"] and l["iters_to_plateau"] else None)
    out["nmi_diff"] = l["nmi"] - p["nmi"]
    return out


def learned_ab(args):
    """Time to the plain chain's log-posterior plateau, learned vs plain, for
    each of --ab-seeds seeds (the chains' trajectories, and so the time to a
    plateau, vary with the seed); the first seed's result is reported at the
    top level, every seed's under `seeds`, with the median wall-clock speed-up."""
    import torch
    from paper_2204_08988_amd import datagen
    spec = datagen.WORKLOADS[AB_WORKLOAD]
    x_np, labels = datagen.workload(AB_WORKLOAD, 3)
    n, d = x_np.shape
    m = x_np.mean(0).astype(np.float64)
    x = torch.from_numpy(x_np).cuda()
    runs = [ab_one(args, torch, x, n, d, m, labels, SEED + i) for i in range(args.ab_seeds)]
    out = {"metric": "time-to-plateau learned vs plain", "unit": "s", "higher_is_better": False,
           "workload": f"{AB_WORKLOAD}: Gaussian DPMM, N={n}, d={d}, {spec.k} true clusters, means N(0,4I), "
                       "covariances Wishart(d+2, I/d), weights Dir(1); start K=1; BF16 cluster scoring",
           "learned_config": {"axes": args.ab_axes, "features": 2 * args.ab_axes, "hidden": [128, 128],
                              "train_every": args.ab_train_every, "train_until": args.ab_train_until,
                              "train_steps": args.ab_train_steps,
                              "batch": args.ab_batch, "lr": args.ab_lr}}
    out.update({k: v for k, v in runs[0].items() if k != "seed"})
    sp = [r["speedup_wall"] for r in runs if r["speedup_wall"] is not None]
    out["seeds"] = [{k: v for k, v in r.items() if k not in ("plain", "learned")} |
                    {f: {k: r[f][k] for k in ("time_to_plateau_s", "iters_to_plateau", "final_K", "final_logpost",
                                                "nmi", "learned_accepted", "train_s")} for f in ("plain", "learned")}
                    for r in runs]
    out["median_speedup_wall"] = float(np.median(sp)) if sp else None
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "bf16x3"],
                    help="form reported as `value` (the other forms are reported beside it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", action="store_true", help="time only the --precision form")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy a device buffer of BYTES five times (calibrates HBM byte counters)")
    ap.add_argument("--label-step", metavar="WORKLOAD",
                    help="instead of the throughput line: label-step throughput at WORKLOAD's true mixture")
    ap.add_argument("--n", default=None, help="points for --label-step (default: the workload's N)")
    ap.add_argument("--learned-ab", action="store_true",
                    help="instead of the throughput line: time to the plain chain's log-posterior plateau, "
                         "learned proposal vs plain, on the learned-proposal workload")
    ap.add_argument("--ab-iters", type=int, default=200)
    ap.add_argument("--ab-seeds", type=int, default=1, help="seeds of the learned-vs-plain comparison")
    ap.add_argument("--ab-axes", type=int, default=8)
    ap.add_argument("--ab-train-every", type=int, default=10)
    ap.add_argument("--ab-train-until", type=int, default=60)
    ap.add_argument("--ab-train-steps", type=int, default=20)
    ap.add_argument("--ab-batch", type=int, default=4096)
    ap.add_argument("--ab-lr", type=float, default=1e-3)
    args = ap.parse_args()
    if args.gpus == 1 and args.learned_ab:
        learned_ab(args)
        return
    if args.gpus == 1 and args.label_step:
        label_step(args)
        return
    if args.copy_probe:
        import torch
        a = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_08988_amd import datagen
    from oracle import nmi as nmi_mod

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    spec = datagen.WORKLOADS[WORKLOAD]
    x_np, labels = datagen.workload(WORKLOAD, SEED)
    n, d = x_np.shape
    m = x_np.mean(0).astype(np.float64)
    x = torch.from_numpy(x_np).cuda()
    forms = [args.precision] if args.only else [args.precision] + [f for f in ("fp32", "bf16", "bf16x3")
                                                                     if f != args.precision]
    results = {}
    main_state = None
    for f in forms:
        S, z, zs, res = run_form(torch, x, n, d, m, f, args.steps, args.warmup, spec.k)
        res["nmi"] = nmi_mod.nmi(labels, z.cpu().numpy())
        results[f] = res
        if f == args.precision:
            main_state = (z.cpu().numpy(), zs.cpu().numpy(), S.K)
        S.close()
    r = results[args.precision]
    label_s = r["label_kernel_ms"] / 1e3
    stats_s = r["stats_kernel_ms"] / 1e3
    algo_label = n * r["k_mean"] * flops_per_eval(d)  # the cluster draw scores K clusters per point
    if args.precision == "fp32":
        label_roof = {"bound": "alu", "achieved": algo_label / label_s / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                      "unit": "TFLOP/s", "frac": algo_label / label_s / PEAK_FP32_VALU,
                      "kernel": "k_label_gauss_z<32> (FP32 VALU cluster draw)"}
    else:
        label_roof = {"bound": "mfma", "achieved": algo_label / label_s / 1e12, "peak": PEAK_BF16_MFMA / 1e12,
                      "unit": "TFLOP/s", "frac": algo_label / label_s / PEAK_BF16_MFMA,
                      "kernel": f"k_label_gauss_mfma32<{'true' if args.precision == 'bf16x3' else 'false'}> "
                                "(BF16 matrix-core cluster draw)"}
    label_roof["algorithmic_flops_per_eval"] = flops_per_eval(d)
    # sub-label draw + statistics over the cluster-sorted order, a phase of
    # three kernels: the two FP32 sub-cluster scores on the FP32 matrix cores
    # (k_sub_labels_mfma), then the FP64 moments (sum x, upper triangle of
    # x x^T) on the FP64 matrix cores (k_sub_stats_w, k_sub_stats_fix).  The
    # kernels run one after the other, so the phase takes at least the sum of
    # the two parts' times at their units' peaks; "peak" is the phase's flops
    # over that time.
    score_flops, moment_flops = 2 * flops_per_eval(d), d + d * (d + 1)
    stats_flops = score_flops + moment_flops
    t_min = n * (score_flops / PEAK_FP32_MFMA + moment_flops / PEAK_FP64_MFMA)
    stats_roof = {"bound": "mfma", "achieved": n * stats_flops / stats_s / 1e12,
                  "peak": n * stats_flops / t_min / 1e12, "unit": "TFLOP/s", "frac": t_min / stats_s,
                  "kernel": "sub-label + statistics phase: k_sub_labels_mfma<32>, k_sub_stats_w<32,false>, "
                            "k_sub_stats_fix",
                  "algorithmic_flops_per_point": stats_flops,
                  "hbm_bytes_per_point": 2 * (4 * d + 4 + 4 + 1)}
    stats_roof["traffic"] = MEASURED_TRAFFIC.get("k_sub_labels_mfma<32>+k_sub_stats_w<32,false>")
    label_roof["traffic"] = (MEASURED_TRAFFIC.get("k_label_gauss_mfma32<false,false>")
                             if args.precision == "bf16" else None)
    # the dominant single kernel is the cluster draw (the statistics phase is
    # split over three kernels, the largest of them shorter than the draw),
    # timed alone by events right around its launch on the sampler's stream
    label_roof["kernel_ms"] = r["label_kernel_ms"]
    roof, other = label_roof, stats_roof
    out = {
        "metric": "point-cluster evals/s in label step; iters/s; time-to-plateau learned vs plain",
        "value": r["value"],
        "unit": "point-cluster evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: Gaussian DPMM, N={n}, d={d}, {spec.k} true clusters, "
                               "means N(0,25I), covariances Wishart(d+2, I/d), weights Dir(1); "
                               f"cluster scoring {args.precision}, sub-labels FP32, statistics and "
                               "parameters FP64", "n": n, "d": d, "k_mean": r["k_mean"],
                   "alpha": ALPHA, "parallelism": "single GPU"},
        "iters_per_s": r["iters_per_s"],
        "phase_ms": r["phase_ms"],
        "label_kernel_ms": r["label_kernel_ms"],
        "label_evals_per_s": r["label_evals_per_s"],
        "nmi": r["nmi"],
        "forms": {f: {k: v for k, v in res.items() if k != "precision"} for f, res in results.items()
                  if f != args.precision},
        "roofline": roof,
        "roofline_other_kernel": other,
    }
    if not args.no_cpu_baseline:
        z_np, zs_np, K = main_state
        out["cpu_baseline"] = cpu_baseline(x_np, z_np, zs_np, K, d)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
