"""Throughput of the DPMM sub-cluster sampler hot path on one MI355X.

A step is one full sampler iteration through the C ABI (dpmm_step: FP64
parameter draws, the cluster draw, the sort by cluster, the sub-label draw and
the statistics, split / merge bookkeeping and relabelling) over the whole data
set, resident in HBM before the clock starts.

Headline workload: the largest configuration, gauss_d128 -- N = 1e7 points,
d = 128, 100 true clusters (means N(0, 9 I), covariances Wishart(d + 2, I/d),
weights Dirichlet(1)), cluster scoring in BF16 on the matrix cores with the
FP32 guard, sub-labels in bf16x3 with FP32 on the rows it leaves undecided
(the same sub-labels as the FP32 pass), statistics and parameters FP64.  The chain
starts at its converged state (the generating labels, random sub-labels,
every cluster old enough to split or merge); the warm-up steps let the
sub-clusters settle and every timed step is a full iteration.

Prints one JSON line: `value` = point-cluster evaluations per second over the
whole step (N (K + 2) scores per iteration), iterations per second, the
roofline of the dominant kernel (the d = 128 BF16 cluster draw, timed by HIP
events around its own dispatch on the sampler's stream), the other
configurations (gauss_d32, mult_v100, the d = 2 label step at N = 1e8, the
d = 2 chain at N = 1e4, the sparse-row multinomial of the 20newsgroups shape:
its chain at N = 11 314 and its label step at N = 2e5) as extra keys, and the FP64 oracle's label step on a
bounded sample on the host cores (all cores and one core).

Other modes: --label-step WORKLOAD (label step at a workload's generating
mixture), --learned-ab (time to the log-posterior plateau, learned proposal
vs plain, over several seeds), --width-compare (the K-wide cluster draw
against the 3K-wide whitening form at the headline shape).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SEED = 1
ALPHA = 10.0
PEAK_HBM = 8.0e12          # bytes/s
PEAK_FP32_VALU = 78.6e12   # 256 CU x 64 FMA lanes x 2 flop x 2.4 GHz (non-packed FP32)
PEAK_BF16_MFMA = 2.5e15    # dense BF16 matrix-core peak
PEAK_FP32_MFMA = 157.3e12  # dense FP32 matrix-core peak
PEAK_FP64_MFMA = 78.6e12   # dense FP64 matrix-core peak
HEADLINE = "gauss_d128"
HEADLINE_KERNEL = "k_label_gauss_mfma_uc<128, 512, 8>"
# HBM bytes per launch of the headline kernel at the headline workload (N = 1e7,
# d = 128, K = 100) from rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB), the
# factors being what a 1 GiB device copy reads on the same counters (FETCH_SIZE
# 0.5 GiB, WRITE_SIZE 1 GiB); empty whenever the kernel changes until the
# counters are taken again
MEASURED_TRAFFIC = {HEADLINE_KERNEL: (2.5282e6 * 2.0 + 7.5822e4) * 1024}


def flops_per_eval(d):
    # centring (d), triangular whitening d(d+1)/2 FMAs, squared norm d FMAs
    return d * (d + 1) + 2 * d


def _sampler(family, d, k_max, m, precision="fp32", burn_out=5, learned=0, seed=SEED):
    from paper_2204_08988_amd.sampler import Sampler
    if family == "gaussian":
        return Sampler("gaussian", d, k_max, ALPHA, seed, kappa=1.0, nu=d + 3.0, m=m, psi=np.eye(d),
                       burn_out=burn_out, precision=precision, learned=learned)
    return Sampler("multinomial", d, k_max, ALPHA, seed, beta=np.ones(d), burn_out=burn_out)


def converged_chain(torch, name, n, precision, steps, warmup, seed=SEED):
    """Full iterations from the converged state of a workload: labels = the
    generating labels, sub-labels random, ages at burn_out.  Returns the
    timing record and the final labels."""
    from paper_2204_08988_amd import datagen
    spec = datagen.WORKLOADS[name]
    gauss = isinstance(spec, datagen.GaussianSpec)
    x_np, labels = datagen.workload(name, seed, n)
    n, d = x_np.shape
    labels = np.unique(labels, return_inverse=True)[1]  # the occupied clusters, renumbered
    K = int(labels.max()) + 1
    m = x_np.mean(0).astype(np.float64) if gauss else None
    x = torch.from_numpy(x_np).cuda()
    del x_np
    burn = 5
    S = _sampler("gaussian" if gauss else "multinomial", d, 2 * K + 16, m, precision, burn_out=burn, seed=seed)
    z = torch.from_numpy(labels.astype(np.int32)).cuda()
    zs = torch.from_numpy((np.random.Generator(np.random.PCG64(seed + 7)).integers(0, 2, n)).astype(np.uint8)).cuda()
    S.set_state(K, [burn] * K)
    t = 1
    for _ in range(warmup):
        S.step(x, t, z, zs)
        t += 1
    torch.cuda.synchronize()
    ms = {"params": 0.0, "labels": 0.0, "sort": 0.0, "stats": 0.0, "splitmerge": 0.0}
    kernel_ms = 0.0
    evals = 0
    k_sum = 0
    moves = [0, 0]
    t0 = time.perf_counter()
    for _ in range(steps):
        info = S.step(x, t, z, zs)
        t += 1
        evals += n * (info["K"] + 2)
        k_sum += info["K"]
        moves[0] += info["splits"]
        moves[1] += info["merges"]
        for key in ms:
            ms[key] += info["ms_" + key]
        kernel_ms += info["ms_label_kernel"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    from paper_2204_08988_amd import _lib
    rec = {"n": n, "d": d, "k_true": K, "k_mean": k_sum / steps, "value": evals / el, "ms_per_step": 1e3 * el / steps,
           "iters_per_s": steps / el, "phase_ms": {k: v / steps for k, v in ms.items()},
           "label_kernel_ms": kernel_ms / steps,
           "label_evals_per_s": n * (k_sum / steps) / (ms["labels"] / steps / 1e3),
           "splits": moves[0], "merges": moves[1],
           "nmi": _lib.nmi(labels, z.cpu().numpy())}
    S.close()
    del x
    torch.cuda.empty_cache()
    return rec


def mfma_roofline(rec, d, kernel):
    """The BF16 cluster draw: algorithmic flops N K (d(d+1) + 2d) per launch
    over the launch's own duration."""
    flops = rec["n"] * rec["k_mean"] * flops_per_eval(d)
    s = rec["label_kernel_ms"] / 1e3
    return {"bound": "mfma", "achieved": flops / s / 1e12, "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
            "frac": flops / s / PEAK_BF16_MFMA, "traffic": MEASURED_TRAFFIC.get(kernel), "traffic_unit": "bytes per launch",
            "algorithmic_bytes_per_launch": rec["n"] * (4 * d + 4), "kernel": kernel,
            "kernel_ms": rec["label_kernel_ms"], "algorithmic_flops_per_eval": flops_per_eval(d),
            "evals_per_launch": rec["n"] * rec["k_mean"]}


def label_step_run(torch, name, n, precision, steps, warmup, thirds=False):
    """Label-step throughput at a workload's true mixture: the statistics come
    from the generating labels, nothing splits or merges (burn_out beyond the
    run), and each timed iteration redraws the parameters and the labels.
    thirds: every true cluster split into three interleaved clusters (3K
    components scored per point, the work of the 3K-wide whitening form)."""
    from paper_2204_08988_amd import datagen
    spec = datagen.WORKLOADS[name]
    gauss = isinstance(spec, datagen.GaussianSpec)
    x_np, labels = datagen.workload(name, 5, n)
    n, d = x_np.shape
    labels = np.unique(labels, return_inverse=True)[1]  # the occupied clusters, renumbered
    if thirds:
        labels = 3 * labels + np.arange(n) % 3
    K = int(labels.max()) + 1
    x = torch.from_numpy(x_np).cuda()
    del x_np
    prec = precision if gauss and d in (32, 64, 128) else "fp32"
    S = _sampler("gaussian" if gauss else "multinomial", d, max(2 * K, 16), np.zeros(d), prec, burn_out=10 ** 9)
    z = torch.from_numpy(labels.astype(np.int32)).cuda()
    zs = torch.from_numpy((np.arange(n) % 2).astype(np.uint8)).cuda()
    S.set_state(K, [0] * K)
    S.suffstats(x, z, zs)
    ms = {"params": 0.0, "labels": 0.0, "sort": 0.0, "stats": 0.0, "splitmerge": 0.0}
    kernel_ms = 0.0
    for t in range(1, warmup + 1):
        S.step(x, t, z, zs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(warmup + 1, warmup + steps + 1):
        info = S.step(x, t, z, zs)
        for key in ms:
            ms[key] += info["ms_" + key]
        kernel_ms += info["ms_label_kernel"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.close()
    del x
    torch.cuda.empty_cache()
    ms = {k: v / steps for k, v in ms.items()}
    kernel_ms /= steps
    ker_s = kernel_ms / 1e3
    fpe = flops_per_eval(d) if gauss else 2 * d  # multinomial: sum_v x_v log theta_kv
    flops = n * K * fpe / ker_s
    fused = d <= 4 or not gauss  # these label kernels also draw the sub-labels
    bpp = 4 * d + 4 + (1 if fused else 0)  # x read, z (and zsub) written
    hbm = bpp * n / ker_s
    if not gauss:  # on the FP32 matrix cores; HBM-bound at this shape
        roof = {"bound": "hbm", "achieved": hbm / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": hbm / PEAK_HBM,
                "mfma_fp32_frac": flops / PEAK_FP32_MFMA}
    elif d <= 4:
        roof = {"bound": "hbm", "achieved": hbm / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": hbm / PEAK_HBM,
                "valu_fp32_frac": flops / PEAK_FP32_VALU}
    elif prec == "fp32":
        roof = {"bound": "alu", "achieved": flops / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                "frac": flops / PEAK_FP32_VALU}
    else:
        roof = {"bound": "mfma", "achieved": flops / 1e12, "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
                "frac": flops / PEAK_BF16_MFMA}
    roof.update({"kernel_ms": kernel_ms, "hbm_GBs": hbm / 1e9, "algorithmic_flops_per_eval": fpe,
                 "hbm_bytes_per_point": bpp})
    return {"workload": f"{name}: N={n}, d={d}, {K} true clusters at the generating mixture (statistics from the "
                        "true labels, no split or merge)", "n": n, "d": d, "K": K, "dtype": prec,
            "label_evals_per_s": n * K / (ms["labels"] / 1e3), "ms_per_step": 1e3 * el / steps, "phase_ms": ms,
            "label_kernel": roof}


def sparse_run(torch, n, steps, warmup, chain):
    """The sparse-row multinomial on the 20newsgroups-shaped stand-in
    (news_v20k, V = 20 000, 20 topics).  chain=True: full iterations from the
    converged state (generating labels, every cluster old enough to move);
    chain=False: the label step at the generating mixture (statistics from
    the true labels, no split or merge).  The label phase is one kernel
    (k_label_csr); its HBM roofline counts the rows once: row pointers (8 B a
    row), entries (4 B word + 4 B count) and the labels written (5 B a row)."""
    from paper_2204_08988_amd import datagen, _lib
    from paper_2204_08988_amd.sampler import Sampler, SparseCounts
    xh, labels = datagen.workload("news_v20k", SEED, n)
    n, V = xh.shape
    nnz = int(xh.indices.size)
    x = SparseCounts.from_numpy(xh.indptr, xh.indices, xh.data, V)
    del xh
    labels = np.unique(labels, return_inverse=True)[1]
    K = int(labels.max()) + 1
    burn = 5 if chain else 10 ** 9
    S = Sampler("multinomial", V, 2 * K + 16, ALPHA, SEED, beta=np.full(V, 0.1), burn_out=burn, sparse=True)
    z = torch.from_numpy(labels.astype(np.int32)).cuda()
    zs = torch.from_numpy((np.random.Generator(np.random.PCG64(SEED + 7)).integers(0, 2, n)).astype(np.uint8)).cuda()
    S.set_state(K, [burn if chain else 0] * K)
    if not chain:
        S.suffstats(x, z, zs)
    t = 1
    for _ in range(warmup):
        S.step(x, t, z, zs)
        t += 1
    torch.cuda.synchronize()
    ms = {"params": 0.0, "labels": 0.0, "sort": 0.0, "stats": 0.0, "splitmerge": 0.0}
    k_sum = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        info = S.step(x, t, z, zs)
        t += 1
        k_sum += info["K"]
        for key in ms:
            ms[key] += info["ms_" + key]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = {k: v / steps for k, v in ms.items()}
    bytes_launch = 8 * (n + 1) + 8 * nnz + 5 * n
    ker_s = ms["labels"] / 1e3
    rec = {"workload": f"news_v20k: sparse rows (CSR), N={n} documents, V={V}, {K} topics, nnz={nnz}; "
                       + ("converged chain" if chain else "label step at the generating mixture"),
           "n": n, "V": V, "nnz": nnz, "k_true": K, "k_mean": k_sum / steps, "ms_per_step": 1e3 * el / steps,
           "iters_per_s": steps / el, "phase_ms": ms,
           "label_evals_per_s": n * (k_sum / steps) / ker_s,
           "label_kernel": {"bound": "hbm", "kernel": "k_label_csr", "kernel_ms": ms["labels"],
                            "achieved": bytes_launch / ker_s / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                            "frac": bytes_launch / ker_s / PEAK_HBM, "algorithmic_bytes_per_launch": bytes_launch},
           "nmi": _lib.nmi(labels, z.cpu().numpy())}
    S.close()
    del x
    torch.cuda.empty_cache()
    return rec


def chain_from_one(torch, name, n, iters, precision="fp32"):
    """Iterations per second of a chain from K = 1 (every iteration timed)."""
    from paper_2204_08988_amd import datagen, _lib
    x_np, labels = datagen.workload(name, SEED, n)
    n, d = x_np.shape
    S = _sampler("gaussian", d, 64, x_np.mean(0).astype(np.float64), precision, burn_out=5)
    x = torch.from_numpy(x_np).cuda()
    z, zs = S.init_labels(n)
    S.step(x, 1, z, zs)  # first call: lazy buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(2, iters + 2):
        info = S.step(x, t, z, zs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"workload": f"{name}: N={n}, d={d}, chain from K=1", "iters": iters, "iters_per_s": iters / el,
           "final_K": info["K"], "nmi": _lib.nmi(labels, z.cpu().numpy())}
    S.close()
    return out


def cpu_baseline(name, n_sample, budget_s):
    """The FP64 oracle's label step (component log-likelihoods of the K true
    clusters and their 2K sub-clusters, Gumbel-max and logistic draws) on the
    first n_sample points of the workload, with all host cores and with one."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import niw, sampler
    from paper_2204_08988_amd import datagen
    x, labels = datagen.workload(name, SEED, n_sample)
    x = x.astype(np.float64)
    d = x.shape[1]
    used, z = np.unique(labels, return_inverse=True)  # the clusters the sample holds
    K = used.size
    model = sampler.Model("gaussian", ALPHA, niw.NIWPrior(1.0, x.mean(0), d + 3.0, np.eye(d)), seed=SEED)
    zs = (np.arange(x.shape[0]) % 2).astype(np.int64)
    stats = sampler.suffstats(model, x, z.astype(np.int64), zs, K)
    params = sampler.sample_params(model, stats, 1)

    def rate(nrows, limit_s):
        reps, t0 = 0, time.perf_counter()
        while True:
            sampler.sample_labels(model, x[:nrows], params, 2 + reps)
            reps += 1
            if time.perf_counter() - t0 > limit_s:
                break
        el = time.perf_counter() - t0
        return nrows * (K + 2) * reps / el, reps, el

    cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    v_all, r_all, e_all = rate(x.shape[0], 0.6 * budget_s)
    with threadpool_limits(limits=1):
        n1 = max(1000, x.shape[0] // 8)
        v_one, r_one, e_one = rate(n1, 0.4 * budget_s)
    return {"value": v_all, "unit": "point-cluster evals/s", "cores": int(cores), "kind": "oracle",
            "sample": f"FP64 oracle label step (K + 2 = {K + 2} components scored and drawn per point) on the first "
                      f"{x.shape[0]} points of {name}: {r_all} repetitions in {e_all:.1f} s",
            "value_1core": v_one,
            "sample_1core": f"the same on {n1} points with BLAS limited to one thread: {r_one} repetitions in "
                            f"{e_one:.1f} s"}


def headline(args):
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rec = converged_chain(torch, HEADLINE, None, args.precision, args.steps, args.warmup)
    d = rec["d"]
    kernel = HEADLINE_KERNEL if args.precision == "bf16" else f"cluster draw ({args.precision})"
    out = {
        "metric": "point-cluster evals/s in label step; iters/s; time-to-plateau learned vs plain",
        "value": rec["value"],
        "unit": "point-cluster evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{HEADLINE}: Gaussian DPMM, N={rec['n']}, d={d}, {rec['k_true']} true clusters, "
                               "means N(0,9I), covariances Wishart(d+2, I/d), weights Dir(1); converged state "
                               f"(generating labels); cluster scoring {args.precision} with the FP32 guard, "
                               "sub-labels bf16x3 with the FP32 guard, statistics and parameters FP64",
                   "n": rec["n"], "d": d, "k_mean": rec["k_mean"], "alpha": ALPHA, "parallelism": "single GPU"},
        "iters_per_s": rec["iters_per_s"],
        "phase_ms": rec["phase_ms"],
        "label_kernel_ms": rec["label_kernel_ms"],
        "label_evals_per_s": rec["label_evals_per_s"],
        "nmi": rec["nmi"],
        "roofline": mfma_roofline(rec, d, kernel),
    }
    if not args.headline_only:
        extra = {}
        r2 = converged_chain(torch, "gauss_d32", None, "bf16", max(args.steps, 20), args.warmup)
        r2["roofline"] = mfma_roofline(r2, 32, "k_label_gauss_mfma32<false,false>")
        extra["gauss_d32"] = r2
        extra["mult_v100"] = label_step_run(torch, "mult_v100", None, "fp32", 20, 3)
        extra["mult_v100_chain"] = converged_chain(torch, "mult_v100", None, "fp32", 20, 3)
        extra["gauss_d2_label_step_n1e8"] = label_step_run(torch, "gauss_d2", 100_000_000, "fp32", 10, 3)
        extra["gauss_d2_chain_n1e4"] = chain_from_one(torch, "gauss_d2", None, 100)
        extra["news_v20k_chain"] = sparse_run(torch, None, 50, 5, True)
        extra["news_v20k_label_step_n2e5"] = sparse_run(torch, 200_000, 20, 3, False)
        out["configs"] = extra
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(HEADLINE, 20_000, 24.0)
    print(json.dumps(out), flush=True)


def width_compare(args):
    """The K-wide cluster draw (this build: K cluster components per point, the
    sub-clusters in their own pass over the sorted rows) against the 3K-wide
    form (every cluster and sub-cluster scored for every point), timed as the
    same main-pass kernel over K and over 3K components at the headline shape."""
    import torch
    n = int(float(args.n)) if args.n else None
    kw = label_step_run(torch, HEADLINE, n, "bf16", args.steps, args.warmup)
    w3 = label_step_run(torch, HEADLINE, n, "bf16", args.steps, args.warmup, thirds=True)
    d, N, K = kw["d"], kw["n"], kw["K"]
    exe = 1.25 * d * d  # executed MFMA flops per point-component (zero tiles above the diagonal skipped)
    alg = N * (K + 2) * flops_per_eval(d)
    rec = {"metric": "whitening form: K-wide + sub-cluster pass vs 3K-wide", "workload": kw["workload"],
           "algorithmic_flops_per_step": alg,
           "k_wide": {"components": K, "cluster_draw_ms": kw["label_kernel"]["kernel_ms"],
                      "executed_flops_cluster_draw": N * K * exe,
                      "executed_flops_sub_labels_bf16x3": N * 2 * 3 * exe},
           "three_k_wide": {"components": 3 * K, "cluster_draw_ms": w3["label_kernel"]["kernel_ms"],
                            "executed_flops": N * 3 * K * exe}}
    print(json.dumps(rec), flush=True)


def yardstick(args):
    """Library GEMM references (torch.matmul in BF16 with FP32 accumulation, served
    by hipBLASLt on this stack), a ceiling reference only: (1) a large square
    product, the BF16 rate library code reaches on this chip; (2) the K-wide
    whitening product of the headline shape, N x d by d x Kd (the K whiteners side
    by side), in row chunks: it writes the N x Kd product that the fused cluster
    draw keeps in registers, and none of the norms or the draw."""
    import torch

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    g = torch.Generator(device="cuda").manual_seed(7)
    out = {"metric": "library BF16 GEMM references (hipBLASLt through torch.matmul)"}
    s = 8192
    a = torch.randn(s, s, device="cuda", dtype=torch.bfloat16, generator=g)
    b = torch.randn(s, s, device="cuda", dtype=torch.bfloat16, generator=g)
    c = torch.empty(s, s, device="cuda", dtype=torch.bfloat16)
    ms = timed(lambda: torch.matmul(a, b, out=c), 20)
    fl = 2.0 * s ** 3
    out["square_8192"] = {"ms": ms, "tflops": fl / ms / 1e9, "frac_of_peak": fl / (ms * 1e-3) / PEAK_BF16_MFMA}
    del a, b, c
    d, K, N, m = 128, 100, 10_000_000, 1 << 18
    xa = torch.randn(m, d, device="cuda", dtype=torch.bfloat16, generator=g)
    w = torch.randn(d, K * d, device="cuda", dtype=torch.bfloat16, generator=g)
    y = torch.empty(m, K * d, device="cuda", dtype=torch.bfloat16)
    ms_chunk = timed(lambda: torch.matmul(xa, w, out=y), 5)
    ms_step = ms_chunk * N / m
    fl_step = 2.0 * N * d * K * d
    out["whitening_k_wide_gauss_d128"] = {
        "rows_per_chunk": m, "ms_per_chunk": ms_chunk, "ms_per_1e7_rows": ms_step,
        "executed_tflops": fl_step / ms_step / 1e9, "frac_of_peak": fl_step / (ms_step * 1e-3) / PEAK_BF16_MFMA,
        "product_bytes_written_per_1e7_rows": 2.0 * N * K * d}
    print(json.dumps(out), flush=True)


def label_step(args):
    import torch
    res = label_step_run(torch, args.label_step, int(float(args.n)) if args.n else None, args.precision, args.steps,
                         args.warmup)
    out = {"metric": "point-cluster evals/s in label step", "value": res["label_evals_per_s"],
           "unit": "point-cluster evals/s", "higher_is_better": True, "data": "synthetic",
           "steps": args.steps, "warmup": args.warmup, **res}
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------------------------- learned vs plain

AB_WORKLOAD = "gauss_d64"


def run_chain(torch, x, n, d, m, iters, learned, train_every, train_until, train_steps, batch, lr, seed):
    """One chain from K = 1 with the BF16 form: per iteration (t, seconds since
    the start, K, log posterior).  The learned chain trains every `train_every`
    iterations up to iteration `train_until`; its training time is inside the
    clock."""
    S = _sampler("gaussian", d, 512, m, "bf16", burn_out=5, learned=learned, seed=seed)
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


def plateau_time(rec, level, rel, window=5):
    """First (iteration, seconds) at which the `window`-iteration moving average
    of the log posterior enters level - rel |level|; None if it never does."""
    lp = np.array([r[3] for r in rec])
    thr = level - rel * abs(level)
    for j in range(window - 1, lp.size):
        if lp[j - window + 1: j + 1].mean() >= thr:
            return rec[j][0], rec[j][1]
    return None


def ab_one(args, torch, x, n, d, m, labels, seed):
    """Both chains under one seed; the plateau is that seed's plain chain's:
    P* = median log posterior over its last 20% iterations; a chain reaches it
    when its 5-iteration moving average enters P* - rel |P*| (rel = 1e-4, and
    1e-5 and 1e-3 for the sensitivity).  A chain that never does has speed-up 0."""
    from paper_2204_08988_amd import _lib
    chains = {}
    for form, learned in (("plain", 0), ("learned", args.ab_axes)):
        S, z, rec, extra = run_chain(torch, x, n, d, m, args.ab_iters, learned, args.ab_train_every,
                                     args.ab_train_until, args.ab_train_steps, args.ab_batch, args.ab_lr, seed)
        chains[form] = (rec, extra, _lib.nmi(labels, z.cpu().numpy()), S.K)
        S.close()
    tail = np.array([r[3] for r in chains["plain"][0][-max(1, args.ab_iters // 5):]])
    level = float(np.median(tail))
    out = {"seed": seed, "plateau_logpost": level}
    for rel in (1e-5, 1e-4, 1e-3):
        hits = {f: plateau_time(chains[f][0], level, rel) for f in chains}
        p, l = hits["plain"], hits["learned"]
        sp = None if p is None else (0.0 if l is None else p[1] / l[1])
        out[f"speedup_wall@{rel:g}"] = sp
        out[f"plain_to_plateau@{rel:g}"] = p
        out[f"learned_to_plateau@{rel:g}"] = l
    for form, (rec, extra, nmi, K) in chains.items():
        out[form] = {"total_s": rec[-1][1], "final_K": K, "final_logpost": rec[-1][3], "nmi": nmi,
                     "trace": [[r[0], round(r[1], 4), r[2], r[3]] for r in rec if r[0] % 5 == 0], **extra}
    out["nmi_diff"] = out["learned"]["nmi"] - out["plain"]["nmi"]
    return out


def learned_ab(args):
    """Time to the plain chain's log-posterior plateau, learned vs plain, for
    each of --ab-seeds seeds; the median wall-clock speed-up over the seeds
    (a learned chain that never reaches the plateau counts as 0)."""
    import torch
    from paper_2204_08988_amd import datagen
    spec = datagen.WORKLOADS[AB_WORKLOAD]
    x_np, labels = datagen.workload(AB_WORKLOAD, 3)
    n, d = x_np.shape
    m = x_np.mean(0).astype(np.float64)
    x = torch.from_numpy(x_np).cuda()
    runs = []
    for i in range(args.ab_seeds):
        runs.append(ab_one(args, torch, x, n, d, m, labels, SEED + i))
        print(json.dumps({"seed_done": SEED + i, "speedup_wall@0.0001": runs[-1]["speedup_wall@0.0001"]}),
              file=sys.stderr, flush=True)
    out = {"metric": "time-to-plateau learned vs plain", "unit": "s", "higher_is_better": False,
           "workload": f"{AB_WORKLOAD}: Gaussian DPMM, N={n}, d={d}, {spec.k} true clusters, means N(0,4I), "
                       "covariances Wishart(d+2, I/d), weights Dir(1); start K=1; BF16 cluster scoring",
           "plateau_rule": "P* = median log posterior of the plain chain's last 20% iterations; reached when the "
                           "5-iteration moving average enters P* - rel |P*|; never reached = speed-up 0",
           "learned_config": {"axes": args.ab_axes, "features": 2 * args.ab_axes, "hidden": [128, 128],
                              "train_every": args.ab_train_every, "train_until": args.ab_train_until,
                              "train_steps": args.ab_train_steps, "batch": args.ab_batch, "lr": args.ab_lr},
           "seeds": runs}
    for rel in (1e-5, 1e-4, 1e-3):
        sp = [r[f"speedup_wall@{rel:g}"] for r in runs if r[f"speedup_wall@{rel:g}"] is not None]
        out[f"median_speedup_wall@{rel:g}"] = float(np.median(sp)) if sp else None
    out["median_nmi_diff"] = float(np.median([r["nmi_diff"] for r in runs]))
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "bf16x3"],
                    help="cluster scoring of the headline workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="skip the other configurations")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy a device buffer of BYTES five times (calibrates HBM byte counters)")
    ap.add_argument("--sparse", action="store_true",
                    help="instead of the throughput line: the sparse-row (news_v20k) chain and label step only")
    ap.add_argument("--width-compare", action="store_true",
                    help="instead of the throughput line: the K-wide cluster draw against the 3K-wide form at the "
                         "headline shape")
    ap.add_argument("--label-step", metavar="WORKLOAD",
                    help="instead of the throughput line: label-step throughput at WORKLOAD's true mixture")
    ap.add_argument("--n", default=None, help="points for --label-step (default: the workload's N)")
    ap.add_argument("--yardstick", action="store_true",
                    help="instead of the throughput line: library BF16 GEMM references (a ceiling reference only)")
    ap.add_argument("--learned-ab", action="store_true",
                    help="instead of the throughput line: time to the plain chain's log-posterior plateau, "
                         "learned proposal vs plain, on the learned-proposal workload")
    ap.add_argument("--ab-iters", type=int, default=200)
    ap.add_argument("--ab-seeds", type=int, default=5, help="seeds of the learned-vs-plain comparison")
    ap.add_argument("--ab-axes", type=int, default=8)
    ap.add_argument("--ab-train-every", type=int, default=10)
    ap.add_argument("--ab-train-until", type=int, default=60)
    ap.add_argument("--ab-train-steps", type=int, default=20)
    ap.add_argument("--ab-batch", type=int, default=4096)
    ap.add_argument("--ab-lr", type=float, default=1e-3)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        import torch
        a = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.learned_ab:
        learned_ab(args)
        return
    if args.label_step:
        label_step(args)
        return
    if args.width_compare:
        width_compare(args)
        return
    if args.yardstick:
        yardstick(args)
        return
    if args.sparse:
        import torch
        out = {"news_v20k_chain": sparse_run(torch, int(float(args.n)) if args.n else None, args.steps, args.warmup,
                                             True),
               "news_v20k_label_step_n2e5": sparse_run(torch, 200_000, args.steps, args.warmup, False)}
        print(json.dumps(out), flush=True)
        return
    headline(args)


if __name__ == "__main__":
    main()
