"""Benchmark: correlated-chains Monte Carlo inversion on one MI355X.

Workload (default): pedigree-structured real non-symmetric C, n = 100000
(~6.7 stored entries per row), fp32 sweeps, 4096 chain pairs in 64 groups,
diagonal + 256 x 256 block + trace requested.  One step = one sampling sweep
of the whole path: every colour's coupled z/w update with fused diagonal and
trace moments, the per-sweep trace reduction and the block moments.

Prints one JSON line: nonzero-updates/s (2 nnz(C) P per sweep: z and w are
the two chains of each pair), the sweep kernel's fraction of the HBM roofline
(algorithmic bytes per sweep / measured sweep-kernel time), the oracle's CPU
throughput on a bounded sample, and the time to reach 1% relative standard
error on every diagonal entry.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_sweep(n, nnz, P, s_state, s_val):
    """State streamed once per sweep (z and w, read and written) plus the
    matrix: CSR of C and of C^dagger and three per-row constants."""
    nnz_off = nnz - n
    M = 2 * (nnz_off * (s_val + 4) + 4 * (n + 1)) + 3 * n * s_val
    return 2 * 2 * P * n * s_state + M


PROFILE = {"pedigree": "profiles/k_sweep_pedigree_n100000_P4096_f32.md",
           "lattice": "profiles/k_sweep_lattice16_P1024_c64.md"}
KERNEL_SOURCES = ("sweep.hip", "sweep.h", "device_common.h")


def profiled_traffic(workload):
    """HBM bytes per sweep-kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when the
    kernel sources changed since those counters were taken."""
    import hashlib
    if workload not in PROFILE:
        return None
    path = os.path.join(ROOT, PROFILE[workload])
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_cs_0412107_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    for line in open(path):
        parts = line.strip().split(": ")
        if len(parts) == 2 and parts[0] in ("traffic_bytes_per_launch", "kernel_sources_sha256"):
            vals[parts[0]] = parts[1]
    if vals.get("kernel_sources_sha256") != h.hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"])


BURN_TOL = 5e-5   # coupling tolerance of the paper's numerical tests
ORDER_NAMES = ("natural", "XCD-contiguous", "XCD runs of 16 row blocks", "pair tiles fastest")


def tuned_order(pkg, m, P, G, dtype, hermitian=False):
    """The fastest sweep workgroup order for this matrix and pair count, timed
    on a scratch context (setup; not part of any timed region)."""
    with pkg.Sampler(m, pairs=P, groups=G, dtype=dtype, seed=0, hermitian=hermitian) as s:
        order, _ = s.tune_launch(2)
    return order


def time_to_1pct(pkg, torch, m, P, G, seed, dtype, moments, burn_in, rel=0.01, check=2, max_sweeps=20000,
                 hermitian=False, xcd_order=0, noise=0, keep_pairs=None):
    """Wall time to max_i SE_i/|est_i| <= rel on the whole diagonal, counted
    from the start of burn-in (a fixed count, or "coupled": until the coupled
    paths agree to BURN_TOL), sampling checked every `check` sweeps; the
    context set-up before it (matrix preparation and upload) is reported
    separately.  keep_pairs: chain pairs whose final z and w columns are
    returned (under "_state"), for a comparison with the oracle."""
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    s = pkg.Sampler(m, pairs=P, groups=G, dtype=dtype, seed=seed, moments=moments, use_torch_stream=True,
                    hermitian=hermitian, xcd_order=xcd_order, noise=noise)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_setup = t0 - t_setup
    if burn_in == "coupled":
        nb, _, _ = s.burn_in_coupled(BURN_TOL, 10000)
        burn_desc = f"coupled to {BURN_TOL:g}"
    else:
        s.burn_in(burn_in)
        nb, burn_desc = burn_in, "fixed"
    s.request(diag=True, trace=False)
    done, ach = s.sample_until(rel, max_sweeps, check)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"seconds": t, "setup_seconds": t_setup, "burn_in": nb, "burn_in_rule": burn_desc,
           "sample_sweeps": done, "max_rel_se": ach, "form": f"{dtype} sweeps, {moments} blocks",
           "noise": ["normal", "Z2"][noise], "xcd_order": ORDER_NAMES[xcd_order], "check_every": check}
    if keep_pairs is not None:
        out["_state"] = {"pairs": np.asarray(keep_pairs), "z": s.state(0)[:, keep_pairs],
                         "w": s.state(1)[:, keep_pairs], "sweeps": nb + done, "seed": seed}
    if dtype == "f32":
        # the same chains in fp64 (same matrix values, noise, burn-in and sample
        # sweeps; the fp64 path is the one tested against the oracle to 1e-12):
        # how far the fp32 sweeps move the estimates, next to their SE
        est, se = s.diag()
        s.close()
        with pkg.Sampler(m, pairs=P, groups=G, dtype="f64", seed=seed, use_torch_stream=True,
                         hermitian=hermitian, xcd_order=xcd_order, noise=noise) as r:
            r.burn_in(nb)
            r.request(diag=True, trace=False)
            r.sample(done)
            ref, _ = r.diag()
        err = np.abs(np.asarray(est) - np.asarray(ref))
        se = np.asarray(se)
        pos = se > 0   # Z2 noise makes rows without off-diagonal entries exact (SE 0)
        out["vs_fp64_same_noise"] = {"max_abs": float(err.max()),
                                     "max_rel": float((err / np.abs(ref)).max()),
                                     "max_over_se": float((err[pos] / se[pos]).max())}
    else:
        s.close()
    return out


def batched_forms(pkg, torch, gen, rel=0.01, check=10):
    """Batched workload: 512 pedigree matrices, n log-uniform in [1e3, 5e4],
    64 chain pairs each.  Time to 1% on every diagonal entry of every matrix:
    one batched context (persistent launches) versus the plain path run
    matrix by matrix; plus the batched sampling throughput."""
    w = gen.WORKLOADS["batched"]
    mats = [gen.round_values(x, np.float32) for x in gen.batched_pedigrees(w["m"], w["lo"], w["hi"], w["seed"])]
    P, G, seed, burn = w["pairs"], w["groups"], w["noise_seed"], w["burn_in"]
    nnz = sum(x.nnz for x in mats)
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    b = pkg.BatchSampler(mats, pairs=P, groups=G, seed=seed, use_torch_stream=True)
    sched, r, g, tune_ms = b.autotune(1)   # set-up: the autotuner's sweeps count as burn-in
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_setup = t0 - t_setup
    burn_b, _ = b.burn_in_coupled(BURN_TOL, 10000)
    b.request(diag=True, block_dim=w["block"], expected_samples=200)
    done, ach = b.sample_until_each(rel, 20000, check)   # each matrix stops at its own 1%
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    msamples, _ = b.matrix_samples()
    ns = np.array([x.nnz for x in mats], dtype=np.float64)
    # batched sampling throughput (block moments on the matrix cores included)
    K = 20
    b.request(diag=True, block_dim=w["block"], expected_samples=200)   # every matrix active again
    b.sample(K)
    ms_call = b.info()["last_call_ms"]
    info = b.info()
    b.close()
    alg = sum(algorithmic_bytes_per_sweep(x.n, x.nnz, P, 4, 4) for x in mats)
    log(f"batched form: {t_batch:.2f} s to 1% ({done} sample sweeps); plain form, matrix by matrix ...")
    # plain form, matrix by matrix (same seeds: stream id = matrix index)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    worst = 0.0
    sweeps_plain = []
    setup_plain = 0.0
    for j, x in enumerate(mats):
        ts = time.perf_counter()
        s = pkg.Sampler(x, pairs=P, groups=G, dtype="f32", seed=seed, stream_id=j, moments="bf16x3",
                        use_torch_stream=True)
        torch.cuda.synchronize()
        setup_plain += time.perf_counter() - ts
        s.burn_in_coupled(BURN_TOL, 10000)
        s.request(diag=True, trace=False)
        dj, aj = s.sample_until(rel, 20000, check)
        worst = max(worst, aj)
        if j % 64 == 63:
            log(f"plain form: {j + 1} matrices, {time.perf_counter() - t1:.1f} s")
        sweeps_plain.append(dj)
        s.close()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t1 - setup_plain
    return {"workload": f"{len(mats)} pedigree matrices, n log-uniform in [{w['lo']}, {w['hi']}] "
                        f"(sum n = {sum(x.n for x in mats)}, nnz = {nnz}), {P} pairs each, fp32",
            "burn_in": f"coupled to {BURN_TOL:g} (batched: {burn_b} sweeps for all matrices; plain: per matrix)",
            "timing": "from the start of burn-in; context set-up (matrix preparation, upload, batched "
                      "autotuning) reported separately",
            "batched_seconds": t_batch, "batched_setup_seconds": t_setup,
            "batched_sample_sweeps": done, "batched_max_rel_se": ach,
            "stopping": "per matrix: each matrix leaves the launches at its first check at 1%, as the plain runs do",
            "batched_sample_sweeps_per_matrix": {"min": int(msamples.min()), "median": float(np.median(msamples)),
                                                 "max": int(msamples.max()),
                                                 "nnz_weighted_mean": float((ns * msamples).sum() / ns.sum())},
            "plain_sample_sweeps_per_matrix": {"min": int(min(sweeps_plain)), "median": float(np.median(sweeps_plain)),
                                               "max": int(max(sweeps_plain)),
                                               "nnz_weighted_mean": float((ns * np.array(sweeps_plain)).sum() / ns.sum())},
            "autotune": {"schedule": ["phased graph", "persistent"][sched], "rows_per_item": r, "grab": g,
                         "ms_per_sweep": tune_ms},
            "plain_seconds": t_plain, "plain_setup_seconds": setup_plain,
            "plain_sample_sweeps_max": max(sweeps_plain), "plain_max_rel_se": worst,
            "speedup_vs_plain": t_plain / t_batch,
            "throughput": {"nonzero_updates_per_s": 2.0 * nnz * P * K / (ms_call / 1e3),
                           "ms_per_sweep": ms_call / K, "items_per_sweep": info["items_per_sweep"],
                           "algorithmic_GBps": alg * K / (ms_call / 1e3) / 1e9,
                           "note": "one graph launch of 20 sampling sweeps with 128x128 bf16x3 block moments, "
                                   "autotuned schedule"}}


def hermitian_form(pkg, torch, gen, w, steps=20):
    """Symmetric pedigree (lambda = 0, symmetric jitter; same size as the
    headline workload): single-draw sweeps (w = z, eq 2) versus the two-chain
    sweeps on the same matrix -- sampling throughput and time to 1%."""
    P, G, seed = w["pairs"], w["groups"], w["noise_seed"]
    m = gen.round_values(gen.pedigree(w["n"], seed=w["seed"], lam=0.0, symmetric=True), np.float32)
    out = {"workload": f"symmetric pedigree n={m.n} nnz={m.nnz} (lambda=0), {P} pairs, fp32"}
    for name, herm in (("two_chain", False), ("single_draw", True)):
        s = pkg.Sampler(m, pairs=P, groups=G, dtype="f32", seed=seed, use_torch_stream=True, hermitian=herm)
        s.burn_in(5)
        s.request(diag=True, trace=True)
        s.sample(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.sample(steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        s.close()
        ttt = time_to_1pct(pkg, torch, m, P, G, seed + 1, "f32", "fp64", "coupled", hermitian=herm)
        out[name] = {"ms_per_sweep": ms, "nonzero_updates_per_s": 2.0 * m.nnz * P / (ms / 1e3),
                     "time_to_1pct_s": ttt["seconds"], "burn_in": ttt["burn_in"],
                     "sample_sweeps": ttt["sample_sweeps"]}
    out["note"] = ("single-draw sweeps give bit-identical estimates to the two-chain sweeps; its "
                   "nonzero_updates_per_s counts the two-chain work it replaces")
    out["speedup_sweep"] = out["two_chain"]["ms_per_sweep"] / out["single_draw"]["ms_per_sweep"]
    out["speedup_time_to_1pct"] = out["two_chain"]["time_to_1pct_s"] / out["single_draw"]["time_to_1pct_s"]
    return out


def paper_dirac_values():
    """The paper's printed values for its second example (Sec. 3.2): exact
    traces (Tables 4, 5, two decimals) and the CC method's burn-in, sample
    count, effective length, variance, MC standard error and estimate."""
    gold = os.path.join(ROOT, "tests", "golden")
    with open(os.path.join(gold, "dirac_free_field.json")) as f:
        cases = {c["N"]: c for c in json.load(f)["cases"]}
    with open(os.path.join(gold, "paper_tables.json")) as f:
        rows = {r["case"]: r for r in json.load(f)["rows"]}
    burn = {18: 18, 20: 18}   # Tables 4, 5: burn-in cycles N
    out = {}
    for N in (18, 20):
        r = rows[f"{N}^4"]
        out[N] = {"exact": cases[N]["exact_trace"], "burn_in": burn[N], "samples": r["samples"],
                  "n_eff": r["n_eff"], "var": r["var"], "se": r["se"], "estimate_re": r["estimate"],
                  "table": cases[N]["table"]}
    return out


def dirac_form(pkg, torch, gen, N):
    """The paper's second example: free Wilson-Dirac matrix on an N^4 lattice
    (K = 0.1, 14 nonzeros per row; case 1 N = 18, case 2 N = 20), trace of
    the inverse to the paper's stopping rule (Geyer standard error below 1e-5
    of the estimate), coupled burn-in to 5e-5; compared with the exact value
    and the run statistics the paper prints (Tables 3-5)."""
    w = gen.WORKLOADS["dirac"]
    paper = paper_dirac_values()[N]
    m = gen.round_values(gen.dirac(N, w["K"]), np.complex64)
    P, G, seed = w["pairs"], w["groups"], w["noise_seed"]
    exact = paper["exact"]
    order = tuned_order(pkg, m, P, G, "c64")

    def run(noise):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = pkg.Sampler(m, pairs=P, groups=G, dtype="c64", seed=seed, use_torch_stream=True, xcd_order=order,
                        noise=noise)
        nb, _, _ = s.burn_in_coupled(BURN_TOL, 10000)
        s.request(diag=False, trace=True)
        done, ach = s.sample_until_trace(w["rel_se"], 20000, 20)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = s.trace_stats()
        est, se = st["mean"], st["se"]
        t1 = time.perf_counter()
        s.sample(10)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / 10
        s.close()
        z = float((est.real - exact) / se)
        return {"seconds": t, "burn_in": nb, "sample_sweeps": done, "rel_se": ach,
                "estimate": [est.real, est.imag], "se": se, "z_score": z, "within_5se": abs(z) <= 5.0,
                "variance_series": st["var"], "effective_length_series": st["n_eff"],
                "variance_per_pair": st["var"] * P, "variance_per_pair_re": st["var_re"] * P,
                "variance_per_pair_im": st["var_im"] * P, "effective_length_pair_sweeps": st["n_eff"] * P,
                "ms_per_sweep": ms}

    out = {"workload": f"free Wilson-Dirac {N}^4 (n={m.n}, nnz={m.nnz}), K={w['K']}, {P} pairs, complex64",
           "exact_paper": exact, **run(pkg.MCINV_NOISE_NORMAL), "xcd_order": ORDER_NAMES[order],
           "paper": {"table": paper["table"], "chain_pairs": 1, "burn_in": paper["burn_in"],
                     "samples": paper["samples"], "effective_length": paper["n_eff"], "variance": paper["var"],
                     "mc_se": paper["se"], "estimate_re": paper["estimate_re"], "exact": exact},
           "note": ("one sweep advances all P pairs; the series averages them, so variance_per_pair and "
                    "effective_length_pair_sweeps are the single-chain figures the paper's tables print")}
    out["nonzero_updates_per_s"] = 2.0 * m.nnz * P / (out["ms_per_sweep"] / 1e3)
    # the paper's preferred Z2 noise (Sec. 1) on the same workload and rule
    out["z2_noise"] = run(pkg.MCINV_NOISE_RADEMACHER)
    return out


def lattice_form(pkg, torch, gen, steps=20, check=2):
    """Random-phase complex non-hermitian 16^4 lattice operator (c64 sweeps,
    fp64 sums, 1024 pairs): sampling throughput with the sweep kernel's
    roofline fraction, and the time to 1% on every diagonal entry."""
    w = gen.WORKLOADS["lattice"]
    m = gen.round_values(gen.lattice(w["L"], k=w["k"], seed=w["seed"]), np.complex64)
    P, G, seed = w["pairs"], w["groups"], w["noise_seed"]
    order = tuned_order(pkg, m, P, G, "c64")
    s = pkg.Sampler(m, pairs=P, groups=G, dtype="c64", seed=seed, use_torch_stream=True, profile=True,
                    xcd_order=order)
    s.burn_in(10)
    s.request(diag=True, trace=True)
    s.sample(3)
    s.reset_profile()
    torch.cuda.synchronize()
    e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    e0.record()
    s.sample(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    info = s.info()
    s.close()
    B = algorithmic_bytes_per_sweep(m.n, m.nnz, P, 8, 8)
    sweep_ms = info["sweep_kernel_ms"] / steps
    launches = info["sweep_kernel_launches"] / steps
    ttt = time_to_1pct(pkg, torch, m, P, G, seed + 1, "c64", "fp64", "coupled", xcd_order=order, check=check)
    return {"workload": f"random-phase lattice {w['L']}^4 (n={m.n}, nnz={m.nnz}), {P} chain pairs in {G} groups, "
                        "complex64 sweeps, fp64 sums, diag + trace",
            "nonzero_updates_per_s": 2.0 * m.nnz * P / (ms / 1e3), "ms_per_step": ms,
            "roofline": {"bound": "hbm", "achieved": B / (sweep_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": B / (sweep_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                         "traffic": profiled_traffic("lattice"),
                         "algorithmic_bytes_per_launch": B / launches, "avg_launch_ms": sweep_ms / launches,
                         "algorithmic_bytes_per_sweep": B, "sweep_kernel_ms": sweep_ms,
                         "launches_per_sweep": launches,
                         "kernel": "k_sweep<Cx<float>, true, false> (all colour launches of one sweep)"},
            "launch_order": ORDER_NAMES[order],
            "time_to_1pct": ttt}


def qtrace_form(pkg, torch, gen, w, steps=20):
    """General-Q trace tr(Q C^-1) (eq tr) on the headline pedigree: a random
    sparse Q with about 5 nonzeros per row; sampling sweeps with diag + trace
    versus diag + trace + Q trace."""
    import scipy.sparse as sp
    P, G, seed = w["pairs"], w["groups"], w["noise_seed"]
    m = gen.round_values(gen.pedigree(w["n"], seed=w["seed"]), np.float32)
    rng = np.random.default_rng(7)
    Q = (sp.random(m.n, m.n, density=4.0 / m.n, random_state=rng, format="csr") + sp.identity(m.n)).tocsr()
    out = {"workload": f"pedigree n={m.n}, {P} pairs, Q: {Q.nnz} nonzeros"}
    for name, with_q in (("diag_trace", False), ("diag_trace_qtrace", True)):
        with pkg.Sampler(m, pairs=P, groups=G, dtype="f32", seed=seed, use_torch_stream=True) as s:
            s.set_trace_matrix(Q)
            s.burn_in(5)
            s.request(diag=True, trace=True, qtrace=with_q)
            s.sample(3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.sample(steps)
            torch.cuda.synchronize()
            out[name] = {"ms_per_sweep": (time.perf_counter() - t0) * 1e3 / steps}
            if with_q:
                est, se = s.qtrace()
                out[name]["estimate"] = float(np.real(est))
                out[name]["se"] = float(se)
    out["qtrace_ms_per_sample"] = out["diag_trace_qtrace"]["ms_per_sweep"] - out["diag_trace"]["ms_per_sweep"]
    # algorithmic bytes of one Q-trace evaluation: Q's CSR, the gathered z slices and the w rows
    qbytes = Q.nnz * (8 + 4) + 8 * (m.n + 1) + (Q.nnz + m.n) * P * 4
    out["qtrace_algorithmic_GBps"] = qbytes / max(out["qtrace_ms_per_sample"], 1e-6) / 1e6
    return out


MLP_FLOP_PER_ROW_STEP = 2 * (32 * 128 + 128 * 128 + 128) + 2 * (2 * 128 + 2 * 128 * 128 + 32 * 128)


def surrogate_form(pkg, torch, gen, n_train, n_val, rel_label=0.005, rel=0.01, steps=2000, batch=65536,
                   noise=None):
    """Learned-surrogate workload: pedigree matrices with random generator
    parameters (n = 2e4) labelled by the batched sampler to rel_label, 32
    features per row, the network trained on the labelled rows, a gate fitted
    on validation matrices, then a held-out matrix (n = 1e6): surrogate plus
    sampler fallback versus the plain sampler to 1% on every row.  Every
    sampler of the form (labels, fallback rows, the plain comparison) draws
    the same noise law: Z2 by default (Sec. 1's preferred law, which on these
    diagonal-dominant matrices needs fewer sweeps)."""
    from paper_cs_0412107_amd import surrogate as sur
    noise = pkg.MCINV_NOISE_RADEMACHER if noise is None else noise
    w = gen.WORKLOADS["surrogate"]
    qs = gen.surrogate_params(n_train + n_val + 1, seed=w["seed"])

    def make(q, n):
        return gen.round_values(gen.pedigree(n, seed=q["seed"], founders=q["founders"], lam=q["lam"],
                                             factor=q["factor"]), np.float32)

    t0 = time.perf_counter()
    mats = [make(q, w["train_n"]) for q in qs[:n_train + n_val]]
    log(f"surrogate: {len(mats)} matrices generated in {time.perf_counter() - t0:.1f} s; labelling ...")
    bw = gen.WORKLOADS["batched"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = pkg.BatchSampler(mats, pairs=bw["pairs"], groups=bw["groups"], seed=w["noise_seed"], noise=noise,
                         use_torch_stream=True)
    b.autotune(1)
    b.burn_in_coupled(BURN_TOL, 10000)
    b.request(diag=True)
    lab_sweeps, lab_ach = 0, float("inf")
    while lab_sweeps < 40000:
        d, lab_ach = b.sample_until_each(rel_label, 1000, 50)
        lab_sweeps += d
        log(f"surrogate: labelling, {lab_sweeps} sample sweeps, max rel SE {lab_ach:.4f}")
        if lab_ach <= rel_label:
            break
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    Y, YSE = [], []
    for j in range(len(mats)):
        y, yse = b.labels(j)
        Y.append(y)
        YSE.append(yse)
    b.close()
    log(f"surrogate: labels in {t_label:.1f} s ({lab_sweeps} sample sweeps, max rel SE {lab_ach:.4f}); features ...")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = []
    for j, x in enumerate(mats):
        F.append(sur.features(x))
        if j % 500 == 499:
            log(f"surrogate: features of {j + 1} matrices")
    t_feat = time.perf_counter() - t0
    Xtr, ytr, setr = np.concatenate(F[:n_train]), np.concatenate(Y[:n_train]), np.concatenate(YSE[:n_train])
    Xv, yv, sev = np.concatenate(F[n_train:]), np.concatenate(Y[n_train:]), np.concatenate(YSE[n_train:])
    net = sur.Network(seed=w["seed"])
    net.set_data(Xtr, ytr, pkg.mcinv_mlp_label_weights(setr))
    net.train(20, batch, 1e-3, 1)  # warm-up (part of the training)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = net.train(steps, batch, 1e-3, 2)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    pv = net.predict(Xv).astype(np.float64)
    rv = (pv - yv) / yv
    # a bin is trusted when a one-sided 95% upper bound of its error meets the
    # tolerance (few validation rows need a smaller observed error)
    gate = sur.Gate(Xv, pv, yv, sev, feature_a=1, feature_b=5, bins=8, min_rows=20, tol=rel, ucb_z=1.645)
    log(f"surrogate: trained {steps} steps x {batch} rows in {t_train:.2f} s; held-out matrix ...")

    m = make(qs[-1], w["eval_n"])
    P, G = 1024, 16
    plain = time_to_1pct(pkg, torch, m, P, G, w["noise_seed"] + 1, "f32", "fp64", "coupled", rel=rel, noise=noise)
    burn = plain["burn_in"]
    with pkg.Sampler(m, pairs=P, groups=G, dtype="f32", seed=w["noise_seed"] + 1, noise=noise) as s:
        s.burn_in(burn)
        s.request(diag=True, trace=False)
        s.sample(plain["sample_sweeps"])
        d_plain, se_plain = s.diag()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est, src, info = sur.estimate_diag(
        m, net, gate, lambda mm: pkg.Sampler(mm, pairs=P, groups=G, dtype="f32", seed=w["noise_seed"] + 1,
                                             noise=noise, use_torch_stream=True),
        rel_se=rel, max_sweeps=20000, check_every=10, burn_in="coupled")
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    acc = src == 0
    r = (est - d_plain) / d_plain
    s_rel = se_plain / np.abs(d_plain)
    net.close()
    gate_tab = gate.table()
    gate.close()
    # rows in bins with fewer than 200 validation rows (which a fixed 200-row
    # floor would send to the sampler): their difference from the plain run
    Xh = sur.features(m)
    hb = np.searchsorted(gate_tab["edges_a"], Xh[:, 1].astype(np.float64), side="right") * 8 + \
        np.searchsorted(gate_tab["edges_b"], Xh[:, 5].astype(np.float64), side="right")
    sparse = acc & (gate_tab["count"][hb] < 200)
    return {
        "workload": f"{n_train} train + {n_val} validation pedigree matrices (n={w['train_n']}, random "
                    f"dominance 1.2-2.0, lambda 0-0.5, founders 2-20%), held-out n={m.n}",
        "noise": "Z2 (Rademacher)" if noise == pkg.MCINV_NOISE_RADEMACHER else "normal",
        "labels": {"seconds": t_label, "sample_sweeps": lab_sweeps, "max_rel_se": lab_ach,
                   "rows": int(sum(x.n for x in mats)), "form": "batched sampler, 64 pairs per matrix, each matrix stopped at its own 0.5%"},
        "features": {"seconds": t_feat, "rows": int(sum(x.n for x in mats)),
                     "rows_per_s": sum(x.n for x in mats) / t_feat, "note": "host preparation included"},
        "training": {"seconds": t_train, "steps": steps, "batch_rows": batch,
                     "rows_per_s": steps * batch / t_train,
                     "TFLOPs": MLP_FLOP_PER_ROW_STEP * steps * batch / t_train / 1e12,
                     "mfma_frac_bf16_peak": MLP_FLOP_PER_ROW_STEP * steps * batch / t_train / 2.5e15,
                     "loss_first": float(hist[0]), "loss_last": float(hist[-1])},
        "validation": {"rms_rel_err": float(np.sqrt(np.mean(rv ** 2))),
                       "rms_rel_err_neumann2": float(np.sqrt(np.mean(((Xv[:, 25] - yv) / yv) ** 2))),
                       "rms_rel_err_jacobi": float(np.sqrt(np.mean(((1.0 - yv) / yv) ** 2))),
                       "gate_bins_fallback": int(gate_tab["fallback"].sum()),
                       "gate_bins": int(gate_tab["fallback"].size)},
        "held_out": {"n": int(m.n), "plain_seconds": plain["seconds"],
                     "plain_setup_seconds": plain["setup_seconds"],
                     "plain_sample_sweeps": plain["sample_sweeps"], "surrogate_seconds": t_sur,
                     "note": "surrogate_seconds starts from the matrix in host memory (features include their "
                             "preparation); speedup_vs_plain compares it with the plain sampler's set-up + burn-in "
                             "+ sampling",
                     "speedup_vs_plain": (plain["seconds"] + plain["setup_seconds"]) / t_sur,
                     "one_off_cost_seconds": t_label + t_feat + t_train,
                     "break_even_matrices": (t_label + t_feat + t_train) /
                     max(plain["seconds"] + plain["setup_seconds"] - t_sur, 1e-9),
                     "break_even_note": ("held-out matrices of this size after which labelling, features and "
                                         "training are paid back by the per-matrix saving"),
                     "accepted_rows": int(acc.sum()), "fallback_rows": int((~acc).sum()),
                     "fallback_sweeps": info["sweeps"],
                     "accepted_rms_rel_diff_vs_plain": float(np.sqrt(np.mean(r[acc] ** 2))) if acc.any() else None,
                     "accepted_model_err_est": float(np.sqrt(max(np.mean(r[acc] ** 2) - np.mean(s_rel[acc] ** 2),
                                                                 0.0))) if acc.any() else None,
                     "plain_pairs": P,
                     "sparse_bin_rows": {
                         "rows": int(sparse.sum()),
                         "rms_rel_diff_vs_plain": float(np.sqrt(np.mean(r[sparse] ** 2))) if sparse.any() else None,
                         "plain_rms_rel_se": float(np.sqrt(np.mean(s_rel[sparse] ** 2))) if sparse.any() else None}},
    }


def host_description():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": allowed}


def cpu_baseline(m, seed, P, G, budget_s, check=None):
    """The oracle (C, fp64, one thread per chain-pair subset) on a bounded
    sample of the same workload: a few chain pairs, as many sweeps as fit a
    time budget.  Three legs: the plain test build on one core, the same
    source built for the host (FAST_FLAGS) on one core, and that build on
    every allowed core (independent chain pairs per thread, no algorithmic
    change; ctypes releases the interpreter lock during each oracle call).
    With ``check`` (a GPU run's seed, sweep count, sampled pairs and their
    final states) the one-core leg of the host build sweeps exactly those
    pairs for exactly those sweeps, and the GPU states' error against it is
    reported."""
    import threading

    import oracle
    host = host_description()
    threads = max(1, min(host["cpus_allowed"] or 1, 16))
    per = 8   # chain pairs per oracle run (thread)

    def pair_ids(k, t):
        # k pairs spread over the P pairs, offset per thread
        return (np.arange(k, dtype=np.int64) * (P // k) + t) % P

    def leg(fast, nthreads, seconds):
        runs = [oracle.Run(m, seed=seed, pairs=P, groups=G, pair_ids=pair_ids(per, t), fast=fast)
                for t in range(nthreads)]
        counts = [0] * nthreads

        def work(t):
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < seconds:
                runs[t].burn_in(1)
                counts[t] += 1
        t0 = time.perf_counter()
        ths = [threading.Thread(target=work, args=(t,)) for t in range(nthreads)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        t = time.perf_counter() - t0
        ups = 2.0 * m.nnz * per * sum(counts) / t
        return ups, sum(counts), t

    u_plain, sw_plain, t_plain = leg(False, 1, budget_s / 3)
    prec = None
    if check is None:
        u_fast, sw_fast, t_fast = leg(True, 1, budget_s / 3)
    else:
        pids = np.asarray(check["pairs"], dtype=np.int64)
        run = oracle.Run(m, seed=check["seed"], pairs=P, groups=G, pair_ids=pids, fast=True)
        t0 = time.perf_counter()
        run.burn_in(check["sweeps"])
        t_fast = time.perf_counter() - t0
        sw_fast = check["sweeps"]
        u_fast = 2.0 * m.nnz * pids.size * sw_fast / t_fast
        prec = {"pairs": pids.tolist(), "sweeps": int(sw_fast)}
        for name, gpu, ora in (("z", check["z"], run.z), ("w", check["w"], run.w)):
            g = np.asarray(gpu).astype(np.complex128)
            prec[f"max_rel_err_{name}"] = float(np.max(np.abs(g - ora)) / np.max(np.abs(ora)))
            prec[f"max_abs_err_{name}"] = float(np.max(np.abs(g - ora)))
        prec["note"] = ("chain states of the precision form (32-bit sweeps) after its burn-in and sample sweeps "
                        "against the fp64 oracle on the same noise, on sampled pairs")
    u_all, sw_all, t_all = leg(True, threads, budget_s / 3)
    import oracle as _o
    extra = {} if prec is None else {"precision_check": prec}
    return dict(value=u_all, unit="nonzero-updates/s", cores=threads, kind="oracle", **extra,
                value_1core=u_fast, value_1core_plain_build=u_plain, value_all_cores=u_all,
                flags={"plain": "-O2", "fast": " ".join(_o.FAST_FLAGS)},
                cpu_model=host["cpu_model"], nproc=host["nproc"], cpus_allowed=host["cpus_allowed"],
                sample=(f"n={m.n}, {per} of {P} chain pairs per thread; plain build 1 thread {sw_plain} sweeps "
                        f"in {t_plain:.1f} s, fast build 1 thread {sw_fast} sweeps in {t_fast:.1f} s, fast build "
                        f"{threads} threads {sw_all} pair-block sweeps in {t_all:.1f} s"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["pedigree", "lattice", "dirac"], default="pedigree")
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=18.0, help="seconds for the three CPU-baseline legs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-1%% phase")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form comparison")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate form")
    ap.add_argument("--no-dirac", action="store_true", help="skip the free Wilson-Dirac forms (18^4 and 20^4)")
    ap.add_argument("--no-lattice", action="store_true", help="skip the random-phase lattice form")
    ap.add_argument("--surrogate-train", type=int, default=2000,
                    help="training matrices of the surrogate form (the full workload has 2000)")
    ap.add_argument("--surrogate-val", type=int, default=100)
    ap.add_argument("--stores", type=int, default=0,
                    help="sweep state stores of the headline sampler: 0 automatic, 1 non-temporal, 2 temporal")
    ap.add_argument("--pairs", type=int, default=0,
                    help="chain pairs of the headline sampler (0: the workload's own)")
    ap.add_argument("--pass-tiles", type=int, default=0,
                    help="256-pair tiles per pass of the headline sampler (0: all tiles in every colour launch)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also report the plain 1 GiB device copy in full (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the chain pairs would "
              "split across GPUs with one fp64 all-reduce of the moment sums, which the "
              "library does not implement.", file=sys.stderr)
        sys.exit(2)

    import torch

    import gen
    import paper_cs_0412107_amd as pkg

    w = gen.WORKLOADS[args.workload]
    P, G, seed, dtype = w["pairs"], w["groups"], w["noise_seed"], w["dtype"]
    if args.pairs > 0:
        P, G = args.pairs, min(G, max(1, args.pairs // 4))
    if args.workload == "pedigree":
        m = gen.round_values(gen.pedigree(w["n"], seed=w["seed"]), np.float32)
        desc = f"pedigree n={m.n} nnz={m.nnz}, {P} chain pairs in {G} groups, fp32 sweeps, " \
               f"diag + {w['block']}x{w['block']} block + trace"
    elif args.workload == "lattice":
        m = gen.round_values(gen.lattice(w["L"], k=w["k"], seed=w["seed"]), np.complex64)
        desc = f"random-phase lattice {w['L']}^4 (n={m.n}, nnz={m.nnz}), {P} chain pairs in {G} groups, " \
               f"complex64 sweeps, diag + trace"
    else:
        m = gen.round_values(gen.dirac(w["N"], w["K"]), np.complex64)
        desc = f"free Wilson-Dirac {w['N']}^4 (n={m.n}, nnz={m.nnz}), K={w['K']}, {P} chain pairs in {G} " \
               f"groups, complex64 sweeps, diag + trace"
    n = m.n
    s_elem = {"f32": 4, "c64": 8}[dtype]
    blk = np.arange(n - w["block"], n) if "block" in w else None
    torch.cuda.set_device(0)

    s = pkg.Sampler(m, pairs=P, groups=G, dtype=dtype, seed=seed, use_torch_stream=True, profile=True,
                    moments="bf16x3" if dtype == "f32" else "fp64", pass_tiles=args.pass_tiles, stores=args.stores)
    info0 = s.info()
    s.burn_in(w.get("burn_in", 60))
    order, ms_orders = s.tune_launch(2)   # setup: picks the fastest workgroup order
    s.request(diag=True, trace=True, block_rows=blk, block_cols=blk)
    s.sample(args.warmup)
    s.reset_profile()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record()
    s.sample(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1)
    info = s.info()
    K = args.steps
    ups = 2.0 * m.nnz * P * K / (ms / 1e3)

    B = algorithmic_bytes_per_sweep(n, m.nnz, P, s_elem, s_elem)
    sweep_ms = info["sweep_kernel_ms"] / K
    launches = info["sweep_kernel_launches"] / K
    # per launch: algorithmic bytes of an average colour launch over its
    # average duration (the same ratio as per sweep)
    achieved = (B / launches) / (sweep_ms / launches / 1e3) / 1e9
    d, se = s.diag()
    rel = se / np.abs(d)
    s.close()

    result = {
        "metric": "nonzero-updates/s",
        "value": ups,
        "unit": "nonzero-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": desc,
                   "n": n, "nnz": int(m.nnz), "pairs": P, "groups": G, "colors": info0["n_colors"],
                   "step": "one sampling sweep (all colours, fused diag/trace moments, trace reduction"
                           + (", block moments)" if blk is not None else ")"),
                   "tiles_per_pass": args.pass_tiles if args.pass_tiles > 0 else "all",
                   "stores": ["automatic", "non-temporal", "temporal"][args.stores],
                   "launch_order": {"chosen": ORDER_NAMES[order],
                                    "burn_in_ms_per_sweep": dict(zip(ORDER_NAMES, map(float, ms_orders)))}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(args.workload)
                     if args.pass_tiles == 0 and args.stores == 0 and args.pairs == 0 else None,
                     "algorithmic_bytes_per_launch": B / launches,
                     "avg_launch_ms": sweep_ms / launches,
                     "kernel": f"k_sweep<{'float' if dtype == 'f32' else 'Cx<float>'}, true, false> "
                               "(all colour launches of one sweep)",
                     "algorithmic_bytes_per_sweep": B, "sweep_kernel_ms": sweep_ms,
                     "launches_per_sweep": launches},
        "moments_ms_per_step": info["moment_kernel_ms"] / K,
        "wall_s_timed": t_wall,
        "diag_rel_se": {"max": float(np.max(rel)), "median": float(np.median(rel)),
                        "p99": float(np.quantile(rel, 0.99)), "samples": args.warmup + K},
    }

    log(f"throughput: {ups:.3e} nonzero-updates/s, {ms / K:.3f} ms per step")
    if not args.no_ttt:
        forms = {}
        if args.workload == "pedigree":
            m64 = gen.pedigree(n, seed=w["seed"])
            order64 = tuned_order(pkg, m64, P, G, "f64")
            forms["plain_fp64"] = time_to_1pct(pkg, torch, m64, P, G, seed + 1, "f64", "fp64", w["burn_in"],
                                               xcd_order=order64)
        forms["precision"] = time_to_1pct(pkg, torch, m, P, G, seed + 1, dtype,
                                          "bf16x3" if dtype == "f32" else "fp64", w.get("burn_in", 60),
                                          xcd_order=order)
        check_pairs = np.array([0, 1, 2, 3, P // 2, P // 2 + 1, P - 2, P - 1])
        forms["precision_coupled"] = time_to_1pct(pkg, torch, m, P, G, seed + 1, dtype,
                                                  "bf16x3" if dtype == "f32" else "fp64", "coupled",
                                                  xcd_order=order, keep_pairs=check_pairs)
        precision_state = forms["precision_coupled"].pop("_state")
        # the paper's preferred Z2 noise (Sec. 1): no transcendental functions, and a
        # diagonal-dominant C loses the variance its diagonal would add
        forms["precision_coupled_z2"] = time_to_1pct(pkg, torch, m, P, G, seed + 1, dtype,
                                                     "bf16x3" if dtype == "f32" else "fp64", "coupled",
                                                     xcd_order=order, noise=pkg.MCINV_NOISE_RADEMACHER)
        if args.workload == "pedigree":
            forms["plain_fp64_coupled"] = time_to_1pct(pkg, torch, m64, P, G, seed + 1, "f64", "fp64", "coupled",
                                                       xcd_order=order64)
        if "plain_fp64" in forms:
            for k in ("precision", "precision_coupled"):
                forms[k]["speedup_vs_plain"] = forms["plain_fp64"]["seconds"] / forms[k]["seconds"]
            forms["precision_coupled"]["speedup_vs_plain_coupled"] = \
                forms["plain_fp64_coupled"]["seconds"] / forms["precision_coupled"]["seconds"]
        log(f"time to 1%: {forms['precision']['seconds']:.2f} s (burn-in {forms['precision']['burn_in']}), "
            f"{forms['precision_coupled']['seconds']:.3f} s (coupled burn-in, "
            f"{forms['precision_coupled']['burn_in']} sweeps), "
            f"{forms['precision_coupled_z2']['seconds']:.3f} s (Z2 noise, "
            f"{forms['precision_coupled_z2']['sample_sweeps']} sample sweeps)")
        if args.workload == "pedigree" and not args.no_batched:
            forms["batched"] = batched_forms(pkg, torch, gen)
        if args.workload == "pedigree":
            forms["hermitian"] = hermitian_form(pkg, torch, gen, w)
            log(f"hermitian single-draw: {forms['hermitian']['speedup_sweep']:.2f}x per sweep")
        if args.workload == "pedigree":
            forms["qtrace"] = qtrace_form(pkg, torch, gen, w)
            log(f"Q trace: {forms['qtrace']['qtrace_ms_per_sample']:.3f} ms per sample")
        if args.workload == "pedigree" and not args.no_lattice:
            forms["lattice"] = lattice_form(pkg, torch, gen)
            log(f"lattice 16^4: {forms['lattice']['nonzero_updates_per_s']:.3e} nonzero-updates/s, roofline "
                f"{forms['lattice']['roofline']['frac']:.3f}, time to 1% "
                f"{forms['lattice']['time_to_1pct']['seconds']:.3f} s")
        if args.workload == "pedigree" and not args.no_dirac:
            for N in (18, 20):
                f = dirac_form(pkg, torch, gen, N)
                forms[f"dirac{N}"] = f
                log(f"dirac {N}^4: {f['seconds']:.2f} s to 1e-5 ({f['burn_in']} + {f['sample_sweeps']} sweeps), "
                    f"z = {f['z_score']:.2f}; Z2 noise {f['z2_noise']['seconds']:.2f} s "
                    f"({f['z2_noise']['sample_sweeps']} sweeps, z = {f['z2_noise']['z_score']:.2f})")
        if args.workload == "pedigree" and not args.no_surrogate:
            forms["surrogate"] = surrogate_form(pkg, torch, gen, args.surrogate_train, args.surrogate_val)
        result["forms"] = forms
        result["time_to_1pct"] = forms["precision_coupled"]

    # reference rate of a plain streaming kernel on this GPU: a 1 GiB device
    # copy (its counters also calibrate FETCH_SIZE / WRITE_SIZE)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    c0.record()
    dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    cms = c0.elapsed_time(c1)
    result["roofline"]["measured_copy_GBps"] = 2 * nbytes / (cms / 1e3) / 1e9
    if args.copy_calibration:
        result["copy_calibration"] = {"bytes_read": nbytes, "bytes_written": nbytes, "ms": cms,
                                      "GBps": 2 * nbytes / (cms / 1e3) / 1e9}
        # two more reference kernels for the counter scale: a read-only 1 GiB
        # sum and a write-only 1 GiB fill
        tot = src.sum()
        dst.fill_(2.0)
        torch.cuda.synchronize()
        result["copy_calibration"]["sum_check"] = float(tot)
    del src, dst

    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(m, seed, P, G, args.cpu_budget,
                          None if args.no_ttt else precision_state)
        if "precision_check" in cb and "forms" in result:
            result["forms"]["precision_coupled"]["vs_fp64_oracle_sampled_pairs"] = cb["precision_check"]
        ttt = result.get("time_to_1pct")
        if ttt is not None:
            # the same sweeps (burn-in + samples) the GPU needed, at the oracle's rate for all P pairs
            sweeps = ttt["burn_in"] + ttt["sample_sweeps"]
            cb["time_to_1pct_s_extrapolated"] = sweeps * 2.0 * m.nnz * P / cb["value"]
            cb["time_to_1pct_s_extrapolated_1core"] = sweeps * 2.0 * m.nnz * P / cb["value_1core"]
            cb["time_to_1pct_note"] = (f"{sweeps} sweeps of {P} pairs (the GPU run's coupled burn-in and "
                                       f"samples) at the measured oracle rates (all cores; one core)")
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
