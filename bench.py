"""Benchmark: nnTucker MU sweeps/s and TTM TFLOP/s on 512^3 (BF16-MFMA form vs FP32 form at
equal final residual), whole Algorithm 1 per step (nnTucker -> nnCP of the core -> lift ->
residual), on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sweeps 500] [--no-cpu]

Prints ONE JSON line.  `value` is the BF16 form's nnTucker sweeps per second over the whole
timed step (nnCP, lift and the final residual included).  The FP32 form is timed the same
way and reported under "fp32_form"; both start from identical initial values and run the
same number of sweeps, and their final relative residuals (both measured against the FP32
X) are reported with their difference.

The "alg2" object times Algorithm 2 on the same tensor (nnCP of X at rank 10 with the same
sweep count and refinement, then an NMF of each CP factor with m = 20, lift, residuals), both
forms, beside one oracle sweep of the nnCP of X.

The roofline object describes the dominant kernel of the BF16 fit (its second X pass,
pass2y_k of the fused three-way schedule, which also forms Y_1, S_0 and M_1), timed per
launch with HIP events on the fit's stream around every pass (nnc_set_timing), median of five
eager 20-sweep fits.  The plain pass kernels (the FP32 form's) are timed the same way through
nnc_ttm.  The cpu_baseline object times the FP64 oracle on a bounded sample (whole sweeps of
the same 512^3 problem), with a 1-thread estimate from one n-mode product of X.

"other_configs" measures the rest of the benchmark set, never the headline: 128^4 stored as
BF16, the 256^3 adjoint (forward + backward), 64^5 with 64 batched nnCP restarts, and the
real-valued CANDELINC path at 512^3.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "nnTucker MU iters/s + TTM TFLOP/s, 512³: BF16-MFMA vs FP32 at equal residual"
HBM_PEAK_GBS = 8000.0
SEED = 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PASS_SOURCES = ["paper_1909_07570_amd/csrc/pass_kernels.hip", "paper_1909_07570_amd/csrc/fused3_kernels.hip"]
COUNTERS = os.path.join(ROOT, "profiles", "pass_counters_512cubed.json")
N_COPY = 128 << 20
# The R = 20 (two 16-wide rank tiles) instantiations of the four pass kernels, X bytes per entry.
PASS_BYTES = (("ttm_last_lds_k<true, 2", 512 ** 3 * 2 + 512 * 512 * 20 * 4),
              ("ttm_mid_lds_k<2, false>", 512 ** 3 * 2 + 512 * 512 * 20 * 4),
              ("ttm_last_lds_k<false, 2", 512 ** 3 * 4 + 512 * 512 * 20 * 4),
              ("ttm_mid_lds_f32_k<2", 512 ** 3 * 4 + 512 * 512 * 20 * 4),
              # fused three-way passes of the BF16 fit: X once, plus Y_0 (pass 1) or T and Y_1 (pass 2)
              ("pass1y_k", 512 ** 3 * 2 + 512 * 400 * 4),
              ("pass2y_k", 512 ** 3 * 2 + 512 * 512 * 20 * 4 + 512 * 400 * 4))


def sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in PASS_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_only(args):
    """Launch each plain X-streaming pass kernel (512^3, R = 20, both forms) and a plain
    512 MiB device copy a few times, then three sweeps of the BF16 fit (its fused passes):
    the workload of the rocprofv3 counter runs."""
    import torch

    import paper_1909_07570_amd as nnc
    import synth
    dev = torch.device("cuda:0")
    N, R = args.n, 20
    X32 = torch.from_numpy(synth.planted_tensor(SEED, (N, N, N), 10, zero_prob=0.5, noise=1e-3,
                                                dtype="f32")[0]).to(dev)
    Xb = nnc.nnc_convert_f32_bf16(X32)
    A = [torch.from_numpy(a).to(dev) for a in synth.init_factors(SEED, (N, N, N), (R, R, R))]
    G = torch.from_numpy(synth.init_core(SEED, (R, R, R))).to(dev)
    src = torch.ones(N_COPY, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)  # calibration: reads and writes N_COPY floats
        for Xt in (Xb, X32):
            nnc.nnc_ttm(Xt, 2, A[2])
            nnc.nnc_ttm(Xt, 0, A[0])
    # three eager sweeps of the BF16 fit: the fused passes pass1y_k / pass2y_k
    nnc.nntucker_fit(Xb, (R, R, R), 3, G, A, use_graph=False, report=False)
    torch.cuda.synchronize()
    print("kernel-only done", flush=True)


def _find(d, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit("no *%s under %s" % (suffix, d))
    return hits[0]


def summarize(args):
    """Write the profiles/ summaries from three rocprofv3 CSV output folders (kernel trace
    with --stats; --pmc FETCH_SIZE; --pmc WRITE_SIZE).  Needs no GPU."""
    import csv
    if len(args.summarize) not in (3, 5):
        raise SystemExit("--summarize takes PROF FETCH WRITE [MFMA_UTIL MFMA_FLOPS]")
    prof_dir, fetch_dir, write_dir = args.summarize[:3]
    dirs = " ".join(args.summarize)
    lines = ["# Kernel time of the bench run, 512^3 step in both forms (rocprofv3 --kernel-trace --stats)", "",
             "Command (repo root):", "",
             "    rocprofv3 --kernel-trace --stats --output-format csv -d %s -o run -- "
             "python -u bench.py --steps 1 --warmup 0 --no-cpu" % prof_dir, "",
             "The step runs 500 nnTucker sweeps per form (BF16 form: 480 sweeps of the fused three-way",
             "schedule -- pass1y_k, mu_rows_k<0>, pass2y_k, mu_rows_k<0>, small_mrows_k, mu_rows_k<1>,",
             "coreL_k -- on BF16 X + 20 general sweeps on FP32 X), nnCP rank 10 x 300 sweeps, lift and",
             "residuals.  Then Algorithm 2 twice per form, the Section 4.2 study (tiny_candelinc_k), the",
             "Section 4.3 sample, the other configurations (128^4 BF16, the 256^3 adjoint, 64^5 with",
             "64 batched restarts, long-mode passes, real-valued CANDELINC at 512^3), the plain pass",
             "kernels timed through nnc_ttm and five eager 20-sweep BF16 fits with per-pass events.",
             "Every kernel of the run is listed.", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    with open(_find(prof_dir, "kernel_stats.csv")) as f:
        rows = list(csv.DictReader(f))
    for r in rows:
        lines.append("| %s | %s | %.2f | %.2f | %.2f | %.2f | %.2f |" % (
            r["Name"].split("(")[0], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "kernel_stats_512cubed.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def counter(d, name):
        per = {}
        with open(_find(d, "counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != name:
                    continue
                key = (r["Kernel_Name"], r["Dispatch_Id"])
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        out = {}
        for (kn, _), v in per.items():
            out.setdefault(kn, []).append(v)
        return out
    fetch = counter(fetch_dir, "FETCH_SIZE")
    write = counter(write_dir, "WRITE_SIZE")

    def pick(d, key):
        ks = [k for k in d if key in k]
        if not ks:
            return None
        v = sorted(d[ks[0]])
        return v[len(v) // 2]  # median dispatch, KiB
    copy_bytes = 2 * N_COPY * 4  # the calibration kernel reads and writes N_COPY floats each
    copy_f, copy_w = pick(fetch, "MulFunctor"), pick(write, "MulFunctor")
    f_scale = (copy_bytes / 2) / (copy_f * 1024.0)
    w_scale = (copy_bytes / 2) / (copy_w * 1024.0)
    res = {"source_sha": sources_sha(), "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    alg = {}
    for key, ab in PASS_BYTES:
        fk, wk = pick(fetch, key), pick(write, key)
        if fk is None or wk is None:
            continue
        alg[key] = ab
        res["kernels"][key] = {"fetch_kib": fk, "write_kib": wk,
                               "traffic_bytes": fk * 1024 * f_scale + wk * 1024 * w_scale,
                               "alg_bytes": alg[key]}
    with open(COUNTERS, "w") as f:
        json.dump(res, f, indent=1)
    md = ["# HBM traffic of the X-streaming pass kernels, 512^3, R = 20 (rocprofv3 --pmc)", "",
          "Commands (repo root), one counter per run:", "",
          "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s -o run -- "
          "python -u bench.py --kernel-only" % fetch_dir,
          "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s -o run -- "
          "python -u bench.py --kernel-only" % write_dir,
          "    python bench.py --summarize %s" % dirs, "",
          "Calibration: a plain elementwise copy of %d MiB (FP32 multiply by 1) reads FETCH_SIZE = %.0f KiB "
          "and writes WRITE_SIZE = %.0f KiB per dispatch (the torch fill that creates its source is not used); "
          "counter KiB are scaled by %.4f (fetch) and "
          "%.4f (write) to HBM bytes." % (copy_bytes // 2 >> 20, copy_f, copy_w, f_scale, w_scale), "",
          "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled HBM bytes | algorithmic bytes | ratio |",
          "|---|---|---|---|---|---|"]
    for k, v in res["kernels"].items():
        md.append("| %s | %.0f | %.0f | %.0f | %d | %.3f |" % (
            k, v["fetch_kib"], v["write_kib"], v["traffic_bytes"], alg[k], v["traffic_bytes"] / alg[k]))
    md += ["", "Algorithmic bytes: X once (2 B or 4 B per entry) + the FP32 outputs (512 x 512 x 20 for the "
           "plain passes; Y_0 = 512 x 20 x 20 for pass1y_k, T and Y_1 = 20 x 512 x 20 for pass2y_k).",
           "Source hash of the pass kernels when measured: %s" % res["source_sha"]]
    with open(os.path.join(ROOT, "profiles", "pass_traffic_512cubed.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    if len(args.summarize) == 5:
        res["mfma"] = summarize_mfma(args.summarize[3], args.summarize[4], rows, counter, pick, dirs)
        with open(COUNTERS, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


PASS_KEYS = (("ttm_last_lds_k<true, 2", "bf16"), ("ttm_mid_lds_k<2, false>", "bf16"),
             ("ttm_last_lds_k<false, 2", "f32"), ("ttm_mid_lds_f32_k<2", "f32"),
             ("pass1y_k", "bf16"), ("pass2y_k", "bf16"))
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3}


def summarize_mfma(util_dir, flops_dir, stats_rows, counter, pick, dirs):
    """MFMA busy fraction (rocprofv3 derived metric MfmaUtil) and MFMA FLOP per dispatch
    (MfmaFlopsBF16 / MfmaFlopsF32) of the pass kernels; achieved MFMA TFLOP/s uses the
    average kernel durations of the kernel-trace run."""
    util = counter(util_dir, "MfmaUtil")
    fb, ff = counter(flops_dir, "MfmaFlopsBF16"), counter(flops_dir, "MfmaFlopsF32")
    alg = 2.0 * 512 ** 3 * 20
    out = {}
    md = ["# MFMA use of the X-streaming pass kernels, 512^3, R = 20 (rocprofv3 --pmc)", "",
          "Commands (repo root), one counter set per run:", "",
          "    rocprofv3 --pmc MfmaUtil --output-format csv -d %s -o run -- "
          "python -u bench.py --kernel-only" % util_dir,
          "    rocprofv3 --pmc MfmaFlopsBF16 MfmaFlopsF32 --output-format csv -d %s "
          "-o run -- python -u bench.py --kernel-only" % flops_dir,
          "    python bench.py --summarize %s" % dirs, "",
          "MfmaUtil is rocprofv3's derived metric: summed SQ_VALU_MFMA_BUSY_CYCLES over "
          "(max GRBM_GUI_ACTIVE x SIMD count), in percent.  MFMA FLOP counts what the matrix cores "
          "executed: the rank is padded to 32 (two 16-wide tiles) and the BF16 kernels multiply each X "
          "tile by the high and the low BF16 half of the FP32 factor (two MFMAs per tile), so they "
          "execute 2 x 32/20 and the FP32 kernels 32/20 times the algorithmic 2 x 512^3 x 20.  Achieved MFMA TFLOP/s divides the counted FLOP by the kernel's average "
          "duration in the kernel-trace run.", "",
          "| kernel | MfmaUtil % | MFMA GFLOP | algorithmic GFLOP | avg us | MFMA TFLOP/s | peak (dtype) | frac |",
          "|---|---|---|---|---|---|---|---|"]
    for key, dt in PASS_KEYS:
        u = pick(util, key)
        fl = pick(fb if dt == "bf16" else ff, key)
        hit = [r for r in stats_rows if key in r["Name"]]
        if u is None or fl is None or not hit:
            continue
        avg_us = float(hit[0]["AverageNs"]) / 1e3
        tf = fl / (avg_us * 1e-6) / 1e12
        out[key] = {"mfma_util_pct": u, "mfma_flop": fl, "alg_flop": alg, "avg_us": avg_us,
                    "mfma_tflops": tf, "peak_tflops": MFMA_PEAK_TFLOPS[dt]}
        md.append("| %s | %.2f | %.2f | %.2f | %.2f | %.2f | %.0f (%s) | %.4f |" % (
            key, u, fl / 1e9, alg / 1e9, avg_us, tf, MFMA_PEAK_TFLOPS[dt], dt, tf / MFMA_PEAK_TFLOPS[dt]))
    md += ["", "Source hash of the pass kernels when measured: %s" % sources_sha()]
    with open(os.path.join(ROOT, "profiles", "pass_mfma_512cubed.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    return out


def extra_studies(args, nnc, dev, Xb, X32, dims, ranks, rank, R):
    """Algorithm 2 on the 512^3 tensor, the Section 4.2 study and a sample of the Section 4.3
    study (the objects "alg2", "restart_study" and "sec43_study" of the JSON line)."""
    import torch

    import synth
    # ---- Algorithm 2 on the same tensor: nnCP of X (rank 10), NMF of each factor (m = 20),
    # lift, residual; both forms from identical initial values.
    Bx0 = [torch.from_numpy(b).to(dev) for b in synth.init_cp_factors(SEED, dims, rank)]
    W0, H0 = synth.init_nmf(SEED, dims, ranks, rank)
    W0 = [torch.from_numpy(w).to(dev) for w in W0]
    H0 = [torch.from_numpy(h).to(dev) for h in H0]
    wsx = torch.empty(nnc.nncpx_workspace_bytes(dims, rank), dtype=torch.uint8, device=dev)
    Bx = [torch.empty_like(b) for b in Bx0]
    Wf = [torch.empty_like(w) for w in W0]
    Hf = [torch.empty_like(h) for h in H0]

    def alg2_step(bf16: bool):
        for b, b0 in zip(Bx, Bx0):
            b.copy_(b0)
        for w, w0 in zip(Wf, W0):
            w.copy_(w0)
        for h, h0 in zip(Hf, H0):
            h.copy_(h0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        if bf16:
            nnc.nncpx_fit(Xb, rank, args.sweeps, Bx, x_fp32=X32, fp32_final_sweeps=args.fp32_final,
                          report=False, workspace=wsx)
        else:
            nnc.nncpx_fit(X32, rank, args.sweeps, Bx, report=False, workspace=wsx)
        torch.cuda.synchronize()
        t_cp = time.perf_counter() - t
        t = time.perf_counter()
        nnc.nmf_fit_batched(Bx, [R] * 3, args.cp_sweeps, Wf, Hf, residual=False)
        C = nnc.nncandelinc_lift(Wf, Hf)
        torch.cuda.synchronize()
        t_nmf = time.perf_counter() - t
        return t_cp, t_nmf, nnc.reconstruct_residual(X32, Bx), nnc.reconstruct_residual(X32, C)

    alg2 = {}
    for form, bf16 in (("bf16", True), ("fp32", False)):
        alg2_step(bf16)  # warm-up
        t_cp, t_nmf, rel_x, rel_l = alg2_step(bf16)
        alg2[form] = {"sweeps_per_s": round(args.sweeps / t_cp, 2), "nncp_x_ms": round(t_cp * 1e3, 3),
                      "nmf_lift_ms": round(t_nmf * 1e3, 3), "cp_x_rel": rel_x, "lifted_rel": rel_l}
        log("alg2 %s: nnCP of X %.1f ms (%.0f sweeps/s), NMF+lift %.1f ms, rel %.6g, lifted rel %.6g"
            % (form, t_cp * 1e3, args.sweeps / t_cp, t_nmf * 1e3, rel_x, rel_l))
    alg2["abs_diff_cp_x_rel"] = abs(alg2["bf16"]["cp_x_rel"] - alg2["fp32"]["cp_x_rel"])
    alg2["config"] = ("Algorithm 2 on the same 512^3 tensor: nnCP rank %d, %d MU sweeps (BF16 form: last %d "
                      "on FP32 X); NMF of each factor with m = %d, %d sweeps; lift; residuals"
                      % (rank, args.sweeps, args.fp32_final, R, args.cp_sweeps))

    # ---- the Section 4.2 study: 1000 starts x 5000 sweeps per sub-fit, both algorithms, four
    # assumed multiranks, on the 4x4x4 example with known nnCPD (rank 4)
    from tests.paper_fixtures import examples
    ex = examples()["ex5_rank_not_preserved_nn"]
    At = [np.asarray(ex[k], dtype=np.float64) for k in ("A1", "A2", "A3")]
    Xs = torch.from_numpy(np.einsum("ir,jr,kr->ijk", *At).astype(np.float32)).to(dev)
    truth = [torch.from_numpy(a.astype(np.float32)).to(dev) for a in At]
    study = {"config": "Section 4.2: the 4x4x4 example (nonnegative rank 4, unique nnCPD), %d random starts "
                       "per (algorithm, multirank), %d sweeps per sub-fit, one launch per configuration"
                       % (args.restarts, args.restart_sweeps), "runs": []}
    for alg in (1, 2):
        for m in ((3, 3, 3), (3, 4, 4), (4, 4, 4), (5, 5, 5)):
            inits = torch.from_numpy(synth.init_restarts(SEED, alg, (4, 4, 4), m, 4, args.restarts)).to(dev)
            nnc.nncandelinc_restarts(Xs, alg, m, 4, inits[:8], 10, 10, truth=truth)  # warm-up
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = nnc.nncandelinc_restarts(Xs, alg, m, 4, inits, args.restart_sweeps, args.restart_sweeps,
                                           truth=truth)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            rel = res.rel_errors.cpu().numpy()
            cg = res.congruences.cpu().numpy()
            study["runs"].append({"algorithm": alg, "multirank": list(m), "seconds": round(el, 4),
                                  "starts_per_s": round(args.restarts / el, 1),
                                  "rel_error": {"mean": float(rel.mean()), "median": float(np.median(rel)),
                                                "std": float(rel.std()), "min": float(rel.min())},
                                  "congruence": {"mean": float(cg.mean()), "std": float(cg.std())}})
            log("study alg %d m %s: %.1f ms, rel mean %.4g median %.4g, congruence %.4f"
                % (alg, m, el * 1e3, rel.mean(), np.median(rel), cg.mean()))

    sec43 = sec43_study(nnc, dev, args.sec43_tensors, args.restart_sweeps)
    return alg2, study, sec43


def sec43_study(nnc, dev, n_tensors: int, sweeps: int, progress_every: int = 0):
    """The Section 4.3 study on tensors 0 .. n_tensors - 1 of its generator: 40^3, nonnegative
    rank 5, canonical multiranks [3, 4, 5] (factors C_n = F_n B_n meeting Kruskal's criterion);
    Algorithms 1 and 2 on each, `sweeps` sweeps per sub-fit, scored against the generating C_n."""
    import torch

    import synth
    d43, m43, r43 = (40, 40, 40), (3, 4, 5), 5
    rows43, t43 = [], {1: 0.0, 2: 0.0}

    def T(a):
        return torch.from_numpy(a).to(dev)
    for j in range(n_tensors):
        X43, _, _, Ctrue = synth.rank_deficient_tensor(43, j, d43, m43, r43)
        ini = synth.init_sec43(43, j, d43, m43, r43)
        Xd43 = T(X43)
        Ct = [T(c) for c in Ctrue]
        torch.cuda.synchronize()
        t = time.perf_counter()
        G43, A43, Bc43 = T(ini["G"]), [T(a) for a in ini["A"]], [T(b) for b in ini["Bc"]]
        nnc.nntucker_fit(Xd43, m43, sweeps, G43, A43, report=False)
        nnc.nncp_fit(G43, r43, sweeps, Bc43, residual=False)
        C1 = nnc.nncandelinc_lift(A43, Bc43)
        torch.cuda.synchronize()
        t43[1] += time.perf_counter() - t
        t = time.perf_counter()
        Bx43, W43, H43 = [T(b) for b in ini["Bx"]], [T(w) for w in ini["W"]], [T(h) for h in ini["H"]]
        nnc.nncandelinc_alg2(Xd43, r43, m43, sweeps, sweeps, Bx43, W43, H43)
        C2 = nnc.nncandelinc_lift(W43, H43)
        torch.cuda.synchronize()
        t43[2] += time.perf_counter() - t
        rows43.append((nnc.reconstruct_residual(Xd43, C1), nnc.mean_congruence(C1, Ct),
                       nnc.reconstruct_residual(Xd43, C2), nnc.mean_congruence(C2, Ct)))
        if progress_every and (j + 1) % progress_every == 0:
            log("sec43: %d / %d tensors" % (j + 1, n_tensors))
    a43 = np.array(rows43)
    out = {"config": "Section 4.3: %d generated 40^3 tensors (nonnegative rank 5, canonical multiranks "
                     "[3,4,5], Kruskal criterion), Algorithms 1 and 2 at multirank [3,4,5], rank 5, %d sweeps "
                     "per sub-fit" % (n_tensors, sweeps)}
    for alg, (cr, cc) in ((1, (0, 1)), (2, (2, 3))):
        out["algorithm_%d" % alg] = {
            "seconds_per_tensor": round(t43[alg] / max(1, n_tensors), 4),
            "rel_error": {"mean": float(a43[:, cr].mean()), "median": float(np.median(a43[:, cr])),
                          "p90": float(np.percentile(a43[:, cr], 90))},
            "congruence": {"mean": float(a43[:, cc].mean()), "median": float(np.median(a43[:, cc])),
                           "p10": float(np.percentile(a43[:, cc], 10))}}
    out["alg2_lower_error_fraction"] = float(np.mean(a43[:, 2] < a43[:, 0]))
    out["alg2_higher_congruence_fraction"] = float(np.mean(a43[:, 3] > a43[:, 1]))
    log("sec43: alg1 rel median %.3g cong %.4f (%.2f s/tensor); alg2 rel median %.3g cong %.4f (%.2f s/tensor)"
        % (np.median(a43[:, 0]), a43[:, 1].mean(), t43[1] / max(1, n_tensors), np.median(a43[:, 2]),
           a43[:, 3].mean(), t43[2] / max(1, n_tensors)))
    return out


def pass_split(nnc, fit):
    """Run `fit()` (a fit with a report) with per-pass timing on: ((ms, launches) of pass 1,
    (ms, launches) of pass 2), HIP events on the fit's stream around every X-pass launch."""
    nnc.set_timing(True)
    try:
        fit()
    finally:
        nnc.set_timing(False)
    return nnc.last_pass_times()


def pass_roofline(times, bytes1, bytes2, names):
    """Per-pass average launch time and achieved HBM rate from pass_split's result."""
    out = {}
    for (ms, n), b, name in zip(times, (bytes1, bytes2), names):
        if n <= 0:
            continue
        us = ms / n * 1e3
        out[name] = {"avg_us": round(us, 2), "alg_bytes_per_launch": int(b),
                     "GB/s": round(b / (us * 1e-6) / 1e9, 1), "frac": round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "launches": int(n)}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def one_thread_ratio(oracle, X64, A):
    """Seconds of one n-mode product of X (the oracle's unit of work on X) at all cores and at
    1 thread; their ratio scales an all-cores rate to a 1-thread estimate."""
    n = X64.ndim - 1
    t = time.perf_counter()
    oracle.ttm_t(X64, n, A)
    t_all = time.perf_counter() - t
    threads = oracle.get_threads()
    oracle.set_threads(1)
    try:
        t = time.perf_counter()
        oracle.ttm_t(X64, n, A)
        t_one = time.perf_counter() - t
    finally:
        oracle.set_threads(threads)
    return t_all, t_one


def extra_workloads(args, nnc, dev):
    """The other configurations of the benchmark set, each with its own timing (never the
    headline): 128^4 stored BF16, the 256^3 adjoint, 64^5 with batched nnCP restarts, and the
    real-valued CANDELINC path at 512^3."""
    import torch

    import synth
    from tests.gpu_util import planted_tensor_dev, signed_planted_dev
    out = {}

    def timed(fn, reps=1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, r

    # ---- 128^4 stored as BF16: nnTucker 16^4, 500 sweeps (BF16 form: last 20 on the exact FP32
    # widening of the stored values; FP32 form: every sweep on that widening), nnCP rank 8, lift
    dims, ranks, seed = (128,) * 4, (16,) * 4, 3
    Xb = nnc.nnc_convert_f32_bf16(planted_tensor_dev(seed, dims, 8))
    X32 = Xb.float()
    G0 = torch.from_numpy(synth.init_core(seed, ranks)).to(dev)
    A0 = [torch.from_numpy(a).to(dev) for a in synth.init_factors(seed, dims, ranks)]
    B0 = [torch.from_numpy(b).to(dev) for b in synth.init_cp_factors(seed, ranks, 8)]
    ws = torch.empty(nnc.nntucker_workspace_bytes(dims, ranks), dtype=torch.uint8, device=dev)
    c3 = {"workload": "128^4 planted rank-8 tensor stored as BF16 (X formed on the GPU from the seeded draws); "
                      "nnTucker multirank 16^4, %d sweeps; nnCP rank 8, 300 sweeps; lift" % args.sweeps}
    for form, bf in (("bf16", True), ("fp32", False)):
        G = G0.clone()
        A = [a.clone() for a in A0]
        B = [b.clone() for b in B0]
        if bf:
            fit = lambda: nnc.nntucker_fit(Xb, ranks, args.sweeps, G, A, x_fp32=X32, fp32_final_sweeps=20,
                                           report=False, workspace=ws)
        else:
            fit = lambda: nnc.nntucker_fit(X32, ranks, args.sweeps, G, A, report=False, workspace=ws)
        el, _ = timed(fit)
        elc, _ = timed(lambda: nnc.nncp_fit(G, 8, 300, B, residual=False))
        C = nnc.nncandelinc_lift(A, B)
        c3[form] = {"sweeps_per_s": round(args.sweeps / el, 1), "nncp_ms": round(elc * 1e3, 3),
                    "tucker_rel": nnc.reconstruct_residual(X32, A, G), "lifted_rel": nnc.reconstruct_residual(X32, C)}
        G = G0.clone()
        A = [a.clone() for a in A0]
        Xs = Xb if bf else X32
        times = pass_split(nnc, lambda: nnc.nntucker_fit(Xs, ranks, 20, G, A, workspace=ws))
        size, esz = 128 ** 4, (2 if bf else 4)
        c3[form]["passes"] = pass_roofline(times, size * esz + size // 128 * 16 * 4, size * esz + size // 128 * 16 * 4,
                                           ("pass1_x_x3", "pass2_x_x0"))
        log("c3 %s: %s" % (form, json.dumps(c3[form])))
    del Xb, X32, ws
    out["c3_128x4_bf16"] = c3

    # ---- 256^3 adjoint: L = 0.5 ||X - G x {A}||^2 and its gradient (core 32^3, factors 256 x 32)
    dims, ranks, seed = (256,) * 3, (32,) * 3, 4
    X = planted_tensor_dev(seed, dims, 12, zero_prob=0.3)
    G = torch.from_numpy(synth.init_core(seed, ranks)).to(dev).requires_grad_(True)
    A = [torch.from_numpy(a).to(dev).requires_grad_(True) for a in synth.init_factors(seed, dims, ranks)]

    def fwd_bwd():
        for t in [G] + A:
            t.grad = None
        loss = nnc.nntucker_loss(X, G, A)
        loss.backward()
        return loss
    timed(fwd_bwd, 3)
    el, loss = timed(fwd_bwd, 20)
    size = 256 ** 3
    alg = 3 * size * 4 + 2 * (size // 256) * 32 * 4  # three reads of X, P and T written once each
    out["c4_256x3_adjoint"] = {
        "workload": "256^3 FP32 planted rank-12 tensor (30 % zeros); loss and gradient at the seeded point, "
                    "core 32^3, factors 256 x 32 (autograd: forward residual pass + nntucker_grad)",
        "fwd_bwd_ms": round(el * 1e3, 3), "loss": float(loss.detach()),
        "alg_bytes": alg, "GB/s": round(alg / el / 1e9, 1), "frac_of_hbm": round(alg / el / 1e9 / HBM_PEAK_GBS, 4),
        "note": "X (64 MiB) fits in the 256 MiB MALL, so the three reads of one call can exceed the HBM rate"}
    log("c4: %s" % json.dumps(out["c4_256x3_adjoint"]))
    del X, G, A

    # ---- 64^5 FP32 (4 GiB): nnTucker 8^5, 300 sweeps; 64 batched nnCP restarts of its core
    dims, ranks, seed = (64,) * 5, (8,) * 5, 5
    X = planted_tensor_dev(seed, dims, 6)
    G = torch.from_numpy(synth.init_core(seed, ranks)).to(dev)
    A = [torch.from_numpy(a).to(dev) for a in synth.init_factors(seed, dims, ranks)]
    A5 = [a.clone() for a in A]
    ws = torch.empty(nnc.nntucker_workspace_bytes(dims, ranks), dtype=torch.uint8, device=dev)
    el, _ = timed(lambda: nnc.nntucker_fit(X, ranks, 300, G, A, report=False, workspace=ws))
    rks = [2 + (j % 15) for j in range(64)]
    Bs = [[torch.from_numpy(b).to(dev) for b in synth.init_cp_factors(seed, ranks, r, restart=j)]
          for j, r in enumerate(rks)]
    nnc.nncp_fit_batched(G, rks, 1, [[b.clone() for b in bs] for bs in Bs])  # tunes (or reads the cache)
    tune = nnc.last_tune()
    elb, res = timed(lambda: nnc.nncp_fit_batched(G, rks, 300, Bs))
    Gt = torch.from_numpy(synth.init_core(seed, ranks)).to(dev)
    At = [a.clone() for a in A5]
    times = pass_split(nnc, lambda: nnc.nntucker_fit(X, ranks, 10, Gt, At, workspace=ws))
    size = 64 ** 5
    out["c5_64x5"] = {
        "workload": "64^5 FP32 planted rank-6 tensor (4 GiB, formed on the GPU); nnTucker multirank 8^5, "
                    "300 sweeps; 64 nnCP restarts of the 8^5 core (ranks 2..16), 300 sweeps each, one launch",
        "sweeps_per_s": round(300 / el, 1), "tucker_rel": nnc.reconstruct_residual(X, A, G),
        "batched_nncp_ms": round(elb * 1e3, 3), "best_restart_rel": float(min(res)),
        "batched_nncp_launch": tune,
        "passes": pass_roofline(times, size * 4 + size // 64 * 8 * 4, size * 4 + size // 64 * 8 * 4,
                                ("pass1_x_x4", "pass2_x_x0"))}
    log("c5: %s" % json.dumps(out["c5_64x5"]))
    del X, ws

    # ---- X passes over modes longer than one launch's factor in LDS (chunked contracted index)
    longm = {}
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    for shape, mode in (((1024, 512, 512), 0), ((512, 512, 1024), 2)):
        X = torch.rand(shape, generator=gen, device=dev)
        Fm = torch.rand((shape[mode], 20), generator=gen, device=dev)
        for form, Xt, esz in (("bf16", nnc.nnc_convert_f32_bf16(X), 2), ("fp32", X, 4)):
            o_t = nnc.nnc_ttm(Xt, mode, Fm)
            timed(lambda: nnc.nnc_ttm(Xt, mode, Fm, o_t), 3)
            el, _ = timed(lambda: nnc.nnc_ttm(Xt, mode, Fm, o_t), 10)
            b = X.numel() * esz + o_t.numel() * 4
            longm["%dx%dx%d_mode%d_%s" % (shape + (mode, form))] = {
                "kernel": nnc.last_ttm_kernel(), "avg_us": round(el * 1e6, 2), "alg_bytes": b,
                "GB/s": round(b / el / 1e9, 1), "frac": round(b / el / 1e9 / HBM_PEAK_GBS, 4),
                "note": "back-to-back launches timed with host clocks around a synchronize"}
            del o_t
        del X
    out["long_mode_passes"] = longm
    log("long modes: %s" % json.dumps(longm))

    # ---- real-valued CANDELINC, 512^3 signed planted rank-20 CP: Tucker 20^3 by alternating
    # least squares (25 sweeps), CP rank 20 of the core by alternating least squares (300), lift
    dims, ranks, seed = (512,) * 3, (20,) * 3, 7
    X = signed_planted_dev(seed, dims, 20, noise=1e-3)
    Xb = nnc.nnc_convert_f32_bf16(X)
    G0 = torch.from_numpy(synth.init_core(seed, ranks)).to(dev)
    A0 = [torch.from_numpy(a).to(dev) for a in synth.init_factors(seed, dims, ranks)]
    B0 = [torch.from_numpy(2.0 * b - 1.0).to(dev) for b in synth.init_cp_factors(seed, ranks, 20)]
    real = {"workload": "512^3 FP32 real tensor: planted rank-20 CP with U[-1,1) factors + U[-1e-3,1e-3) noise; "
                        "Tucker 20^3 by alternating least squares with orthonormalized factors, 25 sweeps; "
                        "CP rank 20 of the core by alternating least squares, 300 sweeps; lift"}
    for form, bf in (("bf16", True), ("fp32", False)):
        G = G0.clone()
        A = [a.clone() for a in A0]
        B = [b.clone() for b in B0]
        if bf:
            fit = lambda: nnc.tucker_ls_fit(Xb, ranks, 25, G, A, x_fp32=X, fp32_final_sweeps=5, report=False)
        else:
            fit = lambda: nnc.tucker_ls_fit(X, ranks, 25, G, A, report=False)
        el, _ = timed(fit)
        elc, _ = timed(lambda: nnc.cp_ls_fit(G, 20, 300, B, residual=False))
        C = nnc.nncandelinc_lift(A, B)
        real[form] = {"sweeps_per_s": round(25 / el, 1), "cp_ls_ms": round(elc * 1e3, 3),
                      "tucker_rel": nnc.reconstruct_residual(X, A, G), "lifted_rel": nnc.reconstruct_residual(X, C)}
        log("real %s: %s" % (form, json.dumps(real[form])))
    out["real_candelinc_512"] = real

    if not args.no_cpu:
        import oracle
        cpu = {"cpu_model": cpu_model(), "threads": oracle.get_threads()}
        # the real path: one oracle sweep at all cores, the 1-thread figure from one n-mode product
        X64 = X.double().cpu().numpy()
        g0 = synth.init_core(seed, ranks).astype(np.float64)
        a0 = [a.astype(np.float64) for a in synth.init_factors(seed, dims, ranks)]
        t = time.perf_counter()
        oracle.tucker_ls(X64, g0, a0, 1)
        el = time.perf_counter() - t
        t_all, t_one = one_thread_ratio(oracle, X64, a0[2])
        cpu["real_candelinc_512"] = {
            "value": round(1.0 / el, 4), "unit": "least-squares sweeps/s", "kind": "oracle",
            "sample": "1 FP64 sweep (with the orthonormalization of the initial factors), %.1f s" % el,
            "one_thread_estimate": round(1.0 / el * t_all / t_one, 5),
            "one_thread_basis": "one 512^3 x 20 n-mode product of X: %.2f s at %d threads, %.2f s at 1 thread; "
                                "the all-cores rate scaled by that ratio" % (t_all, oracle.get_threads(), t_one)}
        del X64
        log("cpu extras: %s" % json.dumps(cpu))
        out["cpu_baseline"] = cpu
    del X, Xb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=500)
    ap.add_argument("--fp32-final", type=int, default=20)
    ap.add_argument("--cp-sweeps", type=int, default=300)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="the oracle baseline runs whole sweeps until this much time has passed")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--restarts", type=int, default=1000)
    ap.add_argument("--restart-sweeps", type=int, default=5000)
    ap.add_argument("--sec43-tensors", type=int, default=8)
    ap.add_argument("--no-studies", action="store_true",
                    help="skip Algorithm 2 and the Section 4.2 / 4.3 studies (diagnostic runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 128^4, 256^3 adjoint, 64^5 and real-valued CANDELINC measurements")
    ap.add_argument("--sec43-only", action="store_true",
                    help="only the Section 4.3 study (progress on stderr, one JSON line)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only launch the pass kernels and a calibration copy (counter runs)")
    ap.add_argument("--summarize", nargs="+", metavar="DIR",
                    help="PROF FETCH WRITE [MFMA_UTIL MFMA_FLOPS]: write profiles/ summaries from "
                         "rocprofv3 CSV output folders (no GPU needed)")
    args = ap.parse_args()
    if args.summarize:
        summarize(args)
        return
    if args.kernel_only:
        kernel_only(args)
        return
    if args.sec43_only:
        import torch

        import paper_1909_07570_amd as nnc
        if not torch.cuda.is_available() or not nnc.device_ok():
            raise SystemExit("bench.py needs an MI355X (gfx950) GPU and the built library")
        print(json.dumps(sec43_study(nnc, torch.device("cuda:0"), args.sec43_tensors, args.restart_sweeps,
                                     progress_every=25)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1909_07570_amd as nnc
    import synth

    if not torch.cuda.is_available() or not nnc.device_ok():
        raise SystemExit("bench.py needs an MI355X (gfx950) GPU and the built library")
    dev = torch.device("cuda:0")
    N, R, rank = args.n, 20, 10
    dims, ranks = (N, N, N), (R, R, R)

    t0 = time.time()
    X32h, _ = synth.planted_tensor(SEED, dims, 10, zero_prob=0.5, noise=1e-3, dtype="f32")
    log("generated X %s in %.1fs" % (dims, time.time() - t0))
    X32 = torch.from_numpy(X32h).to(dev)
    G0 = torch.from_numpy(synth.init_core(SEED, ranks)).to(dev)
    A0 = [torch.from_numpy(a).to(dev) for a in synth.init_factors(SEED, dims, ranks)]
    B0 = [torch.from_numpy(b).to(dev) for b in synth.init_cp_factors(SEED, ranks, rank)]
    torch.cuda.synchronize()
    tc = time.time()
    Xb = nnc.nnc_convert_f32_bf16(X32)
    torch.cuda.synchronize()
    convert_ms = (time.time() - tc) * 1e3

    ws = torch.empty(nnc.nntucker_workspace_bytes(dims, ranks), dtype=torch.uint8, device=dev)
    G = torch.empty_like(G0)
    A = [torch.empty_like(a) for a in A0]
    B = [torch.empty_like(b) for b in B0]

    def step(bf16: bool):
        G.copy_(G0)
        for a, a0 in zip(A, A0):
            a.copy_(a0)
        for b, b0 in zip(B, B0):
            b.copy_(b0)
        if bf16:
            nnc.nntucker_fit(Xb, ranks, args.sweeps, G, A, x_fp32=X32,
                             fp32_final_sweeps=args.fp32_final, report=False, workspace=ws)
        else:
            nnc.nntucker_fit(X32, ranks, args.sweeps, G, A, report=False, workspace=ws)
        nnc.nncp_fit(G, rank, args.cp_sweeps, B, residual=False)
        C = nnc.nncandelinc_lift(A, B)
        cp_rel = nnc.reconstruct_residual(X32, C)
        tucker_rel = nnc.reconstruct_residual(X32, A, G)
        return tucker_rel, cp_rel

    results = {}
    for form, bf16 in (("bf16", True), ("fp32", False)):
        for _ in range(args.warmup):
            step(bf16)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            tucker_rel, cp_rel = step(bf16)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        results[form] = dict(seconds=el, ms_per_step=el / args.steps * 1e3,
                             sweeps_per_s=args.sweeps * args.steps / el,
                             tucker_rel=tucker_rel, cp_rel=cp_rel)
        log("%s: %.1f ms/step, %.0f sweeps/s, tucker rel %.6g, lifted rel %.6g"
            % (form, results[form]["ms_per_step"], results[form]["sweeps_per_s"], tucker_rel, cp_rel))

    alg2, study, sec43 = {}, {}, {}
    if not args.no_studies:
        alg2, study, sec43 = extra_studies(args, nnc, dev, Xb, X32, dims, ranks, rank, R)
    extras = {}
    if not args.no_extras:
        extras = extra_workloads(args, nnc, dev)

    # ---- per-launch timing of the two X-streaming contractions (same kernels, same launch
    # configuration as inside the fit), HIP events on the stream they are launched on:
    # kGroups groups of back-to-back launches, each group's average, and the median group
    # (one disturbed group of launches does not move it; every group is reported).
    size = N ** 3
    kGroups = 5
    def time_kernel(Xt, mode, A_):
        out = torch.empty([N, N, R] if mode == 2 else [R, N, N], dtype=torch.float32, device=dev)
        for _ in range(3):
            nnc.nnc_ttm(Xt, mode, A_, out)
        s = torch.cuda.current_stream()
        groups = []
        for _ in range(kGroups):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(args.kernel_reps):
                nnc.nnc_ttm(Xt, mode, A_, out)
            e1.record(s)
            torch.cuda.synchronize()
            groups.append(e0.elapsed_time(e1) / args.kernel_reps)
        return sorted(groups)[kGroups // 2], groups
    kern = {}
    for name, Xt, esz in (("bf16", Xb, 2), ("fp32", X32, 4)):
        for mode, kname in ((2, "ttm_last"), (0, "ttm_mid")):
            ms, groups = time_kernel(Xt, mode, A0[mode])
            bytes_ = size * esz + size // N * R * 4
            kern["%s_%s" % (kname, name)] = dict(
                avg_us=ms * 1e3, gbs=bytes_ / (ms * 1e-3) / 1e9,
                tflops=2.0 * size * R / (ms * 1e-3) / 1e12, alg_bytes=bytes_,
                group_avg_us=[round(g * 1e3, 2) for g in groups])
            log("%s_%s: %.1f us, %.0f GB/s, %.1f TFLOP/s" % (kname, name, ms * 1e3,
                kern["%s_%s" % (kname, name)]["gbs"], kern["%s_%s" % (kname, name)]["tflops"]))
    # The BF16 fit's own passes (the fused three-way schedule: pass1y_k forms Y_0 = X x_2 A_2^T
    # x_1 A_1^T and M_0, pass2y_k writes T = X x_0 A_0^T and forms Y_1, S_0 and M_1), timed
    # per launch with HIP events around each pass on the fit's stream, over an eager fit of
    # 20 sweeps: kGroups such fits, the median group's per-launch averages.
    size_yx = N * R * R  # Y_0 = N x R x R,  Y_1 = R x N x R
    alg_p1 = size * 2 + size_yx * 4
    alg_p2 = size * 2 + size // N * R * 4 + size_yx * 4
    fused = []
    for _ in range(kGroups):
        G.copy_(G0)
        for a, a0 in zip(A, A0):
            a.copy_(a0)
        fused.append(pass_roofline(pass_split(nnc, lambda: nnc.nntucker_fit(Xb, ranks, 20, G, A, workspace=ws)),
                                   alg_p1, alg_p2, ("pass1y_k", "pass2y_k")))
    infit = {}
    for key in ("pass1y_k", "pass2y_k"):
        us = sorted(f[key]["avg_us"] for f in fused)
        med = us[kGroups // 2]
        b = fused[0][key]["alg_bytes_per_launch"]
        infit[key] = {"avg_us": med, "group_avg_us": us, "alg_bytes_per_launch": b,
                      "GB/s": round(b / (med * 1e-6) / 1e9, 1), "frac": round(b / (med * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        log("%s in the BF16 fit: %.2f us, %.0f GB/s" % (key, med, infit[key]["GB/s"]))
    dom = max(infit, key=lambda k: infit[k]["avg_us"])
    dk = infit[dom]
    traffic = None
    if os.path.exists(COUNTERS):
        cnt = json.load(open(COUNTERS))
        if cnt.get("source_sha") == sources_sha() and dom in cnt.get("kernels", {}):
            traffic = round(cnt["kernels"][dom]["traffic_bytes"])
    roofline = {"bound": "hbm", "achieved": dk["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["frac"], "traffic": traffic, "kernel": dom,
                "avg_us": dk["avg_us"], "alg_bytes_per_launch": dk["alg_bytes_per_launch"]}

    cpu = None
    if not args.no_cpu:
        import oracle
        X64 = X32h.astype(np.float64)
        g0 = synth.init_core(SEED, ranks).astype(np.float64)
        a0 = [a.astype(np.float64) for a in synth.init_factors(SEED, dims, ranks)]
        t = time.perf_counter()
        done = 0
        while True:
            g0, a0, _, _ = oracle.nntucker(X64, g0, a0, 1)
            done += 1
            el = time.perf_counter() - t
            if el >= args.cpu_seconds:
                break
        t_all, t_one = one_thread_ratio(oracle, X64, a0[2])
        cpu = {"value": round(done / el, 5), "unit": "MU sweeps/s", "cores": oracle.get_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": "%d whole FP64 nnTucker sweeps of the same 512^3 problem (multirank 20^3) from the "
                         "same initial values, %.1f s (no extrapolation)" % (done, el),
               "one_thread_estimate": round(done / el * t_all / t_one, 5),
               "one_thread_basis": "one 512^3 x 20 n-mode product of X: %.2f s at %d threads, %.2f s at 1 "
                                   "thread; the all-cores rate scaled by that ratio"
                                   % (t_all, oracle.get_threads(), t_one)}
        if not args.no_studies:
            t = time.perf_counter()
            b0x = [b.astype(np.float64) for b in synth.init_cp_factors(SEED, dims, rank)]
            oracle.nncp(X64, b0x, 1)
            el_cpx = time.perf_counter() - t
            alg2["cpu_baseline"] = {"value": round(1.0 / el_cpx, 5), "unit": "nnCP-of-X MU sweeps/s",
                                    "cores": oracle.get_threads(), "kind": "oracle",
                                    "sample": "1 FP64 nnCP sweep of the 512^3 tensor, rank %d, %.1f s"
                                              % (rank, el_cpx)}
            from tests.paper_fixtures import examples
            ex = examples()["ex5_rank_not_preserved_nn"]
            At = [np.asarray(ex[k], dtype=np.float64) for k in ("A1", "A2", "A3")]
            Xe = np.einsum("ir,jr,kr->ijk", *At)
            inits1 = synth.init_restarts(SEED, 1, (4, 4, 4), (4, 4, 4), 4, 2)
            t = time.perf_counter()
            done = 0
            for j in range(2):
                parts = synth.unpack_restart(inits1[j].astype(np.float64), 1, (4, 4, 4), (4, 4, 4), 4)
                oracle.restart_fit(Xe, 1, parts, args.restart_sweeps, args.restart_sweeps, truth=At)
                done += 1
            el_rs = time.perf_counter() - t
            study["cpu_baseline"] = {"value": round(done / el_rs, 3),
                                     "unit": "starts/s (Algorithm 1, multirank [4,4,4])",
                                     "cores": oracle.get_threads(), "kind": "oracle",
                                     "sample": "%d starts of %d + %d sweeps, %.1f s"
                                               % (done, args.restart_sweeps, args.restart_sweeps, el_rs)}
        del X64

    bf, fp = results["bf16"], results["fp32"]
    sweep_flops = 2.0 * size * (R + R)  # the two X-streaming contractions of one sweep
    line = {
        "metric": METRIC, "value": round(bf["sweeps_per_s"], 2), "unit": "MU sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(bf["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "512^3 FP32 planted rank-10 tensor (U[0,1) factors zeroed w.p. 0.5, "
                               "U[0,1e-3) noise); nnTucker multirank (20,20,20), %d MU sweeps "
                               "(BF16-MFMA, last %d on FP32 X); nnCP rank %d, %d sweeps; lift; "
                               "residuals" % (args.sweeps, args.fp32_final, rank, args.cp_sweeps),
                   "dims": list(dims), "multirank": list(ranks), "cp_rank": rank,
                   "sweeps": args.sweeps, "fp32_final_sweeps": args.fp32_final},
        "ttm_tflops": round(sweep_flops * args.sweeps / (bf["seconds"] / args.steps) / 1e12, 2),
        "ttm_kernel_tflops": {k: round(v["tflops"], 2) for k, v in kern.items()},
        "plain_pass_kernels": {k: {"avg_us": round(v["avg_us"], 2), "GB/s": round(v["gbs"], 1),
                                   "frac": round(v["gbs"] / HBM_PEAK_GBS, 4),
                                   "group_avg_us": v["group_avg_us"]} for k, v in kern.items()},
        "bf16_fit_passes": infit,
        "residuals": {"bf16_tucker": bf["tucker_rel"], "fp32_tucker": fp["tucker_rel"],
                      "bf16_lifted_cp": bf["cp_rel"], "fp32_lifted_cp": fp["cp_rel"],
                      "abs_diff_tucker": abs(bf["tucker_rel"] - fp["tucker_rel"])},
        "fp32_form": {"value": round(fp["sweeps_per_s"], 2), "unit": "MU sweeps/s",
                      "ms_per_step": round(fp["ms_per_step"], 3)},
        "bf16_speedup_vs_fp32": round(bf["sweeps_per_s"] / fp["sweeps_per_s"], 3),
        "x_to_bf16_ms": round(convert_ms, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "alg2": alg2,
        "restart_study": study,
        "sec43_study": sec43,
        "other_configs": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
