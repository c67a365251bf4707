#!/usr/bin/env python3
"""Throughput of the plain BFAST Monitor path on one MI355X.

Workload: one 1024 x 1024 tile (1,048,576 pixels), N = 400 FP32 observations,
history n = 200, k = 3 harmonics (p = 8 regressors), h = 0.25 (H = 50),
lambda = 2.5, f = 23, seeded synthetic season-trend series with 20% planted
steps (see paper_1807_01751_amd/synth.py).  Y is device-resident before the
timed region; one step is one bfm_fit_monitor call over the whole tile
(fit, sigma, MOSUM, boundary test, break index and magnitude), FP64 arithmetic.
Before the W warmup steps of every leg the step runs untimed for at least a
quarter of a second: the first tens of milliseconds of work after the GPU was
idle run at lower clocks (measured: the same launch 2x slower in the first
batch, steady after about 50 ms).

After the headline leg, the same tile with 25% of its observations missing
(NaN: half independent, half cloud runs of 3-15 rows) is timed through the
masked path (per-pixel Gram and Cholesky); it is reported under "masked".  The
mixed-precision leg ("mixed") stores the tile in FP16 (half the bytes) with the
same FP64 arithmetic, and reports how its break indices and magnitudes compare
with the float32 leg.  A serving leg ("serving") runs a stream of requests of
mixed sizes and parameters through the serving runtime under Poisson arrivals
and reports latency percentiles beside throughput.  Three method variants
follow under "variants": the tile with 10% missing observations filled forward
(fill), a scene of the Chile experiment's shape (2400 x 1851 pixels, 288
unevenly spaced acquisitions, day numbers with f = 365, n = 144, h = 72) on
the table-driven kernel (times), and the simulated critical value from one
million no-change paths (lambda).

Two more legs follow: the small tile of the first configuration (64 x 64
pixels, N = 228) timed call by call, warm and with the L2 caches and the MALL
flushed before each call, and with 25% NaN on the missing-value path, unsplit
and with the history split bfm_autotune picks ("latency_tile"), and the
largest tile (4096 x 4096
pixels, N = 512, 10% NaN, p = 8 and 10, float32 and FP16 storage) on the
missing-value kernel ("config4").  The masked tile and the p = 8 config-4
tiles are also timed with the MOSUM in FP32 (BFM_PREC_FP32: "masked_fp32",
"config4" keys ending in _fp32).  In the CPU-baseline leg the oracle also
checks sampled pixels of every leg against the GPU's FP64 outputs of the same
kernels ("accuracy": sigma, magnitude and MOSUM errors, break agreement,
marginal and non-marginal break mismatches).

Prints one JSON line.  Run with --gpus 1 (the default); more GPUs are not
supported by this benchmark.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s at N=400,k=8 (plain vs mixed-precision); p50/p99 tile latency"
P, N, n, ORDER, H_FRAC, LAM, FREQ = 1 << 20, 400, 200, 3, 0.25, 2.5, 23.0
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1807_01751_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
MISSING = 0.25
# The kernels bfm_fit_monitor launches for the two legs (f = 23 is an integer
# period, so the period-blocked kernels are used), the rocprofv3 summaries kept
# for each, and the workload each is timed on.
LEGS = {
    "plain": {"kernel": "::periodic_kernel<3, 23, false, float, false>(",
              "traffic": os.path.join(PROFILES, "traffic_plain_1024x1024_N400.json"),
              "trace_md": os.path.join(PROFILES, "plain_periodic_k3_f23_1024x1024_N400_kernel_trace.md"),
              "workload": "1024x1024 pixels, N=400"},
    "mixed": {"kernel": "::periodic_kernel<3, 23, false, bfm::dev::f16_t, false>(",
              "traffic": os.path.join(PROFILES, "traffic_mixed_f16_1024x1024_N400.json"),
              "trace_md": os.path.join(PROFILES, "mixed_periodic_f16_k3_f23_1024x1024_N400_kernel_trace.md"),
              "workload": "1024x1024 pixels, N=400, FP16-stored", "y_bytes": 2},
    "masked": {"kernel": "::masked_periodic_kernel<3, 23, false, false, float, false>(",
               "traffic": os.path.join(PROFILES, "traffic_masked_1024x1024_N400_nan25.json"),
               "trace_md": os.path.join(PROFILES,
                                        "masked_periodic_k3_f23_1024x1024_N400_nan25_kernel_trace.md"),
               "workload": "1024x1024 pixels, N=400, 25% NaN"},
    "fill": {"kernel": "::periodic_kernel<3, 23, false, float, true>(",
             "traffic": os.path.join(PROFILES, "traffic_fill_1024x1024_N400_miss10.json"),
             "trace_md": os.path.join(PROFILES, "fill_periodic_k3_f23_1024x1024_N400_miss10_kernel_trace.md"),
             "workload": "1024x1024 pixels, N=400, 10% missing, filled"},
    "times": {"kernel": "::plain_kernel<8, false, false>(",
              "traffic": os.path.join(PROFILES, "traffic_times_2400x1851_N288.json"),
              "trace_md": os.path.join(PROFILES, "times_plain_k3_f365_2400x1851_N288_kernel_trace.md"),
              "workload": "2400x1851 pixels, N=288 acquisition days, f=365",
              "pixels": 2400 * 1851, "n_obs": 288},
}
for _k, _ord in (("k8", 3), ("k10", 4)):
    for _st, _yb in (("f32", 4), ("f16", 2)):
        _T = "float" if _st == "f32" else "bfm::dev::f16_t"
        LEGS[f"config4_{_k}_{_st}"] = {
            "kernel": f"::masked_periodic_kernel<{_ord}, 23, false, false, {_T}, false>(",
            "traffic": os.path.join(PROFILES, f"traffic_config4_{_k}_{_st}_4096x4096_N512_nan10.json"),
            "trace_md": os.path.join(PROFILES, f"config4_masked_periodic_{_k}_{_st}_4096x4096_N512_nan10"
                                                "_kernel_trace.md"),
            "workload": f"4096x4096 pixels, N=512, 10% NaN, p={2 + 2 * _ord}, {_st} storage",
            "pixels": 1 << 24, "n_obs": 512, "y_bytes": _yb,
            # 5 timed and 5 latency-pass launches, then the untimed FP64 sample call
            "launches": 10, "skip_last": 1}
LEGS["masked_fp32"] = {
    "kernel": "::masked_periodic_kernel<3, 23, false, false, float, true>(",
    "traffic": os.path.join(PROFILES, "traffic_masked_fp32_1024x1024_N400_nan25.json"),
    "trace_md": os.path.join(PROFILES, "masked_periodic_fp32_k3_f23_1024x1024_N400_nan25_kernel_trace.md"),
    "workload": "1024x1024 pixels, N=400, 25% NaN, MOSUM in FP32"}
for _st, _yb in (("f32", 4), ("f16", 2)):
    _T = "float" if _st == "f32" else "bfm::dev::f16_t"
    LEGS[f"config4_k8_{_st}_fp32"] = {
        "kernel": f"::masked_periodic_kernel<3, 23, false, false, {_T}, true>(",
        "traffic": os.path.join(PROFILES, f"traffic_config4_k8_{_st}_fp32_4096x4096_N512_nan10.json"),
        "trace_md": os.path.join(PROFILES, f"config4_masked_periodic_fp32_k8_{_st}_4096x4096_N512_nan10"
                                            "_kernel_trace.md"),
        "workload": f"4096x4096 pixels, N=512, 10% NaN, p=8, {_st} storage, MOSUM in FP32",
        "pixels": 1 << 24, "n_obs": 512, "y_bytes": _yb, "launches": 10, "skip_last": 1}
CHILE_P, CHILE_N, CHILE_n, CHILE_H = 2400 * 1851, 288, 144, 72
FILL_MISSING = 0.10
LAMBDA_PATHS = 1 << 20
ACC_STRIDE = 128  # every 128th pixel of a 1024x1024 tile is checked against the oracle
PROFILE_CMD = ("rocprofv3 {flags} -f csv -d <dir> -o run -- python3 bench.py --steps 10 "
               "--warmup 2 --no-cpu-baseline --no-serving --copy-calibration")
PROFILED_LAUNCHES = 20  # the --steps 10 timed launches of PROFILE_CMD and the 10 of the latency pass


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha():
    """Hash of the kernel sources, the .hip translation units and the headers
    they include (a change invalidates the stored counters; host-only .cpp
    files do not take part)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_per_launch(leg):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernel source changed since the counters were taken."""
    try:
        with open(LEGS[leg]["traffic"]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(Y, seconds):
    """The FP64 oracle on host cores over a bounded sample of the same tile."""
    import numpy as np

    from oracle import oracle
    threads = oracle.threads(0)
    probe = Y[:, :2048].cpu().numpy()
    t0 = time.perf_counter()
    oracle.fit_monitor(probe, n=n, order=ORDER, h=H_FRAC, lam=LAM, freq=FREQ, threads=threads,
                       extras=False)
    rate = probe.shape[1] / (time.perf_counter() - t0)
    S = int(min(Y.shape[1], max(4096, rate * seconds)))
    S -= S % 64
    sample = np.ascontiguousarray(Y[:, :S].cpu().numpy())
    t0 = time.perf_counter()
    oracle.fit_monitor(sample, n=n, order=ORDER, h=H_FRAC, lam=LAM, freq=FREQ, threads=threads,
                       extras=False)
    dt = time.perf_counter() - t0
    return {"value": S / dt / 1e6, "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "sample": f"first {S} pixels of the same tile (all {N} observations each), "
                      f"{dt:.1f} s on {threads} host threads"}


# Sampled pixels of each leg, checked against the oracle in the CPU-baseline leg:
# the leg's tile (or a sample of its columns), the GPU's FP64 outputs for those
# pixels from the same kernels the leg times, and the oracle's arguments.
SAMPLES = []


def gpu_sample(leg, bfm, Y, idx, *, n_hist, lam, mask_mode=0, mosum=True, ref=None, **kw):
    """Run the leg's call once more (untimed) with FP64 outputs and keep the
    sampled pixels.  The lean and exporting kernels compute identically, so a
    MOSUM export does not change what is compared.  `ref` names another
    sample's GPU result to compare break indices with (storage agreement)."""
    import torch
    outs = ("brk", "mag", "sigma", "status") + (("mosum",) if mosum else ())
    g = bfm.fit_monitor(Y, n=n_hist, lam=lam, mask_mode=mask_mode, outputs=outs,
                        out_dtype=torch.float64, **kw)
    sel = torch.as_tensor(idx, device=Y.device)
    g = {k: (v[:, sel] if v.dim() == 2 else v[sel]).cpu().numpy() for k, v in g.items()}
    SAMPLES.append({"leg": leg, "Y": Y[:, sel].float().cpu().numpy(), "g": g, "n": n_hist,
                    "lam": lam, "mask_mode": mask_mode, "kw": kw, "ref": ref})


def accuracy(s, o):
    """FP64-oracle error of one sample (the parity rule of the tests): relative
    error of sigma and the magnitude, normwise MOSUM error per pixel, break
    agreement, and mismatched break indices split into marginal ones (the
    oracle's MOSUM within 1e-8, relative, of the boundary at a position up to
    the later break) and the rest."""
    import numpy as np
    g, n, lam = s["g"], s["n"], s["lam"]
    ok = (o["status"] == 0) & (g["status"] == 0)
    rep = {"pixels": int(ok.size), "status_agreement": float((g["status"] == o["status"]).mean()),
           "not_ok": int((o["status"] != 0).sum())}
    for k in ("sigma", "mag"):
        e = np.abs(g[k][ok] - o[k][ok]) / np.maximum(np.abs(o[k][ok]), 1e-300)
        rep[f"max_rel_{k}"] = float(e.max()) if e.size else 0.0
        rep[f"p999_rel_{k}"] = float(np.quantile(e, 0.999)) if e.size else 0.0
    mo = o["mosum"]
    if "mosum" in g:
        a, b = g["mosum"][:, ok], mo[:, ok]
        e = np.nanmax(np.abs(a - b), axis=0) / np.maximum(np.nanmax(np.abs(b), axis=0), 1e-300)
        rep["max_rel_mosum"] = float(e.max()) if e.size else 0.0
        rep["p999_rel_mosum"] = float(np.quantile(e, 0.999)) if e.size else 0.0
    M = mo.shape[0]
    fin = np.isfinite(mo)
    if s["mask_mode"] == 1:  # compacted positions u / n_v
        nv = np.isfinite(s["Y"][:n]).sum(0).astype(np.float64)
        x = (nv[None, :] + np.cumsum(fin, axis=0)) / nv[None, :]
    else:
        x = np.broadcast_to(((n + 1 + np.arange(M)) / n)[:, None], mo.shape)
    bnd = lam * np.sqrt(np.where(x <= np.e, 1.0, np.log(np.maximum(x, 1.0))))
    with np.errstate(invalid="ignore"):
        rel = np.abs(np.abs(mo) - bnd) / bnd
    last = np.maximum(g["brk"], o["brk"])
    last = np.where(last < 0, M - 1, last)
    rel = np.where((np.arange(M)[:, None] <= last[None, :]) & fin, rel, np.inf)
    margin = rel.min(axis=0)
    diff = g["brk"] != o["brk"]
    rep["brk_agreement"] = float(1.0 - diff.mean())
    rep["brk_mismatch_marginal"] = int((diff & (margin < 1e-8)).sum())
    rep["brk_mismatch_not_marginal"] = int((diff & ~(margin < 1e-8)).sum())
    return rep


def check_samples(threads):
    """The oracle on every leg's sample: accuracy per leg (the oracle runs here
    only, in the CPU-baseline leg)."""
    import numpy as np

    from oracle import oracle
    res, by_leg = {}, {}
    t0 = time.perf_counter()
    for s in SAMPLES:
        kw = {k: v for k, v in s["kw"].items() if k in ("order", "freq", "h", "h_window", "times")}
        o = oracle.fit_monitor(s["Y"], n=s["n"], lam=s["lam"], mask_mode=s["mask_mode"], threads=threads,
                               **kw)
        rep = accuracy(s, o)
        if s["ref"] is not None:  # break agreement with the float32 series' GPU result
            rep[f"brk_agreement_with_{s['ref']}"] = float((s["g"]["brk"] == by_leg[s["ref"]]["brk"]).mean())
            oref = by_leg[s["ref"] + "/oracle"]
            rep[f"brk_agreement_with_{s['ref']}_oracle"] = float((s["g"]["brk"] == oref["brk"]).mean())
        by_leg[s["leg"]], by_leg[s["leg"] + "/oracle"] = s["g"], o
        res[s["leg"]] = rep
    log(f"bench: oracle check of {len(SAMPLES)} samples in {time.perf_counter() - t0:.1f} s")
    return res


def _csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def summarize_profiles(d, bench_line=None):
    """Turn rocprofv3 CSV output of the three passes under ``d`` (trace/, fetch/,
    write/) into the summaries kept in profiles/, one set per leg.  With
    ``bench_line`` (the JSON line of a plain bench.py run in the same job), each
    summary also records that line's step time and the leg's HIP-event mean."""
    import glob
    import re
    P_ALG = (4 * N + 8) * P
    shas = set()
    for sub in ("trace", "fetch", "write"):
        with open(os.path.join(d, sub + ".log")) as f:
            shas |= set(re.findall(r"kernel_sha=([0-9a-f]+)", f.read()))
    assert shas == {kernel_sha()}, f"profiles were taken on other sources: {shas}"
    trace = _csv(glob.glob(os.path.join(d, "trace", "*kernel_trace.csv"))[0])
    counters = {sub: _csv(glob.glob(os.path.join(d, sub, "*counter_collection.csv"))[0])
                for sub in ("fetch", "write")}
    os.makedirs(PROFILES, exist_ok=True)
    for leg, spec in LEGS.items():
        KERNEL = spec["kernel"]
        pixels = spec.get("pixels", P)
        P_ALG = (spec.get("y_bytes", 4) * spec.get("n_obs", N) + 8) * pixels
        # The leg's own launches: its kernel over the whole tile (one lane per
        # pixel, 64-lane workgroups; the serving leg runs the same kernels on
        # smaller requests), and of those the last PROFILED_LAUNCHES (the
        # warmup and timed steps; the untimed pre-warm of the plain leg comes
        # before them).
        grid = (pixels + 63) // 64 * 64
        take, skip = spec.get("launches", PROFILED_LAUNCHES), spec.get("skip_last", 0)
        disp = sorted((r for r in trace if KERNEL in r["Kernel_Name"] and int(r["Grid_Size_X"]) == grid),
                      key=lambda r: int(r["Start_Timestamp"]))
        disp = disp[len(disp) - skip - take:len(disp) - skip]
        assert disp, f"{leg} kernel missing from the trace"
        dur = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in disp]
        st = {"Name": disp[0]["Kernel_Name"], "Calls": len(dur), "MinNs": min(dur), "MaxNs": max(dur),
              "AverageNs": sum(dur) / len(dur)}
        per = {}
        for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
            rows = counters[sub]
            k = [float(r["Counter_Value"]) for r in sorted(
                     (r for r in rows if KERNEL in r["Kernel_Name"] and int(r["Grid_Size"]) == grid),
                     key=lambda r: int(r["Dispatch_Id"]))]
            k = k[len(k) - skip - take:len(k) - skip]
            copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
            calib = float(copies[-1]["Counter_Value"])  # the 1 GiB copy runs last
            factor = (1 << 30) / (calib * 1024.0)       # bytes per counted byte
            per[counter] = {"kib_per_dispatch": sum(k) / len(k), "dispatches": len(k),
                            "copy_1GiB_kib": calib, "factor": factor}
        hbm = sum(v["kib_per_dispatch"] * 1024.0 * v["factor"] for v in per.values())
        avg_ns = float(st["AverageNs"])
        traffic = {"kernel": KERNEL.strip(":("), "kernel_sha": kernel_sha(),
                   "workload": spec["workload"],
                   "hbm_bytes_per_launch": round(hbm), "algorithmic_bytes_per_launch": P_ALG,
                   "traffic_over_algorithmic": hbm / P_ALG, "counters": per,
                   "commands": [PROFILE_CMD.format(flags="--pmc FETCH_SIZE"),
                                PROFILE_CMD.format(flags="--pmc WRITE_SIZE")]}
        with open(spec["traffic"], "w") as f:
            json.dump(traffic, f, indent=1)
        with open(spec["trace_md"], "w") as f:
            f.write(f"# rocprofv3 kernel trace: {KERNEL.strip(':(')}, {spec['workload']}\n\n")
            f.write("Command (from the repository root, on one MI355X):\n\n    "
                    + PROFILE_CMD.format(flags="--kernel-trace --stats") + "\n\n")
            f.write(f"The leg's timed and latency-pass launches over the whole workload (grid of "
                    f"{grid} work-items) only.\n\n")
            f.write("| kernel | calls | average ns | min ns | max ns |\n|---|---|---|---|---|\n")
            f.write(f"| {st['Name']} | {st['Calls']} | {avg_ns:.0f} | {st['MinNs']} | "
                    f"{st['MaxNs']} |\n\n")
            f.write(f"Algorithmic bytes per launch: {P_ALG} ({spec.get('y_bytes', 4)}N + 8 per pixel, "
                    f"N = {spec.get('n_obs', N)}, {spec.get('pixels', P)} pixels). "
                    f"At the average "
                    f"duration this is {P_ALG / avg_ns:.1f} GB/s "
                    f"({P_ALG / avg_ns / HBM_PEAK_GBS:.3f} of 8 TB/s).\n\n")
            f.write(f"HBM traffic (FETCH_SIZE and WRITE_SIZE passes, each scaled by its reading "
                    f"for a 1 GiB device copy): {hbm:.0f} B per launch = "
                    f"{hbm / P_ALG:.4f} x algorithmic.\n\n| counter | KiB per dispatch | "
                    f"1 GiB copy reads (KiB) | scale |\n|---|---|---|---|\n")
            for c, v in per.items():
                f.write(f"| {c} | {v['kib_per_dispatch']:.1f} | {v['copy_1GiB_kib']:.1f} | "
                        f"{v['factor']:.4f} |\n")
            if bench_line:
                f.write("\n" + bench_line_note(bench_line, leg, avg_ns) + "\n")
        print(spec["trace_md"])
        print(spec["traffic"])


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAVE_CYCLES",
               "SQ_ACTIVE_INST_VALU", "SQ_WAIT_INST_ANY", "SQ_BUSY_CYCLES")


SQ_CMD = ("rocprofv3 --pmc " + " ".join(SQ_COUNTERS) + " -f csv -d <dir>/sq -o run -- python3 bench.py "
          "--steps 10 --warmup 2 --no-cpu-baseline --no-serving > <dir>/sq.log 2>&1")


def summarize_sq(d):
    """Instruction counters of each leg's kernel (one rocprofv3 --pmc pass of
    the eight SQ counters under ``d``/sq) into profiles/sq_counters.md: per
    wave and per row of the series, and the share of a wave's cycles spent
    issuing VALU instructions or waiting."""
    import collections
    import glob
    import re
    with open(os.path.join(d, "sq.log")) as f:
        shas = set(re.findall(r"kernel_sha=([0-9a-f]+)", f.read()))
    assert shas == {kernel_sha()}, f"counters were taken on other sources: {shas}"
    rows = _csv(glob.glob(os.path.join(d, "sq", "*counter_collection.csv"))[0])
    out = os.path.join(PROFILES, "sq_counters.md")
    with open(out, "w") as f:
        f.write("# SQ instruction counters per kernel\n\nCommand (from the repository root, on one "
                "MI355X):\n\n    " + SQ_CMD
                + "\n\nAverages over each leg's last ten whole-workload launches. Per row = per "
                "wave / N (one lane per pixel, one row per observation). VALU share = "
                "SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES, wait share = SQ_WAIT_INST_ANY / "
                "SQ_WAVE_CYCLES (both per wave).\n\n| leg | kernel | waves | VALU / wave | SALU / wave "
                "| LDS / wave | VALU / row | SALU / row | VALU share | wait share |\n"
                "|---|---|---|---|---|---|---|---|---|---|\n")
        for leg, spec in LEGS.items():
            grid = (spec.get("pixels", P) + 63) // 64 * 64
            per = collections.defaultdict(list)
            for r in rows:
                if spec["kernel"] in r["Kernel_Name"] and int(r["Grid_Size"]) == grid:
                    per[r["Counter_Name"]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
            if not per:
                continue
            avg = {c: sum(v for _, v in sorted(x)[-10:]) / len(sorted(x)[-10:]) for c, x in per.items()}
            w, nobs = avg["SQ_WAVES"], spec.get("n_obs", N)
            f.write(f"| {leg} | {spec['kernel'].strip(':(')} | {w:.0f} | {avg['SQ_INSTS_VALU'] / w:.0f} | "
                    f"{avg['SQ_INSTS_SALU'] / w:.0f} | {avg['SQ_INSTS_LDS'] / w:.0f} | "
                    f"{avg['SQ_INSTS_VALU'] / w / nobs:.1f} | {avg['SQ_INSTS_SALU'] / w / nobs:.1f} | "
                    f"{avg['SQ_ACTIVE_INST_VALU'] / avg['SQ_WAVE_CYCLES']:.3f} | "
                    f"{avg['SQ_WAIT_INST_ANY'] / avg['SQ_WAVE_CYCLES']:.3f} |\n")
    print(out)


def bench_line_note(path, leg, avg_ns):
    """The same job's bench line beside a profiled kernel: its step time and
    the leg's HIP-event mean launch duration."""
    with open(path) as f:
        line = json.loads([x for x in f.read().splitlines() if x.startswith("{")][-1])
    parts = leg.split("_", 2)
    node = (line if leg == "plain" else line.get(leg) or line.get("variants", {}).get(leg)
            or line.get("config4", {}).get("_".join(parts[1:])) or {})
    roof = node.get("roofline", {})
    mean_ms = (roof.get("algorithmic_bytes_per_launch", 0) / (roof["achieved"] * 1e9) * 1e3
               if roof.get("achieved") else None)
    return (f"Bench line of the same job (`python3 bench.py`, unprofiled): ms_per_step "
            f"{node.get('ms_per_step')} ms, HIP-event mean launch "
            f"{'%.4f' % mean_ms if mean_ms else 'n/a'} ms; profiled average "
            f"{avg_ns / 1e6:.4f} ms.")


PREWARM_S = 0.25  # --prewarm-s


def prewarm(step, seconds):
    """Runs ``step`` untimed, synchronising after each call, for ``seconds``;
    returns the number of calls."""
    import torch
    t0, k = time.perf_counter(), 0
    while time.perf_counter() - t0 < seconds:
        step()
        torch.cuda.synchronize()
        k += 1
    return k


def timed(step, steps, warmup, stream):
    """Run the step untimed for PREWARM_S seconds (the clocks ramp up over the
    first tens of milliseconds of work: without it a leg of ten 1.3 ms steps
    read 1.37 instead of 1.15 ms per step), warm up, then time exactly
    ``steps`` calls back to back: wall clock over
    all of them, and two HIP events on the stream the kernel runs on around the
    whole region (their span / steps is the mean launch duration).  Per-launch
    latencies (p50, p99) come from a separate pass of as many calls, each
    bracketed by its own events (which add a short gap between launches, so they
    are kept out of the timed region)."""
    import torch
    prewarm(step, PREWARM_S)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        step()
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mean = a.elapsed_time(b) / steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for x, y in ev:
        x.record(stream)
        step()
        y.record(stream)
    torch.cuda.synchronize()
    lat = sorted(x.elapsed_time(y) for x, y in ev)  # ms, per launch
    return {"ms_per_step": wall * 1e3 / steps, "mean": mean,
            "p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]}


def serving_leg(bfm, dev, requests=2000, payloads=32, slots=4, load=0.8, seed=5):
    """Continuous batching under Poisson arrivals (the serving workload):
    requests of log-uniform pixel count in [256^2, 2048^2], N ~ U{200..600},
    n = N/2, harmonic order in {2, 3, 4} (6, 8 or 10 regressors), NaN rate
    U(0, 0.4), 15% planted steps, each on one of ``payloads`` device-resident
    tiles generated before timing (the requests reuse them in turn).  First the capacity is measured with every request
    queued at once; then requests arrive as a Poisson process at ``load`` times
    that capacity.  Latency = submit to completion (server clock)."""
    import ctypes
    import math
    import random

    import numpy as np
    import torch

    from paper_1807_01751_amd.synth import apply_missing, make_missing, make_series, split_rate
    rng = np.random.default_rng(seed)
    tiles = []
    for i in range(payloads):
        P = int(math.exp(rng.uniform(math.log(256 ** 2), math.log(2048 ** 2))))
        N = int(rng.integers(200, 601))
        order = int(rng.choice([2, 3, 4]))
        miss = float(rng.uniform(0.0, 0.4))
        Yt, _ = make_series(P, N, N // 2, order, seed=seed * 100 + i, step_frac=0.15, device=dev)
        if miss > 0:
            r = split_rate(miss)
            Yt = apply_missing(Yt, make_missing(N, P, iid=r, runs=r, seed=seed * 100 + i, device=dev))
        tiles.append((Yt, order, 1 if miss > 0 else 0))
    torch.cuda.synchronize()
    lib = bfm.load()
    with bfm.Server(device=dev.index or 0, slots=slots, pool_bytes=1 << 30) as srv:
        reqs = []
        for j in range(requests):
            Yt, order, mode = tiles[j % payloads]
            reqs.append(srv.request(Yt, n=Yt.shape[0] // 2, order=order, mask_mode=mode,
                                    outputs=("brk", "mag"), out_dtype=torch.float32))
        pixels = sum(r.P for r in reqs)

        def run(gaps):
            # A client thread takes each result as it completes and releases its
            # outputs (the pool holds a small share of all the outputs), while
            # this thread submits at the arrival times.
            import queue
            import threading
            tickets, lat = queue.Queue(), []

            def consume():
                res = bfm.Result()
                while True:
                    tk = tickets.get()
                    if tk is None:
                        return
                    assert lib.bfm_server_wait(srv.handle, tk, -1, ctypes.byref(res)) == 0 and res.rc == 0
                    lat.append(res.latency_us)
                    lib.bfm_server_release(srv.handle, tk)

            client = threading.Thread(target=consume)
            client.start()
            t = ctypes.c_uint64()
            t0 = time.perf_counter()
            due = t0
            for r, g in zip(reqs, gaps):
                due += g
                while True:
                    left = due - time.perf_counter()
                    if left <= 0:
                        break
                    if left > 3e-4:
                        time.sleep(left - 2e-4)
                rc = lib.bfm_server_submit(srv.handle, ctypes.byref(r), ctypes.byref(t))
                assert rc == 0, rc
                tickets.put(t.value)
            tickets.put(None)
            client.join()
            return time.perf_counter() - t0, sorted(lat)

        run([0.0] * len(reqs))  # warm: operators of every parameter set built once
        wall, _ = run([0.0] * len(reqs))
        capacity = len(reqs) / wall
        rnd = random.Random(seed)
        gaps = [rnd.expovariate(load * capacity) for _ in reqs]
        wall2, lat = run(gaps)
        st = srv.stats()
    del tiles
    q = lambda f: lat[min(len(lat) - 1, int(round(f * (len(lat) - 1))))] / 1e3
    return {"requests": len(reqs), "slots": slots, "offered_load": load,
            "capacity_requests_per_s": round(capacity, 1),
            "saturated_mpixel_s": round(pixels / wall / 1e6, 1),
            "mpixel_s": round(pixels / wall2 / 1e6, 1), "p50_ms": round(q(0.5), 4),
            "p99_ms": round(q(0.99), 4), "max_running": st["max_running"],
            "config": {"workload": f"{len(reqs)} Poisson-arriving requests, tiles of 256^2-2048^2 "
                                   "pixels (log-uniform), N 200-600, n = N/2, 6/8/10 regressors, "
                                   "NaN rate U(0, 0.4), 15% planted steps, "
                                   f"{payloads} device-resident payloads reused in turn",
                       "pixels_total": pixels}}


def latency_leg(bfm, dev, stream, calls=200, seed=1):
    """Tile latency at the small tile of the first configuration: 64x64 pixels,
    N = 228, n = 114 (H = 28), k = 3, one call per tile, per-call HIP events.
    Warm: calls back to back on a resident tile.  Cold: before each call the
    L2 caches and the MALL are flushed by writing a 1 GiB buffer (outside the
    events), so the call reads its 3.7 MB from HBM.  Then the same tile with
    25% NaN on the missing-value path, warm: one wave per 64 pixels, and the
    history split that bfm_autotune picks for this tile shape."""
    import torch

    from paper_1807_01751_amd.synth import apply_missing, make_missing, make_series, split_rate
    Pl, Nl, nl = 4096, 228, 114
    Y, _ = make_series(Pl, Nl, nl, ORDER, seed=seed, device=dev)
    out = {"brk": torch.empty(Pl, dtype=torch.int32, device=dev),
           "mag": torch.empty(Pl, dtype=torch.float32, device=dev)}
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    common = dict(n=nl, order=ORDER, freq=FREQ, h=H_FRAC, lam=LAM)

    def step():
        bfm.fit_monitor(Y, outputs=("brk", "mag"), out_dtype=torch.float32, out=out, **common)

    def per_call(f, cold):
        for _ in range(10):
            f()
        torch.cuda.synchronize()
        lat = []
        for _ in range(calls):
            if cold:
                flush.fill_(1.0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            f()
            b.record(stream)
            b.synchronize()
            lat.append(a.elapsed_time(b))
        lat.sort()
        q = lambda x: lat[min(len(lat) - 1, int(round(x * (len(lat) - 1))))]
        return {"p50_ms": round(q(0.5), 5), "p99_ms": round(q(0.99), 5), "calls": calls}

    res = {}
    for mode in ("warm", "cold"):
        res[mode] = per_call(step, mode == "cold")
        log(f"bench: latency tile ({mode}) p50 {res[mode]['p50_ms'] * 1e3:.1f} us, "
            f"p99 {res[mode]['p99_ms'] * 1e3:.1f} us")
    r = split_rate(MISSING)
    Ym = apply_missing(Y.clone(), make_missing(Nl, Pl, iid=r, runs=r, seed=seed + 7, device=dev))

    def mstep():
        bfm.fit_monitor(Ym, mask_mode=bfm.MASK_NAN, outputs=("brk", "mag"), out_dtype=torch.float32, out=out,
                        **common)

    bfm.tune_set(Ym, 1, mask_mode=bfm.MASK_NAN, **common)
    res["masked_warm"] = per_call(mstep, False)
    split, times = bfm.autotune(Ym, mask_mode=bfm.MASK_NAN, stream=stream, **common)
    res["masked_warm_tuned"] = {**per_call(mstep, False), "split": split,
                                "autotune_median_us": {str(k): round(v, 2) for k, v in times.items()}}
    log(f"bench: latency tile, 25% NaN: p50 {res['masked_warm']['p50_ms'] * 1e3:.1f} us with one wave per "
        f"64 pixels, {res['masked_warm_tuned']['p50_ms'] * 1e3:.1f} us with the tuned split {split}")
    res["config"] = {"workload": "64x64 = 4096 pixels, N=228 FP32 observations, n=114, k=3 (p=8), "
                                 "h=0.25 (H=28), lambda=2.5, f=23, 20% planted steps; one call per "
                                 "tile; cold = L2 and MALL flushed by a 1 GiB write before each call; "
                                 "masked = the same tile with 25% NaN (missing-value path), warm"}
    del flush
    return res


def config4_leg(bfm, dev, stream, warmup, steps=5):
    """The largest tile: 4096x4096 = 16,777,216 pixels, N = 512, n = 256,
    h = 0.25 (H = 64), 10% missing as NaN (half iid, half cloud runs of 3-15
    rows), harmonic orders 3 and 4 (p = 8 and 10), series stored as float32 and
    as FP16; the missing-value kernel, FP64 arithmetic.  The missing-value mask
    is drawn per slab of 2^20 pixels (the generator's temporaries stay small)."""
    import numpy as np
    import torch

    from paper_1807_01751_amd.synth import apply_missing, make_missing, make_series, split_rate
    P4, N4, n4 = 1 << 24, 512, 256
    r = split_rate(0.1)
    rng = np.random.default_rng(44)
    idx = np.unique(np.r_[np.arange(32), np.arange(P4 - 32, P4), rng.integers(0, P4, 4032)])
    res = {}
    for order in (3, 4):
        Y, _ = make_series(P4, N4, n4, order, seed=40 + order, device=dev)
        for s0 in range(0, P4, 1 << 20):
            apply_missing(Y[:, s0:s0 + (1 << 20)],
                          make_missing(N4, 1 << 20, iid=r, runs=r, seed=400 + s0 // (1 << 20), device=dev))
        miss = float(torch.isnan(Y[:, :: 4096]).float().mean())
        out = {"brk": torch.empty(P4, dtype=torch.int32, device=dev),
               "mag": torch.empty(P4, dtype=torch.float32, device=dev)}
        runs = [("f32", "fp64"), ("f16", "fp64")]
        if order == 3:
            runs += [("f32", "fp32"), ("f16", "fp32")]
        Yh = Y.to(torch.float16)
        for name, prec in runs:
            Yd = Y if name == "f32" else Yh

            def step():
                bfm.fit_monitor(Yd, n=n4, order=order, freq=FREQ, h=H_FRAC, lam=LAM, mask_mode=bfm.MASK_NAN,
                                outputs=("brk", "mag"), out_dtype=torch.float32, out=out, precision=prec)

            t = timed(step, steps, min(warmup, 2), stream)
            yb = 4 if name == "f32" else 2
            alg = (yb * N4 + 8) * P4
            key = f"k{2 + 2 * order}_{name}" + ("_fp32" if prec == "fp32" else "")
            res[key] = {"value": round(P4 / (t["ms_per_step"] * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
                        "ms_per_step": round(t["ms_per_step"], 4), "p50_ms": round(t["p50"], 4),
                        "p99_ms": round(t["p99"], 4), "storage": name, "p": 2 + 2 * order,
                        "mosum": "f32" if prec == "fp32" else "f64",
                        "missing_fraction": round(miss, 4),
                        "roofline": {"bound": "hbm", "achieved": round(alg / (t["mean"] * 1e-3) / 1e9, 1),
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": round(alg / (t["mean"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                     "algorithmic_bytes_per_launch": alg}}
            log(f"bench: config 4 {key}: {t['ms_per_step']:.3f} ms/step, kernel mean {t['mean']:.3f} ms")
            ref = None if key == f"k{2 + 2 * order}_f32" else f"config4_k{2 + 2 * order}_f32"
            gpu_sample(f"config4_{key}", bfm, Yd, idx, n_hist=n4, lam=LAM, mask_mode=bfm.MASK_NAN,
                       mosum=False, ref=ref, order=order, freq=FREQ, h=H_FRAC, precision=prec)
            del Yd
        del Y, Yh, out
        torch.cuda.empty_cache()
    res["config"] = {"workload": "4096x4096 = 16777216 pixels, N=512, n=256, h=0.25 (H=64), lambda=2.5, "
                                 "f=23, 10% NaN (half iid, half cloud runs of 3-15 rows), p=8 and 10, "
                                 "float32 and FP16 storage, FP64 arithmetic; for p=8 also the MOSUM "
                                 "in FP32 (_fp32: BFM_PREC_FP32)"}
    return res


def roofline(leg, mean_ms, y_bytes=4):
    spec = LEGS[leg]
    bytes_per_px = y_bytes * spec.get("n_obs", N) + 4 + 4  # read y once; write int32 brk + FP32 mag
    alg_bytes = bytes_per_px * spec.get("pixels", P)
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_per_launch(leg),
            "kernel": LEGS[leg]["kernel"].strip(":("), "algorithmic_bytes_per_launch": alg_bytes}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--prewarm-s", type=float, default=0.25,
                    help="seconds of untimed steps before the warmup steps (clock ramp)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="leave out the serving leg (the profiling runs: no summary uses it)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 output under DIR and exit")
    ap.add_argument("--bench-line", metavar="FILE",
                    help="with --summarize-profiles: the JSON line of an unprofiled run of the same job")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run one 1 GiB device-to-device copy (the known-size "
                         "reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_profiles:
        if os.path.isdir(os.path.join(args.summarize_profiles, "sq")):
            summarize_sq(args.summarize_profiles)
        if os.path.isdir(os.path.join(args.summarize_profiles, "trace")):
            summarize_profiles(args.summarize_profiles, args.bench_line)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "pixels are independent, so several GPUs would each take a range of pixels with "
              "no traffic between them; that form is not run here.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1807_01751_amd import bfm
    from paper_1807_01751_amd.synth import make_series

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: generating {P} x {N} series on {torch.cuda.get_device_name(dev)}; "
        f"kernel_sha={kernel_sha()}")
    Y, _ = make_series(P, N, n, ORDER, freq=FREQ, seed=2, device=dev)
    out = {"brk": torch.empty(P, dtype=torch.int32, device=dev),
           "mag": torch.empty(P, dtype=torch.float32, device=dev)}
    torch.cuda.synchronize()

    def step():
        bfm.fit_monitor(Y, n=n, order=ORDER, freq=FREQ, h=H_FRAC, lam=LAM,
                        outputs=("brk", "mag"), out_dtype=torch.float32, out=out)

    stream = torch.cuda.current_stream(dev)
    global PREWARM_S
    PREWARM_S = args.prewarm_s
    log(f"bench: plain leg, pre-warm {PREWARM_S} s, warmup {args.warmup}, timing {args.steps} steps")
    tp = timed(step, args.steps, args.warmup, stream)
    log(f"bench: {tp['ms_per_step']:.4f} ms/step wall, kernel mean {tp['mean']:.4f} ms")
    ref = {k: v.clone() for k, v in out.items()}
    import numpy as np
    idx = np.arange(0, P, ACC_STRIDE)  # pixels checked against the oracle
    common = dict(order=ORDER, freq=FREQ, h=H_FRAC)
    gpu_sample("plain", bfm, Y, idx, n_hist=n, lam=LAM, **common)

    # Mixed-precision leg: FP16-stored tile, FP64 arithmetic.
    Yh = Y.to(torch.float16)
    outh = {k: torch.empty_like(v) for k, v in out.items()}

    def hstep():
        bfm.fit_monitor(Yh, n=n, order=ORDER, freq=FREQ, h=H_FRAC, lam=LAM,
                        outputs=("brk", "mag"), out_dtype=torch.float32, out=outh)

    log(f"bench: mixed leg (FP16 storage), warmup {args.warmup}, timing {args.steps} steps")
    th = timed(hstep, args.steps, args.warmup, stream)
    log(f"bench: mixed {th['ms_per_step']:.4f} ms/step wall, kernel mean {th['mean']:.4f} ms")
    agree = float((outh["brk"] == ref["brk"]).float().mean())
    # |mag| (the size of the largest MOSUM excursion) is compared: where the
    # largest and the smallest MOSUM values are nearly opposite, the signed
    # magnitude may flip sign between the two runs.
    dmag = float((outh["mag"].abs() - ref["mag"].abs()).abs().max())
    gpu_sample("mixed", bfm, Yh, idx, n_hist=n, lam=LAM, ref="plain", **common)
    del Yh

    # Masked leg: the same tile with NaN at 25% of (time, pixel) positions.
    from paper_1807_01751_amd.synth import apply_missing, make_missing, split_rate
    r = split_rate(MISSING)
    Ym = apply_missing(Y.clone(), make_missing(N, P, iid=r, runs=r, seed=7, device=dev))
    miss = float(torch.isnan(Ym).float().mean())

    def mstep():
        bfm.fit_monitor(Ym, n=n, order=ORDER, freq=FREQ, h=H_FRAC, lam=LAM, mask_mode=bfm.MASK_NAN,
                        outputs=("brk", "mag"), out_dtype=torch.float32, out=out)

    log(f"bench: masked leg ({miss:.3f} missing), warmup {args.warmup}, timing {args.steps} steps")
    tm = timed(mstep, args.steps, args.warmup, stream)
    log(f"bench: masked {tm['ms_per_step']:.4f} ms/step wall, kernel mean {tm['mean']:.4f} ms")
    gpu_sample("masked", bfm, Ym, idx, n_hist=n, lam=LAM, mask_mode=bfm.MASK_NAN, **common)

    # The same tile with the MOSUM in FP32 (BFM_PREC_FP32; the fit stays FP64).
    def m32step():
        bfm.fit_monitor(Ym, n=n, order=ORDER, freq=FREQ, h=H_FRAC, lam=LAM, mask_mode=bfm.MASK_NAN,
                        outputs=("brk", "mag"), out_dtype=torch.float32, out=out, precision="fp32")

    log(f"bench: masked leg with FP32 MOSUM, warmup {args.warmup}, timing {args.steps} steps")
    tm32 = timed(m32step, args.steps, args.warmup, stream)
    log(f"bench: masked FP32 {tm32['ms_per_step']:.4f} ms/step wall, kernel mean {tm32['mean']:.4f} ms")
    gpu_sample("masked_fp32", bfm, Ym, idx, n_hist=n, lam=LAM, mask_mode=bfm.MASK_NAN, ref="masked",
               precision="fp32", **common)
    del Ym

    # Fill leg: 10% missing (half iid, half cloud runs), filled forward as read.
    r = split_rate(FILL_MISSING)
    Yf = apply_missing(Y.clone(), make_missing(N, P, iid=r, runs=r, seed=8, device=dev))

    def fstep():
        bfm.fit_monitor(Yf, n=n, order=ORDER, freq=FREQ, h=H_FRAC, lam=LAM, mask_mode=bfm.MASK_FILL,
                        outputs=("brk", "mag"), out_dtype=torch.float32, out=out)

    log(f"bench: fill leg, warmup {args.warmup}, timing {args.steps} steps")
    tf = timed(fstep, args.steps, args.warmup, stream)
    log(f"bench: fill {tf['ms_per_step']:.4f} ms/step wall, kernel mean {tf['mean']:.4f} ms")
    gpu_sample("fill", bfm, Yf, idx, n_hist=n, lam=LAM, mask_mode=bfm.MASK_FILL, **common)
    del Yf

    # Irregular-time leg: a scene of the Chile experiment's shape at synthetic
    # acquisition days (f = 365), table-driven plain kernel.
    from paper_1807_01751_amd.synth import acquisition_days
    days = acquisition_days(CHILE_N, seed=3)
    Yc, _ = make_series(CHILE_P, CHILE_N, CHILE_n, ORDER, freq=365.0, times=days, trend=2e-5, seed=4,
                        device=dev)
    outc = {"brk": torch.empty(CHILE_P, dtype=torch.int32, device=dev),
            "mag": torch.empty(CHILE_P, dtype=torch.float32, device=dev)}

    def cstep():
        bfm.fit_monitor(Yc, n=CHILE_n, order=ORDER, freq=365.0, h_window=CHILE_H, lam=LAM, times=days,
                        outputs=("brk", "mag"), out_dtype=torch.float32, out=outc)

    log(f"bench: times leg ({CHILE_P} pixels x {CHILE_N} days), timing {max(5, args.steps // 5)} steps")
    tc = timed(cstep, max(5, args.steps // 5), min(args.warmup, 2), stream)
    log(f"bench: times {tc['ms_per_step']:.4f} ms/step wall, kernel mean {tc['mean']:.4f} ms")
    gpu_sample("times", bfm, Yc, np.arange(0, CHILE_P, 4 * ACC_STRIDE), n_hist=CHILE_n, lam=LAM,
               order=ORDER, freq=365.0, h_window=CHILE_H, times=days)
    del Yc, outc

    latency = latency_leg(bfm, dev, stream)
    config4 = config4_leg(bfm, dev, stream, args.warmup)

    # Critical value by simulation: one million no-change paths at n = 200, N = 400, H = 50.
    def lstep():
        bfm.mosum_null_sup(n=n, N=N, h=H_FRAC, seed=1, paths=LAMBDA_PATHS)

    tl = timed(lstep, 5, 1, stream)
    t0 = time.perf_counter()
    lam_crit = bfm.critical_value(0.05, n=n, N=N, h=H_FRAC, paths=LAMBDA_PATHS, seed=1)
    lam_ms = (time.perf_counter() - t0) * 1e3
    log(f"bench: lambda {lam_crit:.5f} from {LAMBDA_PATHS} paths: sup kernel {tl['mean']:.3f} ms, "
        f"call {lam_ms:.2f} ms")

    serving = None
    if not args.no_serving:
        log("bench: serving leg (Poisson arrivals, continuous batching)")
        serving = serving_leg(bfm, dev)
        log(f"bench: serving {serving['mpixel_s']} Mpixel/s, p50 {serving['p50_ms']} ms, "
            f"p99 {serving['p99_ms']} ms, max running {serving['max_running']}")

    # Context (not the metric): the tile's host-to-device transfer from pinned
    # memory, the phase that dominates the paper's GPU timings.
    host = torch.empty((N, P), dtype=torch.float32, pin_memory=True)
    host.copy_(Y)
    dst = torch.empty_like(Y)
    h2d = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(host, non_blocking=True)
        b.record(stream)
        torch.cuda.synchronize()
        h2d.append(a.elapsed_time(b))
    assert torch.equal(dst[:: N // 4], Y[:: N // 4])
    h2d_ms = sorted(h2d)[1]
    del host, dst
    log(f"bench: host-to-device {h2d_ms:.3f} ms for {4 * N * P / 1e9:.3f} GB")
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration: 1 GiB read + 1 GiB written")
        del src, dst

    ms_per_step = tp["ms_per_step"]
    res = {"metric": METRIC, "value": round(P / (ms_per_step * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "plain BFAST Monitor, one 1024x1024 tile (1048576 pixels), "
                                  "N=400 FP32 observations, n=200, k=3 harmonics (p=8), "
                                  "h=0.25 (H=50), lambda=2.5, f=23, 20% planted steps",
                      "pixels": P, "n_obs": N, "n_hist": n, "p": 2 + 2 * ORDER,
                      "outputs": "brk int32 + mag f32", "parallelism": "single GPU"},
           "p50_ms": round(tp["p50"], 5), "p99_ms": round(tp["p99"], 5),
           "roofline": roofline("plain", tp["mean"]),
           "masked": {"value": round(P / (tm["ms_per_step"] * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
                      "ms_per_step": round(tm["ms_per_step"], 5), "p50_ms": round(tm["p50"], 5),
                      "p99_ms": round(tm["p99"], 5), "dtype": "f64",
                      "config": {"workload": "masked BFAST Monitor, the same tile with "
                                             f"{100 * MISSING:.0f}% NaN (half iid, half cloud runs "
                                             "of 3-15 rows), per-pixel Gram and Cholesky",
                                 "missing_fraction": round(miss, 4)},
                      "roofline": roofline("masked", tm["mean"])},
           "masked_fp32": {"value": round(P / (tm32["ms_per_step"] * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
                           "ms_per_step": round(tm32["ms_per_step"], 5), "p50_ms": round(tm32["p50"], 5),
                           "p99_ms": round(tm32["p99"], 5), "dtype": "f64 fit, f32 MOSUM",
                           "config": {"workload": "the masked leg's tile with the MOSUM in FP32 "
                                                  "(BFM_PREC_FP32): residuals formed in FP64 and rounded "
                                                  "to float, window sums and boundary test in FP32; "
                                                  "Gram, Cholesky and sigma in FP64"},
                           "roofline": roofline("masked_fp32", tm32["mean"])},
           "mixed": {"value": round(P / (th["ms_per_step"] * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
                     "ms_per_step": round(th["ms_per_step"], 5), "p50_ms": round(th["p50"], 5),
                     "p99_ms": round(th["p99"], 5), "dtype": "f64", "storage": "f16",
                     "config": {"workload": "plain BFAST Monitor, the same tile stored as FP16 "
                                            "(11 significant bits), FP64 arithmetic"},
                     "vs_f32_leg": {"brk_agreement": round(agree, 6), "max_abs_d_abs_mag": round(dmag, 5)},
                     "roofline": roofline("mixed", th["mean"], y_bytes=2)},
           "variants": {
               "fill": {"value": round(P / (tf["ms_per_step"] * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
                        "ms_per_step": round(tf["ms_per_step"], 5), "dtype": "f64",
                        "config": {"workload": "the same tile with 10% missing (half iid, half "
                                               "cloud runs), filled forward (backward for a "
                                               "leading gap) as the rows are read"},
                        "roofline": roofline("fill", tf["mean"])},
               "times": {"value": round(CHILE_P / (tc["ms_per_step"] * 1e-3) / 1e6, 2),
                         "unit": "Mpixel/s", "ms_per_step": round(tc["ms_per_step"], 5),
                         "dtype": "f64",
                         "config": {"workload": "a scene of the Chile experiment's shape: 2400x1851 "
                                                "pixels, 288 acquisitions at synthetic day numbers "
                                                "(gaps of 8-48 days), f=365, n=144, h=72, k=3",
                                    "pixels": CHILE_P, "n_obs": CHILE_N},
                         "roofline": roofline("times", tc["mean"])},
               "lambda": {"value": round(LAMBDA_PATHS / (tl["mean"] * 1e-3) / 1e6, 2),
                          "unit": "Mpaths/s", "sup_kernel_ms": round(tl["mean"], 4),
                          "critical_value_call_ms": round(lam_ms, 3), "lambda": round(lam_crit, 6),
                          "config": {"workload": "critical value for alpha=0.05, h=0.25, N/n=2 "
                                                 "(n=200, N=400) from 1048576 simulated "
                                                 "no-change MOSUM paths"}}},
           "serving": serving,
           "h2d": {"bytes": 4 * N * P, "ms": round(h2d_ms, 3),
                   "gb_per_s": round(4 * N * P / (h2d_ms * 1e-3) / 1e9, 1),
                   "pcie_inclusive_mpixel_s": round(P / ((h2d_ms + tp["mean"]) * 1e-3) / 1e6, 1),
                   "note": "pinned host tile to device, median of 3; context only"}}
    res["latency_tile"] = latency
    res["config4"] = config4
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        res["cpu_baseline"] = cpu_baseline(Y, args.cpu_seconds)
        res["accuracy"] = check_samples(res["cpu_baseline"]["cores"])
        res["accuracy"]["note"] = (
            "FP64 oracle against the GPU's FP64 outputs of each leg's kernels on sampled "
            f"pixels (every {ACC_STRIDE}th pixel of the 1024x1024 tiles, every {4 * ACC_STRIDE}th "
            "of the Chile-shaped scene, 4096 of each 16.8M-pixel config-4 tile); 16-bit legs "
            "against the oracle on the values they decode to")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
