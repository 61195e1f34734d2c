#!/usr/bin/env python3
"""Throughput of conditional simulation by circulant embedding with local
Kriging (arXiv 2109.11044) on one MI355X.

One step is the whole method for one synthetic event, every row of the hot
path inside the timed region:
  ce_setup          torus base + FP64 2D FFT + eigenvalue check
  offgrid_nnkrige   local-Kriging weights and variances of the stations
  ce_simulate       R unconditional grid realizations (CE draw)
  condition         synthetic data, observation Cholesky + solves, and the
                    cross-covariance product onto the grid, in place.
Workload (default): 1024 x 1024 unit-square grid, exponential covariance
(sigma^2 = 1, range 0.02), nugget 0.02, 5000 clustered stations, 6 x 6
local-Kriging windows, R = 1000 realizations per step.  Inputs are seeded
synthetic data already resident on the device when the timed region starts
(station coordinates and values are host arrays the ABI copies, as a caller
would).  The headline value is the mixed-precision path; the plain FP64 path
is measured beside it for the speed ratio.

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}   # dense peaks
SPLIT_PARAM = {"fp16": 0, "bf16": 1, "fp32": 2}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--m", type=int, default=1024)
    ap.add_argument("--n", type=int, default=5000)
    ap.add_argument("--nreal", type=int, default=1000)
    ap.add_argument("--batch", type=int, default=0, help="realizations per call (0: all)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--gemm-tile", type=int, default=0,
                    help="mixed GEMM tile 1-3 (0: tuning table or library default)")
    ap.add_argument("--chunk-pairs", type=int, default=0)
    ap.add_argument("--split", choices=["fp16", "bf16", "fp32"], default="fp16",
                    help="mixed GEMM arithmetic: FP16 or BF16 three-product split, or plain FP32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--json-out", default="")
    ap.add_argument("--se-chunk", type=int, default=0,
                    help="se1024: grid nodes per chunk (0: the library's choice)")
    ap.add_argument("--configs", type=int, default=100,
                    help="accuracy61: random station configurations per case")
    ap.add_argument("--workload", choices=["dm", "events64", "grad512", "accuracy61", "se1024",
                                           "nn1024"],
                    default="dm",
                    help="dm: the 1024^2 single-event workload; events64: 64 uneven events "
                         "run as one batch (one graph launch per step)")
    ap.add_argument("--pad", action="store_true",
                    help="accuracy61: widen the grid by n_p on every side (Section 2.1) and "
                         "score the original 61x61 nodes")
    ap.add_argument("--joint", action="store_true",
                    help="sample the observations that share a grid box jointly "
                         "(CESIM_PARAM_JOINT_BOXES)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip the one-off tuning of launch shapes that precedes the warm-up "
                         "(by default the library's autotuner picks the draw and GEMM tiles "
                         "outside the timed region; results do not depend on them)")
    ap.add_argument("--no-unbatched", action="store_true",
                    help="events64: skip the one-context-per-event comparison")
    ap.add_argument("--record-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "this benchmark with --copy-probe-mib into profiles/hbm_traffic_*.json")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB once (a "
                         "reference kernel of known traffic for hardware-counter runs)")
    return ap.parse_args()


def algorithmic_units(name, wl, R, t1, t2, bytes_per_real, nobs=None):
    """Algorithmic bytes (or flops) of one step for a stage, by its I/O
    contract: traffic of the pair buffer between the two draw passes and of
    the fields (the noise is generated in registers; sqrt(lambda) is read
    once per call in principle and not counted), 2 M n R flops for the grid
    GEMM."""
    M = wl.m * wl.m
    kept = t1 * wl.m                      # complex entries per pair kept after pass A
    b = bytes_per_real                    # 4 (FP32) or 8 (FP64) per real value
    per_real = {                          # per realization = half a pair
        "draw_noise_colfft": (2 * b * kept) / 2,               # writes the kept rows
        "draw_rowfft_crop": (2 * b * kept + 2 * b * M) / 2,    # reads them, writes 2 fields
    }
    if name in per_real:
        return per_real[name] * R, "bytes"
    if name == "krige_grid_gemm":
        return 2.0 * M * (nobs or wl.n) * R, "flops"
    return None, None


def run_path(prec, wl, xy, z, args, torch, cesim):
    R = wl.nreal
    batch = args.batch or R
    dtype = torch.float64 if prec == "fp64" else torch.float32
    fields = torch.empty((R, wl.m, wl.m), dtype=dtype, device="cuda")
    cov = cesim.make_cov(wl.nu, wl.sigma2, wl.range)
    grid = cesim.unit_square_grid(wl.m)
    info = {}
    nn = args.workload == "nn1024"

    def stations(ctx):
        """Local Kriging of the stations, or the nearest-neighbour surrogate
        sites; the values to condition on."""
        if nn:
            return ctx.nn_surrogate(xy, z, wl.tau2, wl.k)[1]
        ctx.offgrid(xy, wl.k)
        return z

    def step():
        ctx = cesim.Context(cov, grid, prec)
        if args.gemm_tile:
            ctx.set_param(cesim.PARAM_GEMM_TILE, args.gemm_tile)
        if args.chunk_pairs:
            ctx.set_param(cesim.PARAM_DRAW_CHUNK_PAIRS, args.chunk_pairs)
        ctx.set_param(cesim.PARAM_GEMM_SPLIT, SPLIT_PARAM[args.split])
        ctx.set_param(cesim.PARAM_JOINT_BOXES, 1 if args.joint else 0)
        zc = stations(ctx)
        for b0 in range(0, R, batch):
            nb = min(batch, R - b0)
            f = fields[b0:b0 + nb]
            ctx.simulate(nb, args.seed, b0, out=f)
            ctx.condition(zc, wl.tau2, f)
        st = ctx.stage_times(reset=True)
        info.update(ctx.info())
        ctx.close()
        return st

    if args.autotune:
        t0 = time.perf_counter()
        with cesim.Context(cov, grid, prec) as ctx:
            ctx.set_param(cesim.PARAM_GEMM_SPLIT, SPLIT_PARAM[args.split])
            stations(ctx)
            ctx.autotune(batch, fields[:batch])
        info["tune_ms"] = 1000.0 * (time.perf_counter() - t0)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stages = {}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    step_ms = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        st = step()                      # ends with the context's streams drained
        step_ms.append(1000.0 * (time.perf_counter() - ts))
        for k, (ms, calls) in st.items():
            a = stages.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += calls
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1000.0 * wall / args.steps
    finite = bool(torch.isfinite(fields).all().item())
    del fields
    torch.cuda.empty_cache()
    kernels = []
    bpr = 8 if prec == "fp64" else 4
    for name, (ms, calls) in stages.items():
        if calls == 0:
            continue
        units, kind = algorithmic_units(name, wl, R, info["t1"], info["t2"], bpr, info["nobs"])
        k = {"name": name, "ms_per_step": ms / args.steps, "launches_per_step": calls / args.steps,
             "avg_launch_ms": ms / calls}
        if kind == "bytes":
            gbs = units / (ms / args.steps / 1000.0) / 1e9
            k.update(bound="hbm", achieved=gbs, unit="GB/s", peak=HBM_PEAK_GBS,
                     frac=gbs / HBM_PEAK_GBS, algorithmic_bytes_per_launch=units / (calls / args.steps))
        elif kind == "flops":
            tf = units / (ms / args.steps / 1000.0) / 1e12
            peak = PEAK_TFLOPS["fp64" if prec == "fp64" else args.split]
            k.update(bound="mfma", achieved=tf, unit="TFLOP/s", peak=peak, frac=tf / peak,
                     algorithmic_flops_per_launch=units / (calls / args.steps))
        kernels.append(k)
    kernels.sort(key=lambda k: -k["ms_per_step"])
    return dict(ms_per_step=ms_step, value=R / (ms_step / 1000.0), kernels=kernels,
                step_ms=step_ms, median_ms_per_step=float(np.median(step_ms)),
                event_ms_per_step=ev0.elapsed_time(ev1) / args.steps, t1=info["t1"],
                nobs=info["nobs"],
                finite=finite, gamma_max=info.get("gamma_max"), tune_ms=info.get("tune_ms"))


# Stage -> (kernel name fragment, source files whose text the kernel is
# built from) for the recorded HBM counters.
COUNTED_STAGES = {
    "draw_noise_colfft": ("k_p2_cols_noise<float", ["ce.hip", "fft_pow2.hpp", "fft.hpp", "devmath.hpp"]),
    "draw_rowfft_crop": ("k_p2_rows_crop<float", ["ce.hip", "fft_pow2.hpp", "fft.hpp"]),
    "krige_grid_gemm": ("k_krige_split3", ["krige_mixed.hpp", "krige_tile1.hip", "devmath.hpp"]),
    "krige_predict_fp64": ("k_predict_f64", ["krige.hip", "devmath.hpp"]),
    "synth_obs_rhs": ("k_synth_rhs<float, false,", ["lk.hip", "devmath.hpp"]),
}


def _digest(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def recorded_traffic(stage, workload):
    """HBM bytes per launch of a stage from the counter runs recorded under
    profiles/, or None when a source of the kernel has changed since (its hash
    no longer matches) or no record exists for this workload."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.json")):
        try:
            with open(path) as f:
                rec = json.load(f)
            if rec.get("workload") != workload or stage not in rec.get("kernels", {}):
                continue
            srcs = rec["sources"].get(stage, [])
            if not srcs or any(_digest(rel) != digest for rel, digest in srcs):
                return None
            k = rec["kernels"][stage]
            return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
        except (OSError, ValueError, KeyError, TypeError):
            continue
    return None


def record_counters(fetch_csv, write_csv, probe_mib, workload):
    """Turn two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) of ``bench.py --copy-probe-mib probe_mib`` into HBM bytes per
    launch for the counted stages, each counter scaled by what it reads for
    the device copy of known size; writes profiles/hbm_traffic_<workload>.json
    and prints a markdown table."""
    import csv
    probe = probe_mib * (1 << 20)

    def load(path):
        rows = list(csv.DictReader(open(path)))
        cp = max((r for r in rows if "copyBuffer" in r["Kernel_Name"]),
                 key=lambda r: float(r["Counter_Value"]))
        return rows, float(cp["Counter_Value"]) * 1024.0

    frows, fprobe = load(fetch_csv)
    wrows, wprobe = load(write_csv)
    fs, ws = probe / fprobe, probe / wprobe
    rec = {"workload": workload, "precision": "mixed",
           "calibration": {"probe_bytes_each_way": probe, "fetch_scale": fs, "write_scale": ws},
           "sources": {}, "kernels": {}}
    lines = ["| stage | kernel | launches | FETCH_SIZE KiB/launch (raw) | WRITE_SIZE KiB/launch (raw) "
             "| HBM read GB/launch (scaled) | HBM write GB/launch (scaled) |",
             "|---|---|---:|---:|---:|---:|---:|"]
    for stage, (frag, files) in COUNTED_STAGES.items():
        fr = [float(r["Counter_Value"]) for r in frows if frag in r["Kernel_Name"]]
        wr = [float(r["Counter_Value"]) for r in wrows if frag in r["Kernel_Name"]]
        if not fr or not wr:
            continue
        name = next(r["Kernel_Name"] for r in frows if frag in r["Kernel_Name"])
        f_kib, w_kib = sum(fr) / len(fr), sum(wr) / len(wr)
        rec["kernels"][stage] = {"kernel": name, "launches": len(fr),
                                 "fetch_bytes_per_launch": f_kib * 1024.0 * fs,
                                 "write_bytes_per_launch": w_kib * 1024.0 * ws}
        rec["sources"][stage] = [[f"paper_2109_11044_amd/csrc/{f}",
                                  _digest(f"paper_2109_11044_amd/csrc/{f}")] for f in files]
        lines.append(f"| {stage} | `{name.split('(')[0][:60]}` | {len(fr)} | {f_kib:.1f} | {w_kib:.1f} "
                     f"| {f_kib * 1024 * fs / 1e9:.3f} | {w_kib * 1024 * ws / 1e9:.3f} |")
    out = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"calibration: FETCH_SIZE x {fs:.4f}, WRITE_SIZE x {ws:.4f}")
    print("\n".join(lines))
    print(f"wrote {out}")


def cpu_baseline(wl, xy, z, seed, nn=False):
    """The oracle timed on a bounded sample of the same workload, scaled to
    one step of R realizations (nn: the nearest-neighbour variant)."""
    from oracle import ce, kriging, localkrige, philox
    from oracle import nnkrige as onn
    from oracle.pipeline import Grid as OGrid
    from oracle.covariance import Cov
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = 1
    cov = Cov(wl.nu, wl.sigma2, wl.range)
    dx = wl.dx
    R = wl.nreal
    t = {}
    s0 = time.perf_counter()
    t1, t2, s, _ = ce.ce_setup(cov, dx, dx, wl.m, wl.m)
    t["setup"] = time.perf_counter() - s0
    s0 = time.perf_counter()
    if nn:
        sur = onn.surrogate(cov, OGrid.unit_square(wl.m), xy, z, wl.tau2, wl.k)
        sites, z = sur["xy"], sur["zN"]
    else:
        a, b, W, gamma = localkrige.local_krige(xy, cov, 0.0, 0.0, dx, dx, wl.m, wl.m, wl.k)
        sites = xy
    t["offgrid"] = time.perf_counter() - s0
    s0 = time.perf_counter()
    fac = (onn.surrogate_factor(cov, sites, wl.tau2, sur["sigmaN2"]) if nn
           else kriging.factor(xy, cov, wl.tau2))
    t["cholesky"] = time.perf_counter() - s0
    nd = 24
    s0 = time.perf_counter()
    y = ce.ce_draw(s, seed, range(nd), wl.m, wl.m)
    xi = philox.offgrid_noise(seed, len(sites), range(nd))
    if nn:
        zs = (y.reshape(nd, -1)[:, sur["idx"]]
              + np.sqrt(wl.tau2 + sur["sigmaN2"])[None, :] * xi)
    else:
        zs = localkrige.synthetic_obs(y, a, b, W, gamma, wl.tau2, xi)
    t["per_real_draw_synth"] = (time.perf_counter() - s0) / nd
    zsR = np.repeat(zs, R // nd + 1, axis=0)[:R]
    s0 = time.perf_counter()
    B = kriging.coefficients(fac, z, zsR)
    t["solve_R"] = time.perf_counter() - s0
    rows = np.arange(192)
    s0 = time.perf_counter()
    kriging.krige_to_grid(B, sites, cov, 0.0, 0.0, dx, dx, wl.m, wl.m, rows=rows, chunk_rows=8)
    t["krige_rows"] = time.perf_counter() - s0
    step = (t["setup"] + t["offgrid"] + t["cholesky"] + R * t["per_real_draw_synth"]
            + t["solve_R"] + t["krige_rows"] * wl.m / rows.size)
    return {"value": R / step, "unit": "conditional realizations/s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"full setup, {'surrogate sites' if nn else 'local Kriging'} and "
                       f"Cholesky; {nd} of {R} CE draws and "
                       f"synthetic data; solves for all {R}; {rows.size} of {wl.m} grid rows "
                       f"of the K12 product; scaled to one step of {R} realizations"),
            "seconds_measured": sum(t.values()), "host_cpus": len(os.sched_getaffinity(0))}


def events_main(args, torch, cesim, workloads):
    """64 uneven events (grids 128^2 / 256^2 / 512^2, Matern 1/2 or 3/2,
    anisotropic, 100-3000 clustered stations, 200 realizations each) planned
    as one batch; a step is one graph launch drawing the next 200 conditional
    realizations of every event.  The one-context-per-event path is timed
    beside it on the same events (steady state, factorisations reused)."""
    prec = "mixed" if args.precision in ("both", "mixed") else "fp64"
    table = workloads.event_table(64)
    evs = [dict(cov=cesim.make_cov(d["nu"], d["sigma2"], d["range"], d["aniso_ratio"],
                                   d["aniso_angle"]),
                grid=cesim.unit_square_grid(d["m"]), obs_xy=d["obs_xy"], z=d["z"],
                nugget=d["nugget"], k=d["k"], nreal=d["nreal"], first_real=0, seed=args.seed,
                event_id=d["event_id"])
           for d in workloads.event_inputs(table)]
    R = sum(ev["nreal"] for ev in evs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = cesim.Batch(evs, prec, autotune=args.autotune)
    plan_ms = 1000.0 * (time.perf_counter() - t0)
    tori = [b.info(e)["t1"] for e in range(len(evs))]
    for w in range(args.warmup):
        b.run(w * 200)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for st in range(args.steps):
        b.run((args.warmup + st) * 200)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1000.0 * wall / args.steps
    finite = all(bool(torch.isfinite(f).all().item()) for f in b.fields)
    b.close()
    out = {
        "metric": "conditional realizations/sec, 64 uneven events in one graph launch",
        "value": R / (ms_step / 1000.0), "unit": "conditional realizations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 FFT / fp16x3 GEMM (f64 setup, Cholesky, solves)" if prec == "mixed"
                 else "f64",
        "data": "synthetic",
        "config": {"workload": "events64_uneven_R200", "events": len(evs),
                   "realizations_per_step": R, "grids": sorted({wl.m for wl in table}),
                   "tori": sorted(set(tori)), "stations_total": sum(wl.n for wl in table),
                   "per_event": [[wl.m, t, wl.n] for wl, t in zip(table, tori)]},
        "events_per_s": len(evs) / (ms_step / 1000.0),
        "plan_ms": plan_ms, "autotuned_in_plan": bool(args.autotune),
        "graph_ms_per_step": ev0.elapsed_time(ev1) / args.steps,
        "finite": finite,
    }
    if not args.no_unbatched:
        ctxs = []
        for ev in evs:
            c = cesim.Context(ev["cov"], ev["grid"], prec)
            c.set_param(cesim.PARAM_EVENT_ID, ev["event_id"])
            c.offgrid(ev["obs_xy"], ev["k"])
            ctxs.append((c, torch.empty((ev["nreal"], ev["grid"].m2, ev["grid"].m1),
                                        dtype=torch.float32 if prec == "mixed"
                                        else torch.float64, device="cuda")))

        def unbatched(off):
            for (c, f), ev in zip(ctxs, evs):
                c.simulate(ev["nreal"], ev["seed"], off, out=f)
                c.condition(ev["z"], ev["nugget"], f)
        unbatched(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for st in range(args.steps):
            unbatched((1 + st) * 200)
        torch.cuda.synchronize()
        ms_u = 1000.0 * (time.perf_counter() - t0) / args.steps
        for c, _ in ctxs:
            c.close()
        out["unbatched"] = {"ms_per_step": ms_u, "value": R / (ms_u / 1000.0),
                            "batched_speedup": ms_u / ms_step}
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def grad_main(args, torch, cesim, workloads):
    """Gradient of the linear ensemble statistic at the differentiation
    workload (512^2 grid, Matern nu = 1, range 0.1, nugget 0.05, 2000
    clustered stations, 200 realizations): a step is one new context, the
    station set-up and ce_grad_linear (L and dL/d(range, sigma^2, nugget, z)).
    The forward ensemble (draw + condition of the 200 realizations and the
    weighted mean) is timed beside it."""
    wl = workloads.C4
    xy = wl.obs_xy()
    z = workloads.iid_values(wl.n, wl.sigma2 + wl.tau2)
    w = torch.as_tensor(np.random.default_rng(4).standard_normal((wl.m, wl.m)), device="cuda")
    cov = cesim.make_cov(wl.nu, wl.sigma2, wl.range)
    grid = cesim.unit_square_grid(wl.m)

    def step():
        with cesim.Context(cov, grid, "fp64") as ctx:
            ctx.offgrid(xy, wl.k)
            return ctx.grad_linear(z, wl.tau2, wl.nreal, args.seed, w)

    def forward(f):
        with cesim.Context(cov, grid, "fp64") as ctx:
            ctx.offgrid(xy, wl.k)
            ctx.simulate(wl.nreal, args.seed, out=f)
            ctx.condition(z, wl.tau2, f)
            return float((f * w).sum(dim=(1, 2)).mean())

    for _ in range(args.warmup):
        g = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = step()
    torch.cuda.synchronize()
    ms_step = 1000.0 * (time.perf_counter() - t0) / args.steps
    f = torch.empty((wl.nreal, wl.m, wl.m), dtype=torch.float64, device="cuda")
    Lf = forward(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Lf = forward(f)
    torch.cuda.synchronize()
    ms_fwd = 1000.0 * (time.perf_counter() - t0) / args.steps
    del f
    # a non-linear statistic: the weighted sum of the per-node ensemble
    # variances, differentiated through cesim.conditional_fields (forward
    # draw + condition, backward ce_grad_vjp over the 200 realizations)
    spec = dict(nu=wl.nu, grid=grid, obs_xy=xy, k=wl.k, nreal=wl.nreal, seed=args.seed)

    def variance_step():
        f64 = dict(dtype=torch.float64, requires_grad=True)
        th, s2 = torch.tensor(wl.range, **f64), torch.tensor(wl.sigma2, **f64)
        nug, zt = torch.tensor(wl.tau2, **f64), torch.tensor(z, **f64)
        v = cesim.conditional_fields(th, s2, nug, zt, spec)
        S = (w * v.var(dim=0, unbiased=False)).sum()
        S.backward()
        return float(S), float(th.grad), float(s2.grad), float(nug.grad)

    variance_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vs = variance_step()
    torch.cuda.synchronize()
    ms_var = 1000.0 * (time.perf_counter() - t0)
    out = {
        "metric": "gradients/sec of a linear ensemble statistic (range, sigma2, nugget, 2000 z)",
        "value": 1000.0 / ms_step, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "grad512_matern1_n2000cl_R200", "grid": "512x512", "nu": wl.nu,
                   "range": wl.range, "nugget": wl.tau2, "n_obs": wl.n, "k": wl.k,
                   "realizations": wl.nreal},
        "gradient": {"L": g["L"], "d_range": g["d_range"], "d_sigma2": g["d_sigma2"],
                     "d_nugget": g["d_nugget"], "d_z_norm": float(np.linalg.norm(g["d_z"]))},
        "forward_ensemble": {"ms": ms_fwd, "L": Lf,
                             "rel_diff_L": abs(Lf - g["L"]) / max(1.0, abs(Lf))},
        "variance_gradient": {"ms": ms_var, "S": vs[0], "d_range": vs[1], "d_sigma2": vs[2],
                              "d_nugget": vs[3],
                              "note": "S = sum_g w_g Var_r v_r[g] over the 200 realizations; "
                                      "forward ensemble + backward ce_grad_vjp"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = grad_cpu_baseline()
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as fh:
            fh.write(line + "\n")


def grad_cpu_baseline():
    """The oracle's reference adjoint on a bounded sample of the gradient
    workload: the same covariance, nugget, window and 200 realizations on a
    192^2 grid (384^2 torus) with 750 clustered stations."""
    from oracle import gradient as ograd
    from oracle.covariance import Cov as OCov
    from oracle.pipeline import Grid as OGrid
    from paper_2109_11044_amd import workloads
    wl = workloads.C4
    m, n = 192, 750
    xy = workloads.locations("clustered", n, seed=1)
    z = workloads.iid_values(n, wl.sigma2 + wl.tau2)
    w = np.random.default_rng(4).standard_normal((m, m))
    threads = os.environ.get("OMP_NUM_THREADS") or str(len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    ograd.linear_stat_gradient(OCov(wl.nu, wl.sigma2, wl.range), OGrid.unit_square(m), xy, z,
                               wl.tau2, wl.k, 2, wl.nreal, w, 2 * m, 2 * m)
    sec = time.perf_counter() - t0
    return {"value": 1.0 / sec, "unit": "gradients/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{m}^2 grid, {2 * m}^2 torus, {n} clustered stations, same covariance, "
                      f"nugget, window and {wl.nreal} realizations (not scaled)",
            "seconds_measured": sec}


def _sig3(x):
    """Values rounded to three significant figures (x > 0), on the device."""
    import torch
    s = torch.pow(10.0, torch.floor(torch.log10(x)) - 2.0)
    return torch.round(x / s) * s


def accuracy_main(args, torch, cesim, workloads):
    """Accuracy study of Sections 3.3-3.4 on the GPU: for each of the 18
    cases and each random configuration of 35 stations, the exact and the
    local-Kriging prediction standard errors on the 61 x 61 grid for
    n_p = 1..4 (ce_prediction_se, FP64).  Reports the fraction of nodes
    correct to three significant figures (Table 1's score) and the 95th
    percentile over the grid of E_L = 100 (SE_L - SE_E) / SE_E (the quantity
    behind the 1 % claim), mean and spread over configurations.  The timed
    region is the whole study: 18 contexts, and per configuration and n_p one
    station set-up and one standard-error map pair."""
    pads = [p if args.pad else 0 for p in workloads.STUDY_NP]
    grids = [cesim.Grid(*workloads.study_grid(p), 0, 0) for p in pads]
    m1, m2 = workloads.STUDY_GRID[:2]
    cases = workloads.study_cases()
    C = args.configs
    ks = [(2 * p) ** 2 for p in workloads.STUDY_NP]
    locs = [workloads.study_locations(c) for c in range(C)]

    zero = np.zeros(workloads.STUDY_NOBS)

    def study(ncases, nconf):
        frac = torch.zeros((2, ncases, len(ks), nconf), dtype=torch.float64, device="cuda")
        p95 = torch.zeros_like(frac)
        for ci, case in enumerate(cases[:ncases]):
            tau2 = case["tau"] ** 2
            for ki, k in enumerate(ks):
                p = pads[ki]
                with cesim.Context(cesim.make_cov(case["nu"], 1.0, case["theta"]), grids[ki],
                                   "fp64") as ctx:
                    for c in range(nconf):
                        ctx.offgrid(locs[c], k)
                        e, l = ctx.prediction_se(tau2)
                        ctx.nn_surrogate(locs[c], zero, tau2, k)
                        nn_e, _ = ctx.prediction_se(tau2)
                        # scored on the original 61 x 61 nodes
                        e = e.reshape(m2 + 2 * p, m1 + 2 * p)[p:p + m2, p:p + m1]
                        for mi, a in enumerate((l, nn_e)):
                            a = a.reshape(m2 + 2 * p, m1 + 2 * p)[p:p + m2, p:p + m1]
                            frac[mi, ci, ki, c] = (_sig3(a) == _sig3(e)).double().mean()
                            p95[mi, ci, ki, c] = torch.quantile(
                                (100.0 * (a - e) / e).reshape(-1), 0.95)
        return frac.cpu().numpy(), p95.cpu().numpy()

    study(1, 2)                                        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fr2, p2 = study(len(cases), C)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    frac, p95 = fr2[0], p2[0]
    maps = len(cases) * C * len(ks)
    rows = []
    for ci, case in enumerate(cases):
        rows.append({"nu": case["nu"], "theta": round(float(case["theta"]), 4), "tau": case["tau"],
                     "frac_sig3_mean": [float(v) for v in frac[ci].mean(axis=1)],
                     "frac_sig3_sd": [float(v) for v in frac[ci].std(axis=1, ddof=1)],
                     "p95_EL_pct_median": [float(v) for v in np.median(p95[ci], axis=1)],
                     "p95_EL_pct_max": [float(v) for v in p95[ci].max(axis=1)],
                     "configs_p95_under_1pct": [float(v) for v in (p95[ci] < 1.0).mean(axis=1)],
                     "nn_frac_sig3_mean": [float(v) for v in fr2[1, ci].mean(axis=1)],
                     "nn_p95_EN_pct_median": [float(v) for v in np.median(p2[1, ci], axis=1)],
                     "nn_configs_p95_abs_under_1pct": [float(v) for v in
                                                       (np.abs(p2[1, ci]) < 1.0).mean(axis=1)]})
    paper, paper_nn = {}, {}
    for name, dest in (("table1_local_kriging_sig3.txt", paper), ("table2_nn_kriging_sig3.txt",
                                                                   paper_nn)):
        golden = os.path.join(ROOT, "tests", "golden", name)
        if os.path.exists(golden):
            for r in np.loadtxt(golden):
                dest[f"theta={r[0]:g},tau={r[1]:g}"] = [float(r[2]), float(r[4]), float(r[6])]
    out = {
        "metric": "prediction-SE map triples/s (exact, local and nearest-neighbour Kriging) over "
                  "the 18-case accuracy study, 61x61 grid, 35 uniform stations",
        "value": maps / sec, "unit": "SE map triples/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": 1000.0 * sec, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"accuracy61_18cases_C{C}_np1-4" + ("_padded" if args.pad else ""),
                   "grid": "61x61 on [0,60]^2" + (", widened by n_p on every side for the "
                                                  "simulation, scored on the 61x61 nodes"
                                                  if args.pad else ""),
                   "n_obs": workloads.STUDY_NOBS, "configs_per_case": C, "n_p": list(workloads.STUDY_NP),
                   "maps": maps},
        "roofline": None,
        "roofline_note": "35 stations and 3721 nodes per map: launch and latency bound; the "
                         "standard-error kernels are measured against their roofline at scale by "
                         "--workload se1024",
        "cases": rows,
        "table1_paper_np1-3_means": paper,
        "table2_paper_np1-3_means": paper_nn,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = accuracy_cpu_baseline(workloads)
    _emit(out, args)


def accuracy_cpu_baseline(workloads, nconf=24):
    """The oracle's se_exact, se_local and se_nn on a bounded sample of the
    study: the first case, 24 configurations, n_p = 1..4."""
    from oracle import accuracy as acc
    from oracle import nnkrige as onn
    from oracle.covariance import Cov as OCov
    from oracle.pipeline import Grid as OGrid
    og = OGrid(*workloads.STUDY_GRID)
    case = workloads.study_cases()[0]
    cov = OCov(case["nu"], 1.0, case["theta"])
    threads = os.environ.get("OMP_NUM_THREADS") or str(len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    nmaps = 0
    for c in range(nconf):
        xy = workloads.study_locations(c)
        for p in workloads.STUDY_NP:
            acc.se_exact(cov, og, xy, case["tau"] ** 2)
            acc.se_local(cov, og, xy, case["tau"] ** 2, (2 * p) ** 2)
            onn.se_nn(cov, og, xy, case["tau"] ** 2, (2 * p) ** 2)
            nmaps += 1
    sec = time.perf_counter() - t0
    return {"value": nmaps / sec, "unit": "SE map triples/s", "cores": int(threads),
            "kind": "oracle", "sample": f"{nmaps} map triples: first case (nu 1/2, theta 6.68, "
                                        f"tau 0.1), {nconf} configurations, n_p = 1..4",
            "seconds_measured": sec}


def se_main(args, torch, cesim, workloads):
    """Prediction standard-error maps at scale: the 1024^2 headline workload
    (exponential, range 0.02, nugget 0.02, 5000 clustered stations, 6 x 6
    windows); a step is one ce_prediction_se call (both maps, every grid
    node).  Roofline of the GEMM of the solved rows with W1 K11 W1^T
    (2 M n^2 flops per map, FP64 matrix cores) and of the observation solves
    (2 M n^2 flops: two triangular solves per node)."""
    wl = workloads.DM
    xy = wl.obs_xy()
    grid = cesim.unit_square_grid(wl.m)
    M, n = wl.m * wl.m, wl.n
    with cesim.Context(cesim.make_cov(wl.nu, wl.sigma2, wl.range), grid, "fp64") as ctx:
        ctx.offgrid(xy, wl.k)
        ctx.set_param(cesim.PARAM_SE_CHUNK_NODES, args.se_chunk)
        ctx.set_timing(True)
        for _ in range(args.warmup):
            e, l = ctx.prediction_se(wl.tau2)
        ctx.stage_times(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            # a different nugget each step would refactor; the same one reuses
            # the observation factor, as repeated maps for one event do
            e, l = ctx.prediction_se(wl.tau2)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        st = ctx.stage_times(reset=True)
    finite = bool(torch.isfinite(e).all().item() and torch.isfinite(l).all().item())
    ratio = float((l / e).median())
    kern = []
    for name, (ms, calls) in st.items():
        if calls == 0:
            continue
        k = {"name": name, "ms_per_step": ms / args.steps,
             "launches_per_step": calls / args.steps, "avg_launch_ms": ms / calls}
        if name in ("se_gemm_xq", "obs_solve"):
            fl = 2.0 * M * n * n
            tf = fl / (ms / args.steps / 1000.0) / 1e12
            k.update(bound="mfma", achieved=tf, unit="TFLOP/s", peak=PEAK_TFLOPS["fp64"],
                     frac=tf / PEAK_TFLOPS["fp64"],
                     algorithmic_flops_per_launch=fl / (calls / args.steps))
        kern.append(k)
    kern.sort(key=lambda k: -k["ms_per_step"])
    dom = next(k for k in kern if k["name"] == "se_gemm_xq")
    out = {
        "metric": "prediction-SE map pairs/s (exact + local Kriging, every node) at 1024^2",
        "value": 1.0 / sec, "unit": "SE map pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * sec, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "se_" + wl.name.replace("_R1000", ""), "grid": f"{wl.m}x{wl.m}",
                   "n_obs": n, "k": wl.k, "covariance": "exponential sigma2=1 range=0.02",
                   "nugget": wl.tau2},
        "roofline": {"bound": "mfma", "kernel": dom["name"], "achieved": dom["achieved"],
                     "peak": dom["peak"], "unit": "TFLOP/s", "frac": dom["frac"],
                     "traffic": None, "avg_launch_ms": dom["avg_launch_ms"]},
        "kernels": kern, "finite": finite, "median_se_local_over_exact": ratio,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = se_cpu_baseline(workloads)
    _emit(out, args)


def se_cpu_baseline(workloads):
    """The oracle's se_exact and se_local on a bounded sample of the 1024^2
    map: 1100 clustered stations (the oracle's W1 K11 W1^T at 5000 stations
    alone is hours of host work) and 4096 sampled grid nodes."""
    from oracle import accuracy as acc
    from oracle.covariance import Cov as OCov
    from oracle.pipeline import Grid as OGrid
    wl = workloads.DM
    n, nodes = 1100, 8192
    xy = workloads.locations("clustered", n, seed=1)
    rows = np.random.default_rng(0).choice(wl.m * wl.m, nodes, replace=False)
    cov = OCov(wl.nu, wl.sigma2, wl.range)
    threads = os.environ.get("OMP_NUM_THREADS") or str(len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    acc.se_exact(cov, OGrid.unit_square(wl.m), xy, wl.tau2, rows)
    acc.se_local(cov, OGrid.unit_square(wl.m), xy, wl.tau2, wl.k, rows)
    sec = time.perf_counter() - t0
    return {"value": nodes / sec / (wl.m * wl.m), "unit": "SE map pairs/s", "cores": int(threads),
            "kind": "oracle", "sample": f"{nodes} sampled nodes of the 1024^2 grid with {n} "
                                        "clustered stations (not 5000), scaled to whole maps",
            "seconds_measured": sec}


def _emit(out, args):
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as fh:
            fh.write(line + "\n")


def main():
    args = parse()
    if args.record_counters:
        from paper_2109_11044_amd import workloads
        record_counters(args.record_counters[0], args.record_counters[1],
                        args.copy_probe_mib or 1024, workloads.DM.name)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py: the library runs on one GPU; multi-GPU runs are not supported "
              "(realizations would shard across GPUs with no per-realization exchange).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_2109_11044_amd import cesim, workloads
    cesim.lib()
    if args.workload == "events64":
        return events_main(args, torch, cesim, workloads)
    if args.workload == "grad512":
        return grad_main(args, torch, cesim, workloads)
    if args.workload == "accuracy61":
        return accuracy_main(args, torch, cesim, workloads)
    if args.workload == "se1024":
        return se_main(args, torch, cesim, workloads)
    cesim.set_default_timing(True)
    nn = args.workload == "nn1024"
    if nn:
        wl = workloads.NN
    else:
        wl = workloads.DM
        wl.m, wl.n, wl.nreal = args.m, args.n, args.nreal
    xy = wl.obs_xy()
    z = workloads.iid_values(wl.n, wl.sigma2 + wl.tau2)
    res = {}
    for prec in (["mixed", "fp64"] if args.precision == "both" else [args.precision]):
        res[prec] = run_path(prec, wl, xy, z, args, torch, cesim)
    head = res.get("mixed") or res["fp64"]
    dom = head["kernels"][0]
    gemm = [k for k in head["kernels"] if k.get("bound")]
    dom_k = max(gemm, key=lambda k: k["ms_per_step"]) if gemm else dom
    default_size = nn or (args.m, args.n, args.nreal) == (1024, 5000, 1000)
    wname = wl.name if default_size else "custom"
    head_prec = "mixed" if "mixed" in res else "fp64"
    for k in head["kernels"]:
        if head_prec == "mixed" and not args.batch and args.split == "fp16" and not nn:
            k["hbm_traffic_bytes_per_launch"] = recorded_traffic(k["name"], wname)
    roof = {"bound": dom_k.get("bound"), "kernel": dom_k["name"],
            "achieved": dom_k.get("achieved"), "peak": dom_k.get("peak"),
            "unit": dom_k.get("unit"), "frac": dom_k.get("frac"),
            "traffic": dom_k.get("hbm_traffic_bytes_per_launch"),
            "avg_launch_ms": dom_k["avg_launch_ms"]}
    out = {
        "metric": ("nearest-neighbour " if nn else "")
                  + "conditional realizations/sec at 1024^2 grid (mixed vs FP64 path); HBM GB/s %",
        "value": head["value"],
        "unit": "conditional realizations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ((f"f32 FFT / {args.split}x3 GEMM (f64 setup, Cholesky, solves)"
                   if args.split != "fp32" else "f32 FFT / f32 GEMM (f64 setup, Cholesky, solves)")
                  if "mixed" in res
                  else "f64"),
        "data": "synthetic",
        "config": {"workload": (wl.name if default_size
                                else f"exp{args.m}_n{args.n}cl_k36_R{args.nreal}")
                               + ("_joint" if args.joint else ""),
                   "grid": f"{wl.m}x{wl.m}", "torus": head["t1"], "n_obs": wl.n, "k": wl.k,
                   "method": "nearest-neighbour Kriging" if nn else "local Kriging",
                   "stations_conditioned_on": head["nobs"],
                   "covariance": "exponential sigma2=1 range=0.02", "nugget": wl.tau2,
                   "realizations_per_step": wl.nreal, "batch": args.batch or wl.nreal,
                   "joint_boxes": bool(args.joint)},
        "roofline": roof,
    }
    out["step_ms"] = {p: r["step_ms"] for p, r in res.items()}
    out["median_ms_per_step"] = {p: r["median_ms_per_step"] for p, r in res.items()}
    if "fp64" in res and "mixed" in res:
        out["fp64_path"] = {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_per_step"]}
        out["mixed_over_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    out["kernels"] = {p: r["kernels"] for p, r in res.items()}
    out["fft_passes_hbm_frac"] = {k["name"]: k["frac"] for k in head["kernels"]
                                  if k.get("bound") == "hbm"}
    out["finite"] = all(r["finite"] for r in res.values())
    out["autotune"] = {"enabled": bool(args.autotune),
                       "tune_ms": {p: r["tune_ms"] for p, r in res.items()}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, xy, z, args.seed, nn)
    if args.copy_probe_mib:
        nel = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * nel * 4
        del src, dst
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
