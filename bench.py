#!/usr/bin/env python3
"""Energy points/s of the fused outer-region R-matrix loop on one MI355X.

One step = the whole hot path (R-matrix contraction, near-pole FP64 correction
in split mode, channel split + asymptotic functions, matching + LU K solve,
S/T/Omega) over every energy of the workload, with the partial wave's poles and
amplitudes resident in HBM and the energies already on the device.

Workload: one partial wave with 1500 channels (375 targets), 60000 poles in
[-2, 60] Ry, z = 5, a = 12 bohr, 1000 energies uniform in [0.01, 8] Ry, seeded
synthetic data.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "f64": 78.6}  # MI355X dense MFMA TFLOP/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rform_c4_traffic.md")
RFORM_SOURCES = [os.path.join(ROOT, "paper_1909_07321_amd", "csrc", f)
                 for f in ("k_rform.hip", "k_common.h", "rm_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rform_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in RFORM_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` (name and tile shape, e.g. "k_rform_f32
    tile=32x4") from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (already scaled by the copy-kernel calibration), or None if there is none or
    the kernel's sources changed since it was taken."""
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"^traffic: %s fetch_bytes=(\S+) write_bytes=(\S+) source_sha256=(\S+)" % re.escape(kernel),
                  text, re.M)
    if not m or m.group(3) != rform_source_sha():
        return None
    return float(m.group(1)) + float(m.group(2))


def request_cost(pw, ne: int) -> float:
    """Flops of a request: per energy the R contraction n(n+1)M (symmetric half)
    plus the LU of the n x n matching matrix, (2/3) n^3."""
    n = float(pw.nchan)
    return ne * (n * (n + 1) * pw.npole + 2.0 / 3.0 * n ** 3)


def serve_measure(ctx, nreq: int, block_max: int, load: float = 0.7) -> dict:
    """Open-loop Poisson streams through rm_submit/rm_poll on a pool of 16
    resident partial waves (channel counts log-uniform in 10..2000, 30-40 poles
    per channel, energies in [0.01, 8] Ry, blocks log-uniform in
    100..block_max energies), once all-FP64 and once all-FP32-split.

    Per-point cost spans about seven decades over the pool, so the load is set
    in flops: a closed-loop burst of the stream's first 16 requests measures
    the capacity in flop/s, and the arrival rate is load x capacity / mean
    request cost.  Reported beside the latencies: the offered rate and the
    served rate (both in flop/s and energy points/s) and the capacity."""
    import numpy as np

    from paper_1909_07321_amd import rm, synth

    pool = synth.config5_pool(16, 2000)
    ids = [ctx.pw_upload(p) for p in pool]
    block = (100, block_max)

    def run_stream(reqs, prec, scale=None):
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            if scale:
                wait = t0 + r.arrival_s * scale - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
            t, _ = ctx.submit(ids[r.pw_index], r.energies, prec=prec)
            tickets.append(t)
        stats, pending = [], set(tickets)
        while pending:
            for t in list(pending):
                st = ctx.poll(t)
                if st is not None:
                    stats.append(st)
                    pending.discard(t)
            time.sleep(0.0005)
        return time.perf_counter() - t0, stats

    out = {}
    base = synth.config5_requests(pool, nreq=nreq, rate_hz=1.0, block_range=block)  # arrivals at 1 request/s
    cost = np.array([request_cost(pool[r.pw_index], r.energies.size) for r in base])
    pts = int(sum(r.energies.size for r in base))
    for name, prec in (("fp64", rm.FP64), ("split", rm.FP32_SPLIT)):
        burst = base[:16]
        dt, _ = run_stream(burst, prec)
        capacity = float(cost[:16].sum()) / dt                       # flop/s, closed loop
        rate = load * capacity / float(cost.mean())                   # requests/s
        log(f"serving {name}: capacity {capacity / 1e12:.1f} TFLOP/s from the first 16 requests ({dt:.1f} s); "
            f"stream of {nreq} requests at {rate:.2f}/s follows")
        dt, stats = run_stream(base, prec, scale=1.0 / rate)
        lat = np.array([(st["t_done_ns"] - st["t_arrive_ns"]) * 1e-6 for st in stats])
        span = base[-1].arrival_s / rate                              # offered over the arrival window
        out[name] = dict(requests=nreq, load=load, arrival_rate_hz=rate,
                         capacity_tflops=capacity / 1e12,
                         offered_tflops=float(cost.sum()) / span / 1e12,
                         served_tflops=float(cost.sum()) / dt / 1e12,
                         offered_points_per_s=pts / span, points=pts, points_per_s=pts / dt,
                         p50_ms=float(np.median(lat)), p99_ms=float(np.quantile(lat, 0.99)),
                         max_ms=float(lat.max()))
        o_ = out[name]
        log(f"serving {name}: {nreq} requests at {rate:.2f}/s, capacity {o_['capacity_tflops']:.1f} TFLOP/s, offered "
            f"{o_['offered_tflops']:.1f}, served {o_['served_tflops']:.1f} TFLOP/s ({o_['points_per_s']:.0f} points/s), "
            f"p50 {o_['p50_ms']:.0f} ms, p99 {o_['p99_ms']:.0f} ms")
    for i in ids:
        ctx.pw_release(i)
    out["pool"] = "16 partial waves, n log-uniform 10..2000, 30-40 poles/channel"
    out["blocks"] = (f"log-uniform {block[0]}..{block[1]} energies"
                     + ("" if block_max >= 20000 else " (capped below the 20000 of the full stream to bound the run)"))
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pw, E, threads: int, budget_s: float) -> dict:
    """The FP64 oracle (plain long-double C, OpenMP over the R rows of one
    energy) on the host cores, over an evenly spaced subsample of the grid: the
    planned sample is every 31st energy (32 points); as many of those as fit in
    budget_s are timed, spread evenly over the grid, starting mid-grid."""
    import numpy as np

    import oracle
    threads = threads or len(os.sched_getaffinity(0))
    plan = np.arange(0, E.size, 31)
    o = oracle.Oracle(pw, nthreads=threads)
    order = [plan[plan.size // 2]]
    t3 = time.perf_counter()
    o.run(E[order], want_K=False)
    t_one = time.perf_counter() - t3
    n_fit = int(min(plan.size, max(1, budget_s // t_one)))
    if n_fit > 1:
        spread = [int(i) for i in plan[np.linspace(0, plan.size - 1, n_fit).round().astype(int)]]
        rest = [i for i in spread if i != order[0]][:n_fit - 1]
        o.run(E[rest], want_K=False)
        order += rest
    dt = time.perf_counter() - t3
    idx = sorted(int(i) for i in order)
    out = dict(value=len(idx) / dt, unit="energy points/s", cores=threads, kind="oracle",
               cpu_model=cpu_model(),
               sample=f"{len(idx)} of the 32 planned energies (every 31st grid point; fitted to a {budget_s:.0f} s "
                      f"budget) at grid indices {idx}, full path R -> asymptotics -> K -> Omega in long double, "
                      f"{dt:.1f} s on {threads} threads ({cpu_model()})")
    log(f"cpu oracle: {out['value']:.4f} points/s on {threads} threads, {len(idx)} energies in {dt:.1f} s")
    # the 200-channel workload: 32 evenly spaced energies of its 2000
    from paper_1909_07321_amd import synth
    pw2, E2 = synth.config2()
    sel = E2[np.linspace(0, E2.size - 1, 32).round().astype(int)]
    o2 = oracle.Oracle(pw2, nthreads=threads)
    t4 = time.perf_counter()
    o2.run(sel, want_K=False)
    dt2 = time.perf_counter() - t4
    out["c2"] = dict(value=sel.size / dt2, unit="energy points/s", cores=threads,
                     sample=f"32 evenly spaced energies of the 200-channel workload's 2000, {dt2:.1f} s")
    log(f"cpu oracle, 200 channels: {sel.size / dt2:.2f} points/s on {threads} threads")
    return out


STAGES = ("rform", "nearpole", "asym", "ksolve", "somega", "prop")


def drain_prof(ctx):
    return {s_: ctx.prof_read(s_) for s_ in STAGES}


def config_measure(ctx) -> dict:
    """Throughput on the other workloads: the 200-channel wave (2000 energies,
    both modes, one rm_run each) and the batch of 64 waves of 20..600 channels
    (5000 energies each, FP64, one rm_run_batch).  R-stage points/s come from
    the same run's R-contraction launch times."""
    import torch

    from paper_1909_07321_amd import rm, synth

    dev = torch.device("cuda", 0)
    out = {}
    pw, E = synth.config2()
    pid = ctx.pw_upload(pw)
    Ed = torch.tensor(E, dtype=torch.float64, device=dev)
    om = torch.empty((E.size, pw.ntarget, pw.ntarget), dtype=torch.float64, device=dev)
    st = torch.empty(E.size, dtype=torch.int32, device=dev)
    for name, prec in (("fp64", rm.FP64), ("split", rm.FP32_SPLIT)):
        ctx.run(pid, Ed, prec=prec, want_K=False, out=(om, None, st))
        torch.cuda.synchronize()
        drain_prof(ctx)
        ctx.prof_enable(True)
        t1 = time.perf_counter()
        ctx.run(pid, Ed, prec=prec, want_K=False, out=(om, None, st))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ctx.prof_enable(False)
        rf_ms, _, rf_e = drain_prof(ctx)["rform"]
        out[f"c2_{name}"] = dict(points_per_s=E.size / dt, r_stage_points_per_s=rf_e / (rf_ms * 1e-3),
                                 workload="one wave, 200 channels, 6000 poles, 2000 energies in [0.01, 6] Ry")
        log(f"c2 {name}: {E.size / dt:.0f} points/s (R stage {rf_e / (rf_ms * 1e-3):.0f} points/s)")
    ctx.pw_release(pid)

    t0 = time.time()
    pws, E = synth.config3()
    ids = [ctx.pw_upload(p) for p in pws]
    log(f"c3 workload generated in {time.time() - t0:.1f}s: {len(pws)} waves, {E.size} energies each")
    Ed = torch.tensor(E, dtype=torch.float64, device=dev)
    # tile autotuner: up to 4 waves of each size bucket, every R tile shape, one choice per bucket
    byb = {}
    for p, i in zip(pws, ids):
        byb.setdefault(rm.tile_bucket(p.nchan), []).append(i)
    t0 = time.time()
    for b, lst in sorted(byb.items()):
        ctx.tune(rm.FP64, lst[:4], E[::20][:256], reps=1)
    tiles = {b: rm.tile_shapes(rm.FP64)[ctx.get_tile(rm.FP64, b)] for b in sorted(byb)}
    log(f"c3 tuned in {time.time() - t0:.1f}s: tile shape per size bucket {tiles}")
    ctx.run_batch([(i, Ed[:64]) for i in ids], prec=rm.FP64)  # warm-up: workspaces and code
    torch.cuda.synchronize()
    drain_prof(ctx)
    ctx.prof_enable(True)
    t1 = time.perf_counter()
    res = ctx.run_batch([(i, Ed) for i in ids], prec=rm.FP64)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    ctx.prof_enable(False)
    rf_ms, _, rf_e = drain_prof(ctx)["rform"]
    flagged = int(sum(int((r[2] != 0).sum().item()) for r in res))
    del res
    pts = len(ids) * E.size
    flops = sum(float(p.nchan) * (p.nchan + 1) * p.npole for p in pws) * E.size
    out["c3_fp64"] = dict(points_per_s=pts / dt, r_stage_points_per_s=rf_e / (rf_ms * 1e-3),
                          r_tflops=flops / (rf_ms * 1e-3) / 1e12, seconds=dt, flagged_energies=flagged,
                          tiles={str(b): dict(side=t[0], energies_per_task=t[1]) for b, t in tiles.items()},
                          workload="64 waves, 20..600 channels, 30 poles per channel, 5000 energies each, "
                                   "one rm_run_batch call")
    log(f"c3 fp64: {pts / dt:.0f} points/s over {dt:.1f}s (R stage {rf_e / (rf_ms * 1e-3):.0f} points/s, "
        f"{flops / (rf_ms * 1e-3) / 1e12:.1f} TFLOP/s)")
    for i in ids:
        ctx.pw_release(i)

    # sum over partial waves with the load-balance family (16 waves of 72..634
    # channels sharing 150 targets), wave order and the permuted (J pi, E) order
    pws, E = synth.config_imbalance()
    out["imbalance"] = imbalance_measure(ctx, pws, E)
    out["coupled"] = coupled_measure(ctx)
    return out


def coupled_measure(ctx) -> dict:
    """The coupled workload (100 channels with dipole and quadrupole potentials,
    1000 energies, Numerov propagation from r1 = 30 to a = 12 on 3201 points):
    points/s of rm_run and the propagation stage against the FP64 MFMA peak.
    The propagation's model flops per energy are those of its two coupling
    products per step, (npts - 1) * 2 * 2 n^2 m lamax with m = n + n_o solution
    columns (the series W + P W + P^2 W and U Y = U W + U P W)."""
    import torch

    from paper_1909_07321_amd import rm, synth

    pw, cp, E = synth.config_coupled()
    pid = ctx.pw_upload(pw, cp)
    ctx.set_propagation(cp["npts"], cp["stab"])
    Ed = torch.tensor(E, dtype=torch.float64, device="cuda")
    om = torch.empty((E.size, pw.ntarget, pw.ntarget), dtype=torch.float64, device="cuda")
    st = torch.empty(E.size, dtype=torch.int32, device="cuda")
    ctx.run(pid, Ed, prec=rm.FP64, want_K=False, out=(om, None, st))  # warm-up: workspace, graphs
    torch.cuda.synchronize()
    drain_prof(ctx)
    ctx.prof_enable(True)
    t1 = time.perf_counter()
    ctx.run(pid, Ed, prec=rm.FP64, want_K=False, out=(om, None, st))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    ctx.prof_enable(False)
    stages = drain_prof(ctx)
    n, lam = pw.nchan, cp["cf"].shape[0]
    m = n + (E[:, None] - pw.e_thr[None, :] > 0).sum(axis=1)  # solution columns per energy
    flops = float(((cp["npts"] - 1) * 2 * 2 * n * n * lam * m).sum())
    pr_ms = stages["prop"][0]
    achieved = flops / (pr_ms * 1e-3) / 1e12
    flagged = int((st.cpu().numpy() != 0).sum())
    ctx.pw_release(pid)
    ctx.set_propagation()
    res = dict(points_per_s=E.size / dt, seconds=dt, flagged_energies=flagged,
               stage_ms={k: v[0] for k, v in stages.items()},
               roofline=dict(bound="mfma", achieved=achieved, peak=PEAK["f64"], unit="TFLOP/s",
                             frac=achieved / PEAK["f64"], kernel="propagation stage (k_prop_start, k_numerov, "
                             "k_prop_stab)", model_flops=flops),
               workload=f"one coupled wave, {n} channels, lamax {lam}, {pw.npole} poles, {E.size} energies in "
                        f"[{E[0]}, {E[-1]}] Ry, Numerov from r1 = {cp['r1']} to a = {pw.a} on {cp['npts']} "
                        f"points, recombination every {cp['stab']} steps, FP64")
    log(f"coupled: {res['points_per_s']:.0f} points/s over {dt:.2f}s; propagation {pr_ms:.1f} ms "
        f"({achieved:.2f} TFLOP/s model, {100 * achieved / PEAK['f64']:.1f}% of the FP64 peak); stages "
        + ", ".join(f"{k}={v:.1f}ms" for k, v in res["stage_ms"].items()))
    return res


def mqdt_measure(ctx) -> dict:
    """The quantum-defect workload (the Rydberg series below the highest
    threshold: 1500 channels, 60000 poles, 2000 energies in the 0.4 Ry below
    it, coarse step 8): fine-mesh points/s of rm_run_mqdt against rm_run on
    the same mesh, both FP64 with Omega only, and Omega of the interpolated
    points against the direct one (elementwise above 1e-12 of each energy's
    largest entry, the points that are not coarse)."""
    import numpy as np
    import torch

    from paper_1909_07321_amd import rm, synth

    t0 = time.time()
    pw, E, ieq, fnumin = synth.config_mqdt()
    log(f"mqdt workload generated in {time.time() - t0:.1f}s")
    pid = ctx.pw_upload(pw)
    Ed = torch.tensor(E, dtype=torch.float64, device="cuda")
    ctx.run_mqdt(pid, Ed[:64], ieq, fnumin, want_K=False)  # warm-up: workspace and code
    ctx.run(pid, Ed[:64], want_K=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    om, _, co, st = ctx.run_mqdt(pid, Ed, ieq, fnumin, want_K=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    t1 = time.perf_counter()
    om2, _, st2 = ctx.run(pid, Ed, want_K=False)
    torch.cuda.synchronize()
    dt2 = time.perf_counter() - t1
    fine = ((co == 0) & (st == 0) & (st2 == 0)).cpu().numpy()
    b = om2.reshape(E.size, -1)
    top = b.abs().amax(dim=1, keepdim=True)
    den = torch.maximum(b.abs(), 1e-12 * top)

    def err(x):
        return ((x.reshape(E.size, -1) - b).abs() / den).amax(dim=1).cpu().numpy()

    eo = err(om)[fine]
    co_n, st_n = int(co.sum().item()), int((st != 0).sum().item())
    del om
    # the same in FP32-split precision (the coarse points' R contraction and the
    # direct path's), Omega against the FP64 direct one
    ctx.run_mqdt(pid, Ed[:64], ieq, fnumin, want_K=False, prec=rm.FP32_SPLIT)
    ctx.run(pid, Ed[:64], want_K=False, prec=rm.FP32_SPLIT)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    oms, _, _, sts = ctx.run_mqdt(pid, Ed, ieq, fnumin, want_K=False, prec=rm.FP32_SPLIT)
    torch.cuda.synchronize()
    dts = time.perf_counter() - t1
    t1 = time.perf_counter()
    oms2, _, sts2 = ctx.run(pid, Ed, want_K=False, prec=rm.FP32_SPLIT)
    torch.cuda.synchronize()
    dts2 = time.perf_counter() - t1
    ok = ((sts == 0) & (sts2 == 0)).cpu().numpy()
    es, es2 = err(oms)[ok & fine], err(oms2)[ok & fine]
    del oms, oms2, om2, b, den
    split = dict(points_per_s=E.size / dts, direct_points_per_s=E.size / dts2, speedup=dts2 / dts,
                 omega_err_vs_fp64_direct=dict(median=float(np.median(es)), p99=float(np.quantile(es, 0.99))),
                 direct_omega_err_vs_fp64_direct=dict(median=float(np.median(es2)),
                                                      p99=float(np.quantile(es2, 0.99))))
    log(f"mqdt split: {split['points_per_s']:.0f} points/s against {split['direct_points_per_s']:.0f} points/s "
        f"direct split ({split['speedup']:.2f}x); Omega vs the FP64 direct one median "
        f"{split['omega_err_vs_fp64_direct']['median']:.1e} (direct split "
        f"{split['direct_omega_err_vs_fp64_direct']['median']:.1e})")
    ctx.pw_release(pid)
    res = dict(points_per_s=E.size / dt, seconds=dt, direct_points_per_s=E.size / dt2, direct_seconds=dt2,
               speedup=dt2 / dt, coarse_points=co_n, flagged_energies=st_n,
               omega_err_vs_direct=dict(median=float(np.median(eo)), p99=float(np.quantile(eo, 0.99)),
                                        max=float(eo.max())),
               split=split,
               workload=f"one wave, {pw.nchan} channels, {pw.npole} poles in [9.5, 60] Ry, {E.size} energies in "
                        f"[{E[0]:.4f}, {E[-1]:.4f}] Ry (0.4 Ry below the highest threshold), coarse step {ieq}, "
                        f"fnumin {fnumin:.3f}, FP64")
    log(f"mqdt: {res['points_per_s']:.0f} points/s over {dt:.2f}s ({co_n} coarse of {E.size}) against "
        f"{res['direct_points_per_s']:.0f} points/s direct ({res['speedup']:.2f}x); Omega vs direct median "
        f"{res['omega_err_vs_direct']['median']:.1e} p99 {res['omega_err_vs_direct']['p99']:.1e} max "
        f"{res['omega_err_vs_direct']['max']:.1e}")
    return res


def imbalance_measure(ctx, pws, E) -> dict:
    """Omega summed over a family of partial waves in both chunk orders, with
    the per-chunk GPU time distribution: max/mean and coefficient of variation
    of the chunk times, and how chunk time follows the chunk's model flops and
    open fraction n_o/n (the single-GPU view of the paper's per-processor load
    balance)."""
    import numpy as np
    import torch

    from paper_1909_07321_amd import rm

    ids = [ctx.pw_upload(p) for p in pws]
    Ed = torch.tensor(E, dtype=torch.float64, device="cuda")
    ctx.run_sum(ids, Ed[:64])
    torch.cuda.synchronize()
    res = {}
    for name, order in (("wave", rm.ORDER_WAVE), ("permuted", rm.ORDER_PERMUTED)):
        ctx.run_sum(ids, Ed, prec=rm.FP64, order=order)   # warm-up: workspaces, graphs
        torch.cuda.synchronize()
        drain_prof(ctx)
        ctx.prof_chunks()
        ctx.prof_enable(True)
        t1 = time.perf_counter()
        ctx.run_sum(ids, Ed, prec=rm.FP64, order=order)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ctx.prof_enable(False)
        ch = ctx.prof_chunks()
        drain_prof(ctx)
        ms, fl, of = ch["ms"], ch["model_flops"], ch["open_frac"]
        rate = fl / (ms * 1e-3) / 1e12
        res[name] = dict(points_per_s=len(ids) * E.size / dt, seconds=dt, chunks=int(ms.size),
                         chunk_ms=dict(mean=float(ms.mean()), max=float(ms.max()), min=float(ms.min()),
                                       max_over_mean=float(ms.max() / ms.mean()), cv=float(ms.std() / ms.mean()),
                                       sum=float(ms.sum())),
                         chunk_model_tflop=dict(mean=float(fl.mean() / 1e12), max=float(fl.max() / 1e12),
                                                max_over_mean=float(fl.max() / fl.mean())),
                         chunk_tflops=dict(min=float(rate.min()), median=float(np.median(rate)),
                                           max=float(rate.max())),
                         corr_ms_vs_model=float(np.corrcoef(ms, fl)[0, 1]) if ms.size > 2 else None,
                         open_frac=dict(min=float(of.min()), max=float(of.max())))
        r = res[name]
        log(f"imbalance ({name} order): {r['points_per_s']:.0f} points/s over {dt:.2f}s, {r['chunks']} chunks, "
            f"chunk ms mean {r['chunk_ms']['mean']:.1f} max/mean {r['chunk_ms']['max_over_mean']:.2f} "
            f"cv {r['chunk_ms']['cv']:.2f}, model TFLOP/s per chunk {r['chunk_tflops']['min']:.1f}.."
            f"{r['chunk_tflops']['max']:.1f}, corr(ms, model) {r['corr_ms_vs_model']:.2f}, "
            f"open fraction {r['open_frac']['min']:.2f}..{r['open_frac']['max']:.2f}")
    for i in ids:
        ctx.pw_release(i)
    res["workload"] = (f"{len(pws)} waves sharing {pws[0].ntarget} targets, {min(p.nchan for p in pws)}.."
                       f"{max(p.nchan for p in pws)} channels, 30 poles per channel, {E.size} energies in "
                       f"[{E[0]}, {E[-1]}] Ry, FP64, Omega summed over the waves")
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["split", "fp64", "both"], default="both",
                    help="headline mode is FP32-split; 'both' also times FP64")
    ap.add_argument("--nenergy", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads for the CPU baseline (0 = every core this process may run on)")
    ap.add_argument("--cpu-budget", type=float, default=30.0,
                    help="seconds of oracle time for the CPU baseline sample")
    ap.add_argument("--serving", type=int, default=100, metavar="NREQ",
                    help="requests per mode in the serving measurement (0 = skip)")
    ap.add_argument("--serving-block-max", type=int, default=2000,
                    help="largest energy block of a serving request (the full stream goes to 20000)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 200-channel and 64-wave batch throughput measurements")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default R tile shapes instead of running the tile autotuner first")
    ap.add_argument("--coupled-only", action="store_true",
                    help="run only the coupled-wave (Numerov propagation) measurement and print its JSON block")
    ap.add_argument("--mqdt-only", action="store_true",
                    help="only the quantum-defect workload (coarse/fine mesh against the direct path)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a 1 GiB read + 1 GiB write kernel (HBM counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; there is no multi-GPU path "
              "(each partial wave and energy is independent, so points would be dealt out over GPUs; that is not built)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1909_07321_amd import rm, synth

    if args.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)  # one elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB write elementwise kernel done")
        del src, dst

    if args.coupled_only:
        ctx = rm.Context(0)
        print(json.dumps({"coupled": coupled_measure(ctx)}), flush=True)
        ctx.close()
        return 0
    if args.mqdt_only:
        ctx = rm.Context(0)
        print(json.dumps({"mqdt": mqdt_measure(ctx)}), flush=True)
        ctx.close()
        return 0

    # the quantum-defect leg first, in a context of its own that is closed
    # before the headline's (both paths of its comparison need a full-size
    # workspace); a failure there is recorded, never fatal to the headline
    mqdt = None
    if not args.no_configs:
        try:
            mctx = rm.Context(0)
            mqdt = mqdt_measure(mctx)
            mctx.close()
        except Exception as exc:  # noqa: BLE001 -- reported in the JSON line
            log(f"mqdt leg failed: {exc}")
            mqdt = dict(error=str(exc))
        torch.cuda.empty_cache()

    t0 = time.time()
    pw, E = synth.config4(args.nenergy)
    log(f"workload generated in {time.time() - t0:.1f}s: n={pw.nchan} M={pw.npole} ne={E.size}")
    ctx = rm.Context(0)
    pid = ctx.pw_upload(pw)
    dev = torch.device("cuda", 0)
    Ed = torch.tensor(E, dtype=torch.float64, device=dev)
    om = torch.empty((E.size, pw.ntarget, pw.ntarget), dtype=torch.float64, device=dev)
    st = torch.empty(E.size, dtype=torch.int32, device=dev)
    flops_R = float(pw.nchan) * (pw.nchan + 1) * pw.npole  # per energy: n(n+1)M, symmetric half

    modes = {"split": [("split", rm.FP32_SPLIT)], "fp64": [("fp64", rm.FP64)],
             "both": [("split", rm.FP32_SPLIT), ("fp64", rm.FP64)]}[args.prec]
    results = {}
    for name, prec in modes:
        # tile autotuner: time every R tile shape on a slice of the grid, keep the fastest
        tune_ms = None
        if not args.no_tune:
            tune_ms = ctx.tune(prec, [pid], E[::4][:256], reps=1)[0].tolist()
        shape = ctx.get_tile(prec, rm.tile_bucket(pw.nchan))
        tile = rm.tile_shapes(prec)[shape]
        log(f"{name}: tile shapes {rm.tile_shapes(prec)} tuned at "
            f"{[round(x, 1) for x in tune_ms] if tune_ms else 'default'} ms -> {tile}")
        for _ in range(args.warmup):
            ctx.run(pid, Ed, prec=prec, want_K=False, out=(om, None, st))
        torch.cuda.synchronize()
        for s in ("rform", "nearpole", "asym", "ksolve", "somega"):
            ctx.prof_read(s)
        ctx.prof_enable(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            ctx.run(pid, Ed, prec=prec, want_K=False, out=(om, None, st))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ctx.prof_enable(False)
        stages = {s: ctx.prof_read(s) for s in ("rform", "nearpole", "asym", "ksolve", "somega")}
        stat = st.cpu().numpy()
        ms_step = (t2 - t1) * 1e3 / args.steps
        rf_ms, rf_n, rf_e = stages["rform"]
        achieved = flops_R * rf_e / (rf_ms * 1e-3) / 1e12 if rf_ms > 0 else None
        dt = "f32" if prec == rm.FP32_SPLIT else "f64"
        kname = ("k_rform_f32" if dt == "f32" else "k_rform_f64") + f" tile={tile[0]}x{tile[1]}"
        results[name] = dict(
            value=E.size * args.steps / (t2 - t1), ms_per_step=ms_step,
            flagged_energies=int((stat != 0).sum()),
            tile=dict(side=tile[0], energies_per_task=tile[1], tuned_ms=tune_ms),
            stage_ms_per_step={s: v[0] / args.steps for s, v in stages.items()},
            roofline=dict(bound="mfma", achieved=achieved, peak=PEAK[dt], unit="TFLOP/s",
                          frac=(achieved / PEAK[dt]) if achieved else None, traffic=measured_traffic(kname),
                          traffic_GBps=(measured_traffic(kname) / (rf_ms / rf_n * 1e-3) / 1e9
                                        if measured_traffic(kname) and rf_n else None),
                          kernel=kname,
                          launches=rf_n, avg_launch_ms=rf_ms / max(rf_n, 1),
                          flops_per_launch=flops_R * rf_e / max(rf_n, 1)))
        log(f"{name}: {results[name]['value']:.1f} points/s, {ms_step:.1f} ms/step, stages "
            + ", ".join(f"{s}={v[0] / args.steps:.1f}ms" for s, v in stages.items())
            + (f", R contraction {achieved:.1f} TFLOP/s" if achieved else ""))

    serving = None
    if args.serving > 0:
        serving = serve_measure(ctx, args.serving, args.serving_block_max)
    configs = None if args.no_configs else config_measure(ctx)
    if configs is not None:
        configs["mqdt"] = mqdt

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(pw, E, args.cpu_threads, args.cpu_budget)

    head = results.get("split") or results.get("fp64")
    head_name = "split" if "split" in results else "fp64"
    line = {
        "metric": "energy points/s at 1500 ch (FP64 vs FP32-split); MFMA %; p99 latency",
        "value": head["value"], "unit": "energy points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if head_name == "split" else "f64", "data": "synthetic",
        "config": {"workload": "one partial wave, 1500 channels, 60000 poles, 1000 energies in [0.01, 8] Ry "
                               "(z=5, a=12)", "nchan": pw.nchan, "npole": pw.npole, "nenergy": int(E.size),
                   "precision": "fp32-split (delta=0.05 Ry)" if head_name == "split" else "fp64"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "modes": results,
        "serving": serving,
        "configs": configs,
        "graphs": dict(zip(("captured", "replayed"), ctx.graph_stats())),
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
