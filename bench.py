"""Benchmark of the Z4c RHS + RK4 step on one MI355X.

One "step" is one classical RK4 step (four fused substeps, each preceded by
its ghost work) of the whole box.  Default workload: the 256^3 two-puncture
Brill-Lindquist box with 3 Sommerfeld ghosts in float64 (the bandwidth
roofline point), synthetic data, advanced through the batched plan API (one
fused launch per substep, the RK4 step replayed as a HIP graph, tile shape
chosen by the autotuner).  value = zone cycles per second (active cells x
RK4 steps / wall time), the unit the paper uses.

Extras on the same JSON line: the same data on the 128^3 box, the same
workload with float32 arithmetic (Z4C_MIXED), its z >= 0 half with
equatorial symmetry, the 9-box hierarchy in one persistent launch per
substep (float64 and mixed), the binary-black-hole hierarchy with moving
patches (full and equatorial half), the constraint monitor, the roofline of
the fused kernel (HIP events around its launches on the stream it runs on)
and the CPU oracle timed on a bounded sample.  Tile shapes come from the
persisted tuning cache (paper_2607_08743_amd/tune_cache.jsonl; a miss times
every compiled shape once and records the fastest).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
KERNEL_SRC = os.path.join(ROOT, "paper_2607_08743_amd", "csrc", "z4c_kernels.hip")
TUNE_CACHE = os.path.join(ROOT, "paper_2607_08743_amd", "tune_cache.jsonl")

# HBM bytes per fused launch (mean of the four substeps) from rocprofv3
# FETCH_SIZE and WRITE_SIZE passes over `bench.py --tile <tile> --steps 3
# --warmup 1 --no-extras --no-cpu-baseline`, each scaled by what the same
# counter reads for a plain 1 GiB device copy (`bench.py --copy-calibration`).
# Keyed by the SHA-256 of the kernel source the counters were taken on: once
# the source changes the figure no longer applies and `traffic` is null.
MEASURED_TRAFFIC = {
    "db8f8c5328017a29e16dbd7b00e4a944092e5942da345c2043f77e806d292fae": {"tile": (8, 8, 8, 2, 1), "n": 256, "bytes_per_launch": 21932600000,
        "fetch_bytes": 15825700000, "write_bytes": 6106900000,
        "profile": "profiles/fused_stage_256cube_punctures_fp64.md"},
}


def kernel_source_digest():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def copy_calibration(torch):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    n = 1 << 27  # float64 elements: 1 GiB each way
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 8 * n, "bytes_written": 8 * n, "launches": 3}}))


def stream_bandwidth(torch, reps=10):
    """Best rate of two plain 1 GiB streaming kernels over float64 arrays
    (torch's device-to-device copy and its element-wise scale into another
    array; bytes read plus bytes written per second, HIP events): what HBM
    sustains for a streaming kernel on this part, beside the published
    8 TB/s.  The two differ by up to 15% from run to run, the scale usually
    ahead, so the faster of them is the reference."""
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    rates = {}
    for name, fn in (("copy", lambda: dst.copy_(src)),
                     ("scale", lambda: torch.mul(src, 1.0, out=dst))):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        e1.synchronize()
        rates[name] = 2 * 8 * n / (e0.elapsed_time(e1) * 1e-3 / reps) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return rates


def alg_bytes_per_stage(n, ng=3):
    """Algorithmic HBM bytes of the four fused launches of one RK4 step of one
    n^3 box (float64, 25 fields): each stage reads its stencil input once
    over the stored points, plus its pointwise arrays over the active points
    (stage 1: write u1, acc; 2, 3: read u_n, acc, write u_s, acc; 4: read
    acc, write u_n)."""
    stored = (n + 2 * ng) ** 3
    act = n ** 3
    f = 25 * 8
    return [f * (stored + 2 * act), f * (stored + 4 * act), f * (stored + 4 * act), f * (stored + 2 * act)]


def timed_plan_steps(plan, steps, warmup, torch):
    plan.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def fused_kernel_roofline(z4c, I, torch, g, u_dev, dt, tile, params, reps=5):
    """Time each fused substep launch alone with HIP events on the stream it
    is launched on.  A periodic box of the same size launches only the fused
    kernel (its ghost fill is a separate call, left out of the events)."""
    gp = I.Grid(g.n, g.h, g.x0, I.BC_PERIODIC, g.ng)
    z4c.select_tile(params.precision, tile)
    a = torch.empty_like(u_dev)
    b = torch.empty_like(u_dev)
    acc = torch.empty_like(u_dev)
    s = torch.cuda.current_stream()
    seq = ((u_dev, a), (a, b), (b, a), (a, u_dev))
    ms = [0.0] * 4
    z4c.apply_ghosts(u_dev, gp)
    for rep in range(reps + 1):
        for st, (src, dst) in enumerate(seq, start=1):
            z4c.apply_ghosts(src, gp)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            z4c.rk4_substep(st, dt, src, u_dev, acc, dst, gp, params)
            e1.record(s)
            e1.synchronize()
            if rep > 0:
                ms[st - 1] += e0.elapsed_time(e1) / reps
    z4c.select_tile(params.precision, None)
    del a, b, acc
    return ms


def constraint_monitor_rate(z4c, torch, g, u0, n, reps=5):
    """Constraint monitor (norms only) on the benchmark state: mean time per
    call (HIP events on the launch stream) and its algorithmic bytes (18
    fields read over the active points plus the 2-cell stencil margin); and
    the extra time of the monitor fused into stage 1 of the RK4 step."""
    u = torch.as_tensor(u0, device="cuda")
    ws = torch.empty(z4c.constraints_workspace(g), dtype=torch.float64, device="cuda")
    norms = torch.empty(4, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    z4c.constraints(u, g, norms=norms, ws=ws)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        z4c.constraints(u, g, norms=norms, ws=ws)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = 18 * 8 * (n + 4) ** 3
    out = {"ms_per_call": round(ms, 4), "alg_bytes": alg, "achieved_GBs": round(alg / (ms * 1e-3) / 1e9, 1),
           "zone_per_s": n ** 3 / (ms * 1e-3), "norms": [float(x) for x in norms.cpu()]}
    # the same monitor fused into stage 1 of an RK4 step (rk4_substep_monitor):
    # its cost is the difference to the plain stage 1
    acc, dst = torch.empty_like(u), torch.empty_like(u)
    wsm = torch.empty(z4c.monitor_workspace(g), dtype=torch.float64, device="cuda")
    nm = torch.empty(4, dtype=torch.float64, device="cuda")
    dt = 0.5 * g.h[0]
    z4c.select_tile(z4c.FP64, z4c.Tile(8, 8, 8, 2, 1))  # the monitor's launch shape, for a like-for-like difference
    t = {}
    for mon in (False, True, False, True):
        z4c.rk4_substep_monitor(1, dt, u, None, acc, dst, g, norms=nm, ws=wsm) if mon else \
            z4c.rk4_substep(1, dt, u, None, acc, dst, g)
        e0.record(s)
        for _ in range(reps):
            if mon:
                z4c.rk4_substep_monitor(1, dt, u, None, acc, dst, g, norms=nm, ws=wsm)
            else:
                z4c.rk4_substep(1, dt, u, None, acc, dst, g)
        e1.record(s)
        e1.synchronize()
        t[mon] = e0.elapsed_time(e1) / reps
    z4c.select_tile(z4c.FP64, None)
    out["fused_into_stage1"] = {"ms_stage1_with_monitor": round(t[True], 4), "ms_stage1_plain": round(t[False], 4),
                                "ms_monitor_extra": round(t[True] - t[False], 4),
                                "norms": [float(x) for x in nm.cpu()]}
    del u, ws, acc, dst, wsm
    torch.cuda.empty_cache()
    return out


def hierarchy_run(z4c, torch, boxes, prec, steps):
    plan = z4c.Plan(boxes, params=z4c.default_params(precision=prec))
    plan.step(steps)
    torch.cuda.synchronize()
    out = [u.cpu().numpy() for u in plan.u]
    plan.close()
    return out


def per_field_errors(I, boxes, got, ref):
    """Per field, max over boxes of max|got - ref| / max|ref| (norm-relative)
    and of max|got - ref| / max|ref - initial| (relative to how far the field
    moved), over the active cells."""
    norm = [0.0] * 25
    moved = [0.0] * 25
    for bx, a, b in zip(boxes, got, ref):
        m = bx.grid.active_mask()
        for f in range(25):
            d = float(abs(a[f][m] - b[f][m]).max())
            sc = float(abs(b[f][m]).max())
            mv = float(abs(b[f][m] - bx.state[f][m]).max())
            norm[f] = max(norm[f], d / sc if sc > 0 else d)
            moved[f] = max(moved[f], d / mv if mv > 1e-8 else 0.0)
    return {"per_field_normrel": dict(zip(I.FIELD_NAMES, norm)),
            "per_field_rel_to_change": dict(zip(I.FIELD_NAMES, moved)),
            "max_normrel": max(norm), "max_rel_to_change": max(moved)}


def mixed_hierarchy_error(z4c, I, torch, boxes, steps=50, oracle_boxes=(8, 7)):
    """Mixed precision on the 9-box hierarchy after `steps` RK4 steps.
    Against the float64 ORACLE (its own 50 steps on the host) for the boxes
    oracle_boxes (the smallest: 64^3 and 72^3 -- the whole hierarchy would
    take the oracle several minutes), for both GPU precisions; and, for all
    nine boxes, mixed against the float64 GPU path."""
    import oracle

    oracle.build(force=False)
    res = {prec: hierarchy_run(z4c, torch, boxes, prec, steps) for prec in (z4c.FP64, z4c.MIXED)}
    sub = [boxes[i] for i in oracle_boxes]
    t0 = time.perf_counter()
    ref = []
    for bx in sub:
        r = bx.state.copy()
        oracle.rk4(r, bx.grid.as_dict(), bx.dt, steps, shell=bx.shell)
        ref.append(r)
    t_oracle = time.perf_counter() - t0
    return {"steps": steps,
            "vs_oracle": {"boxes": [f"level {bx.level}: {bx.grid.n[0]}^3" for bx in sub],
                          "oracle_seconds": round(t_oracle, 1),
                          "mixed": per_field_errors(I, sub, [res[z4c.MIXED][i] for i in oracle_boxes], ref),
                          "fp64": per_field_errors(I, sub, [res[z4c.FP64][i] for i in oracle_boxes], ref)},
            "mixed_vs_fp64_gpu_all_boxes": per_field_errors(I, boxes, res[z4c.MIXED], res[z4c.FP64])}


def bbh_moving_rate(z4c, I, torch, steps=5, warmup=1, equatorial=False, lag=0.05):
    """The full hierarchy method on the binary-black-hole layout: Berger-Oliger
    subcycling over fixed levels and moving patch pairs (exchange, tracking,
    regrid), FP64; equatorial: the upper half with every patch on the
    symmetry plane.  The punctures start `lag` inside their patches' centres,
    so that the deepest moving patches shift during the timed root steps.
    Each root step is timed on its own (the hierarchy reads the punctures back
    after every root step anyway); the step after which a patch shifted
    includes the shift, the next one the re-capture of the graph.  Zone
    updates count every patch's active cells once per step of its depth."""
    pt, states, dt0, xp = I.config_bbh_moving(equatorial=equatorial, lag=lag)
    depth = []
    for g, F, par, obj in pt:
        depth.append(0 if par < 0 else depth[par] + 1)
    H = z4c.Hierarchy([(g, u, F, par, obj) for (g, F, par, obj), u in zip(pt, states)], dt0)
    del states
    H.set_moving(xp)
    H.advance(warmup)
    torch.cuda.synchronize()
    _, Fprev, _ = H.puncture()
    per_step, shifted = [], []
    for k in range(steps):
        t0 = time.perf_counter()
        H.advance(1)
        torch.cuda.synchronize()
        per_step.append(time.perf_counter() - t0)
        _, F, _ = H.puncture()
        shifted.append([q for q in range(len(pt)) if tuple(F[q]) != tuple(Fprev[q])])
        Fprev = F
    sec = sum(per_step)
    x, F, x0 = H.puncture()
    finite = all(bool(torch.isfinite(u).all()) for u in H.u)
    H.close()
    upd = sum(g.active * 2 ** d for (g, *_), d in zip(pt, depth))
    quiet = [t for k, t in enumerate(per_step) if not shifted[k] and not (k > 0 and shifted[k - 1])]
    base = sorted(quiet)[len(quiet) // 2] if quiet else None
    regrid = {}
    for k in range(steps):
        if shifted[k] and base is not None:
            regrid[f"timed step {k}"] = {"patches_shifted": shifted[k],
                                         "extra_ms_shift": round(1e3 * (per_step[k] - base), 2),
                                         "extra_ms_next_step_recapture": round(1e3 * (per_step[k + 1] - base), 2)
                                         if k + 1 < steps else None}
    extra = {"full_domain_equivalent_value": 2 * upd * steps / sec} if equatorial else {}
    return {"value": upd * steps / sec, **extra, "unit": "zone-cycles/s", "ms_per_root_step": 1e3 * sec / steps,
            "ms_per_timed_root_step": [round(1e3 * t, 2) for t in per_step],
            "ms_per_root_step_without_regrid": round(1e3 * base, 2) if base else None,
            "regrids": regrid, "patches": len(pt), "depths": max(depth) + 1,
            "active_cells": sum(g.active for g, *_ in pt), "zone_updates_per_root_step": upd,
            "punctures_start": xp.tolist(), "punctures_end": x.tolist(), "lag": lag, "finite": finite}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(I, n=256):
    """The float64 oracle, as it stands, on a bounded sample of the headline
    workload (the n^3 two-puncture box): its right-hand side at every active
    point of a few z-planes through the middle of the box (the same per-point
    routine its full RK4 step runs on every point), at one thread and at all
    host threads.  A zone cycle is four right-hand-side evaluations; the RK4
    combination and the enforcement (pointwise, a few percent of the
    oracle's work) are left out of the sample."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    g, u, _ = I.config_punctures(n)
    ng = g.ng
    nall = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    runs = {}
    for nth, planes in ((1, 24), (nall, 192)):
        k0 = ng + n // 2 - planes // 2
        K, J, X = np.meshgrid(np.arange(k0, k0 + planes), np.arange(ng, ng + n), np.arange(ng, ng + n), indexing="ij")
        pts = np.stack([X.ravel(), J.ravel(), K.ravel()], axis=1).astype(np.int32)
        t0 = time.perf_counter()
        oracle.rhs_points(u, g.as_dict(), pts, nthreads=nth)
        t = time.perf_counter() - t0
        runs[nth] = {"value": len(pts) / t / 4.0, "threads": nth, "seconds": round(t, 2),
                     "sample": f"RHS at all {len(pts)} active points of z-planes {k0}..{k0 + planes - 1}"}
    top = runs[nall]
    return {"value": top["value"], "unit": "zone-cycles/s", "cores": nall, "kind": "oracle",
            "sample": f"{n}^3 two-puncture Sommerfeld box (the headline workload): {top['sample']} "
                      f"on {nall} OpenMP threads ({top['seconds']} s); zone-cycles/s = RHS points/s / 4",
            "one_thread": runs[1], "all_threads": top, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="active cells per side of the puncture box")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the mixed-precision and hierarchy runs")
    ap.add_argument("--tile", default="", help="bx,by,bz,waves,persistent (skip the autotuner)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--only", choices=["bbh_moving", "bbh_moving_equatorial", "constraints"], default="",
                    help="run only this extra measurement and print its JSON")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="tuning cache file (JSON lines); empty string: time every shape, persist nothing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    if args.copy_calibration:
        torch.cuda.set_device(0)
        copy_calibration(torch)
        return

    from paper_2607_08743_amd import inputs as I
    from paper_2607_08743_amd import z4c

    torch.cuda.set_device(0)
    if args.only == "constraints":
        g, u0, _ = I.config_punctures(args.n)
        print(json.dumps({"constraints": constraint_monitor_rate(z4c, torch, g, u0, args.n)}), flush=True)
        return
    if args.only:
        print(json.dumps({args.only: bbh_moving_rate(z4c, I, torch, equatorial=args.only.endswith("equatorial"))}),
              flush=True)
        return
    g, u0, dt = I.config_punctures(args.n)
    box = I.Box(g, u0, None, dt)
    params = z4c.default_params()

    cache = args.tune_cache or None

    def run(box_list, params, tile_arg):
        """Tile from the caller, else the tuning cache (a miss tunes once and
        records the result); the timed plan starts from the initial state."""
        if tile_arg is None:
            best, source = z4c.autotune(box_list, params, tune_cache=cache)
            torch.cuda.empty_cache()
        else:
            best, source = tile_arg, "caller"
        plan = z4c.Plan(box_list, params=params, tile=best)
        sec = timed_plan_steps(plan, args.steps, args.warmup, torch)
        finite = all(bool(torch.isfinite(x).all()) for x in plan.u)
        plan.close()
        torch.cuda.empty_cache()
        return sec, best, source, finite

    tile = None
    if args.tile:
        v = [int(x) for x in args.tile.split(",")]
        tile = z4c.Tile(*v)
    sec, best, tune_source, finite = run([box], params, tile)
    if not finite:
        raise RuntimeError("non-finite state after the timed steps")
    active = g.active
    value = active * args.steps / sec

    # roofline of the dominant (fused) kernel
    u_dev = torch.as_tensor(u0, device="cuda")
    ms = fused_kernel_roofline(z4c, I, torch, g, u_dev, dt, best, params)
    del u_dev
    torch.cuda.empty_cache()
    bytes_stage = alg_bytes_per_stage(args.n)
    achieved = sum(bytes_stage) / (sum(ms) * 1e-3) / 1e9
    digest = kernel_source_digest()
    meas = MEASURED_TRAFFIC.get(digest)
    traffic = meas["bytes_per_launch"] if meas and tuple(meas["tile"]) == tuple(best.as_tuple()) \
        and meas["n"] == args.n else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "fused_stage", "ms_per_launch": [round(x, 4) for x in ms],
            "ms_per_launch_mean": round(sum(ms) / 4, 4),
            "alg_bytes_per_launch": bytes_stage, "alg_bytes_per_launch_mean": sum(bytes_stage) // 4,
            "kernel_resources": z4c.tile_resources(params.precision, best),
            "kernel_source_sha256": digest[:16]}
    stream = stream_bandwidth(torch)
    best_stream = max(stream.values())
    roof["stream_GBs"] = {k: round(v, 1) for k, v in stream.items()}
    roof["frac_of_stream"] = round(achieved / best_stream, 4)

    extras = {}
    extras["constraints"] = constraint_monitor_rate(z4c, torch, g, u0, args.n)
    if not args.no_extras:
        # the same puncture data on the 128^3 box (dx = 0.25), same tile
        g2, u2, dt2 = I.config_punctures(128)
        sec2, best2, src2, fin2 = run([I.Box(g2, u2, None, dt2)], params, None)
        extras["box128"] = {"value": g2.active * args.steps / sec2, "ms_per_step": 1e3 * sec2 / args.steps,
                            "tile": list(best2.as_tuple()), "tune_source": src2, "finite": fin2}
        del u2
        pm = z4c.default_params(precision=z4c.MIXED)
        sec_m, best_m, src_m, fin_m = run([box], pm, None)
        extras["mixed"] = {"value": active * args.steps / sec_m, "ms_per_step": 1e3 * sec_m / args.steps,
                           "tile": list(best_m.as_tuple()), "tune_source": src_m, "finite": fin_m,
                           "kernel_resources": z4c.tile_resources(pm.precision, best_m),
                           "fp64_kernel_resources": z4c.tile_resources(params.precision, best)}
        ge, ue, dte = I.config_punctures_equatorial(args.n)
        sec_e, best_e, src_e, fin_e = run([I.Box(ge, ue, None, dte)], params, None)
        extras["equatorial"] = {"value": ge.active * args.steps / sec_e, "ms_per_step": 1e3 * sec_e / args.steps,
                                "active_cells": ge.active, "full_box_equivalent_value":
                                    2 * ge.active * args.steps / sec_e,
                                "tile": list(best_e.as_tuple()), "tune_source": src_e, "finite": fin_e}
        boxes = I.config_hierarchy()
        act_h = sum(b.grid.active for b in boxes)
        sec_h, best_h, src_h, fin_h = run(boxes, params, None)
        extras["hierarchy9"] = {"value": act_h * args.steps / sec_h, "ms_per_step": 1e3 * sec_h / args.steps,
                                "active_cells": act_h, "tile": list(best_h.as_tuple()), "tune_source": src_h,
                                "finite": fin_h}
        extras["bbh_moving"] = bbh_moving_rate(z4c, I, torch)
        extras["bbh_moving_equatorial"] = bbh_moving_rate(z4c, I, torch, equatorial=True)
        sec_hm, best_hm, src_hm, fin_hm = run(boxes, pm, None)
        extras["hierarchy9_mixed"] = {"value": act_h * args.steps / sec_hm, "ms_per_step": 1e3 * sec_hm / args.steps,
                                      "tile": list(best_hm.as_tuple()), "tune_source": src_hm, "finite": fin_hm,
                                      "error_after_50_steps": mixed_hierarchy_error(z4c, I, torch, boxes)}

    out = {
        "metric": "zone-updates/s for Z4c RHS+RK4 substep (FP64 vs mixed) + % HBM roofline",
        "value": value, "unit": "zone-cycles/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"single {args.n}^3 box + 3 ghosts, two Brill-Lindquist punctures (m=0.5 each, "
                               f"separation 10), alpha=W, Sommerfeld outer boundary, dx={g.h[0]}, FP64, "
                               f"RK4 steps of dt=0.5dx", "tile": list(best.as_tuple()),
                   "tune_source": tune_source, "tune_cache": os.path.relpath(cache, ROOT) if cache else None,
                   "zone_substeps_per_s": 4 * value},
        "roofline": roof,
        "extras": extras,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(I)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
