#!/usr/bin/env python3
"""Benchmark of the TTIE hot path on one MI355X.

One step = the whole hot path over the folded-cloth workload (256 x 256 vertex grid,
130,050 triangles, seed 0): LBVH broad phase -> screening of every candidate pair ->
per-hit interval gradients -> energy, gradient and PSD block-sparse Hessian assembly.
The metric is candidate pairs per second of that step.  Inputs are resident in HBM before
the timed region; nothing is allocated inside it.

Prints one JSON line.  Besides the contract fields it carries:
  fp64          the same step on the all-FP64 path
  hits_per_s    intersecting pairs found per second of the step
  eval_only, broadphase_only
                the step split at the stage timers (candidate pairs/s of the evaluation,
                triangles/s of the broad phase)
  err           relative errors of both paths against the FP64 CPU oracle
  stages        per-stage kernel time from the library's stage timers (warm-up steps)
  roofline      the dominant kernel's algorithmic bytes / its measured duration vs HBM peak
  roofline_issue  the same kernel's VALU issue rate vs the VALU issue peak
  cpu_baseline  the CPU oracle timed on this host on the same workload
  extra         the larger workloads (brute-force icospheres, 1M-triangle sphere, batch of 64,
                Newton on the 4M-triangle sphere, quasi-static cloth)
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "folded cloth 256x256 grid (65,536 verts, 130,050 tris), LBVH broad phase, seed 0"

# Counter figures per launch of a kernel on this workload, valid only for the kernel source and
# the launch parameters they were taken with (otherwise reported as null until taken again):
#   bytes       HBM bytes from two rocprofv3 passes, FETCH_SIZE x 1.9998 and WRITE_SIZE x 1.0 (the
#               factors that make a 256 MiB elementwise copy read and write 256 MiB)
#   valu_wave   SQ_INSTS_VALU, wave-level VALU instructions
MEASURED = {
    "bp_traverse": [
        {"bytes": 16645751, "valu_wave": 13846425, "source": "paper_2606_06511_amd/csrc/broadphase.hip",
         "sha256": "5efb9b997f8b387f40d5c27da6cb45273ad84ac11c0ce1cb456614f836aff4f7", "params": {"trav_budget": 24}},
        {"bytes": 16494401, "valu_wave": 14476783, "source": "paper_2606_06511_amd/csrc/broadphase.hip",
         "sha256": "5efb9b997f8b387f40d5c27da6cb45273ad84ac11c0ce1cb456614f836aff4f7", "params": {"trav_budget": 32}},
    ],
}
# VALU issue peak: 256 CUs x 4 SIMD16 units x 2.4 GHz (a wave64 instruction takes a SIMD 4 cycles)
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9


def measured(stage, what, params=None):
    import hashlib

    for m in MEASURED.get(stage, []):
        if params is not None and any(params.get(k) != v for k, v in m.get("params", {}).items()):
            continue
        with open(os.path.join(ROOT, m["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != m["sha256"]:
                continue
        return m[what]
    return None


def stage_bytes(stage, nv, nt, P, H, nnzb, prec_bytes):
    """Algorithmic HBM bytes one launch of a stage must move (each input read once, each
    output written once)."""
    s = prec_bytes
    table = {
        # pair ids in; each vertex and triangle index read once; hit records (80 B) out
        "screen": 8 * P + 24 * nv + 12 * nt + 80 * H,
        # x and indices in; FP64 boxes (48 B) and FP32 centres (12 B) out
        "bp_boxes": 24 * nv + 12 * nt + 48 * nt + 12 * nt,
        # centres in, bucket + rank out (Morton pass); bucket, rank, offset in and ids out
        # (scatter)
        "bp_sort": 12 * nt + 8 * nt + 12 * nt + 4 * nt,
        # ids, FP64 boxes and indices in; 64-B leaf records, FP32 leaf boxes (32 B) and the
        # inner 4-ary levels (32 B per node, about nt/3 nodes) out
        "bp_build": 4 * nt + 48 * nt + 12 * nt + 64 * nt + 32 * nt + 32 * nt // 3,
        # every leaf record and node box read once, each candidate pair (8 B) written once
        "bp_traverse": 64 * nt + 32 * nt + 32 * nt // 3 + 8 * P,
        "screen_exact": 0,
        "derivs": H * (80 + 6 * 24 + 24 + 8 + s * 57),
        "assembly": 3 * s * nv + (9 * s + 4) * nnzb + 4 * (nv + 1) + H * 6 * 16 * 2,
    }
    return table.get(stage, 0)


def extra_configs(args, np, torch, ttie, workloads, only=None):
    """The larger workloads: the two icospheres by brute force (FP64), the 1,048,576-triangle
    noisy sphere (mixed, BSR on; eager steps, stage breakdown), the batch of 64 two-mesh problems
    (one step = batched broad phase + batched evaluation, captured once in a HIP graph and
    replayed), 20 Newton steps on the 4,194,304-triangle sphere (BSR and matrix-free) and the
    quasi-static cloth.  ``only`` (a set of names) restricts the run to those workloads."""
    dev = torch.device("cuda", 0)
    res = {}
    want = (lambda name: only is None or name in only)

    def run(step, steps):
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    if want("icospheres_brute"):
        # two icospheres, every non-adjacent pair (brute force), FP64
        x, tris = workloads.two_icospheres(seed=0)
        ctx = ttie.Context(0)
        cap = 1 << 22
        ctx.reserve(len(x), len(tris), cap, max_hits=1 << 12, max_blocks=36 << 12)
        xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(tris).to(dev)
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        n = torch.zeros(1, dtype=torch.int64, device=dev)
        out = ctx.evaluate(xd, td, pairs[:1], torch.zeros(1, dtype=torch.int64, device=dev), precision=ttie.FP64)

        def ico_step():
            ctx.broadphase(xd, td, ttie.BROAD_BRUTE, capacity=cap, out=(pairs, n))
            ctx.evaluate(xd, td, pairs, n, precision=ttie.FP64, out=out)

        ms = run(ico_step, 20)
        ctx.check()
        P = int(n.item())
        res["icospheres_brute"] = {"workload": "two icospheres (642 verts / 1280 tris each), all 3,260,220 non-adjacent "
                                               "pairs, FP64, seed 0",
                                   "pairs": P, "hits": int(out["n_hits"].item()), "ms_per_step": ms,
                                   "pairs_per_s": P / (ms * 1e-3)}
        del ctx, pairs, out

    if want("sphere_1m"):
        # noisy sphere, 1024 x 513 bands
        x, tris = workloads.noisy_sphere(seed=0)
        ctx = ttie.Context(0)
        cap, hcap = 1 << 23, 1 << 17
        ctx.reserve(len(x), len(tris), cap, max_hits=hcap, max_blocks=36 * hcap)
        xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(tris).to(dev)
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        n = torch.zeros(1, dtype=torch.int64, device=dev)
        out = ctx.evaluate(xd, td, pairs[:1], torch.zeros(1, dtype=torch.int64, device=dev), precision=ttie.MIXED)

        def sphere_step():
            ctx.broadphase(xd, td, ttie.BROAD_LBVH, capacity=cap, out=(pairs, n))
            ctx.evaluate(xd, td, pairs, n, precision=ttie.MIXED, out=out)

        ms = run(sphere_step, 20)
        ctx.check()
        ctx.set_timing(None)
        for _ in range(5):
            sphere_step()
        torch.cuda.synchronize()
        st = ctx.read_timers()
        ctx.set_timing([])
        P = int(n.item())
        bp_ms = sum(v[1] for k, v in st.items() if k.startswith("bp_")) / 5
        res["sphere_1m"] = {"workload": "noisy UV sphere 1024x513 bands (524,290 verts, 1,048,576 tris), LBVH, seed 0",
                            "pairs": P, "hits": int(out["n_hits"].item()), "ms_per_step": ms,
                            "pairs_per_s": P / (ms * 1e-3), "broadphase_tris_per_s": len(tris) / (bp_ms * 1e-3),
                            "stages_ms_per_step": {k: round(v[1] / 5, 5) for k, v in st.items()}}
        del ctx, pairs, out

    if want("batch64"):
        # 64 two-mesh problems in one batch
        probs = workloads.batch_problems(seed=0)
        x, tris, vert_off, tri_off = workloads.concat_problems(probs)
        ctx = ttie.Context(0)
        cap, hcap = 1 << 23, 1 << 17
        ctx.reserve(len(x), len(tris), cap, max_hits=hcap, max_blocks=36 * hcap)
        n = torch.zeros(1, dtype=torch.int64, device=dev)
        xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(tris).to(dev)
        vo, to = torch.from_numpy(vert_off).to(dev), torch.from_numpy(tri_off).to(dev)
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        out = ctx.batch_evaluate(xd, td, vo, pairs[:1], torch.zeros(1, dtype=torch.int64, device=dev),
                                 precision=ttie.MIXED)

        def batch_step():
            ctx.batch_broadphase(xd, td, to, capacity=cap, out=(pairs, n))
            ctx.batch_evaluate(xd, td, vo, pairs, n, precision=ttie.MIXED, out=out)

        # the launch parameters are tuned on this batch (coordinate descent over the step time),
        # then the tuned step is captured
        from paper_2606_06511_amd import autotune

        tuned, ms_tuned, ms_default = autotune.tune(ctx, batch_step, reps=5, rounds=1)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            batch_step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        ctx.check()
        eager_E = out["energies"].cpu().numpy().copy()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, capture_error_mode="relaxed"):
            batch_step()
        out["energies"].zero_()
        g.replay()
        torch.cuda.synchronize()
        ctx.check()
        same = bool(np.array_equal(out["energies"].cpu().numpy(), eager_E))
        ms_graph = run(g.replay, 20)
        ms_eager = run(batch_step, 10)
        ctx.check()
        P = int(n.item())
        res["batch64"] = {"workload": "64 two-mesh problems (icospheres, tori, bump grids; 2,842,166 verts, "
                                      "5,664,096 tris), batched LBVH, seed 0",
                          "problems": len(probs), "pairs": P, "hits": int(out["n_hits"].item()),
                          "ms_per_step": ms_graph, "pairs_per_s": P / (ms_graph * 1e-3),
                          "ms_per_step_eager": ms_eager, "graph_replay_matches_eager": same,
                          "autotuned": tuned, "ms_eager_default_params": ms_default, "ms_eager_tuned_params": ms_tuned}
        del ctx, pairs, out

    if want("newton_4m"):
        # inexact Newton, 20 steps, on the 4,194,304-triangle sphere (Jacobi-PCG with 50 iterations)
        from paper_2606_06511_amd.energy import TTIE
        from paper_2606_06511_amd.newton import newton

        x, tris = workloads.noisy_sphere(seed=0, n_lon=2048, n_bands=1025)
        model = TTIE(torch.from_numpy(tris), len(x), max_pairs=1 << 25, max_hits=1 << 17, precision=ttie.MIXED)
        xd = torch.from_numpy(x).to(dev)
        newton(model, xd, steps=1)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hist = newton(model, xd, steps=20)
        torch.cuda.synchronize()
        total_ms = (time.perf_counter() - t0) * 1e3
        steps = [h for h in hist if "alpha" in h]
        res["newton_4m"] = {
            "workload": "noisy UV sphere 2048x1025 bands (2,097,154 verts, 4,194,304 tris), 20 inexact Newton steps, "
                        "BSR Hessian + Jacobi-PCG (50), Armijo, swept LBVH candidates",
            "E": [h["E"] for h in hist], "hits": [h["hits"] for h in hist], "pairs": [h["pairs"] for h in hist],
            "alpha": [h["alpha"] for h in steps], "ms_per_newton_step": [round(h["ms"], 3) for h in steps],
            "total_ms": total_ms, "E_final_over_E0": hist[-1]["E"] / hist[0]["E"] if hist[0]["E"] else None,
            "pairs_per_s": sum(h["pairs"] for h in steps) / (sum(h["ms"] for h in steps) * 1e-3)}
        # the same 20 steps matrix-free: the solve applies the PSD Hessian from the hit records
        newton(model, xd, steps=1, matrix_free=True)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hist_mf = newton(model, xd, steps=20, matrix_free=True)
        torch.cuda.synchronize()
        steps_mf = [h for h in hist_mf if "alpha" in h]
        res["newton_4m"]["matrix_free"] = {
            "E": [h["E"] for h in hist_mf], "total_ms": (time.perf_counter() - t0) * 1e3,
            "ms_per_newton_step": [round(h["ms"], 3) for h in steps_mf],
            "E_final_over_E0": hist_mf[-1]["E"] / hist_mf[0]["E"] if hist_mf[0]["E"] else None}
        del model

    if want("quasistatic_cloth"):
        # quasi-static coupling on the folded cloth: springs on the edges (rest = the folded state),
        # proximal weight m, energy weight w scaled with the inverse squared edge length
        from paper_2606_06511_amd.energy import TTIE
        from paper_2606_06511_amd.quasistatic import QuasiStatic

        x, tris = workloads.folded_cloth(seed=0)
        model = TTIE(torch.from_numpy(tris), len(x), max_pairs=1 << 22, max_hits=1 << 16)
        xd = torch.from_numpy(x).to(dev)
        sim = QuasiStatic(model, xd, k=1.0, m=1.0, w=1e6)
        sim.step(xd, newton_iters=1)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hist = sim.run(xd, 5, newton_iters=4, pcg_iters=50)
        torch.cuda.synchronize()
        total_ms = (time.perf_counter() - t0) * 1e3
        its = [r for h in hist for r in h["newton"]]
        res["quasistatic_cloth"] = {
            "workload": "folded cloth 256x256 grid (130,050 tris), 5 quasi-static steps x 4 Newton iterations, springs "
                        "k = 1 on the edges, proximal m = 1, energy weight w = 1e6, FP64, coupled Jacobi-PCG (50)",
            "E": [h["E"] for h in hist], "hits": [h["hits"] for h in hist],
            "phi": [[r["phi"] for r in h["newton"]] for h in hist[:-1]],
            "alpha": [[r["alpha"] for r in h["newton"]] for h in hist[:-1]],
            "ms_per_newton_iter": sum(r["ms"] for r in its) / max(len(its), 1), "total_ms": total_ms}
        del model, sim

    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="CPU oracle sample length")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the larger configurations (1M-triangle sphere, 64-problem batch)")
    ap.add_argument("--params", default="", metavar="NAME=V,...",
                    help="fix launch parameters (trav_budget, screen_blocks, row_blocks) instead of autotuning them; "
                         "a profiler run uses this to time the configuration the autotuner picks")
    ap.add_argument("--extra-only", default="", metavar="NAME,...",
                    help="run only these larger workloads (icospheres_brute, sphere_1m, batch64, newton_4m, "
                         "quasistatic_cloth) and print their records: for profiling one workload alone, "
                         "not a benchmark line")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="finish with one elementwise copy kernel over this many MB (a known-size kernel that "
                         "calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the hot path runs on a single MI355X; sharding by "
                                   "candidate pairs across GPUs is designed but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_06511_amd import ttie, workloads

    if args.extra_only:
        only = set(args.extra_only.split(","))
        print(json.dumps({"extra": extra_configs(args, np, torch, ttie, workloads, only=only)}), flush=True)
        return

    x, tris = workloads.folded_cloth(seed=0, n=256)
    nv, nt = len(x), len(tris)
    dev = torch.device("cuda", 0)
    ctx = ttie.Context(0)
    max_pairs, max_hits = 1 << 21, 1 << 16
    ctx.reserve(nv, nt, max_pairs, max_hits=max_hits, max_blocks=36 * max_hits)
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(tris).to(dev)
    pairs = torch.empty((max_pairs, 2), dtype=torch.int32, device=dev)
    npairs = torch.zeros(1, dtype=torch.int64, device=dev)

    def outputs(dt):
        return {"energy": torch.zeros(1, dtype=torch.float64, device=dev),
                "grad": torch.empty((nv, 3), dtype=dt, device=dev),
                "n_hits": torch.zeros(1, dtype=torch.int64, device=dev),
                "row_ptr": torch.empty(nv + 1, dtype=torch.int32, device=dev),
                "col_idx": torch.empty(36 * max_hits, dtype=torch.int32, device=dev),
                "vals": torch.empty((36 * max_hits, 3, 3), dtype=dt, device=dev),
                "n_blocks": torch.zeros(1, dtype=torch.int64, device=dev)}

    precs = {"mixed": ttie.MIXED, "fp64": ttie.FP64}
    outs = {"mixed": outputs(torch.float32), "fp64": outputs(torch.float64)}

    def step(name):
        ctx.broadphase(xd, td, ttie.BROAD_LBVH, capacity=max_pairs, out=(pairs, npairs))
        ctx.evaluate(xd, td, pairs, npairs, precision=precs[name], hessian=True, out=outs[name])

    def timed(name, steps, warmup, stage=None):
        ctx.set_timing([])
        for _ in range(warmup):
            step(name)
        torch.cuda.synchronize()
        ctx.check()
        ctx.read_timers()
        if stage:
            ctx.set_timing([stage])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(name)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tim = ctx.read_timers()
        ctx.set_timing([])
        ctx.check()
        return (t1 - t0) * 1e3 / steps, tim

    primary = args.precision
    other = "fp64" if primary == "mixed" else "mixed"

    # launch parameters picked by the autotuner on this very step before anything is timed
    # (they change the speed only, never a result)
    from paper_2606_06511_amd import autotune

    if args.params:
        tuned = {}
        for item in args.params.split(","):
            name, val = item.split("=")
            ctx.set_param(autotune.SPACE[name][0], int(val))
            tuned[name] = int(val)
        ms_tuned = ms_default = None
    else:
        tuned, ms_tuned, ms_default = autotune.tune(ctx, lambda: step(primary), reps=20, rounds=1)
    torch.cuda.synchronize()
    ctx.check()

    # stage breakdown from warm-up steps with every timer on
    step(primary)
    torch.cuda.synchronize()
    ctx.read_timers()
    ctx.set_timing(None)
    for _ in range(max(5, args.warmup // 2)):
        step(primary)
    torch.cuda.synchronize()
    stages = ctx.read_timers()
    ctx.set_timing([])
    nsteps_b = max(5, args.warmup // 2)
    stage_avg = {k: v[1] / v[0] for k, v in stages.items()}
    per_step_stage = {k: v[1] / nsteps_b for k, v in stages.items()}
    dominant = max(per_step_stage, key=per_step_stage.get)

    ms, tim = timed(primary, args.steps, args.warmup, stage=dominant)
    ms_other, _ = timed(other, args.steps, args.warmup)

    P = int(npairs.item())
    H = int(outs[primary]["n_hits"].item())
    nnzb = int(outs[primary]["n_blocks"].item())
    value = P / (ms * 1e-3)
    dom_launches, dom_ms = tim.get(dominant, (0, 0.0))
    dom_avg_ms = dom_ms / max(dom_launches, 1)
    prec_bytes = 4 if primary == "mixed" else 8
    alg = stage_bytes(dominant, nv, nt, P, H, nnzb, prec_bytes)
    achieved = alg / (dom_avg_ms * 1e-3) / 1e9 if dom_avg_ms > 0 else 0.0

    rec = {
        "metric": "triangle pairs/s (energy+grad+PSD Hessian assembled), FP32 vs FP64 at stated err",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64pred" if primary == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_verts": nv, "n_tris": nt, "pairs": P, "hits": H, "nnzb": nnzb,
                   "step": "broadphase+screen+derivatives+energy+gradient+BSR Hessian",
                   "launch_params": tuned},
        "hits_per_s": H / (ms * 1e-3),  # intersecting pairs found per second of the whole step
        "autotune": {"ms_per_step_default_params": ms_default, "ms_per_step_tuned_params": ms_tuned},
        other: {"value": P / (ms_other * 1e-3), "ms_per_step": ms_other},
        "stages_ms_per_step": {k: round(v, 5) for k, v in per_step_stage.items()},
        # the same step split at the stage timers: evaluation only (screening through BSR
        # assembly, candidate pairs per second of it) and the broad phase (triangles per second)
        "eval_only": {"ms_per_step": sum(v for k, v in per_step_stage.items() if not k.startswith("bp_")),
                      "pairs_per_s": P / (sum(v for k, v in per_step_stage.items() if not k.startswith("bp_")) * 1e-3)},
        "broadphase_only": {"ms_per_step": sum(v for k, v in per_step_stage.items() if k.startswith("bp_")),
                            "tris_per_s": nt / (sum(v for k, v in per_step_stage.items() if k.startswith("bp_")) * 1e-3)},
        "roofline": {"kernel_stage": dominant, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured(dominant, "bytes", tuned),
                     "traffic_unit": "bytes per launch",
                     "alg_bytes_per_launch": alg, "avg_launch_ms": dom_avg_ms, "launches": dom_launches},
    }

    # the same kernel against the VALU issue rate (its real bound: a latency- and issue-bound
    # tree search), from the committed instruction count and the live duration
    vw = measured(dominant, "valu_wave", tuned)
    if vw and dom_avg_ms > 0:
        rate = vw * 64 / (dom_avg_ms * 1e-3)
        rec["roofline_issue"] = {"kernel_stage": dominant, "bound": "alu", "achieved": rate, "peak": VALU_LANE_PEAK,
                                 "unit": "VALU lane-instructions/s", "frac": rate / VALU_LANE_PEAK,
                                 "valu_wave_instructions_per_launch": vw}

    if not args.no_cpu_baseline:
        import oracle

        res = None
        reps = 0
        t0 = time.perf_counter()
        while True:
            ref_pairs = oracle.pairs(x, tris, oracle.BROAD_BOXES)
            res = oracle.evaluate(x, tris, ref_pairs, psd=oracle.PSD_PER_PART, hessian=True)
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        # the same on one thread (the box broad phase is single-threaded either way)
        reps1 = 0
        t1 = time.perf_counter()
        while True:
            p1 = oracle.pairs(x, tris, oracle.BROAD_BOXES)
            oracle.evaluate(x, tris, p1, psd=oracle.PSD_PER_PART, hessian=True, threads=1)
            reps1 += 1
            if time.perf_counter() - t1 >= args.cpu_seconds / 2:
                break
        el1 = time.perf_counter() - t1
        rec["cpu_baseline"] = {"value": len(ref_pairs) * reps / el, "unit": "pairs/s", "cores": oracle.threads(),
                               "kind": "oracle",
                               "sample": f"the full workload (box broad phase + evaluation + BSR assembly), "
                                         f"{reps} repetitions in {el:.1f} s",
                               "value_1thread": len(p1) * reps1 / el1,
                               "sample_1thread": f"the same on one thread, {reps1} repetitions in {el1:.1f} s"}

        def rel(a, b):
            a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
            return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

        err = {}
        for name in ("mixed", "fp64"):
            o = outs[name]
            nb = int(o["n_blocks"].item())
            err[name] = {"energy_rel": abs(o["energy"].item() - res["E"]) / abs(res["E"]),
                         "grad_rel": rel(o["grad"].cpu().numpy(), res["G"]),
                         "hess_rel": rel(o["vals"][:nb].cpu().numpy(), res["vals"])
                         if nb == len(res["vals"]) else None}
        rec["err"] = err
    if not args.no_extra:
        rec["extra"] = extra_configs(args, np, torch, ttie, workloads)
    print(json.dumps(rec), flush=True)
    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)  # one elementwise kernel: reads and writes exactly MB each
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
