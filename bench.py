#!/usr/bin/env python
"""Benchmark of the space-charge tracking step on one MI355X (gfx950).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Primary line (one JSON object on stdout): the space-charge avalanche cloud --
4,000,000 point charges (2M electrons, 2M cations, Gaussian clouds of sigma
50 um, at rest) in the single-GEM cell (40,776 cells) filled with the
synthetic Ar/CO2-like gas.  One step is one pass of the whole hot path
(track_step, dynamic option): right-hand side from the charging counts and
FP64 re-solve of the cell charges with the cached LU factors, field at every
charge from all cells and all other charges (mixed precision) with the
nearest opposite-species partner, recombination, Euler push with
null-collision Monte Carlo (1 ps), absorption and charging-up, compaction.
Every timed step starts from the same 4M-charge state (restored by a device
copy inside the timed region), so each step does the same work.  `value` is
(pair + charge-cell interactions) per second of that step.

`extra` carries the other measurements of the same metric: the field-only
step (re-solve + field, no transport), the influence of the 4M charges on the
40,776 cell equations, the GEM cell with 1M field points in mixed precision
and in FP64 (interactions/s each, and the relative L2 difference between the
two), the double-GEM tracking run (1000 steps from 200k electrons released
in the holes of the upper foil, with its population, event totals and the
final dL/dsigma), and the adjoint's backward/forward time ratio on 1M
charges with the refined (49,128-cell) mesh.

`roofline` is for the dominant work, the pairwise sum: per step one launch of
the directed kernel (tile pairs inside a super-block or near each other) and
the launches of the pair-once kernel (every other unordered pair evaluated
once for both particles) with their ordered reductions.  `achieved` counts
the work executed: 20 flop per term of the directed kernel (3 sub, 3 FMA for
|d|^2 + s^2, 1 rsqrt, 2 mul for the cube, 1 mul by q, 3 FMA into E) and 26
per pair-once evaluation (the same plus the partner's charge product and its
3 FMA), with the term and pair counts the library reports, divided by the
summed duration of those launches per step, measured with HIP events on the
library's stream inside the timed region, against the published FP32 vector
peak.  `interaction_equivalent` gives the 20-flop-per-interaction figure over
all n (n - 1) interactions beside it.  `cpu_baseline` times the CPU oracle on a sample
of the same workload (its error against the GPU field is reported too).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
FLOP_PER_PAIR = 20           # one directed interaction (3 sub, 3 FMA, rsqrt, 2 mul, 1 mul by q, 3 FMA)
FLOP_PER_ONCE_PAIR = 26      # one pair-once evaluation: the above plus the partner's charge product and 3 FMA


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the translation unit that holds the pairwise kernel (and the
    cell integrals it includes)."""
    h = hashlib.sha256()
    for f in ("field.hip", "cellmath.hpp"):
        with open(os.path.join(ROOT, "paper_2110_09214_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles():
    """HBM bytes per step of the pairwise sum's kernels from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "pairwise_cloud4M_traffic.json")
    try:
        with open(p) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_step")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run one plain 1 GiB device copy, one 1 GiB read-only sum and one tracking step of the "
                         "4M-charge cloud without cells (the same pairwise kernel as the timed step; for "
                         "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs), print the sizes and exit")
    ap.add_argument("--pmc-probe-cells", action="store_true",
                    help="run one 1 GiB device copy and the mixed cell field of the 40,776-cell GEM mesh at the "
                         "4M charges of the cloud (the cell kernels of the timed step, cell charges from a "
                         "smooth synthetic density), print the sizes and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the pairwise sum would shard by "
              "its (super-block, partner) work items with one reduce-scatter of the partial fields per step, "
              "which is not implemented here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2110_09214_amd import binding as B
    from paper_2110_09214_amd import workloads as W

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)

    def dev(a, dtype=torch.float64):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")

    def bind(ctx, m):
        return B.BoundMesh(ctx, dev(m.a), dev(m.b), dev(m.c), dev(m.kind, torch.int8), dev(m.eps1), dev(m.eps2))

    ctx = B.Context(0)
    stream = ctx.stream

    if args.pmc_probe:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)                                     # reads and writes 1 GiB each
        torch.cuda.synchronize()
        float(b.sum())                                 # reads 1 GiB (a second calibration of FETCH_SIZE)
        torch.cuda.synchronize()
        x, q, sp = W.space_charge_cloud()
        gas_s, gas_keep = B.gas_struct(W.synthetic_ar_co2(), "cuda")
        parts = B.Particles(len(q) + len(q) // 4, "cuda", dev(x), dev(np.zeros_like(x)), dev(sp, torch.int8),
                            torch.arange(len(q), dtype=torch.int64, device="cuda"), len(q))
        B.track_step(ctx, None, parts, gas_s, dict(dt=1e-12, step=1, seed=5, max_coll=64, max_ion_per_step=4,
                                                   ion_v_cap=2e4, box_lo=(-1.0, -1.0, -1.0), box_hi=(1.0, 1.0, 1.0),
                                                   soft=1e-7, r_rec=1e-6, precision=B.OBEM_MIXED), None, None)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "n_charges": len(q),
                          "kernel_source_sha256_16": kernel_source_hash()}), flush=True)
        ctx.close()
        return

    work = {}

    if args.pmc_probe_cells:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        mesh = W.gem_cell_mesh()
        x, q, sp = W.space_charge_cloud()
        bm = bind(ctx, mesh)
        c = (mesh.a + mesh.b + mesh.c) / 3
        sig = dev(1e-6 * np.sin(c @ np.array([3e4, 2e4, 1e4])))
        E = B.field_eval(ctx, bm, sig, None, None, dev(x), 0.0, B.OBEM_MIXED)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "n_points": len(q),
                          "n_cells": mesh.n, "E_rms": float(E.pow(2).sum(1).mean().sqrt()),
                          "kernel_source_sha256_16": kernel_source_hash()}), flush=True)
        ctx.close()
        return

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read()
        ctx.profile_work()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        work["directed"], work["once"] = ctx.profile_work()
        ctx.profile(False)
        return e0.elapsed_time(e1) / steps, prof

    # ------------------------------------------------------------------ primary
    t0 = time.time()
    mesh = W.gem_cell_mesh()
    x, q, sp = W.space_charge_cloud()
    n, N = len(q), mesh.n
    log(f"[bench] space-charge cloud: {n} charges, {N} cells (inputs {time.time() - t0:.1f}s)")
    bm = bind(ctx, mesh)
    rhs = dev(mesh.rhs)
    t0 = time.time()
    sigma, info = B.bem_solve_charges(ctx, bm, rhs, max_refine=3)
    torch.cuda.synchronize()
    log(f"[bench] assembly + LU + solve of {N} cells: {time.time() - t0:.1f}s, backward error {info['backward_error']:.2e}")
    X, Q = dev(x), dev(q)
    gas = W.synthetic_ar_co2()
    gas_s, gas_keep = B.gas_struct(gas, "cuda")
    geo = W.GemGeometry()
    top = geo.t_kapton / 2 + geo.t_cu
    params = dict(dt=1e-12, step=0, seed=5, max_coll=64, max_ion_per_step=4, ion_v_cap=2e4,
                  box_lo=(-geo.half_x, -geo.half_y, -(top + 2e-3)), box_hi=(geo.half_x, geo.half_y, top + 3e-3),
                  soft=1e-7, r_rec=1e-6, precision=B.OBEM_MIXED, resolve=1, influence=0)
    ids0 = torch.arange(n, dtype=torch.int64, device="cuda")
    sp0 = dev(sp, torch.int8)
    parts = B.Particles(n + n // 4, "cuda", X, torch.zeros_like(X), sp0, ids0, n)
    counts = torch.zeros(N, dtype=torch.int64, device="cuda")
    step_stats = []

    def restore():
        for k in range(3):
            parts.cols[k][:n].copy_(X[:, k])
            parts.cols[3 + k][:n].zero_()
        parts.species[:n].copy_(sp0)
        parts.id[:n].copy_(ids0)
        parts.n_live, parts.next_id = n, n
        counts.zero_()

    def step():
        restore()
        params["step"] += 1
        st = B.track_step(ctx, bm, parts, gas_s, params, counts, sigma, rhs)
        step_stats.append(st)

    log(f"[bench] timing {args.steps} steps after {args.warmup} warm-up")
    ms, prof = timed(step, args.steps, args.warmup)
    last = step_stats[-1]
    pairs = n * (n - 1)
    inter = pairs + n * N
    value = inter / (ms / 1e3)
    # the pairwise sum: directed launch, its reduction, pair-once launches
    pair_keys = [k for k in ("pair", "pair_reduce", "pair_once") if k in prof]
    pair_ms = sum(prof[k][0] for k in pair_keys) / args.steps
    # executed work: the directed kernel's terms at 20 flop, the pair-once
    # kernel's evaluations (two interactions each) at 26 flop
    directed_terms = work["directed"] / args.steps
    once_pairs = work["once"] / args.steps
    exec_flop = FLOP_PER_PAIR * directed_terms + FLOP_PER_ONCE_PAIR * once_pairs
    achieved = exec_flop / (pair_ms / 1e3) / 1e12
    achieved_equiv = FLOP_PER_PAIR * pairs / (pair_ms / 1e3) / 1e12
    log(f"[bench] step {ms:.1f} ms, {value:.3e} interactions/s; kernels: " +
        ", ".join(f"{k} {v[0] / max(v[1], 1):.2f}ms x{v[1]}" for k, v in prof.items()))
    log(f"[bench] last step: {dict((k, last[k]) for k in ('n_live', 'recombined', 'absorbed', 'left_world', 'children'))}"
        f" collisions {list(last['real_collisions'])} null {last['null_collisions']}")
    traffic = traffic_from_profiles()
    out = {
        "metric": "particle-source interactions/s, mixed vs FP64 at 1e-5 rel err; bwd/fwd ratio",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed-f32/f64",
        "data": "synthetic",
        "config": {
            "workload": "space-charge avalanche cloud: 4,000,000 point charges (2M electrons + 2M cations at rest, "
                        "Gaussian sigma 50 um) in the single-GEM cell of 40,776 cells with a synthetic Ar/CO2-like "
                        "gas; per step the whole tracking step: FP64 cell-charge re-solve (cached LU + refinement), "
                        "mixed-precision field at every charge with nearest opposite-species partner, "
                        "recombination (1 um), 1 ps Euler push with null-collision MC, absorption and charging-up, "
                        "compaction",
            "n_charges": n, "n_cells": N, "softening_m": 1e-7, "precision": "mixed", "dt_s": 1e-12,
            "interactions_per_step": inter, "pair_interactions_per_step": pairs,
        },
        "roofline": {
            "kernel": "pairwise sum: k_pair_sym launches + k_pair_mixed (directed remainder) + reductions",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": traffic,
            "flop_counted": f"executed: {FLOP_PER_PAIR} per directed term x {directed_terms:.4g} + "
                            f"{FLOP_PER_ONCE_PAIR} per pair-once evaluation x {once_pairs:.4g} per step",
            "ms_per_step": pair_ms,
            "interaction_equivalent": {
                "achieved": achieved_equiv, "frac": achieved_equiv / FP32_PEAK_TFLOPS,
                "flop_per_interaction": FLOP_PER_PAIR, "interactions": pairs,
                "note": "20 flop per ordered interaction n(n-1), as if every interaction were evaluated on its own",
            },
        },
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "last_step": {k: (list(v) if k == "real_collisions" else v) for k, v in last.items()},
    }
    E = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]

    # ------------------------------------------------------------ cpu baseline
    if not args.no_cpu_baseline:
        import oracle

        cores = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        rng = np.random.default_rng(11)
        it = rng.choice(n, 1536, replace=False)          # about 10 s of the oracle on 16 cores
        ic = it[:384]
        sig_h = sigma.cpu().numpy()
        B.field_eval(ctx, bm, sigma, X, Q, X, 1e-7, B.OBEM_MIXED, tgt_is_src=True, out=E)
        t0 = time.time()
        Ep = oracle.pair_field(x[it], x, q, 1e-7)        # own term: zero field at zero distance
        tp = time.time() - t0
        t0 = time.time()
        Ec = oracle.panel_field(x[ic], mesh.a, mesh.b, mesh.c, sig_h)
        tc = time.time() - t0
        rate_p = len(it) * n / tp
        rate_c = len(ic) * N / tc
        # transport: the oracle's push + null-collision MC + absorption (every
        # flight chord tested against all cells) on a sample of the cloud in
        # a uniform 1 MV/m drift field
        im = rng.choice(n, 2048, replace=False)
        xm, vm, spm = x[im].copy(), np.zeros((len(im), 3)), sp[im].copy()
        Em = np.zeros((len(im), 3))
        Em[:, 2] = 1e6
        t0 = time.time()
        oracle.mc_step(xm, vm, spm, im.astype(np.int64), Em, gas, params, mesh)
        tm = time.time() - t0
        rate_m = len(im) / tm
        t_full = pairs / rate_p + n * N / rate_c + n / rate_m
        Eg = torch.stack(E, 1).cpu().numpy()
        # oracle total field on the targets that have both parts
        ref = Ep[:len(ic)] + Ec
        err = float(np.linalg.norm(Eg[ic] - ref) / np.linalg.norm(ref))
        out["cpu_baseline"] = {
            "value": inter / t_full, "unit": "interactions/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(it)} of the {n} charges against all {n} charges ({tp:.1f}s), {len(ic)} against all "
                      f"{N} cells ({tc:.1f}s), push + MC + absorption of {len(im)} charges ({tm:.1f}s); per-part "
                      f"rates combined over the full step (solve, recombination and compaction not sampled)",
            "gpu_vs_oracle_rel_l2_on_sample": err,
        }
        log(f"[bench] cpu oracle: {inter / t_full:.3e} interactions/s on {cores} cores; GPU vs oracle rel L2 {err:.2e}")

    # ------------------------------------------------------------------ extras
    if not args.no_extra:
        extra = {}

        def field_step():
            B.bem_solve_charges(ctx, bm, rhs, sigma, max_refine=1, want_info=False)
            B.field_eval(ctx, bm, sigma, X, Q, X, 1e-7, B.OBEM_MIXED, tgt_is_src=True, out=E)

        ms_f, _ = timed(field_step, 2, 1)
        extra["field_only_step_ms"] = ms_f
        extra["field_only_interactions_per_s"] = inter / (ms_f / 1e3)
        rhs_i = torch.empty_like(rhs)

        def infl():
            B.bem_influence(ctx, bm, rhs, X, Q, B.OBEM_MIXED, rhs_out=rhs_i)

        ms_i, _ = timed(infl, 2, 1)
        extra["influence_ms"] = ms_i
        extra["influence_interactions_per_s"] = n * N / (ms_i / 1e3)
        log(f"[bench] field-only step {ms_f:.1f} ms; influence of {n} charges on {N} cells {ms_i:.1f} ms")
        # parallel-plate counter: 4096 cells (FP64 solve), the field at the
        # 4096 electrons from all cells and the other electrons, FP64 and mixed
        m1 = W.parallel_plate_mesh()
        x1, q1 = W.parallel_plate_electrons()
        bm1 = bind(ctx, m1)
        sig1, _ = B.bem_solve_charges(ctx, bm1, dev(m1.rhs))
        X1, Q1 = dev(x1), dev(q1)
        n1 = len(q1)
        inter1 = n1 * m1.n + n1 * (n1 - 1)
        outs1 = {}
        for name, prec in (("fp64", B.OBEM_FP64), ("mixed", B.OBEM_MIXED)):
            res = {}

            def fe1(prec=prec, res=res):
                res["E"] = B.field_eval(ctx, bm1, sig1, X1, Q1, X1, 1e-7, prec, tgt_is_src=True)

            ms1, _ = timed(fe1, 5, 2)
            outs1[name] = res["E"]
            extra[f"parallel_plate_{name}_interactions_per_s"] = inter1 / (ms1 / 1e3)
            extra[f"parallel_plate_{name}_ms"] = ms1
        extra["parallel_plate_mixed_vs_fp64_rel_l2"] = float((outs1["mixed"] - outs1["fp64"]).norm() /
                                                             outs1["fp64"].norm())
        if not args.no_cpu_baseline:
            import oracle

            s1 = sig1.cpu().numpy()
            t0 = time.time()
            ref1 = oracle.panel_field(x1, m1.a, m1.b, m1.c, s1) + oracle.pair_field(x1, x1, q1, 1e-7, tgt_is_src=True)
            t1 = time.time() - t0
            extra["parallel_plate_oracle_interactions_per_s"] = inter1 / t1
            extra["parallel_plate_fp64_vs_oracle_rel_l2"] = float(np.linalg.norm(outs1["fp64"].cpu().numpy() - ref1) /
                                                                  np.linalg.norm(ref1))
            extra["parallel_plate_mixed_vs_oracle_rel_l2"] = float(np.linalg.norm(outs1["mixed"].cpu().numpy() - ref1) /
                                                                   np.linalg.norm(ref1))
        extra["parallel_plate_workload"] = f"{n1} electrons x ({m1.n} cells + {n1 - 1} other electrons), FP64 solve"
        log(f"[bench] parallel plate: fp64 {extra['parallel_plate_fp64_interactions_per_s']:.3e}/s, mixed "
            f"{extra['parallel_plate_mixed_interactions_per_s']:.3e}/s")
        del bm1, outs1
        # GEM cell, 1M field points: mixed vs FP64
        pts = dev(W.gem_cell_points())
        npts = int(pts.shape[0])
        outs = {}
        for name, prec in (("mixed", B.OBEM_MIXED), ("fp64", B.OBEM_FP64)):
            res = {}

            def fe(prec=prec, res=res):
                res["E"] = B.field_eval(ctx, bm, sigma, None, None, pts, 0.0, prec)

            ms_g, pr = timed(fe, 2, 1)
            outs[name] = res["E"]
            extra[f"gem_cell_{name}_interactions_per_s"] = npts * N / (ms_g / 1e3)
            extra[f"gem_cell_{name}_ms"] = ms_g
        d = (outs["mixed"] - outs["fp64"]).norm() / outs["fp64"].norm()
        extra["gem_cell_mixed_vs_fp64_rel_l2"] = float(d)
        if not args.no_cpu_baseline:
            import oracle

            ig = np.random.default_rng(13).choice(npts, 256, replace=False)
            ig_t = torch.as_tensor(ig, device="cuda")
            pts_h = pts[ig_t].cpu().numpy()
            t0 = time.time()
            refg = oracle.panel_field(pts_h, mesh.a, mesh.b, mesh.c, sigma.cpu().numpy())
            tg = time.time() - t0
            extra["gem_cell_oracle_interactions_per_s"] = len(ig) * N / tg
            for name in ("mixed", "fp64"):
                eg = outs[name][ig_t].cpu().numpy()
                extra[f"gem_cell_{name}_vs_oracle_rel_l2_on_sample"] = float(np.linalg.norm(eg - refg) /
                                                                             np.linalg.norm(refg))
            extra["gem_cell_oracle_sample"] = f"{len(ig)} of the {npts} points against all {N} cells ({tg:.1f}s)"
        extra["gem_cell_workload"] = f"{npts} field points x {N} cells, cell charges from the FP64 solve"
        log(f"[bench] gem cell: mixed {extra['gem_cell_mixed_interactions_per_s']:.3e}/s, "
            f"fp64 {extra['gem_cell_fp64_interactions_per_s']:.3e}/s, rel L2 {float(d):.2e}")
        del outs, pts
        # double-GEM run (the tracking configuration): 200k electrons released
        # at rest in the holes of the upper foil, 60,752 cells, 1000 steps of
        # 1 ps with the charging-up re-solve every step, capacity 2M; then the
        # final-step backward dL/dsigma of L = sum w . E(x)
        geo5 = W.GemGeometry(m=10, n_r=5, n_cone=6)
        top5 = geo5.t_kapton / 2 + geo5.t_cu
        m5 = W.double_gem_mesh(geo5)
        x5, sp5 = W.double_gem_avalanche_start(geo=geo5)
        n5 = len(sp5)
        bm5 = bind(ctx, m5)
        rhs5 = dev(m5.rhs)
        t0 = time.time()
        sig5, _ = B.bem_solve_charges(ctx, bm5, rhs5)
        torch.cuda.synchronize()
        t_setup5 = time.time() - t0
        parts5 = B.Particles(2_000_000, "cuda", dev(x5), dev(np.zeros_like(x5)), dev(sp5, torch.int8),
                             torch.arange(n5, dtype=torch.int64, device="cuda"), n5)
        counts5 = torch.zeros(m5.n, dtype=torch.int64, device="cuda")
        p5 = dict(dt=1e-12, step=0, seed=5, max_coll=64, max_ion_per_step=4, ion_v_cap=2e4,
                  box_lo=(-geo5.half_x, -geo5.half_y, -2e-3 - top5 - 2e-3),
                  box_hi=(geo5.half_x, geo5.half_y, top5 + 3e-3), soft=1e-7, r_rec=1e-6,
                  precision=B.OBEM_MIXED, resolve=3)
        steps5 = 1000
        tot5 = dict(children=0, recombined=0, absorbed=0, left_world=0, dd_charge_deposited=0, ionisations=0,
                    attachments=0, children_dropped=0)
        live5, inter5 = [], []

        def step5():
            nl = parts5.n_live
            st = B.track_step(ctx, bm5, parts5, gas_s, p5, counts5, sig5, rhs5)
            p5["step"] += 1
            inter5.append(nl * (nl - 1) + nl * m5.n)
            for k in ("children", "recombined", "absorbed", "left_world", "dd_charge_deposited", "children_dropped"):
                tot5[k] += st[k]
            tot5["ionisations"] += st["real_collisions"][3]
            tot5["attachments"] += st["real_collisions"][4]
            if p5["step"] % 50 == 0:
                live5.append(parts5.n_live)

        ms5, prof5 = timed(step5, steps5, 0)
        rate5 = sum(inter5) / (steps5 * ms5 / 1e3)
        nl5 = parts5.n_live
        X5 = torch.stack([c[:nl5] for c in parts5.cols[:3]], 1).contiguous()
        Q5 = torch.full((nl5,), -W.E_CHARGE, dtype=torch.float64, device="cuda")
        Q5[parts5.species[:nl5] == 1] = W.E_CHARGE
        W5 = dev(np.random.default_rng(6).normal(size=(nl5, 3)))

        def bwd5():
            B.field_eval_backward(ctx, bm5, sig5, X5, Q5, X5, 1e-7, W5, B.OBEM_MIXED, tgt_is_src=True,
                                  want_t=False, want_s=False)

        ms5b, _ = timed(bwd5, 1, 1)
        extra["double_gem_steps"] = steps5
        extra["double_gem_step_ms"] = ms5
        extra["double_gem_kernel_ms_per_step"] = {k: v[0] / steps5 for k, v in prof5.items()}
        extra["double_gem_interactions_per_s"] = rate5
        extra["double_gem_interactions_total"] = int(sum(inter5))
        extra["double_gem_n_live_every_50_steps"] = live5
        extra["double_gem_totals"] = dict(tot5, dd_charges_on_cells=int(counts5.abs().sum()))
        extra["double_gem_final_backward_ms"] = ms5b
        extra["double_gem_workload"] = (f"{n5} electrons released at rest in the holes of the upper foil, "
                                        f"{m5.n} cells, {steps5} steps of 1 ps, charging-up re-solve every "
                                        f"step (from the inverse's columns of the dd cells hit when few changed, "
                                        f"a full refined solve otherwise and every 64 updates), recombination "
                                        f"within 1 um, capacity 2M, mixed; setup (assembly "
                                        f"+ LU + inverse) {t_setup5:.1f} s; then dL/dsigma of L = sum w.E at "
                                        f"the {nl5} final charges")
        log(f"[bench] double GEM: {steps5} steps, {ms5:.1f} ms per step, {rate5:.3e} interactions/s, n_live "
            f"{n5} -> {nl5}, totals {tot5}, backward {ms5b:.1f} ms")
        del bm5, parts5, X5, Q5, W5
        # adjoint bwd/fwd on 1M charges + refined mesh (synthetic cell charges)
        m4 = W.gem_cell_mesh(W.gem_cell_refined_geometry())
        x4, q4, sp4, w4 = W.adjoint_workload()
        bm4 = bind(ctx, m4)
        c4 = (m4.a + m4.b + m4.c) / 3
        s4 = dev(1e-6 * np.sin(c4 @ np.array([3e4, 2e4, 1e4])))
        X4, Q4, W4 = dev(x4), dev(q4), dev(w4)

        def fwd():
            B.field_eval(ctx, bm4, s4, X4, Q4, X4, 1e-7, B.OBEM_MIXED, tgt_is_src=True)

        def bwd():
            B.field_eval_backward(ctx, bm4, s4, X4, Q4, X4, 1e-7, W4, B.OBEM_MIXED, tgt_is_src=True)

        ms_f, _ = timed(fwd, 2, 1)
        ms_b, pb = timed(bwd, 2, 1)
        extra["adjoint_fwd_ms"] = ms_f
        extra["adjoint_bwd_ms"] = ms_b
        extra["adjoint_bwd_fwd_ratio"] = ms_b / ms_f
        extra["adjoint_workload"] = f"{len(q4)} charges (targets = sources) + {m4.n} cells, mixed precision"
        log(f"[bench] adjoint: fwd {ms_f:.1f} ms, bwd {ms_b:.1f} ms, ratio {ms_b / ms_f:.2f}")
        out["extra"] = extra

    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
