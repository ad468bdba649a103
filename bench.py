#!/usr/bin/env python
"""Benchmark of the XM hot path on one MI355X.

Workload: the large unordered scene (N = 10155 frames, M = 2M landmarks, ~8M
observations, 20 camera clusters, 5% outlier observations; synthetic, seeded).
One step = the whole hot path on that scene with the observations resident in
HBM: xm_build_Q (Q assembly, FP64), xm_bm_solve in the FP32 form (FP32
products, tCG and retraction, then an FP64 stage to the FP64 gradient
tolerance; FP64 dual certificate inside the staircase) and
xm_round (FP64).  The reported value is the mean wall time of a step, i.e.
the time from resident observations to certified, rounded optimum (mean,
median, min and max are reported, with the parts: Q assembly; solve +
certificate + rounding with Q resident).  The plain FP64 form is timed with
the same protocol after the steps, the BF16-stored-Q solve with Q resident.

Prints one JSON line.  --gpus N with N > 1 is refused (one GPU per box).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-certified-optimum (s) + BSR SpMM GB/s, FP32 vs FP64, N=10k frames"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6   # MI355X FP64, vector and matrix
# HBM bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain
# copy kernel (profiles/hbm_traffic_sweep_update_large.md,
# profiles/hbm_traffic_spmm_sym_f32_large.md,
# profiles/hbm_traffic_factored_product_large.md); valid for the large workload
# and the kernels as they were profiled -- re-measure after changing one.
PMC_TRAFFIC_BYTES = {("large", "sweep_update_kernel"): 0.948e9,
                     ("large", "spmm_sym_kernel (f32 Q)"): 1.923e9,
                     ("large", "spmm_sym_kernel (f32 G^-1, in the factored product)"): 0.219e9,
                     ("large", "fact_rows pass (f32, in the factored product)"): 0.215e9}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(sc, products, n_timed=4):
    """The FP64 oracle on the full workload, timed on this host's cores: its Q
    assembly in the matrix-free form (sparse landmark elimination + one dense
    Cholesky of the grounded Laplacian: the same elimination as its dense
    construction, which would need 7.4 GB and a cubic solve here), then
    `n_timed` of its Q products at rank 5, measured.  A full oracle solve is
    not run (the bound on the sample): its time is the assembly plus the
    measured per-product time times `products`, the Q products an oracle
    staircase takes for the FP64 solve's iteration counts (its Hessian
    recomputes the product at the point, so two per truncated-CG iteration)."""
    import numpy as np

    from oracle import data_matrix
    threads = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        threads = min(threads, int(omp))
    t0 = time.perf_counter()
    op = data_matrix.QOperator(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w)
    t1 = time.perf_counter()
    Y = np.random.default_rng(0).standard_normal((3 * sc.N, 5))
    for _ in range(n_timed):
        op.matmat(Y)
    t2 = time.perf_counter()
    per = (t2 - t1) / n_timed
    return {
        "value": round((t1 - t0) + products * per, 2),
        "unit": "s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 oracle on the full {sc.N}-frame workload: Q assembly (matrix-free: sparse landmark "
                   f"elimination + dense Cholesky of the {sc.N - 1}-frame grounded Laplacian) measured "
                   f"{t1 - t0:.1f} s; {n_timed} rank-5 Q products measured, {per:.3f} s each; the solve "
                   f"is not run: {products} products (two per truncated-CG iteration and two per trust-region "
                   f"step of the FP64 solve's counts, plus its Lanczos steps) x {per:.3f} s"),
        "measured_s": round(t2 - t0, 2),
        "assembly_s": round(t1 - t0, 2),
        "product_s": round(per, 4),
        "products": products,
    }


def _summary(xs):
    return {"mean": round(statistics.fmean(xs), 4), "median": round(statistics.median(xs), 4),
            "min": round(min(xs), 4), "max": round(max(xs), 4), "n": len(xs)}


WORKLOAD_TEXT = {
    "large": ("large unordered scene: N=10155 frames in 20 Gaussian camera clusters (centres U[-15,15]^3, "
              "sigma_c=6), M=2M landmarks, track length 1+Geom(1/3) (mean 4, min 2) over the 50 nearest cameras, "
              "~8.0M observations, noise sigma=0.02, depth scales U[0.5,2], 5% outlier observations whose "
              "3D point is drawn uniformly in the cube of half-side 3 around the true landmark (local outliers)"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 / BF16 comparison solves")
    ap.add_argument("--no-box", action="store_true", help="skip the box-outlier variant of the workload")
    ap.add_argument("--no-xm2", action="store_true", help="skip the XM^2 run on the workload")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the steps, run one plain FP32 copy kernel (torch.mul by 1) of this many MiB: "
                         "the reference dispatch that scales the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch

    import paper_2502_04640_amd as xm
    import scenes

    t = time.perf_counter()
    sc = scenes.make_scene(args.workload, args.seed)
    log(f"scene {args.workload}: N={sc.N} M={sc.M} n_obs={sc.n_obs} ({time.perf_counter() - t:.1f} s)")
    dev = torch.device("cuda:0")
    fr = torch.from_numpy(sc.frame).to(dev)
    lm = torch.from_numpy(sc.landmark).to(dev)
    u = torch.from_numpy(sc.u).to(dev)
    w = torch.from_numpy(sc.w).to(dev)
    torch.cuda.synchronize()
    opts32 = xm.SolveOptions(compute="f32", verbose=args.verbose)
    opts64 = xm.SolveOptions(compute="f64", verbose=args.verbose)
    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del a, b

    def step(opts, keep, timing=False):
        """One pass of the hot path: observations in HBM -> Q -> certified
        solve -> rounded rotations.  Returns the problem and the part times."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = xm.build_Q(sc.N, sc.M, fr, lm, u, w, keep=keep)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if timing:
            P.spmm_timing(True)
        Y, info = P.solve(opts)
        R, s, rho_hat = P.round(Y)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return P, Y, info, rho_hat, (t1 - t0), (t2 - t1)

    def run_steps(opts, keep, warmup, steps, tag):
        P = None
        for i in range(warmup):
            P, Y, info, rho_hat, tb, ts = step(opts, keep)
            log(f"{tag} warmup {i}: build {tb:.3f} s, solve+cert+round {ts:.3f} s, "
                f"certified={info['certified']} r={info['r']}")
            del P
            P = None
        builds, ttcs, infos, rhos = [], [], [], []
        torch.cuda.synchronize()
        t_all0 = time.perf_counter()
        for i in range(steps):
            if P is not None:
                del P
                P = None
            P, Y, info, rho_hat, tb, ts = step(opts, keep)
            builds.append(tb)
            ttcs.append(ts)
            infos.append(info)
            rhos.append(rho_hat)
            log(f"{tag} step {i}: build {tb:.3f} s, ttc {ts:.3f} s, certified={info['certified']} r={info['r']} "
                f"outer={info['outer_iters']} inner={info['inner_iters']} spmm={info['spmm_count']} "
                f"lanczos={info['lanczos_iters']} cost={info['cost']:.10e}")
        del P
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_all0
        return builds, ttcs, infos, rhos, wall

    # the timed FP32 steps (no per-launch instrumentation inside them)
    builds, ttcs, infos, rhos, wall = run_steps(opts32, ("f32",), args.warmup, args.steps, "f32")
    steps_s = [b + t for b, t in zip(builds, ttcs)]
    last = infos[-1]
    rho = rhos[-1]
    eta = (rho - last["cost"]) / (1 + abs(rho) + abs(last["cost"]))

    # one more step, instrumented: HIP events around every product launch and
    # the main assembly launches give the per-kernel figures (not timed above)
    P, Y, info_i, _, tb_i, ts_i = step(opts32, ("f32",), timing=True)
    log(f"instrumented step: build {tb_i:.3f} s, ttc {ts_i:.3f} s")
    stats = P.spmm_stats(reset=True)
    kernels = {}
    names = {"f64": "spmm_sym_kernel (f64 Q)", "f32": "spmm_sym_kernel (f32 Q)",
             "bf16": "spmm_split_kernel (bf16 Q)",
             "f64_ginv": "spmm_sym_kernel (f64 G^-1, in the factored product)",
             "f32_ginv": "spmm_sym_kernel (f32 G^-1, in the factored product)",
             "f64_factored": "factored product (f64: sparse A_rr, A_rt; dense G^-1)",
             "f32_factored": "factored product (f32: sparse A_rr, A_rt; dense G^-1)",
             "f64_fact_rows": "fact_rows pass (f64, in the factored product)",
             "f32_fact_rows": "fact_rows pass (f32, in the factored product)"}
    composite = {names["f64_factored"], names["f32_factored"]}
    for k in stats:
        if stats[k]["launches"]:
            kernels[names[k]] = {
                "launches": stats[k]["launches"], "total_ms": stats[k]["total_ms"],
                "bytes": stats[k]["bytes_per_launch"] * stats[k]["launches"], "flops": None}
    for name, v in P.build_stats().items():
        kernels[name] = dict(v)
    spmm_kinds = {f"{d} {role}": P.spmm_kind(d, role) for d in ("f64", "f32") for role in ("residual", "curvature")}
    del P
    dom_name = max((k for k in kernels if k not in composite), key=lambda k: kernels[k]["total_ms"])
    dk = kernels[dom_name]
    avg_ms = dk["total_ms"] / dk["launches"]
    bytes_l = dk["bytes"] / dk["launches"]
    flops_l = (dk["flops"] or 0.0) / dk["launches"]
    gbs = bytes_l / (avg_ms * 1e-3) / 1e9
    tfs = flops_l / (avg_ms * 1e-3) / 1e12
    if flops_l and tfs / FP64_PEAK_TFS > gbs / HBM_PEAK_GBS:
        roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                "frac": round(tfs / FP64_PEAK_TFS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    roof.update({"traffic": PMC_TRAFFIC_BYTES.get((args.workload, dom_name)), "kernel": dom_name,
                 "launches": dk["launches"],
                 "bytes_per_launch": bytes_l, "flops_per_launch": flops_l or None,
                 "avg_launch_ms": round(avg_ms, 4)})
    spmm_gbs = {k: (stats[k]["bytes_per_launch"] / (stats[k]["total_ms"] / stats[k]["launches"] * 1e-3) / 1e9
                    if stats[k]["launches"] else None) for k in stats}
    out = {
        "metric": METRIC,
        "value": round(statistics.fmean(steps_s), 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 2),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "precision_note": ("FP32 stage (FP32 products, truncated CG, retraction and iterate) to the FP32 floor, then "
                           "an FP64 stage (FP64 iterate, manifold arithmetic and gradient products; truncated-CG "
                           "Hessian products still FP32) to the FP64 gradient tolerance; Q assembly, the "
                           "certificate Lanczos, the final cost/gradient check and rounding in FP64"),
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT.get(args.workload, args.workload),
                   "N": sc.N, "M": sc.M, "n_obs": sc.n_obs, "seed": args.seed, "outlier_model": "local",
                   "solver": {"r0": opts32.r0, "r_max": opts32.r_max, "lift": opts32.lift}},
        "step_s": _summary(steps_s),
        "build_Q_s": _summary(builds),
        "ttc_q_resident_s": _summary(ttcs),
        "certified": bool(last["certified"]),
        "rank": last["r"],
        "cost": last["cost"],
        "rho_hat": rho,
        "eta": eta,
        "lambda_min": last["lambda_min"],
        "solve_ms": round(last["solve_ms"], 2),
        "cert_ms": round(last["cert_ms"], 2),
        "iters": {"outer": last["outer_iters"], "inner": last["inner_iters"], "spmm": last["spmm_count"],
                  "lanczos": last["lanczos_iters"], "stair_steps": last["stair_steps"]},
        "spmm_GBps": {k: (round(v, 1) if v else None) for k, v in spmm_gbs.items()},
        # the metric's SpMM: the Y Q product over the stored FP32 Q (residual products)
        "spmm_roofline": ({"kernel": names["f32"], "bound": "hbm", "achieved": round(spmm_gbs["f32"], 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(spmm_gbs["f32"] / HBM_PEAK_GBS, 4),
                           "traffic": PMC_TRAFFIC_BYTES.get((args.workload, names["f32"]))}
                          if spmm_gbs.get("f32") else None),
        "spmm_launches": {k: stats[k]["launches"] for k in stats},
        "spmm_kernel": spmm_kinds,
        "roofline": roof,
        "kernels_ms": {k: round(v["total_ms"], 2) for k, v in kernels.items()},
    }
    if not args.no_compare:
        # the plain FP64 form, same protocol (build without reduced copies + FP64 solve + rounding)
        b64, t64, i64s, r64s, wall64 = run_steps(opts64, (), min(args.warmup, 1), args.steps, "f64")
        i64 = i64s[-1]
        out["f64_step_s"] = _summary([b + t for b, t in zip(b64, t64)])
        out["ttc_f64_s"] = _summary(t64)
        out["f64_solve"] = {"certified": bool(i64["certified"]), "rank": i64["r"], "cost": i64["cost"],
                            "outer": i64["outer_iters"], "inner": i64["inner_iters"],
                            "lanczos": i64["lanczos_iters"], "rho_hat": r64s[-1],
                            "cost_gap_vs_f32": abs(i64["cost"] - last["cost"]) / (1 + abs(i64["cost"])
                                                                                   + abs(last["cost"]))}
        # BF16-stored Q (Hessian products) with FP32 gradient and cost: Q resident
        P = xm.build_Q(sc.N, sc.M, fr, lm, u, w, keep=("f32", "bf16"))
        tb16 = []
        for i in range(1 + min(args.steps, 3)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Yc, ic = P.solve(xm.SolveOptions(compute="bf16"))
            Rc, sc_, rc = P.round(Yc)
            torch.cuda.synchronize()
            if i:
                tb16.append(time.perf_counter() - t0)
        out["ttc_bf16_s"] = _summary(tb16)
        out["bf16_solve"] = {"certified": bool(ic["certified"]), "rank": ic["r"], "cost": ic["cost"],
                             "outer": ic["outer_iters"], "inner": ic["inner_iters"],
                             "lanczos": ic["lanczos_iters"], "rho_hat": rc}
        log(f"bf16: ttc {statistics.fmean(tb16):.3f} s certified={ic['certified']} r={ic['r']} "
            f"cost={ic['cost']:.10e}")
        del P
    if not args.no_box and args.workload == "large":
        # the other reading of the outlier model: the outlier's 3D point uniform in
        # the scene's bounding box (cameras +-3); capped, reported whether or not it certifies
        t = time.perf_counter()
        sb = scenes.make_scene("large", args.seed, outlier_model="box")
        log(f"box-outlier scene ({time.perf_counter() - t:.1f} s)")
        P = xm.build_Q(sb.N, sb.M, torch.from_numpy(sb.frame).to(dev), torch.from_numpy(sb.landmark).to(dev),
                       torch.from_numpy(sb.u).to(dev), torch.from_numpy(sb.w).to(dev), keep=("f32",))
        cap = 300
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Yb, ib = P.solve(xm.SolveOptions(compute="f32", max_outer=cap))
        Rb, sb_, rb = P.round(Yb)
        torch.cuda.synchronize()
        tbox = time.perf_counter() - t0
        out["box_outlier_variant"] = {
            "workload": "as above with the outlier's 3D point uniform in the bounding box of the cameras +-3",
            "max_outer_per_rank": cap, "ttc_s": round(tbox, 3), "certified": bool(ib["certified"]),
            "status": "ENOCONV (cap reached)" if ib["status"] != 0 else "ok",
            "rank": ib["r"], "cost": ib["cost"], "rho_hat": rb,
            "eta": (rb - ib["cost"]) / (1 + abs(rb) + abs(ib["cost"])), "lambda_min": ib["lambda_min"],
            "outer": ib["outer_iters"], "inner": ib["inner_iters"],
            "median_scale": float(sb_.median().item())}
        log(f"box variant: {out['box_outlier_variant']}")
        del P
    if not args.no_xm2 and args.workload == "large":
        # XM^2 on the workload (Section "Structure from Motion with XM"): solve,
        # delete the 10% of observations with the largest residuals (frame
        # units), rebuild Q from the rest and solve again from the first solution
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o2 = xm.xm2(sc.N, sc.M, fr, lm, u, w, opts=opts32, frac=0.1, frame_units=True)
        torch.cuda.synchronize()
        txm2 = time.perf_counter() - t0
        R1, s1, rho1, i1 = o2["first"]
        R2, s2, rho2, i2 = o2["second"]
        # the certificate's parts at the second optimum: the smallest eigenvalue
        # of the scaled dual off rows(Y), the deflated block and their coupling
        c2 = o2["problem"].certify(o2["Y"][: i2["r"]])
        kept = o2["keep"].cpu().numpy().astype(bool)
        bad = sc.gt["outlier"]
        out["xm2_variant"] = {
            "workload": "as the timed workload, then XM^2: the 10% largest residuals |e_o|/s_i deleted, re-solved",
            "wall_s": round(txm2, 3), "dropped": o2["n_dropped"], "restored": o2["n_restored"],
            "injected_outliers_deleted": round(float((bad & ~kept).sum() / max(1, bad.sum())), 4),
            "first": {"certified": bool(i1["certified"]), "rank": i1["r"], "cost": i1["cost"], "rho_hat": rho1,
                      "eta": (rho1 - i1["cost"]) / (1 + abs(rho1) + abs(i1["cost"]))},
            "second": {"certified": bool(i2["certified"]), "rank": i2["r"], "cost": i2["cost"], "rho_hat": rho2,
                       "eta": (rho2 - i2["cost"]) / (1 + abs(rho2) + abs(i2["cost"])),
                       "outer": i2["outer_iters"], "inner": i2["inner_iters"],
                       "lambda_bound": c2["lambda_bound"], "lambda_complement_scaled": c2["lambda_min"],
                       "deflated_block_min_scaled": c2["defl_min"], "coupling_scaled": c2["defl_cross"]}}
        log(f"xm2 variant: {out['xm2_variant']}")
        del o2
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        ref = i64 if not args.no_compare else last
        products = 2 * ref["inner_iters"] + 2 * ref["outer_iters"] + ref["lanczos_iters"]
        out["cpu_baseline"] = cpu_baseline(sc, products)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
