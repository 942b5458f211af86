"""Benchmark: solves/sec to a 1e-6 relative residual on a 128^3 mixed-BC scene,
mixed precision vs FP32, with p50/p99 solve latency.

A step is one whole solve (Alg. 1 with the network of Alg. 2 as
preconditioner) of one synthetic 128^3 system whose labels, right-hand side
and weights are already resident in HBM.  The headline `value` is the mixed
path (bf16/fp16 network, fp32 Krylov vectors, fp64 refinement); the plain
FP32 path is timed on the same inputs and reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Also reports the roofline of the dominant kernel
(HIP-event durations recorded by the library on its launch stream, over a
profiled pass of the same solves) and the CPU oracle timed on a bounded
sample of the same workload.
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

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def measured_traffic(kernel: str, workload_ok: bool):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by its reading on a
    known-size kernel), or None when the kernel sources changed since the
    counters were taken or the workload is not the profiled one."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not workload_ok or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in sorted(glob.glob(os.path.join(ROOT, "paper_2310_00177_amd", "csrc", "*"))):
        with open(src, "rb") as f:
            h.update(f.read())
    k = rec["kernels"].get(kernel)
    if h.hexdigest() != rec["source_sha256"] or k is None:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=2000)
    ap.add_argument("--headline", default="mixed_bf16", choices=["mixed_bf16", "mixed_fp16", "fp32", "fp64"])
    ap.add_argument("--compare", default="fp32", help="second precision to time, or 'none'")
    ap.add_argument("--compare2", default="mixed_fp16", help="third precision to time, or 'none'")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with known-size fill and negate kernels (1 GiB each) for the HBM counters")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the solver-variant comparison")
    ap.add_argument("--cpu-iters", type=int, default=4, help="oracle iterations in the CPU sample")
    ap.add_argument("--train", action="store_true", help="training throughput (forward, loss, gradient) instead")
    ap.add_argument("--batch", type=int, default=16, help="systems per training step of --train")
    ap.add_argument("--rhs-gen", action="store_true", help="Ritz-vector right-hand-side generator instead")
    ap.add_argument("--ritz", type=int, default=1600, help="Lanczos steps of --rhs-gen")
    ap.add_argument("--rhs-count", type=int, default=800, help="right-hand sides of --rhs-gen")
    ap.add_argument("--reorth", action="store_true",
                    help="--rhs-gen with full reorthogonalisation (O(m^2 n) traffic: use a small --ritz)")
    ap.add_argument("--serving", action="store_true",
                    help="run the request-server sweep instead (Poisson arrivals, mixed grid sizes)")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--qps", type=float, nargs="+", default=[20.0, 50.0, 100.0, 200.0, 400.0])
    ap.add_argument("--slots", type=int, default=16)
    return ap.parse_args()


# Algorithmic HBM bytes per fine cell and iteration: the method's compulsory
# traffic with labels-only operator reads, per pass, with s = bytes per Krylov
# element and a = bytes per network activation (s = 8, a = 8 in FP64; s = 4,
# a = 4 in FP32; s = 4, a = 2 in the mixed modes):
#   net-down l1 (CConv_1^1 + pool)        r, labels -> x1, r2         s + 1 + 1.125 a
#   coarse levels 2..6, down + up         counts as 2 x u16           0.143 (4.25 a + 8)
#   net-up l1 + the beta dots             x2, labels, x1, Ad_(k-1), Ad_(k-2) -> dhat
#                                                                     3 s + 1.125 a + 1
#   ortho + matvec + the alpha dots       dhat, d_(k-1), d_(k-2), Ad_(k-1), Ad_(k-2), r,
#                                         labels -> d, Ad             8 s + 1
#   update                                x, d, r, Ad -> x, r         6 s
#   mixed modes: FP64 refinement          (8 + 8 + 1 + 4 + 4 + 8) / 20 ~ 1.7
# The library's kernels map onto these passes one to one (`residual` is the
# update, with the literal residual), except that the coarse levels run as
# several launches.
def alg_bytes_per_cell(kernel: str, s: int, a: int) -> float | None:
    table = {
        "net_down_l1": s + 1 + 1.125 * a,
        "net_up_l1": 3 * s + 1.125 * a + 1,
        "ortho_matvec": 8 * s + 1,
        "residual": 6 * s,
    }
    return table.get(kernel)


def iteration_bytes_per_fine_cell(s: int, a: int, mixed: bool) -> float:
    """All passes of one iteration (the sum above, ~83.5 B mixed, ~88 B FP32)."""
    return 18 * s + (1.125 + 1.125 + 0.143 * 4.25) * a + 3 + 0.143 * 8 + (1.7 if mixed else 0.0)


def cpu_baseline(labels, b, params, iters_sample):
    """The FP64 oracle on one host core: setup + `iters_sample` iterations,
    scaled to a whole solve with the oracle's own iteration count."""
    from threadpoolctl import threadpool_limits
    from oracle import network as onet
    from oracle import npsdo as onpsdo

    ref_path = os.path.join(ROOT, "tests", "golden", "oracle_workloads.json")
    ref = json.load(open(ref_path)).get(f"{labels.shape[0]}^3") if os.path.exists(ref_path) else None
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        net = onet.Network(params, 6, labels)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        res = onpsdo.solve(labels, b, net.apply, max_iter=iters_sample, fixed_iters=True)
        t_iter = (time.perf_counter() - t0) / max(res.iterations, 1)
    if ref is None:
        return None
    t_solve = t_setup + ref["iterations"] * t_iter
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup + {iters_sample} NPSDO iterations at {labels.shape[0]}^3 on 1 thread "
                      f"({t_setup:.1f} s + {t_iter:.2f} s/iteration), scaled to the oracle's own "
                      f"{ref['iterations']}-iteration solve of this workload"}


def _serving_request(i):
    """Request i of the serving workload: grid N ~ U{64, 96, 128, 160} (seed
    10000 + i), labels of the 128^3 recipe scaled by N/128 (seed 10000 + i),
    N(0,1) right-hand side on fluid (seed 20000 + i)."""
    import nps_inputs as gi
    n = [64, 96, 128, 160][int(np.random.default_rng(10000 + i).integers(0, 4))]
    lab = gi.gen_labels(gi.scene_serving(n), seed=10000 + i)
    return n, lab, gi.gen_rhs(lab, seed=20000 + i)


def serving_sweep(args):
    """Continuous-batching server: `requests` solves with Poisson arrivals at each
    QPS (seed 77), each request its own seeded grid drawn from {64,96,128,160}^3,
    tol 1e-6, mixed bf16; the offered rates run past the server's capacity,
    whose served rate is the headline.  Back-to-back single solves of the first
    64 requests, mixed bf16 and FP32, give the reference rates (solves/s and
    cell-iterations/s on the same grid mix)."""
    import multiprocessing as mp

    import torch

    import nps_inputs as gi
    import paper_2310_00177_amd as nps

    with mp.get_context("fork").Pool(8) as pool:
        reqs = pool.map(_serving_request, range(args.requests))
    print(f"# serving: {len(reqs)} requests ready", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    net = nps.Net(gi.multilevel_params(6), 6)
    # reference: back-to-back single solves (nps_solve) of the first 64 requests,
    # mixed bf16 and plain FP32
    ref = {}
    for name, prec in (("mixed_bf16", nps.MIXED_BF16), ("fp32", nps.FP32)):
        cells_its, t_ref, n_ok = 0.0, 0.0, 0
        for n, lab, b in reqs[:64]:
            labels_d, b_d = torch.from_numpy(lab).cuda(), torch.from_numpy(b).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = nps.solve(net, labels_d, b_d, tol=1e-6, precision=prec)
            t_ref += time.perf_counter() - t0
            cells_its += float(lab.size) * info.iterations
            n_ok += info.status == 0 and info.rel_residual < 1e-6
        ref[name] = {"solves_per_s": 64 / t_ref, "cell_iterations_per_s": cells_its / t_ref, "converged": n_ok}
        print(f"# single solves back to back, {name}: {64 / t_ref:.1f} solves/s, "
              f"{cells_its / t_ref / 1e9:.2f} G cell-iterations/s, {n_ok}/64 converged", file=sys.stderr, flush=True)
    ref_rate = ref["mixed_bf16"]["cell_iterations_per_s"]
    rng = np.random.default_rng(77)
    results = []
    for qps in args.qps:
        srv = nps.Server(net, hbm_budget=64 << 30, max_slots=args.slots)
        gaps = rng.exponential(1.0 / qps, size=args.requests)
        arrivals = np.cumsum(gaps) - gaps[0]
        for n, lab, b in reqs[:4]:   # warm-up
            rid = srv.submit(lab, b)
            while srv.poll(rid) is None:
                srv.step()
        lat, its, ok, inflight, peak, cells_its = [], [], 0, {}, 0, 0.0
        t0 = time.perf_counter()
        i = 0
        t_end = t0
        while len(lat) < args.requests:
            now = time.perf_counter() - t0
            while i < args.requests and arrivals[i] <= now:
                n, lab, b = reqs[i]
                inflight[srv.submit(lab, b)] = lab.size
                i += 1
            active, queued = srv.step()
            peak = max(peak, active)
            # admission is first in, first out, so every request on the device or
            # finished is among the oldest slots + a few in flight: polling those
            # keeps the host loop short when many requests wait
            for rid in list(inflight)[:2 * args.slots]:
                r = srv.poll(rid)
                if r is not None:
                    x, info, ms = r
                    lat.append(ms)
                    its.append(info.iterations)
                    cells_its += float(inflight[rid]) * info.iterations
                    ok += info.status == 0 and info.rel_residual < 1e-6
                    del inflight[rid]
                    t_end = time.perf_counter()
        wall = t_end - t0
        srv.close()
        lat = np.array(lat)
        row = {"qps": qps, "throughput": args.requests / wall,
               "cell_iterations_per_s": cells_its / wall, "vs_single_solves": cells_its / wall / ref_rate,
               "vs_fp32_single_solves": args.requests / wall / ref["fp32"]["solves_per_s"],
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "mean_iterations": float(np.mean(its)), "converged": int(ok), "peak_active": int(peak)}
        print(f"# serving qps {row['qps']}: {row}", file=sys.stderr, flush=True)
        results.append(row)
    sat = max(results, key=lambda r: r["throughput"])   # offered rates past capacity: the served rate
    out = {"metric": "served solves/sec to 1e-6 rel. residual, grids {64,96,128,160}^3; p50/p99 latency",
           "value": sat["throughput"], "unit": "solves/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "bf16+f32+f64", "data": "synthetic",
           "config": {"workload": f"{args.requests} requests per QPS, Poisson arrivals (seed 77), request i: grid "
                                  "N ~ U{64,96,128,160} and labels seed 10000+i, N(0,1) RHS seed 20000+i, tol 1e-6, "
                                  f"L=6, n_ortho=2, mixed bf16, {args.slots} slots", "weights": "multilevel",
                      "single_solves": ref},
           "sweep": results}
    print(json.dumps(out))


def train_bench(args):
    """Training step (Sec. "Training"; the batch of 16 systems at 128^3): the
    mean over the batch of ||b - A P(b)|| and its gradient with respect to
    every network parameter, through nps_train_step, in FP32 and in the bf16
    leg (kernels from bf16-rounded weights, weight-gradient contraction on
    bf16 matrix cores); the oracle's loss-and-gradient of one 32^3 system on
    one host thread for context."""
    import torch

    import nps_inputs as gi
    import paper_2310_00177_amd as nps

    torch.cuda.set_device(0)
    n, batch = args.size, args.batch
    spec = gi.scene_c1() if n == 32 else gi.scene_serving(n)
    labs = [gi.gen_labels(spec, seed=args.seed + i) for i in range(batch)]
    bs = [gi.gen_rhs(lab, seed=100 + i, normalize=True) for i, lab in enumerate(labs)]
    params = gi.multilevel_params(6)
    labels = torch.from_numpy(np.stack(labs)).cuda()
    b32 = torch.from_numpy(np.stack(bs)).float().cuda()
    net = nps.Net(params, 6)
    legs = {}
    for name, prec in (("fp32", nps.FP32), ("bf16", nps.MIXED_BF16)):
        ws = nps.train_workspace(labs[0].shape, 6, prec)
        grad = torch.zeros(gi.param_count(6), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            nps.train_step(net, labels, b32, grad, ws, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            loss = nps.train_step(net, labels, b32, grad, ws, precision=prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        legs[name] = {"steps_per_s": 1.0 / dt, "systems_per_s": batch / dt, "ms_per_step": dt * 1e3, "loss": loss}
        print(f"# train {name}: {dt * 1e3:.2f} ms per {batch}-system step, {batch / dt:.1f} systems/s, loss {loss:.4f}",
              file=sys.stderr, flush=True)
        del ws
    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import gradient as og
        lab32 = gi.gen_labels(gi.scene_c1(), seed=1)
        b32c = gi.gen_rhs(lab32, seed=2, normalize=True)
        with threadpool_limits(limits=1):
            c0 = time.perf_counter()
            og.loss_and_grad(params, 6, lab32, b32c)
            ct = time.perf_counter() - c0
        cpu = {"value": 1.0 / ct, "unit": "systems/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle loss + adjoint gradient of one 32^3 system on 1 thread ({ct:.2f} s); "
                         f"the GPU line is at {n}^3 ({(n / 32) ** 3:.0f}x the cells)"}
    head = legs["fp32"]
    out = {"metric": f"training steps/s (batch of {batch} systems at {n}^3: forward, loss, full parameter gradient)",
           "value": head["steps_per_s"], "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{batch} systems of the {n}^3 scene recipe (seeds {args.seed}..{args.seed + batch - 1}), "
                                  f"unit-norm N(0,1) right-hand sides, L=6, {gi.param_count(6)} parameters, "
                                  "stored kernels at every level", "systems_per_s": head["systems_per_s"],
                      "bf16_leg": legs["bf16"]},
           "cpu_baseline": cpu}
    print(json.dumps(out))


def rhs_gen_bench(args):
    """Training-data generator (Sec. "Training"): 1600 Lanczos steps with full
    reorthogonalisation on the 128^3 system matrix, then 800 normalised
    random combinations of the Ritz vectors (the paper's counts)."""
    import torch

    import nps_inputs as gi
    import paper_2310_00177_amd as nps

    torch.cuda.set_device(0)
    n = args.size
    lab = gi.gen_labels(gi.scene_c1() if n == 32 else gi.scene_serving(n), seed=args.seed)
    m, k = args.ritz, args.rhs_count
    rng = np.random.default_rng(5)
    labels = torch.from_numpy(lab).cuda()
    v0 = torch.from_numpy(rng.standard_normal(lab.shape)).cuda()
    coef = torch.from_numpy(rng.standard_normal((m, k))).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V, alpha, beta, steps = nps.lanczos(labels, v0, m, reorth=args.reorth)
    t1 = time.perf_counter()
    rhs, theta = nps.ritz_rhs(V[:steps], alpha[:steps].contiguous(), beta[:steps].contiguous(), coef[:steps])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fl = int((lab == gi.FLUID).sum())
    print(f"# rhs-gen: lanczos {m} steps {t1 - t0:.2f} s, ritz + {k} combinations {t2 - t1:.2f} s, "
          f"theta [{theta[0].item():.4g}, {theta[-1].item():.4g}]", file=sys.stderr, flush=True)
    out = {"metric": f"training right-hand sides/s ({m} Ritz vectors -> {k} normalised combinations) at {n}^3",
           "value": k / (t2 - t0), "unit": "rhs/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": (t2 - t0) * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{n}^3 scene ({fl} fluid cells), Lanczos from N(0,1), "
                                  f"{'full reorthogonalisation' if args.reorth else 'three-term recurrence'}, "
                                  f"N(0,1) coefficients", "lanczos_s": t1 - t0,
                      "ritz_s": t2 - t1, "steps": steps, "basis_GB": m * lab.size * 8 / 1e9},
           "cpu_baseline": None}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1 and (args.serving or args.train or args.rhs_gen):
        print("bench.py measures one GPU only", file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving_sweep(args)
        return
    if args.train:
        train_bench(args)
        return
    if args.rhs_gen:
        rhs_gen_bench(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this solver runs a single solve per GPU and the build has "
              f"no multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch

    import nps_inputs as gi
    import paper_2310_00177_amd as nps
    from paper_2310_00177_amd import _lib

    prec_of = {"mixed_bf16": nps.MIXED_BF16, "mixed_fp16": nps.MIXED_FP16, "fp32": nps.FP32, "fp64": nps.FP64}
    torch.cuda.set_device(0)
    n = args.size
    spec = gi.scene_c1() if n == 32 else gi.scene_serving(n)
    lab = gi.gen_labels(spec, seed=args.seed)
    b = gi.gen_rhs(lab, seed=args.seed + 1)
    params = gi.multilevel_params(6)
    labels_d = torch.from_numpy(lab).cuda()
    b_d = torch.from_numpy(b).cuda()
    net = nps.Net(params, 6)
    print(f"# workload {n}^3, fluid {int((lab == 0).sum())} cells", file=sys.stderr, flush=True)

    def run(name, steps, warmup, method=0, n_ortho=2, label=None):
        prec = prec_of[name]
        ws = nps.workspace(lab.shape, 6, prec, n_ortho)
        x = torch.empty_like(b_d)
        kw = dict(tol=args.tol, max_iter=args.max_iter, precision=prec, x=x, ws=ws, method=method, n_ortho=n_ortho)
        for _ in range(warmup):
            nps.solve(net, labels_d, b_d, **kw)
        torch.cuda.synchronize()
        lat = []
        infos = []
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            _, info = nps.solve(net, labels_d, b_d, **kw)
            lat.append(time.perf_counter() - s0)   # nps_solve synchronises its stream
            infos.append(info)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        lat_ms = np.array(lat) * 1e3
        its = [i.iterations for i in infos]
        ok = all(i.status == 0 and i.rel_residual < args.tol for i in infos)
        print(f"# {label or name}: {steps / total:.2f} solves/s, {total / steps * 1e3:.2f} ms/solve, iterations {its[0]}, "
              f"true rel residual {infos[-1].rel_residual:.2e}, converged {ok}", file=sys.stderr, flush=True)
        return {"solves_per_s": steps / total, "ms_per_solve": total / steps * 1e3,
                "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                "iterations": int(np.median(its)), "rel_residual_true": max(i.rel_residual for i in infos),
                "converged": ok, "refinements": infos[-1].refinements,
                "t_setup_us": float(np.median([i.t_setup_ms for i in infos])) * 1e3,
                "t_iter_us": float(np.median([i.t_iter_ms for i in infos])) * 1e3}, ws, x

    head, ws_h, x_h = run(args.headline, args.steps, args.warmup)
    comp = None
    if args.compare and args.compare not in ("none", args.headline):
        comp, _, _ = run(args.compare, args.steps, args.warmup)
    comp2 = None
    if args.compare2 and args.compare2 not in ("none", args.headline, args.compare):
        comp2, _, _ = run(args.compare2, args.steps, args.warmup)

    # solver variants on the same system (the paper's PCG-variant and n_ortho
    # comparisons): NPSDO with n_ortho 0..4 (0 = steepest descent), PCG, flexible PCG
    variants = []
    if not args.no_variants:
        vsteps = max(2, min(args.steps, 3))
        for method, n_ortho, tag in [(0, 0, "psd"), (0, 1, "npsdo1"), (0, 2, "npsdo2"), (0, 3, "npsdo3"),
                                     (0, 4, "npsdo4"), (1, 1, "pcg"), (2, 1, "fpcg")]:
            r, _, _ = run(args.headline, vsteps, 1, method=method, n_ortho=n_ortho, label=f"variant {tag}")
            variants.append({"variant": tag, "method": ["npsdo", "pcg", "fpcg"][method], "n_ortho": n_ortho,
                             "solves_per_s": r["solves_per_s"], "iterations": r["iterations"],
                             "converged": r["converged"]})

    # profiled pass: per-kernel durations from HIP events on the launch stream
    prec = prec_of[args.headline]
    s_bytes = 8 if prec == nps.FP64 else 4
    a_bytes = {nps.FP64: 8, nps.FP32: 4}.get(prec, 2)
    _lib.nps_profile_enable(1)
    prof_solves = max(2, min(args.steps, 5))
    for _ in range(prof_solves):
        nps.solve(net, labels_d, b_d, tol=args.tol, max_iter=args.max_iter, precision=prec, x=x_h, ws=ws_h)
    rc, stats = _lib.nps_profile_read(64)
    _lib.nps_profile_enable(0)
    kstats = {s.name.decode(): (s.launches, s.total_ms, s.cells) for s in stats}
    dom = max((k for k in kstats if alg_bytes_per_cell(k, s_bytes, a_bytes) is not None), key=lambda k: kstats[k][1])
    launches, total_ms, cells = kstats[dom]
    avg_s = total_ms / launches * 1e-3
    bytes_per_launch = alg_bytes_per_cell(dom, s_bytes, a_bytes) * cells / launches
    achieved = bytes_per_launch / avg_s / 1e9
    it_bytes = iteration_bytes_per_fine_cell(s_bytes, a_bytes, prec in (nps.MIXED_BF16, nps.MIXED_FP16)) * lab.size
    kernels = {k: {"launches": v[0], "avg_us": v[1] / v[0] * 1e3, "share": v[1] / sum(w[1] for w in kstats.values())}
               for k, v in kstats.items()}
    print("# kernels: " + ", ".join(f"{k} {v['avg_us']:.1f}us x{v['launches']} ({v['share'] * 100:.1f}%)"
                                    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["share"])),
          file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(lab, b, params, args.cpu_iters)

    dtype = {"mixed_bf16": "bf16+f32+f64", "mixed_fp16": "f16+f32+f64", "fp32": "f32", "fp64": "f64"}[args.headline]
    out = {
        "metric": "solves/sec to 1e-6 rel. residual at 128^3, mixed vs FP32; p50/p99 latency",
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": f"{n}^3 mixed-BC voxel scene (20 solid spheres r 4-20, 3 slabs, solid walls, flat free "
                        f"surface drawn in [64,112]), N(0,1) RHS on fluid, tol {args.tol:g}, L=6, n_ortho=2",
            "precision": args.headline,
            "weights": "multilevel (hand-set blob in the paper's architecture; seeded Xavier weights do not "
                       "precondition: the iteration stalls)",
            "iterations": head["iterations"],
            "rel_residual_true": head["rel_residual_true"],
            "converged": head["converged"],
        },
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "compare": None if comp is None else {
            "precision": args.compare, "value": comp["solves_per_s"], "p50_ms": comp["p50_ms"],
            "p99_ms": comp["p99_ms"], "iterations": comp["iterations"],
            "rel_residual_true": comp["rel_residual_true"], "converged": comp["converged"],
            "speedup_headline_vs_compare": head["solves_per_s"] / comp["solves_per_s"]},
        "compare2": None if comp2 is None else {
            "precision": args.compare2, "value": comp2["solves_per_s"], "p50_ms": comp2["p50_ms"],
            "p99_ms": comp2["p99_ms"], "iterations": comp2["iterations"],
            "rel_residual_true": comp2["rel_residual_true"], "converged": comp2["converged"]},
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom, n == 128 and args.seed == 1 and args.headline == "mixed_bf16"),
            "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_s * 1e6,
            # the timed solves' own per-iteration time (stream events around the
            # iteration loop, no per-launch events)
            "iteration": {"alg_bytes": it_bytes, "us": head["t_iter_us"],
                          "achieved_GBs": it_bytes / (head["t_iter_us"] * 1e-6) / 1e9,
                          "frac": it_bytes / (head["t_iter_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                          "setup_us": head["t_setup_us"]},
        },
        "variants": variants,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    if args.calibrate_copy:
        # A known-size kernel for the HBM counters: fill src (1 GiB), write
        # another 1 GiB so src is evicted from the L2s and the 256 MB
        # Infinity Cache, then negate src into dst (1 GiB read, 1 GiB written).
        n = 256 << 20
        src = torch.full((n,), 1.0, dtype=torch.float32, device="cuda")
        flush = torch.zeros(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del flush
        print(f"# calibration: fill 2 x {4 * n} bytes written; neg {4 * n} bytes read, {4 * n} bytes written",
              file=sys.stderr)

if __name__ == "__main__":
    main()
