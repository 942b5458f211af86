"""Error of the GPU solves against the FP64 oracle at full size (test
infrastructure: run by hand on a GPU machine, not collected by pytest).

    python tests/mixed_error_report.py --size 256 --out report.md
    python tests/mixed_error_report.py --size 256 --reference-out xref.npy   # oracle only (CPU)
    python tests/mixed_error_report.py --size 256 --reference xref.npy --out report.md

The 256^3 scene (60 solid spheres r 8-40, 3 slabs, sinusoidal free surface of
amplitude 16, seed 1; N(0,1) right-hand side on fluid, seed 2) or the 128^3
benchmark scene is solved on the GPU in every precision to each tolerance;
the oracle then solves the same system to a 1e-12 relative residual (x_ref).
Reported per GPU result: iterations, solve time, the FP64 true relative
residual by the oracle's matvec and ||x - x_ref|| / ||x_ref||.  The paper
reports that a single-precision network does not limit the accuracy of the
double-precision iteration (Sec. "Results and Analysis"); here the network is
bf16 / fp16 and the Krylov vectors float.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import nps_inputs as gi  # noqa: E402
from oracle import laplacian as lap  # noqa: E402
from oracle import network as onet  # noqa: E402
from oracle import npsdo as onpsdo  # noqa: E402


def oracle_reference(lab, b, params):
    """x_ref: the oracle's NPSDO (FP64, CPU) to a 1e-12 relative residual."""
    print("oracle: setup", flush=True)
    t0 = time.perf_counter()
    P = onet.Network(params, 6, lab)
    count = [0]

    def precond(r):
        count[0] += 1
        if count[0] % 10 == 0:
            print(f"oracle iteration {count[0]} ({time.perf_counter() - t0:.0f} s)", flush=True)
        return P.apply(r)

    ref = onpsdo.solve(lab, b, precond, tol=1e-12, max_iter=5000)
    return ref, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=256, choices=[128, 256])
    ap.add_argument("--tols", type=float, nargs="+", default=[1e-6, 1e-8])
    ap.add_argument("--precisions", nargs="+", default=["mixed_bf16", "mixed_fp16", "fp32", "fp64"])
    ap.add_argument("--out")
    ap.add_argument("--reference-out", help="oracle only: write x_ref (fluid cells, float64 .npy) and exit")
    ap.add_argument("--reference", help="x_ref written by --reference-out instead of solving here")
    args = ap.parse_args()
    spec = gi.scene_c3() if args.size == 256 else gi.scene_c2()
    lab = gi.gen_labels(spec, seed=1)
    b = gi.gen_rhs(lab, seed=2)
    params = gi.multilevel_params(6)
    fluid = lab == gi.FLUID
    nf = int(fluid.sum())
    print(f"{args.size}^3: {nf} fluid cells", flush=True)
    if args.reference_out:
        ref, t_ref = oracle_reference(lab, b, params)
        np.save(args.reference_out, ref.x[fluid])
        meta = {"iterations": ref.iterations, "rel_residual": ref.rel_residual, "seconds": t_ref}
        with open(args.reference_out + ".json", "w") as f:
            json.dump(meta, f)
        print(f"oracle x_ref: {meta}", flush=True)
        return
    import torch

    import paper_2310_00177_amd as nps
    PREC = {"mixed_bf16": nps.MIXED_BF16, "mixed_fp16": nps.MIXED_FP16, "fp32": nps.FP32, "fp64": nps.FP64}
    net = nps.Net(params, 6)
    labd, bd = torch.from_numpy(lab).cuda(), torch.from_numpy(b).cuda()
    rows = []
    for prec in args.precisions:
        for tol in args.tols:
            nps.solve(net, labd, bd, tol=tol, max_iter=3000, precision=PREC[prec])   # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = nps.solve(net, labd, bd, tol=tol, max_iter=3000, precision=PREC[prec])
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            xs = x.cpu().numpy()
            true_rel = lap.rel_residual(lab, b, xs)
            rows.append(dict(prec=prec, tol=tol, its=info.iterations, status=info.status, ms=ms,
                             reported=info.rel_residual, true_rel=true_rel, x=xs))
            print(f"gpu {prec} tol {tol:.0e}: {info.iterations} its, {ms:.1f} ms, status {info.status}, "
                  f"true rel residual {true_rel:.3e}", flush=True)
    del x
    if args.reference:
        xref = np.zeros(lab.shape)
        xref[fluid] = np.load(args.reference)
        meta = json.load(open(args.reference + ".json"))
        ref_its, ref_res, t_ref = meta["iterations"], meta["rel_residual"], meta["seconds"]
    else:
        ref, t_ref = oracle_reference(lab, b, params)
        xref, ref_its, ref_res = ref.x, ref.iterations, ref.rel_residual
    nref = np.linalg.norm(xref)
    print(f"oracle x_ref: {ref_its} its, rel residual {ref_res:.3e}, {t_ref:.0f} s", flush=True)
    with open(args.out, "w") as f:
        f.write(f"# Solution error vs the FP64 oracle, {args.size}^3\n\n")
        f.write(f"Command: `python tests/mixed_error_report.py --size {args.size} --out <file>` "
                f"(tolerances {args.tols}).\n\n")
        f.write(f"Scene: {'scene_c3()' if args.size == 256 else 'scene_c2()'} seed 1 ({nf} fluid cells), "
                "gen_rhs seed 2, multilevel weights, L = 6, n_ortho = 2, x0 = 0.\n")
        f.write(f"x_ref: oracle NPSDO (FP64, CPU) to a {ref_res:.2e} relative residual in "
                f"{ref_its} iterations ({t_ref:.0f} s{', computed separately with --reference-out' if args.reference else ''}).\n\n")
        f.write("| precision | tol | iterations | ms/solve | FP64 true rel. residual (oracle matvec) "
                "| ‖x − x_ref‖/‖x_ref‖ |\n|---|---|---:|---:|---:|---:|\n")
        for r in rows:
            err = float(np.linalg.norm(r["x"] - xref) / nref)
            f.write(f"| {r['prec']} | {r['tol']:.0e} | {r['its']} | {r['ms']:.1f} | {r['true_rel']:.3e} "
                    f"| {err:.3e} |\n")
            print(f"{r['prec']} tol {r['tol']:.0e}: error vs x_ref {err:.3e}", flush=True)
    print(open(args.out).read(), flush=True)


if __name__ == "__main__":
    main()
