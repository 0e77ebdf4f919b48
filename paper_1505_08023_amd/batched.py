"""Batched uneven solves from the command line.

nsys box meshes with Nx, Ny, Nz drawn uniformly from {lo..hi} and six face
values from U[0, 1) (seeded, inputs.batched_meshes), assembled into one
block-diagonal system and solved together to tol: FP64 CG, the FP32-inner /
FP64-refinement CG restarting its inner solves, and the same keeping each
system's inner direction.  Each solve runs once untimed (graph capture)
and once timed.  Prints one JSON line.
"""
import argparse
import json
import time

import torch

from . import inputs
from .mfe import Batch, Context


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nsys", type=int, default=64)
    ap.add_argument("--lo", type=int, default=16)
    ap.add_argument("--hi", type=int, default=96)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--fmt", default="bcrs13", choices=["bcrs13", "csr"])
    args = ap.parse_args(argv)
    ctx = Context(0)
    sizes, faces = inputs.batched_meshes(nsys=args.nsys, lo=args.lo, hi=args.hi, seed=args.seed)
    B = Batch(ctx, sizes, faces, precisions=("f64", "f32"))
    lanes, factor = B.autotune(args.fmt)
    x = torch.zeros(B.m, dtype=torch.float64, device=ctx.device)
    out = dict(systems=args.nsys, rows=B.m, nnz=B.nnz, tol=args.tol, format=args.fmt,
               autotune=dict(lanes_per_row=lanes, grid_factor=factor))
    runs = (("fp64", lambda: B.cg(x, tol=args.tol, fmt=args.fmt)[1]),
            ("mixed_restart", lambda: B.cg_mixed(x, tol=args.tol, fmt=args.fmt)[1]),
            ("mixed_keep_direction", lambda: B.cg_mixed(x, tol=args.tol, inner_tol=1e-4, fmt=args.fmt,
                                                        keep_direction=True)[1]))
    for name, fn in runs:
        for timed in (False, True):
            with torch.cuda.stream(ctx.stream):
                x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
        its = [s["iterations"] for s in st]
        out[name] = dict(seconds=dt, max_iterations=max(its), sum_iterations=sum(its),
                         worst_rel_res_true=max(s["rel_res_true"] for s in st),
                         all_converged=all(s["status"] == 0 for s in st))
    B.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
