"""One solve of the box-mesh problem from the command line.

Assembles the N^3 heat-conduction mesh (u = 1 on x = 1, 0 on the other
faces) and solves it to tol from x0 = 0 with the chosen method: FP64 CG,
its single-reduction or Jacobi-preconditioned variant, or the FP32-inner /
FP64-refinement CG (restarting its inner solves, or keeping their
direction).  The solve runs once untimed (graph capture) and once timed;
prints one JSON line with the statistics and the error against the series
solution at nodes with x <= 3/4.
"""
import argparse
import json
import time

import torch

from .mfe import Context, Problem


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256, help="elements per axis")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--fmt", default="bcrs13", choices=["bcrs13", "csr"])
    ap.add_argument("--method", default="cg",
                    choices=["cg", "single_reduction", "jacobi", "mixed", "mixed_keep"])
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="inner tolerance of the mixed solves (default 1e-4 restarting, 1e-2 keeping the direction)")
    args = ap.parse_args(argv)
    ctx = Context(0)
    n = args.n
    mixed = args.method.startswith("mixed")
    P = Problem.mesh(ctx, n, n, n, formats=(args.fmt,), precisions=("f64", "f32") if mixed else ("f64",))
    x = torch.zeros(P.m, dtype=torch.float64, device=ctx.device)
    if mixed:
        keep = args.method == "mixed_keep"
        itol = args.inner_tol if args.inner_tol is not None else (1e-2 if keep else 1e-4)
        run = lambda: P.cg_mixed(x, tol=args.tol, inner_tol=itol, fmt=args.fmt, keep_direction=keep)[1]
    else:
        run = lambda: P.cg(x, tol=args.tol, max_iter=100000, fmt=args.fmt, variant=args.method)[1]
    for _ in range(2):
        with torch.cuda.stream(ctx.stream):
            x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
    out = dict(n=n, rows=P.m, method=args.method, format=args.fmt, tol=args.tol, wall_seconds=dt, stats=st)
    out["series_error"] = P.verify_series(x, x_max=0.75)
    P.close()
    print(json.dumps(out, default=float), flush=True)


if __name__ == "__main__":
    main()
