"""Learned initial guess for CG: data generation with the plain method,
training of the encoder-decoder on the GPU, and evaluation against the zero
start.  Every arithmetic step runs in libmfe's kernels (CG, network forward,
backward and Adam); this module only moves data and schedules steps.

    python -m paper_1505_08023_amd.learned --n 64 --train 20000 --epochs 4 \\
        --eval 1000 --out weights.npz

Boundary data: per face, c + sum_{k<8} a_k sin(p_k pi s) sin(q_k pi t) (see
inputs.smooth_faces), seeds 0..train-1 for training, 10^6.. for evaluation.
Targets: FP64 CG solutions to 1e-8 of the Nx = Ny = Nz = n mesh.
"""
import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import inputs
from .mfe import Batch, Context, Net, Problem

HELD_OUT_BASE = 10 ** 6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def layer_shapes():
    """(cin, cout) per layer, in the order of include/mfe.h."""
    return [(8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (128, 64), (64, 64),
            (64, 32), (32, 32), (32, 16), (16, 8)]


def he_init(seed=0):
    """Flat FP32 parameters (natural layout W[o][27][c], b[o] per layer)."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in layer_shapes():
        parts.append(rng.standard_normal(cout * 27 * cin) * math.sqrt(2.0 / (27 * cin)))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def fields(n, seeds):
    """Boundary fields of several seeds, concatenated (host FP64)."""
    return np.concatenate([inputs.node_field(n, n, n, inputs.smooth_faces(int(s))) for s in seeds])


def generate(ctx, n, seeds, chunk=32, tol=1e-8):
    """Solve the plain problem for every seed (chunk systems at a time with the
    batched CG).  Returns (g, u): FP64 CUDA tensors [len(seeds), (n+1)^3]."""
    V = (n + 1) ** 3
    S = len(seeds)
    g_all = torch.empty((S, V), dtype=torch.float64, device=ctx.device)
    u_all = torch.empty((S, V), dtype=torch.float64, device=ctx.device)
    B = Batch(ctx, np.full((chunk, 3), n), formats=("bcrs13",))
    B.autotune("bcrs13")
    x = torch.zeros(B.m, dtype=torch.float64, device=ctx.device)
    t0 = time.time()
    its = []
    for c0 in range(0, S, chunk):
        ids = seeds[c0:c0 + chunk]
        k = len(ids)
        g = np.zeros(chunk * V)
        g[:k * V] = fields(n, ids)
        gt = torch.tensor(g, device=ctx.device)
        B.set_bc(node_g=gt)
        x.zero_()
        x, st = B.cg(x, tol=tol, max_iter=20000)
        if any(s["status"] != 0 for s in st[:k]):
            raise RuntimeError("CG did not converge while generating data")
        its += [s["iterations"] for s in st[:k]]
        g_all[c0:c0 + k] = gt[:k * V].view(k, V)
        u_all[c0:c0 + k] = x[:k * V].view(k, V)
        if (c0 // chunk) % 50 == 0:
            log(f"[learned] generated {c0 + k}/{S} solutions ({time.time() - t0:.0f} s, mean its {np.mean(its):.1f})")
    B.close()
    return g_all, u_all


def train(net, g, u, epochs, batch, lr, seed=0, log_every=60.0, energy=None):
    """Adam with cosine decay over the fields (g, u).  energy: None for the
    mean squared error of the interior prediction, or the mesh's Problem for
    the energy norm e^T A e of the interior error (the norm CG minimises)."""
    S = g.shape[0]
    rng = np.random.default_rng(seed)
    steps_per_epoch = S // batch
    total = epochs * steps_per_epoch
    step, t0, last = 0, time.time(), time.time()
    history = []
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(S), device=g.device)
        run = 0.0
        for i in range(steps_per_epoch):
            idx = perm[i * batch:(i + 1) * batch]
            gb = g.index_select(0, idx).reshape(-1)
            ub = u.index_select(0, idx).reshape(-1)
            loss = net.loss_grad(gb, ub, energy=energy)
            cur = lr * 0.5 * (1 + math.cos(math.pi * step / total))  # cosine decay
            net.adam_step(cur)
            run += loss
            step += 1
            if time.time() - last > log_every:
                last = time.time()
                log(f"[learned] epoch {ep} step {i}/{steps_per_epoch} loss {loss:.3e} ({time.time() - t0:.0f} s)")
        history.append(run / steps_per_epoch)
        log(f"[learned] epoch {ep} mean loss {history[-1]:.3e}")
    return history


def boundary_mask(n):
    """Boolean mask over the (n+1)^3 nodes of an n^3 mesh (node id
    ix + (n+1)(iy + (n+1) iz), x fastest) of the nodes on the six faces,
    where the Dirichlet values sit (Sec. 1)."""
    i = np.arange(n + 1)
    face = (i == 0) | (i == n)
    return (face[None, None, :] | face[None, :, None] | face[:, None, None]).reshape(-1)


def evaluate(ctx, net, n, seeds, tol=1e-8, mixed=True, inner_tol=1e-4, keep_direction=False, errors=True):
    """Per held-out seed: plain FP64 CG from x0 = 0 against CG from the
    network's guess (inference included in its time; the solver falls back to
    the zero start when the guess's residual is not below ||b||), and, with
    mixed, the FP32-inner / FP64-refinement solve from zero and from the guess
    (the learned + mixed-precision form; inner_tol and keep_direction as in
    Problem.cg_mixed), and, for context, plain FP64 CG from the trivial guess
    that holds g on the boundary and 0 inside.  All solves stop at the same
    tolerance on ||b - A x|| / ||b||.  Every variant runs once on the first
    seed before timing (graph capture).  Times are host wall clock,
    GPU-synchronised.  With errors, every solution's ||x - x_ref|| / ||x_ref||
    against FP64 CG to tol / 100 (outside the timed regions)."""
    V = (n + 1) ** 3
    P = Problem.mesh(ctx, n, n, n, formats=("bcrs13",), precisions=("f64", "f32") if mixed else ("f64",))
    x = torch.zeros(V, dtype=torch.float64, device=ctx.device)
    x0 = torch.zeros(V, dtype=torch.float64, device=ctx.device)
    xr = torch.zeros(V, dtype=torch.float64, device=ctx.device)
    # the trivial guess keeps g on the boundary nodes and 0 inside (r = 0 on
    # the Dirichlet rows, as the network's guess, whose boundary values are
    # exact, also has)
    on_b = torch.tensor(boundary_mask(n), device=ctx.device)

    def err(v):
        return float(torch.linalg.norm(v - xr) / torch.linalg.norm(xr))

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, st

    def one(s):
        g = torch.tensor(inputs.node_field(n, n, n, inputs.smooth_faces(int(s))), device=ctx.device)
        P.set_bc(node_g=g)
        r = dict(seed=int(s))
        x.zero_()
        if errors:
            xr.zero_()
            P.cg(xr, tol=tol / 100, max_iter=20000)
        r["t_plain"], st0 = timed(lambda: P.cg(x, tol=tol, max_iter=20000)[1])
        if errors:
            r["err_plain"] = err(x)

        def learned_fp64():
            net.predict_x0(g, x0)
            return P.cg(x0, tol=tol, max_iter=20000, warm=True)[1]
        r["t_learned"], st1 = timed(learned_fp64)
        if errors:
            r["err_learned"] = err(x0)

        def boundary_fp64():
            torch.where(on_b, g, torch.zeros_like(g), out=x)
            return P.cg(x, tol=tol, max_iter=20000)[1]
        r["t_boundary"], stb = timed(boundary_fp64)
        r.update(its_plain=st0["iterations"], its_learned=st1["iterations"], used=not st1["guess_rejected"],
                 res_plain=st0["rel_res_true"], res_learned=st1["rel_res_true"], its_boundary=stb["iterations"])
        if mixed:
            x.zero_()
            r["t_mixed"], st2 = timed(lambda: P.cg_mixed(x, tol=tol, inner_tol=inner_tol,
                                                         keep_direction=keep_direction)[1])
            if errors:
                r["err_mixed"] = err(x)

            def learned_mixed():
                net.predict_x0(g, x0)
                return P.cg_mixed(x0, tol=tol, inner_tol=inner_tol, warm=True, keep_direction=keep_direction)[1]
            r["t_learned_mixed"], st3 = timed(learned_mixed)
            if errors:
                r["err_learned_mixed"] = err(x0)
            r.update(its_mixed=st2["iterations"], its_learned_mixed=st3["iterations"],
                     res_mixed=st2["rel_res_true"], res_learned_mixed=st3["rel_res_true"],
                     used_mixed=not st3["guess_rejected"])
        # the guess's own residual, outside the timed region
        net.predict_x0(g, x0)
        _, chk = P.cg(x0, tol=tol, max_iter=0)
        r["guess_rel_res"] = chk["rel_res_true"]
        return r

    one(seeds[0])  # warm-up
    rows = [one(s) for s in seeds]
    P.close()
    a = lambda k: float(np.mean([r[k] for r in rows]))
    out = dict(samples=len(rows), mean_its_plain=a("its_plain"), mean_its_learned=a("its_learned"),
               mean_time_plain_s=a("t_plain"), mean_time_learned_s=a("t_learned"),
               mean_guess_rel_res=a("guess_rel_res"), guesses_used=int(sum(r["used"] for r in rows)),
               worst_res_learned=max(r["res_learned"] for r in rows),
               speedup_time=a("t_plain") / a("t_learned"),
               # context: the trivial guess (g on the boundary, 0 inside)
               mean_its_boundary_start=a("its_boundary"), mean_time_boundary_start_s=a("t_boundary"),
               speedup_time_vs_boundary_start=a("t_boundary") / a("t_learned"))
    if mixed:
        out.update(mean_its_mixed=a("its_mixed"), mean_its_learned_mixed=a("its_learned_mixed"),
                   mean_time_mixed_s=a("t_mixed"), mean_time_learned_mixed_s=a("t_learned_mixed"),
                   worst_res_learned_mixed=max(r["res_learned_mixed"] for r in rows),
                   guesses_used_mixed=int(sum(r["used_mixed"] for r in rows)),
                   speedup_time_mixed=a("t_plain") / a("t_mixed"),
                   speedup_time_learned_mixed=a("t_plain") / a("t_learned_mixed"))
    if errors:
        out["error_vs_fp64_ref"] = {
            "reference": f"FP64 CG to {tol / 100:g}",
            **{f"{k}_mean": a(f"err_{k}") for k in (("plain", "learned", "mixed", "learned_mixed") if mixed
                                                     else ("plain", "learned"))},
            **{f"{k}_max": max(r[f"err_{k}"] for r in rows) for k in (("plain", "learned", "mixed", "learned_mixed")
                                                                       if mixed else ("plain", "learned"))}}
    out["rows"] = rows
    return out


def save(path, params, meta):
    np.savez_compressed(path, params=params, meta=json.dumps(meta))


def load(path):
    with np.load(path, allow_pickle=False) as f:
        return f["params"].astype(np.float32), json.loads(str(f["meta"]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64, help="elements per axis")
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval", type=int, default=1000)
    ap.add_argument("--init", default=None, help="start from these weights (.npz)")
    ap.add_argument("--loss", choices=("mse", "energy"), default="mse",
                    help="training loss: squared error or energy norm of the interior error")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    ctx = Context(0)
    n = args.n
    net = Net(ctx, n + 1, args.batch)
    if args.init:
        p, _ = load(args.init)
        net.set_params(p)
    else:
        net.set_params(he_init(0))
    result = {"n": n}
    if args.train > 0:
        t = time.time()
        g, u = generate(ctx, n, np.arange(args.train))
        result["generate_s"] = time.time() - t
        t = time.time()
        prob = Problem.mesh(ctx, n, n, n, formats=("bcrs13",)) if args.loss == "energy" else None
        result["loss_history"] = train(net, g, u, args.epochs, args.batch, args.lr, energy=prob)
        if prob is not None:
            prob.close()
        result["train_s"] = time.time() - t
        del g, u
        torch.cuda.empty_cache()
        if args.out:
            save(args.out, net.get_params(), dict(n=n, train=args.train, epochs=args.epochs, batch=args.batch,
                                                  lr=args.lr, init=args.init or "he_init(0)", loss=args.loss,
                                                  loss_history=result["loss_history"]))
    if args.eval > 0:
        ev = evaluate(ctx, net, n, np.arange(HELD_OUT_BASE, HELD_OUT_BASE + args.eval))
        ev.pop("rows")
        result["eval"] = ev
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
