#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X: plain FP64 CG on the 256^3 MiniFE
heat-conduction mesh (unit cube, u = 1 on x = 1, 0 on the other faces, zero
source, x0 = 0) to ||r||/||b|| <= 1e-8 with the 1x3 BCRS SpMV.

One step = one complete CG solve (every iteration: fused SpMV + p.q, r update
+ r.r, x/p update, all scalars on the device).  value = CG iterations per
second over the K timed solves.  Printed as one JSON line, with
  roofline      the fused SpMV + dot kernel (the dominant kernel of the
                loop), its algorithmic bytes per launch over its mean
                launch duration measured with HIP events on its stream;
  cpu_baseline  the CPU oracle's CG on the same matrix, a bounded sample of
                iterations on one host core.
Progress goes to stderr.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# HBM bytes per launch of the fused SpMV + dot kernels from FETCH_SIZE (x 2.0)
# and WRITE_SIZE (x 1.0) counter runs, scaled by streaming kernels of known
# size; taken from the profile named beside each, not in this run.  Reset to
# None whenever the kernel changes.
MEASURED_TRAFFIC = {("bcrs13", 256): (4.305e9, "profiles/spmv_b13_fp64_256cubed_hbm_counters.md"),
                    ("csr", 256): (4.292e9, "profiles/spmv_b13_fp64_256cubed_hbm_counters.md")}
# The paper's own gains of the BCRS format over CRS on its CPU server (it
# prints no absolute numbers): context, not a target.
PAPER_CONTEXT = ("Wu et al. report no absolute times; BCRS over CRS on their CPU server: SpMV +10.42 %, CG "
                 "+10.56 %, whole program +8.31 % on average (best +16.30 %, worst +1.50 %)")
METRIC = "SpMV GB/s & %HBM peak, CG iter/s at 256³; time-to-1e-8 learned vs plain"
# inner tolerance of the mixed-precision refinement that keeps the inner CG
# direction (the fastest of 1e-1 ... 1e-4 at 256^3, to 1e-10 and to 1e-8)
KEEP_INNER_TOL = 1e-2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(fmt, m, nnz, nb, fp=8, layout=None):
    """Algorithmic bytes of one SpMV: matrix streamed once, x read once, y
    written once, int32 indices; for the fused dot p_i is the x entry already
    read.  CRS (layout: the problem's csr_layout): with a group walk, fp nnz
    values, 8 bytes per work item, 4 per group, 12 per other row and 4 per
    entry of the other rows; else fp nnz values, 4 bytes of
    column index per entry outside the descriptor tiles, 112 per descriptor
    tile, 4 (tiles + 1) of tile bounds plus 4 per row of the other tiles,
    2 fp m.  1x3 BCRS (layout: b13_layout): 3 fp nb values, 4 bytes of column
    index per block outside the descriptor slices, 48 per descriptor slice,
    4 (slices + 1) of slice bounds, 2 fp m.  layout None counts every tile or
    slice as indexed (CRS then 4 (m+1) of row pointers)."""
    if fmt == "csr":
        if layout is None:
            return (fp + 4) * nnz + 4 * (m + 1) + 2 * fp * m
        if layout.get("items", 0) > 0:
            # group walk: every value; per item an 8-byte record; per group its
            # first row pointer; the other rows' list entry, two row pointers
            # and column indices
            other_nnz = nnz - 27 * layout["group_rows"]
            return (fp * nnz + 8 * layout["items"] + 4 * layout["groups"] + 12 * layout["other_rows"]
                    + 4 * other_nnz + 2 * fp * m)
        R, tiles, ct = layout["tile_rows"], layout["tiles"], layout["compressed_tiles"]
        return fp * nnz + 4 * (nnz - 27 * R * ct) + 112 * ct + 4 * (tiles + 1) + 4 * (m - R * ct) + 2 * fp * m
    slices = (m + 63) // 64
    cs = cb = 0
    if layout is not None:
        slices, cs, cb = layout["slices"], layout["compressed_slices"], layout["compressed_blocks"]
    return 3 * fp * nb + 4 * (nb - cb) + 48 * cs + 4 * (slices + 1) + 2 * fp * m


def algorithmic_bytes(fmt, m, nnz, nb, fp=8):
    """The bytes one product must move by its format's definition, every
    index stored and read, x read once, y written once, int32 indices:
    CRS (fp + 4) nnz + 4 (m + 1) + 2 fp m; 1x3 BCRS (3 fp + 4) nb + 4 (m + 1)
    + 2 fp m (row pointers counted as for CRS)."""
    if fmt == "csr":
        return (fp + 4) * nnz + 4 * (m + 1) + 2 * fp * m
    return (3 * fp + 4) * nb + 4 * (m + 1) + 2 * fp * m


def time_spmv_dot(P, fmt, reps, torch, flush_bytes=1 << 30, warmup=5, f32=False):
    """Mean duration of the fused SpMV + dot kernel from HIP event pairs
    recorded around each launch on the library's stream.  Before each launch
    flush_bytes of unrelated memory are written on the same stream, as the
    vector updates of a CG iteration do between two products, so that x is
    not left in the memory-side cache by the previous launch."""
    from paper_1505_08023_amd import inputs
    x = torch.tensor(inputs.spmv_vector(P.m, seed=0, dtype="float32" if f32 else "float64"), device=P.ctx.device)
    q = torch.empty_like(x)
    pq = torch.zeros(1, dtype=torch.float64, device=x.device)
    flush = torch.empty(max(flush_bytes // 8, 1), dtype=torch.float64, device=x.device) if flush_bytes else None
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for _ in range(warmup):
        P.spmv_dot(x, q, pq, fmt=fmt)
    for ev in pairs:
        if flush is not None:
            with torch.cuda.stream(P.ctx.stream):
                flush.fill_(0.0)
        P.spmv_dot(x, q, pq, fmt=fmt, events=ev)
    P.ctx.stream.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in pairs)
    time_spmv_dot.median_ms = ms[len(ms) // 2]
    return sum(ms) / len(ms), ms[0]


def host_cpu():
    """CPU model, physical cores and the CPUs this process may use."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                k, _, v = ln.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    if phys is not None:
        cores.add((phys, core))
    return dict(cpu_model=model, physical_cores=len(cores) or None, logical_cpus=os.cpu_count(),
                cpus_available=len(os.sched_getaffinity(0)))


def time_oracle_cg(A, its, library=None):
    """Seconds per CG iteration of a build of the oracle: its[1] - its[0]
    iterations timed as the difference of two capped runs."""
    import oracle
    times = []
    for k in its:
        t = time.perf_counter()
        oracle.cg(A, tol=1e-8, max_iter=k, library=library)
        times.append(time.perf_counter() - t)
    return (times[1] - times[0]) / (its[1] - its[0])


def cpu_baseline(N, gpu_iters, its=(2, 42), its_omp=(4, 204)):
    """The oracle's CG on the host (assembly untimed): as it stands (the
    plain single-threaded build), and for context the same source built on
    this host with -O3 -march=native, single-threaded and with its loops over
    all the cores OpenMP is given.  gpu_iters: the iterations of the GPU
    solve, from which the time to the tolerance is extrapolated."""
    import tempfile

    import oracle
    from oracle import build as obuild
    t = time.perf_counter()
    A = oracle.assemble(N, N, N)
    log(f"[bench] oracle assembly {N}^3: {time.perf_counter() - t:.1f} s")
    sec = time_oracle_cg(A, its)
    n = its[1] - its[0]
    out = dict(value=1.0 / sec, unit="CG iter/s", cores=1, kind="oracle",
               sample=f"{N}^3 FP64 CRS oracle CG, {n} iterations timed as cg(max_iter={its[1]}) minus "
                      f"cg(max_iter={its[0]}) on one host core (gcc -O2, generic x86-64); assembly untimed",
               host=host_cpu(), paper_context=PAPER_CONTEXT)
    tmp = tempfile.TemporaryDirectory(prefix="oracle_timing_")  # removed below; loaded builds stay mapped
    try:
        d = tmp.name
        native = oracle.load_timing_build(obuild.build_timing(d))
        s1 = time_oracle_cg(A, its, native)
        out["native_O3_one_core"] = dict(value=1.0 / s1, unit="CG iter/s", cores=1,
                                         sample=f"same {n} iterations, gcc -O3 -march=native on this host")
        log(f"[bench] oracle -O3 -march=native, one core: {1.0 / s1:.3f} it/s")
        omp = oracle.load_timing_build(obuild.build_timing(d, openmp=True))
        threads = int(omp.orc_num_threads())
        sm = time_oracle_cg(A, its_omp, omp)
        out["native_O3_all_cores"] = dict(value=1.0 / sm, unit="CG iter/s", cores=threads,
                                          sample=f"{its_omp[1] - its_omp[0]} iterations, the same loops with "
                                                 f"OpenMP over {threads} threads, gcc -O3 -march=native -fopenmp")
        log(f"[bench] oracle -O3 -march=native, {threads} threads: {1.0 / sm:.3f} it/s")
        # the CRS and the 1x3 BCRS products alone (median of 10, x ~ U[-1, 1)
        # as on the GPU; the paper's own comparison, on this host) and the
        # time to 1e-8 extrapolated from the iteration rate
        from paper_1505_08023_amd import inputs
        xv = inputs.spmv_vector(A.m, seed=0)
        b13 = oracle.bcrs13(A)
        nb = len(b13[1])

        def median_ms(fn):
            ts = []
            for _ in range(10):
                t = time.perf_counter()
                fn()
                ts.append(time.perf_counter() - t)
            return sorted(ts)[5] * 1e3
        for lib, key in ((native, "native_O3_one_core"), (omp, "native_O3_all_cores")):
            ms = median_ms(lambda: oracle.csr_spmv(A, xv, library=lib))
            out[key]["spmv_ms"] = ms
            out[key]["spmv_GBps"] = algorithmic_bytes("csr", A.m, A.nnz, 0) / (ms * 1e-3) / 1e9
            mb = median_ms(lambda: oracle.bcrs13_spmv(A, b13, xv, library=lib))
            out[key]["bcrs13_spmv_ms"] = mb
            out[key]["bcrs13_spmv_GBps"] = algorithmic_bytes("bcrs13", A.m, A.nnz, nb) / (mb * 1e-3) / 1e9
            out[key]["bcrs13_over_csr_spmv"] = ms / mb
            log(f"[bench] oracle products, {key}: CRS {ms:.1f} ms, 1x3 BCRS {mb:.1f} ms")
        del b13
        out["native_O3_all_cores"]["time_to_1e-8_s_extrapolated"] = gpu_iters * sm
        out["native_O3_all_cores"]["extrapolation"] = (f"{gpu_iters} iterations (the GPU solve's count) x the "
                                                       "measured seconds per iteration")
    except (OSError, subprocess.CalledProcessError) as e:
        out["native_builds_error"] = str(e)
    finally:
        tmp.cleanup()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="elements per axis")
    ap.add_argument("--fmt", default="bcrs13", choices=["bcrs13", "csr"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--spmv-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--learned-samples", type=int, default=1000, help="held-out seeds in the learned section")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision and batched sections (for profiler runs)")
    ap.add_argument("--size-sweep", action="store_true",
                    help="instead of the benchmark: FP64 CG iterations/s for exactly 200 iterations at meshes "
                         "16^3 to 320^3 in both formats, one JSON line per mesh")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.size_sweep:
        size_sweep()
        return

    import torch
    from paper_1505_08023_amd.mfe import Context, Problem

    N = args.n
    ctx = Context(0)
    t = time.perf_counter()
    P = Problem.mesh(ctx, N, N, N, formats=("csr", "bcrs13"), precisions=("f64", "f32"))
    log(f"[bench] assembled {N}^3 on the GPU (m={P.m}, nnz={P.nnz}, 1x3 blocks={P.nblocks}) "
        f"in {time.perf_counter() - t:.2f} s")
    x = torch.zeros(P.m, dtype=torch.float64, device=ctx.device)

    def solve():
        with torch.cuda.stream(ctx.stream):
            x.zero_()
        return P.cg(x, tol=args.tol, max_iter=args.max_iter, fmt=args.fmt)[1]

    for _ in range(args.warmup):
        st = solve()
        log(f"[bench] warm-up solve: {st['iterations']} its, {st['seconds']:.3f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [solve() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    its = sum(s["iterations"] for s in stats)
    log(f"[bench] {args.steps} timed solves: {its} its in {elapsed:.3f} s")

    # dominant kernel: fused SpMV + dot, both formats, FP64 and the FP32
    # product of the mixed-precision inner solves.  bytes: the format's
    # algorithmic bytes (every index read); bytes_moved: what this storage
    # streams (descriptor tiles and slices form their indices)
    spmv = {}
    for fp, suffix in ((8, ""), (4, "_f32")):
        for fmt in ("bcrs13", "csr"):
            mean_ms, min_ms = time_spmv_dot(P, fmt, args.spmv_reps, torch, f32=fp == 4)
            by = algorithmic_bytes(fmt, P.m, P.nnz, P.nblocks, fp=fp)
            moved = spmv_bytes(fmt, P.m, P.nnz, P.nblocks, fp=fp,
                               layout=P.csr_layout if fmt == "csr" else P.b13_layout)
            sec = mean_ms * 1e-3
            spmv[fmt + suffix] = dict(mean_ms=mean_ms, median_ms=time_spmv_dot.median_ms, min_ms=min_ms,
                                      launches=args.spmv_reps, bytes=by, GBps=by / sec / 1e9,
                                      frac_hbm=by / sec / 1e9 / HBM_PEAK_GBS, bytes_moved=moved,
                                      moved_GBps=moved / sec / 1e9)
            log(f"[bench] spmv_dot {fmt}{suffix}: {mean_ms:.4f} ms, {spmv[fmt + suffix]['GBps']:.0f} GB/s algorithmic, "
                f"{spmv[fmt + suffix]['moved_GBps']:.0f} GB/s moved")
    dom = spmv[args.fmt]
    vec_bytes = 64 * P.m
    it_bytes = dom["bytes"] + vec_bytes
    t_asm, t_conv = assembly_and_conversion(ctx, N, torch)
    log(f"[bench] {N}^3 assembly {t_asm:.4f} s, CRS -> 1x3 BCRS {t_conv:.4f} s")

    line = {
        "metric": METRIC,
        "value": its / elapsed,
        "unit": "CG iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"minife_heat_{N}cubed_fp64_cg_{args.fmt}", "mesh": [N, N, N],
                   "rows": P.m, "nnz": P.nnz, "blocks_1x3": P.nblocks, "format": args.fmt,
                   "tol": args.tol, "x0": "zero", "step": "one CG solve to tol"},
        "roofline": {"bound": "hbm", "achieved": dom["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["GBps"] / HBM_PEAK_GBS,
                     "traffic": (MEASURED_TRAFFIC.get((args.fmt, N)) or (None, None))[0],
                     "traffic_source": (MEASURED_TRAFFIC.get((args.fmt, N)) or (None, None))[1],
                     "kernel": "k_spmv_b13s<double, dot>" if args.fmt == "bcrs13" else "k_spmv_csrg<double, dot>",
                     "timing": "HIP events around each launch on the library stream, 1 GiB of other memory "
                               "written before each, as between two products of a CG iteration",
                     "bytes_per_launch": dom["bytes"],
                     "bytes_definition": "(3*8+4) nb + 4 (m+1) + 16 m: the 1x3 BCRS format's algorithmic bytes"
                                         if args.fmt == "bcrs13" else "12 nnz + 4 (m+1) + 16 m: CRS algorithmic bytes",
                     "mean_launch_ms": dom["mean_ms"],
                     "bytes_moved_per_launch": dom["bytes_moved"], "moved_GBps": dom["moved_GBps"]},
        "cg": {"iterations_per_solve": stats[-1]["iterations"], "time_to_tol_s": elapsed / args.steps,
               "time_to_tol_incl_conversion_s": elapsed / args.steps + t_conv,
               "bcrs13_conversion_s": t_conv, "assembly_s": t_asm,
               "rel_res_true": stats[-1]["rel_res_true"], "status": stats[-1]["status"],
               "bytes_per_iteration": it_bytes,
               "effective_GBps": its / elapsed * it_bytes / 1e9},
        "spmv": spmv,
        "bcrs13_over_csr": {"spmv_fp64": spmv["csr"]["mean_ms"] / spmv["bcrs13"]["mean_ms"],
                            "spmv_fp32": spmv["csr_f32"]["mean_ms"] / spmv["bcrs13_f32"]["mean_ms"],
                            "paper_context": PAPER_CONTEXT},
    }
    # a plain 1 GiB device copy: the measured streaming ceiling, and the
    # known-size kernel that scales the HBM byte counters of a profiler run
    line["copy_probe"] = copy_probe(torch, ctx.device)
    log(f"[bench] copy probe: {line['copy_probe']['GBps']:.0f} GB/s")
    # the library's own streaming probes (16-byte non-temporal accesses): the
    # bandwidth a plain stream reaches on this machine, next to the 8 TB/s peak
    line["stream_probe"] = stream_probe(ctx, torch)
    line["roofline"]["frac_of_stream_read"] = dom["GBps"] / line["stream_probe"]["read_GBps"]
    log(f"[bench] stream probe: {line['stream_probe']}")
    if not args.no_extras:
        extras(args, ctx, P, x, line, torch)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (bounded sample) ...")
        line["cpu_baseline"] = cpu_baseline(N, stats[-1]["iterations"])
        log(f"[bench] oracle {line['cpu_baseline']['value']:.3f} it/s")
    print(json.dumps(line), flush=True)


def size_sweep(sizes=(16, 24, 32, 48, 64, 96, 128, 160, 192, 224, 256, 288, 320), its=200):
    """CG iterations per second against mesh size: FP64 CG for exactly `its`
    iterations (tol 0) from x0 = 0 on the paper's problem, fastest of 3 timed
    solves after one untimed, in both formats; `TBps` divides the format's
    algorithmic SpMV bytes plus the 64 m vector bytes of an iteration by the
    iteration time."""
    import torch
    from paper_1505_08023_amd.mfe import Context, Problem
    ctx = Context(0)
    for n in sizes:
        P = Problem.mesh(ctx, n, n, n, formats=("csr", "bcrs13"))
        x = torch.zeros(P.m, dtype=torch.float64, device=ctx.device)
        row = {"mesh": [n, n, n], "rows": P.m, "nnz": P.nnz, "blocks_1x3": P.nblocks, "iterations": its}
        for fmt in ("bcrs13", "csr"):
            def solve():
                with torch.cuda.stream(ctx.stream):
                    x.zero_()
                return P.cg(x, tol=0.0, max_iter=its, fmt=fmt, raise_on_breakdown=False)[1]
            solve()
            times = []
            for _ in range(3):
                torch.cuda.synchronize()
                t = time.perf_counter()
                st = solve()
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t)
            assert st["iterations"] == its
            rate = its / min(times)
            by = algorithmic_bytes(fmt, P.m, P.nnz, P.nblocks) + 64 * P.m
            row[fmt] = {"it_per_s": rate, "TBps": by * rate / 1e12}
        print(json.dumps(row), flush=True)
        P.close()
        del x
        torch.cuda.empty_cache()
    ctx.close()


def assembly_and_conversion(ctx, n, torch, reps=3):
    """Best-of-reps wall time of creating the n^3 problem in CRS only
    (mesh, structure, element sums, Dirichlet elimination, CRS tile
    descriptors) and the extra time when the 1x3 BCRS is built too."""
    from paper_1505_08023_amd.mfe import Problem
    best = {}
    for fmts in (("csr",), ("csr", "bcrs13")):
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            Q = Problem.mesh(ctx, n, n, n, formats=fmts)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            Q.close()
            best[fmts] = min(best.get(fmts, dt), dt)
    return best[("csr",)], max(best[("csr", "bcrs13")] - best[("csr",)], 0.0)


def copy_probe(torch, device, nbytes=1 << 30):
    """Bandwidth of a plain device-to-device copy of nbytes (read + write)."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device=device).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    return dict(bytes_moved=2 * nbytes, ms=ms, GBps=2 * nbytes / (ms * 1e-3) / 1e9)


def stream_probe(ctx, torch, nbytes=2 << 30, reps=10):
    """Median bandwidth of the library's streaming read and copy probes over
    nbytes of source (HIP events around each launch)."""
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device=ctx.device)
    out = {}
    for kind, dst, moved in (("read", torch.empty(4096, dtype=torch.float64, device=ctx.device), nbytes),
                             ("copy", torch.empty(n // 2, dtype=torch.float64, device=ctx.device), nbytes)):
        m = n if kind == "read" else n // 2  # the copy moves nbytes in all (half read, half written)
        src_k = src if kind == "read" else src[:m]
        torch.cuda.synchronize()
        for _ in range(3):
            ctx.stream_probe(kind, src_k, dst)
        pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for ev in pairs:
            ctx.stream_probe(kind, src_k, dst, events=ev)
        ctx.stream.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in pairs)[reps // 2]
        out[f"{kind}_GBps"] = moved / (ms * 1e-3) / 1e9
        out[f"{kind}_ms"] = ms
    out["bytes_moved"] = nbytes
    del src
    return out


def extras(args, ctx, P, x, line, torch):
    from paper_1505_08023_amd import inputs
    from paper_1505_08023_amd.mfe import Batch, Problem

    # FP64 references for the error of every mixed-precision result: FP64 CG
    # to a tolerance 100 times tighter than the compared solves
    refs = {}
    for tol in (1e-10, 1e-8):
        xr = torch.zeros_like(x)
        P.cg(xr, tol=tol / 100, max_iter=args.max_iter, fmt=args.fmt)
        refs[tol] = (xr, float(torch.linalg.norm(xr)))

    def err(tol):
        xr, nr = refs[tol]
        return float(torch.linalg.norm(x - xr)) / nr

    # mixed precision against FP64 CG at equal accuracy (1e-10)
    mixed = {"error_reference": "FP64 CG to 1e-12"}
    for name, fn in (("fp64_cg", lambda: P.cg(x, tol=1e-10, max_iter=args.max_iter, fmt=args.fmt)[1]),
                     ("fp32_inner_fp64_refine", lambda: P.cg_mixed(x, tol=1e-10, inner_tol=1e-4, fmt=args.fmt)[1]),
                     ("fp32_inner_fp64_refine_keep_direction",
                      lambda: P.cg_mixed(x, tol=1e-10, inner_tol=KEEP_INNER_TOL, fmt=args.fmt, keep_direction=True)[1])):
        with torch.cuda.stream(ctx.stream):
            x.zero_()
        fn()  # warm-up (graph capture)
        with torch.cuda.stream(ctx.stream):
            x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = fn()
        torch.cuda.synchronize()
        mixed[name] = dict(seconds=time.perf_counter() - t, iterations=st["iterations"], outer=st["outer"],
                           rel_res_true=st["rel_res_true"], error_vs_fp64=err(1e-10))
        log(f"[bench] {name} to 1e-10: {mixed[name]}")
    mixed["speedup"] = mixed["fp64_cg"]["seconds"] / mixed["fp32_inner_fp64_refine"]["seconds"]
    mixed["speedup_keep_direction"] = (mixed["fp64_cg"]["seconds"]
                                       / mixed["fp32_inner_fp64_refine_keep_direction"]["seconds"])
    line["mixed_precision_1e-10"] = mixed

    # inner tolerance of the FP32 solves, swept at 1e-10 (best first), and
    # mixed against FP64 at the headline tolerance 1e-8
    def timed(fn):
        with torch.cuda.stream(ctx.stream):
            x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, st
    sweep = []
    for keep, itols in ((False, (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)), (True, (1e-1, 1e-2, 1e-3, 1e-4))):
        for itol in itols:
            dt, st = timed(lambda: P.cg_mixed(x, tol=1e-10, inner_tol=itol, fmt=args.fmt, keep_direction=keep)[1])
            sweep.append(dict(inner_tol=itol, keep_direction=keep, seconds=dt, inner_iterations=st["iterations"],
                              outer=st["outer"], rel_res_true=st["rel_res_true"], error_vs_fp64=err(1e-10)))
    sweep.sort(key=lambda r: r["seconds"])
    line["mixed_inner_tol_sweep_1e-10"] = sweep
    log(f"[bench] inner tolerance sweep: best {sweep[0]}")
    m8 = {"error_reference": "FP64 CG to 1e-10"}
    for name, fn in (("fp64_cg", lambda: P.cg(x, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt)[1]),
                     ("fp32_inner_fp64_refine", lambda: P.cg_mixed(x, tol=1e-8, inner_tol=1e-4, fmt=args.fmt)[1]),
                     ("fp32_inner_fp64_refine_keep_direction",
                      lambda: P.cg_mixed(x, tol=1e-8, inner_tol=KEEP_INNER_TOL, fmt=args.fmt, keep_direction=True)[1])):
        dt, st = timed(fn)
        m8[name] = dict(seconds=dt, iterations=st["iterations"], outer=st["outer"], rel_res_true=st["rel_res_true"],
                        error_vs_fp64=err(1e-8))
    m8["speedup"] = m8["fp64_cg"]["seconds"] / m8["fp32_inner_fp64_refine"]["seconds"]
    m8["speedup_keep_direction"] = m8["fp64_cg"]["seconds"] / m8["fp32_inner_fp64_refine_keep_direction"]["seconds"]
    line["mixed_precision_1e-8"] = m8
    log(f"[bench] mixed at 1e-8: {m8}")
    del refs

    # batched uneven solves: 64 meshes, Nx, Ny, Nz ~ U{16..96}, seed 0, to 1e-8 each
    sizes, faces = inputs.batched_meshes(nsys=64, lo=16, hi=96, seed=0)
    B = Batch(ctx, sizes, faces, precisions=("f64", "f32"))
    xb = torch.zeros(B.m, dtype=torch.float64, device=ctx.device)

    def batch_fp64_seconds():
        for _ in range(2):  # warm-up (graph capture), then timed
            with torch.cuda.stream(ctx.stream):
                xb.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            B.cg(xb, tol=1e-8, fmt=args.fmt)
            torch.cuda.synchronize()
        return time.perf_counter() - t
    t_default = batch_fp64_seconds()
    lanes, factor = B.autotune(args.fmt)
    shape = ({"slices_per_wavefront": lanes, "rows_per_wavefront": 64 * lanes} if args.fmt == "bcrs13"
             else {"lanes_per_row": lanes, "rows_per_wavefront": 64 // lanes})
    bat = {"systems": 64, "rows": B.m, "nnz": B.nnz,
           "autotune": {**shape, "grid_factor": factor, "fp64_seconds_untuned": t_default,
                        "untuned_shape": "1 slice per wavefront, grid 1 x resident" if args.fmt == "bcrs13"
                        else "32 lanes per row, grid 1 x resident"}}
    xbr = torch.zeros_like(xb)
    B.cg(xbr, tol=1e-10, fmt=args.fmt)
    offs = B.row_offsets.tolist()

    def worst_err():
        return max(float(torch.linalg.norm(xb[a:b] - xbr[a:b]) / torch.linalg.norm(xbr[a:b]))
                   for a, b in zip(offs[:-1], offs[1:]))
    bat["error_reference"] = "each system's FP64 CG to 1e-10"
    for name, fn in (("fp64", lambda: B.cg(xb, tol=1e-8, fmt=args.fmt)[1]),
                     ("fp32_inner_fp64_refine", lambda: B.cg_mixed(xb, tol=1e-8, fmt=args.fmt)[1]),
                     ("fp32_inner_fp64_refine_keep_direction",
                      lambda: B.cg_mixed(xb, tol=1e-8, inner_tol=1e-4, fmt=args.fmt, keep_direction=True)[1])):
        with torch.cuda.stream(ctx.stream):
            xb.zero_()
        fn()
        with torch.cuda.stream(ctx.stream):
            xb.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        its = [s["iterations"] for s in st]
        bat[name] = dict(seconds=dt, max_iterations=max(its), sum_iterations=sum(its),
                         worst_rel_res_true=max(s["rel_res_true"] for s in st),
                         all_converged=all(s["status"] == 0 for s in st), worst_error_vs_fp64=worst_err())
        if name == "fp64":
            # algorithmic bytes: each system's iterations x (its rows' share of
            # the batch's 1x3 BCRS SpMV bytes + 64 m)
            dims = [((nx + 1) * (ny + 1) * (nz + 1), (nx + 1) * (3 * ny + 1) * (3 * nz + 1))
                    for nx, ny, nz in sizes.tolist()]
            full = spmv_bytes("bcrs13", B.m, 0, sum(nbs for _, nbs in dims), layout=B.b13_layout)
            tot = 0
            for (ms, _), k in zip(dims, its):
                tot += k * (full * ms / B.m + 64 * ms)
            bat[name]["algorithmic_bytes"] = tot
            bat[name]["effective_GBps"] = tot / dt / 1e9
        log(f"[bench] batched {name}: {bat[name]}")
    bat["autotune"]["gain_fp64"] = t_default / bat["fp64"]["seconds"]
    line["batched_64_meshes_1e-8"] = bat
    B.close()

    # CG variants to 1e-8 against the two-reduction loop: single-reduction (one
    # reduction point per iteration) and Jacobi-preconditioned; 256^3 and the
    # 64^3 mesh of the learned section
    sr = {}
    P64 = Problem.mesh(ctx, 64, 64, 64, formats=("bcrs13",))
    for label, PP, xx in (("256cubed", P, x), ("64cubed", P64, None)):
        if xx is None:
            xx = torch.zeros(PP.m, dtype=torch.float64, device=ctx.device)
        row = {}
        for variant in ("cg", "single_reduction", "jacobi"):
            best, st = None, None
            for _ in range(3):
                with torch.cuda.stream(ctx.stream):
                    xx.zero_()
                torch.cuda.synchronize()
                t = time.perf_counter()
                st = PP.cg(xx, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt, variant=variant)[1]
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                best = dt if best is None else min(best, dt)
            row[variant] = dict(seconds=best, iterations=st["iterations"], it_per_s=st["iterations"] / best,
                                rel_res_true=st["rel_res_true"])
        row["speedup_single_reduction"] = row["cg"]["seconds"] / row["single_reduction"]["seconds"]
        row["speedup_jacobi"] = row["cg"]["seconds"] / row["jacobi"]["seconds"]
        sr[label] = row
        log(f"[bench] CG variants {label}: {row}")
    line["cg_variants_1e-8"] = sr
    P64.close()

    # 128^3 plain CG for exactly 200 iterations (tol 0), both formats
    P2 = Problem.mesh(ctx, 128, 128, 128, formats=("csr", "bcrs13"))
    x2 = torch.zeros(P2.m, dtype=torch.float64, device=ctx.device)
    c2 = {"rows": P2.m, "nnz": P2.nnz, "iterations": 200}
    for fmt in ("bcrs13", "csr"):
        best = None
        for _ in range(3):
            with torch.cuda.stream(ctx.stream):
                x2.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = P2.cg(x2, tol=0.0, max_iter=200, fmt=fmt)[1]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        assert st["iterations"] == 200
        it_bytes = spmv_bytes(fmt, P2.m, P2.nnz, P2.nblocks,
                              layout=P2.csr_layout if fmt == "csr" else P2.b13_layout) + 64 * P2.m
        c2[fmt] = dict(it_per_s=200 / best, seconds=best, effective_GBps=200 * it_bytes / best / 1e9)
        log(f"[bench] 128^3 CG x200 {fmt}: {c2[fmt]}")
    line["cg_128cubed_200_iterations"] = c2
    P2.close()

    # time per module at the paper's mesh sizes: assembly (mesh, CRS
    # structure, element sums, Dirichlet elimination), CRS -> 1x3 BCRS
    # conversion, CG to 1e-8 (its SpMV share from the SpMV + dot kernel time),
    # and the device-side verification against the series solution
    mods = {}
    for n in (200, 300):
        t_asm, t_cv = assembly_and_conversion(ctx, n, torch)
        Pb = Problem.mesh(ctx, n, n, n, formats=("csr", "bcrs13"))
        xn = torch.zeros(Pb.m, dtype=torch.float64, device=ctx.device)
        Pb.cg(xn, tol=1e-8, max_iter=args.max_iter, fmt="bcrs13")  # warm-up (graph capture)
        with torch.cuda.stream(ctx.stream):
            xn.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = Pb.cg(xn, tol=1e-8, max_iter=args.max_iter, fmt="bcrs13")[1]
        torch.cuda.synchronize()
        t_cg = time.perf_counter() - t
        spmv_ms = time_spmv_dot(Pb, "bcrs13", 10, torch)[0]
        t = time.perf_counter()
        ver = Pb.verify_series(xn, x_max=0.75)
        t_ver = time.perf_counter() - t
        mods[f"{n}cubed"] = dict(rows=Pb.m, nnz=Pb.nnz, assembly_s=t_asm, bcrs13_conversion_s=t_cv,
                                 cg_s=t_cg, cg_iterations=st["iterations"], cg_rel_res_true=st["rel_res_true"],
                                 spmv_share_of_cg=st["iterations"] * spmv_ms * 1e-3 / t_cg,
                                 verification_s=t_ver, verification_max_err=ver["max_err"],
                                 verification_rms_err=ver["rms_err"], verification_nodes=ver["count"])
        log(f"[bench] modules {n}^3: {mods[f'{n}cubed']}")
        Pb.close()
        del xn
    line["module_times"] = mods

    # learned warm start against the zero start, 64^3, held-out boundary data
    wpath = os.path.join(ROOT, "paper_1505_08023_amd", "weights", "net64.npz")
    if os.path.exists(wpath):
        from paper_1505_08023_amd import learned
        from paper_1505_08023_amd.mfe import Net
        params, meta = learned.load(wpath)
        net = Net(ctx, 65, 1)
        net.set_params(params)
        seeds = list(range(learned.HELD_OUT_BASE, learned.HELD_OUT_BASE + args.learned_samples))
        ev = learned.evaluate(ctx, net, 64, seeds)
        ev.pop("rows")
        ev["weights"] = os.path.relpath(wpath, ROOT)
        ev["trained_on"] = {k: meta[k] for k in ("train", "epochs", "batch", "lr", "schedule") if k in meta}
        line["learned_warm_start_64cubed_1e-8"] = ev
        log(f"[bench] learned vs plain: {ev}")
        # the same with the mixed solves keeping their inner direction (inner
        # tolerance 1e-4, the fastest at 64^3), on the first 200 of those seeds
        evk = learned.evaluate(ctx, net, 64, seeds[:200], inner_tol=1e-4, keep_direction=True)
        evk.pop("rows")
        line["learned_warm_start_64cubed_1e-8_keep_direction"] = {
            k: evk[k] for k in ("samples", "mean_its_plain", "mean_time_plain_s", "mean_its_mixed", "mean_time_mixed_s",
                                "mean_its_learned_mixed", "mean_time_learned_mixed_s", "worst_res_learned_mixed",
                                "guesses_used_mixed", "speedup_time_mixed", "speedup_time_learned_mixed",
                                "error_vs_fp64_ref")}
        log(f"[bench] learned + mixed, direction kept: {line['learned_warm_start_64cubed_1e-8_keep_direction']}")
        if args.n % 64 == 0:
            line[f"guess_at_{args.n}cubed_1e-8"] = guess_at_scale(args, ctx, P, x, net, torch)
        net.close()


def guess_at_scale(args, ctx, P, x, net, torch):
    """Does an initial guess pay on the headline mesh?  The paper's boundary
    data on the 64^3 mesh, either the network's guess there (inference) or
    the 64^3 CG solution to 1e-8, prolonged trilinearly to the n^3 mesh
    (boundary nodes exact), as x0 of the FP64 solve to 1e-8 (mfe_cg_warm),
    timed from the start of the inference or of the coarse solve, against
    the zero start."""
    from paper_1505_08023_amd.mfe import Problem
    n, f = args.n, args.n // 64
    P64 = Problem.mesh(ctx, 64, 64, 64, formats=("bcrs13",))
    with torch.cuda.stream(ctx.stream):
        g64 = (torch.arange(65 ** 3, device=ctx.device) % 65 == 64).to(torch.float64)
        x64 = torch.zeros(65 ** 3, dtype=torch.float64, device=ctx.device)
        xr = torch.zeros_like(x)
    b = P.rhs()
    P.cg(xr, tol=1e-10, max_iter=args.max_iter, fmt=args.fmt)
    nr = float(torch.linalg.norm(xr))
    # the trivial guess keeps b (= g, the boundary rows being identity rows)
    # on the boundary nodes and 0 on the interior ones
    from paper_1505_08023_amd.learned import boundary_mask
    with torch.cuda.stream(ctx.stream):
        inner = ~torch.tensor(boundary_mask(n), device=ctx.device)

    def set_boundary_start():
        with torch.cuda.stream(ctx.stream):
            x.copy_(b).masked_fill_(inner, 0.0)

    def boundary():
        set_boundary_start()
        return P.cg(x, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt)[1]

    def zero():
        with torch.cuda.stream(ctx.stream):
            x.zero_()
        return P.cg(x, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt)[1]

    def learned():
        net.predict_x0(g64, x64)
        ctx.prolong(x64, (64, 64, 64), f, bnd=b, xf=x)
        return P.cg(x, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt, warm=True)[1]

    def coarse():
        with torch.cuda.stream(ctx.stream):
            x64.zero_()
        P64.cg(x64, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt)
        ctx.prolong(x64, (64, 64, 64), f, bnd=b, xf=x)
        return P.cg(x, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt, warm=True)[1]

    # the same guesses followed by the FP32-inner / FP64-refinement solve that
    # keeps its inner direction (the learned + mixed-precision form)
    def learned_mixed():
        net.predict_x0(g64, x64)
        ctx.prolong(x64, (64, 64, 64), f, bnd=b, xf=x)
        return P.cg_mixed(x, tol=1e-8, inner_tol=KEEP_INNER_TOL, fmt=args.fmt, warm=True, keep_direction=True)[1]

    def coarse_mixed():
        with torch.cuda.stream(ctx.stream):
            x64.zero_()
        P64.cg(x64, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt)
        ctx.prolong(x64, (64, 64, 64), f, bnd=b, xf=x)
        return P.cg_mixed(x, tol=1e-8, inner_tol=KEEP_INNER_TOL, fmt=args.fmt, warm=True, keep_direction=True)[1]

    out = {"mesh": [n, n, n], "boundary_data": "paper (u = 1 on x = 1, 0 elsewhere)",
           "error_reference": "FP64 CG to 1e-10"}
    for name, fn in (("zero_start", zero), ("boundary_start", boundary), ("learned_64cubed_guess_prolonged", learned),
                     ("cg_64cubed_solution_prolonged", coarse),
                     ("learned_64cubed_guess_prolonged_mixed_keep_direction", learned_mixed),
                     ("cg_64cubed_solution_prolonged_mixed_keep_direction", coarse_mixed)):
        fn()  # warm-up (graph capture)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out[name] = dict(seconds=dt, iterations=st["iterations"], rel_res_true=st["rel_res_true"],
                         guess_rejected=st["guess_rejected"], error_vs_fp64=float(torch.linalg.norm(x - xr)) / nr)
        if name != "zero_start":
            # the guess's own residual, untimed
            if name == "boundary_start":
                set_boundary_start()
            else:
                if name.startswith("learned"):
                    net.predict_x0(g64, x64)
                else:
                    with torch.cuda.stream(ctx.stream):
                        x64.zero_()
                    P64.cg(x64, tol=1e-8, max_iter=args.max_iter, fmt=args.fmt)
                ctx.prolong(x64, (64, 64, 64), f, bnd=b, xf=x)
            out[name]["guess_rel_res"] = P.cg(x, tol=1e-8, max_iter=0, fmt=args.fmt)[1]["rel_res_true"]
            out[name]["speedup"] = out["zero_start"]["seconds"] / dt
        log(f"[bench] guess at {n}^3, {name}: {out[name]}")
    P64.close()
    return out


if __name__ == "__main__":
    main()
