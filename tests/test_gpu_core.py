"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Same seeded inputs on both sides (paper_1505_08023_amd.inputs); the oracle
assembles its own matrix, so assembly, format conversion, SpMV and CG are
each compared end to end.

Tolerances
  assembly   ptr/col bit-exact; values |d| <= 8 eps max|A| (the GPU uses the
             closed-form element matrix, the oracle Gauss quadrature: both
             exact, they differ by rounding only); b |d| <= 64 eps max(|b|, h)
  SpMV       per row |d_i| <= 1e-12 sum_j |A_ij x_j| and ||d||_2 <= 1e-12 ||y||_2
  CG         both reach ||r||/||b|| <= tol; iteration counts within 2; the
             first 4 recurrence residuals (k = 0..3) within 1e-10 relative; the two
             solutions within ||A^-1|| (||r_gpu|| + ||r_oracle||) of each
             other, with true residuals and the exact smallest eigenvalue of A.
             Only the first residuals are compared entry by entry: the
             identity rows of the Dirichlet nodes put an isolated eigenvalue 1
             far above the rest of the spectrum, and rounding differences in
             its direction grow by orders of magnitude per iteration until CG
             re-converges them (visible as bumps in the residual history); the growth
             starts earlier on finer meshes (from k = 7 at 20^3, k = 5 at 128^3).  The
             oracle against a third-party CG (scipy matvec, numpy dots) shows
             the same O(1) gaps at the bumps.
"""
import math

import numpy as np
import pytest
import torch

import b13_model
import oracle
from paper_1505_08023_amd import inputs

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    from paper_1505_08023_amd.mfe import Context
    c = Context(0)
    yield c
    c.close()


def np_(t):
    return t.detach().cpu().numpy()


def mesh_problem(ctx, N, **kw):
    from paper_1505_08023_amd.mfe import Problem
    return Problem.mesh(ctx, *N, **kw)


MESHES = [(1, 1, 1), (2, 2, 2), (2, 3, 4), (4, 4, 4), (5, 3, 7), (20, 20, 20), (33, 33, 33)]


def bc_variants(N, seed=0):
    m = oracle.num_rows(*N)
    rng = np.random.default_rng(seed)
    field = inputs.node_field(*N, inputs.smooth_faces(seed))
    return [dict(), dict(face_vals=rng.uniform(0, 1, 6)), dict(node_g=field)]


def gpu_kw(ctx, kw):
    if "node_g" in kw:
        return dict(node_g=torch.tensor(kw["node_g"], dtype=torch.float64, device=ctx.device))
    return dict(kw)


# ---------------------------------------------------------------- assembly + Dirichlet

@pytest.mark.parametrize("N", MESHES)
def test_assembly_matches_oracle(ctx, N):
    for kw in bc_variants(N):
        print("assembly", N, list(kw), flush=True)
        A = oracle.assemble(*N, **kw)
        P = mesh_problem(ctx, N, **gpu_kw(ctx, kw))
        ptr, col, val, b = (np_(t) for t in P.export_csr())
        assert P.m == A.m and P.nnz == A.nnz
        assert np.array_equal(ptr, A.ptr.astype(np.int32))
        assert np.array_equal(col, A.col)
        amax = np.abs(A.val).max()
        assert np.abs(val - A.val).max() <= 8 * EPS * amax
        h = 1.0 / max(N)
        assert np.abs(b - A.b).max() <= 64 * EPS * max(np.abs(A.b).max(), h)
        P.close()


@pytest.mark.parametrize("N", MESHES)
def test_bcrs13_matches_oracle(ctx, N):
    A = oracle.assemble(*N)
    bptr, bcol, bval = oracle.bcrs13(A)
    P = mesh_problem(ctx, N)
    gptr, gcol, gval = (np_(t) for t in P.export_bcrs13())
    assert P.nblocks == len(bcol)
    assert np.array_equal(gptr, bptr.astype(np.int32))
    assert np.array_equal(gcol, bcol)
    assert np.abs(gval - bval).max() <= 8 * EPS * np.abs(A.val).max()
    P.close()


@pytest.mark.parametrize("N", [(2, 3, 4), (5, 3, 7), (20, 20, 20), (33, 33, 33), (40, 9, 6)])
def test_bcrs13_descriptor_slices(ctx, N):
    """The per-slice (1x3 BCRS) and per-tile (CRS) descriptors cover exactly
    the slices and tiles the host models find (index work: bit-exact counts),
    and the products through them match the oracle."""
    A = oracle.assemble(*N)
    bptr, bcol, _ = oracle.bcrs13(A)
    want = b13_model.descriptor_slices(bptr, bcol, A.m)
    P = mesh_problem(ctx, N)
    lay = P.b13_layout
    assert lay["slices"] == (A.m + 63) // 64
    assert (lay["compressed_slices"], lay["compressed_blocks"]) == want, (lay, want)
    if min(N) >= 20:
        assert lay["compressed_slices"] >= 0.5 * lay["slices"]
    # the CRS group walk (index work: bit-exact counts against the host model
    # and, for the groups, the closed form)
    cl = P.csr_layout
    want = b13_model.csr_groups(A.ptr, A.col, A.m, N)
    assert (cl["items"], cl["groups"], cl["group_rows"], cl["other_rows"]) == want, (cl, want)
    assert (cl["groups"], cl["group_rows"]) == b13_model.csr_groups_closed_form(*N)
    x = inputs.spmv_vector(A.m, seed=3)
    for fmt in ("bcrs13", "csr"):
        check_spmv(np_(P.spmv(torch.tensor(x, device=ctx.device), fmt=fmt)), A, x, oracle.csr_spmv(A, x))
    P.close()


def shifted_pattern_csr(m, e, offsets, edge, seed):
    """Rows edge..m-edge-1: 9 runs of 3 columns at i + e_i + offsets[k]
    (e_i in {0, 1}); the other rows: their diagonal only.  Random values."""
    rng = np.random.default_rng(seed)
    cols = []
    for i in range(m):
        if edge <= i < m - edge:
            cols.append(np.concatenate([i + e[i] + d + np.arange(3) for d in offsets]))
        else:
            cols.append(np.array([i]))
    ptr = np.concatenate([[0], np.cumsum([len(c) for c in cols])]).astype(np.int64)
    col = np.concatenate(cols).astype(np.int32)
    return oracle.CSR(ptr, col, rng.uniform(-1, 1, len(col)), np.zeros(m))


def test_descriptors_on_a_generic_matrix_with_random_row_shifts(ctx):
    """A CRS matrix (not a mesh) whose middle rows hold 9 runs of 3 columns at
    row + e_row + d_k with random 0/1 shifts e: every full 64-row slice there
    gets a 1x3 BCRS descriptor whatever its shift bits; CRS tiles get one
    only where e is constant over the tile.  Coverage against the host
    models, products against the oracle in both formats and precisions."""
    from paper_1505_08023_amd.mfe import Problem
    m, edge = 64 * 40 + 23, 700
    offsets = [-640, -333, -200, -3, 0, 3, 150, 321, 640]
    rng = np.random.default_rng(9)
    e = rng.integers(0, 2, m)
    e[64 * 20:64 * 22] = 0  # two slices without shifts
    e[64 * 24:64 * 26] = 1  # and two with every row shifted
    A = shifted_pattern_csr(m, e, offsets, edge, seed=10)
    bptr, bcol, _ = oracle.bcrs13(A)
    d = ctx.device
    P = Problem.from_csr(ctx, torch.tensor(A.ptr.astype(np.int32), device=d), torch.tensor(A.col, device=d),
                         torch.tensor(A.val, device=d), formats=("csr", "bcrs13"), precisions=("f64", "f32"))
    want = b13_model.descriptor_slices(bptr, bcol, A.m)
    assert want[0] > 0 and want[0] == sum(1 for s in range(m // 64) if 64 * s >= edge and 64 * s + 64 <= m - edge)
    assert (P.b13_layout["compressed_slices"], P.b13_layout["compressed_blocks"]) == want
    R = P.csr_layout["tile_rows"]
    assert P.csr_layout["compressed_tiles"] == b13_model.csr_descriptor_tiles(A.ptr, A.col, A.m, R) > 0
    x = inputs.spmv_vector(A.m, seed=11)
    y_ref = oracle.csr_spmv(A, x)
    for fmt in ("csr", "bcrs13"):
        check_spmv(np_(P.spmv(torch.tensor(x, device=d), fmt=fmt)), A, x, y_ref)
        x32 = x.astype(np.float32)
        a32 = A.val.astype(np.float32).astype(np.float64)
        ref32 = np.add.reduceat(a32 * x32.astype(np.float64)[A.col], A.ptr[:-1])
        scale32 = np.add.reduceat(np.abs(a32) * np.abs(x32.astype(np.float64))[A.col], A.ptr[:-1])
        y32 = np_(P.spmv(torch.tensor(x32, device=d), fmt=fmt)).astype(np.float64)
        assert np.all(np.abs(y32 - ref32) <= 32 * np.finfo(np.float32).eps * scale32 + 1e-38)
    P.close()


def test_set_bc_matches_fresh_assembly(ctx):
    N = (9, 7, 8)
    fv = np.random.default_rng(5).uniform(0, 1, 6)
    P = mesh_problem(ctx, N)
    P.set_bc(face_vals=fv)
    Q = mesh_problem(ctx, N, face_vals=fv)
    assert torch.equal(P.export_csr()[3], Q.export_csr()[3])
    field = inputs.node_field(*N, inputs.smooth_faces(11))
    P.set_bc(node_g=torch.tensor(field, dtype=torch.float64, device=ctx.device))
    A = oracle.assemble(*N, node_g=field)
    assert np.abs(np_(P.export_csr()[3]) - A.b).max() <= 64 * EPS * np.abs(A.b).max()


# ---------------------------------------------------------------- SpMV

def check_spmv(y_gpu, A, x, y_ref):
    scale = np.abs(A.val) * np.abs(x[A.col])
    rowscale = np.add.reduceat(scale, A.ptr[:-1]) if A.nnz else np.zeros(A.m)
    rowscale[np.diff(A.ptr) == 0] = 0
    d = np.abs(y_gpu - y_ref)
    assert np.all(d <= 1e-12 * rowscale + 1e-300), (d / np.maximum(rowscale, 1e-300)).max()
    assert np.linalg.norm(y_gpu - y_ref) <= 1e-12 * np.linalg.norm(y_ref)


# 64^3: matrices loaded through the caches; 112^3: non-temporal loads with the
# plain 1x3 BCRS walk; 128^3: non-temporal loads with the pipelined walk
# Besides the small meshes, sizes that take each 1x3 BCRS walk and tile order:
# 24^3 runs of 8 tiles per XCD, 48^3 runs of 2, 64^3 and 76^3 the plain walk
# (its grid takes every tile in one pass, the read-ahead walk's would not),
# 77^3 and up the read-ahead walk with runs of 16.
@pytest.mark.parametrize("N", MESHES + [(24, 24, 24), (48, 48, 48), (64, 64, 64), (76, 76, 76), (77, 77, 77),
                                        (112, 112, 112), (128, 128, 128)])
@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
def test_spmv_matches_oracle(ctx, N, fmt):
    print("spmv", N, fmt, flush=True)
    A = oracle.assemble(*N)
    x = inputs.spmv_vector(A.m, seed=0)
    y_ref = oracle.csr_spmv(A, x)
    P = mesh_problem(ctx, N)
    xg = torch.tensor(x, device=ctx.device)
    y = np_(P.spmv(xg, fmt=fmt))
    check_spmv(y, A, x, y_ref)
    # deterministic: a second product is bitwise equal
    assert np.array_equal(np_(P.spmv(xg, fmt=fmt)), y)
    P.close()


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
def test_spmv_full_size_sampled_rows(ctx, fmt):
    """256^3 in the launch configuration of the benchmark; rows sampled and
    rebuilt one by one by the oracle."""
    N = (256, 256, 256)
    P = mesh_problem(ctx, N, formats=(fmt,))
    m = P.m
    if fmt == "bcrs13":
        assert P.b13_layout["compressed_slices"] == b13_model.descriptor_slices_closed_form(*N)
        assert P.b13_layout["compressed_blocks"] == 576 * P.b13_layout["compressed_slices"]
    else:
        cl = P.csr_layout
        assert (cl["groups"], cl["group_rows"]) == b13_model.csr_groups_closed_form(*N)
        assert cl["other_rows"] == m - cl["group_rows"] and cl["compressed_tiles"] == 0
    x = inputs.spmv_vector(m, seed=0)
    y = np_(P.spmv(torch.tensor(x, device=ctx.device), fmt=fmt))
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([rng.integers(0, m, 3000), np.arange(0, 300), np.arange(m - 300, m),
                                     np.arange(m // 2 - 200, m // 2 + 200)]))
    got, _ = oracle.assemble_rows(*N, rows)
    for r, (c, v) in zip(rows, got):
        ref = 0.0
        for cc, vv in zip(c, v):
            ref += vv * x[cc]
        scale = float(np.sum(np.abs(v) * np.abs(x[c])))
        assert abs(y[r] - ref) <= 1e-12 * scale + 1e-300, (r, y[r], ref)
    P.close()


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
def test_spmv_f32_full_size_sampled_rows(ctx, fmt):
    """256^3 FP32 product (the inner product of the mixed-precision solve, in
    its launch configuration: packed FP32 values, non-temporal loads); rows
    sampled and rebuilt by the oracle, bar as in the FP32 SpMV tests: per row
    |d| <= 32 eps32 sum_j |A32_ij x32_j| against the FP64 product of the
    FP32-rounded matrix and vector."""
    N = (256, 256, 256)
    P = mesh_problem(ctx, N, formats=(fmt,), precisions=("f64", "f32"))
    m = P.m
    x32 = inputs.spmv_vector(m, seed=6, dtype=np.float32)
    y = np_(P.spmv(torch.tensor(x32, device=ctx.device), fmt=fmt)).astype(np.float64)
    rng = np.random.default_rng(8)
    rows = np.unique(np.concatenate([rng.integers(0, m, 3000), np.arange(0, 200), np.arange(m - 200, m)]))
    got, _ = oracle.assemble_rows(*N, rows)
    x64 = x32.astype(np.float64)
    eps32 = float(np.finfo(np.float32).eps)
    for r, (c, v) in zip(rows, got):
        a32 = np.asarray(v, np.float32).astype(np.float64)
        ref = float(np.sum(a32 * x64[c]))
        scale = float(np.sum(np.abs(a32) * np.abs(x64[c])))
        assert abs(y[r] - ref) <= 32 * eps32 * scale + 1e-38, (r, y[r], ref)
    P.close()


def test_spmv_generic_csr_ragged(ctx):
    """Rows of length 0..60 with random columns (empty rows, long rows, ragged tail)."""
    from paper_1505_08023_amd.mfe import Problem
    rng = np.random.default_rng(2)
    m = 1000 + 37
    lens = rng.integers(0, 61, m)
    lens[::17] = 0
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([np.sort(rng.choice(m, l, replace=False)) for l in lens]).astype(np.int32)
    val = rng.uniform(-1, 1, ptr[-1])
    A = oracle.CSR(ptr, col, val, np.zeros(m))
    x = inputs.spmv_vector(m, seed=4)
    y_ref = oracle.csr_spmv(A, x)
    d = ctx.device
    P = Problem.from_csr(ctx, torch.tensor(ptr.astype(np.int32), device=d), torch.tensor(col, device=d),
                         torch.tensor(val, device=d), formats=("csr", "bcrs13"))
    xg = torch.tensor(x, device=d)
    for fmt in ("csr", "bcrs13"):
        check_spmv(np_(P.spmv(xg, fmt=fmt)), A, x, y_ref)
    P.close()


def test_from_csr_rejects_bad_structure(ctx):
    from paper_1505_08023_amd._lib import MfeError
    from paper_1505_08023_amd.mfe import Problem
    d = ctx.device
    ptr = torch.tensor([0, 2, 3], dtype=torch.int32, device=d)
    for col in ([1, 0, 1], [0, 5, 1]):  # descending / out of range
        with pytest.raises(MfeError, match="EINVAL"):
            Problem.from_csr(ctx, ptr, torch.tensor(col, dtype=torch.int32, device=d),
                             torch.ones(3, dtype=torch.float64, device=d))


def test_stream_probe(ctx):
    """The bandwidth probes do what they time: the copy is exact, the read's
    per-workgroup partials sum to the sum of the input (ones: exact)."""
    d = ctx.device
    for n in (0, 1, 7, 1000, 2_000_003):
        src = torch.arange(n, dtype=torch.float64, device=d)
        dst = torch.full((n,), -1.0, dtype=torch.float64, device=d)
        ctx.stream_probe("copy", src, dst)
        ctx.stream.synchronize()
        assert torch.equal(dst, src)
        ones = torch.ones(n, dtype=torch.float64, device=d)
        part = torch.zeros(4096, dtype=torch.float64, device=d)
        ctx.stream_probe("read", ones, part)
        ctx.stream.synchronize()
        assert float(part.sum()) == float(n)


def test_dot_matches_oracle_and_is_reproducible(ctx):
    for n in (0, 1, 63, 1000, 2_000_003):
        x = inputs.spmv_vector(n, seed=1)
        y = inputs.spmv_vector(n, seed=2)
        ref = math.fsum(x * y)
        xg, yg = torch.tensor(x, device=ctx.device), torch.tensor(y, device=ctx.device)
        got = ctx.dot(xg, yg)
        assert abs(got - ref) <= 1e-13 * max(1.0, float(np.sum(np.abs(x * y))))
        assert ctx.dot(xg, yg) == got


# ---------------------------------------------------------------- CG

def lam_min(N):
    """Smallest eigenvalue of the assembled A (closed form).  The free block
    is S(x)M(x)M + M(x)S(x)M + M(x)M(x)S of 1-D linear-element stiffness S and
    mass M with Dirichlet ends, whose eigenvectors are sine modes:
    s(h) = (2 - 2 cos(pi h)) / h, m(h) = h (4 + 2 cos(pi h)) / 6 at mode 1.
    The Dirichlet identity rows add the eigenvalue 1."""
    def s(h):
        return (2 - 2 * math.cos(math.pi * h)) / h

    def m(h):
        return h * (4 + 2 * math.cos(math.pi * h)) / 6
    hx, hy, hz = (1.0 / n for n in N)
    lf = s(hx) * m(hy) * m(hz) + m(hx) * s(hy) * m(hz) + m(hx) * m(hy) * s(hz)
    return min(lf, 1.0) if min(N) >= 2 else 1.0


def check_solution_gap(x, ref, st, N, A):
    """||x - x_ref|| <= ||A^-1|| (||r|| + ||r_ref|| + rounding of the two
    residual evaluations, 27 eps || |A| |x| || each)."""
    bnorm = np.linalg.norm(A.b)
    absAx = np.add.reduceat(np.abs(A.val) * np.abs(ref["x"][A.col]), A.ptr[:-1])
    floor = 2 * 27 * EPS * (np.linalg.norm(absAx) + bnorm)
    bound = ((st["rel_res_true"] + ref["rel_res_true"]) * bnorm + floor) / lam_min(N)
    gap = float(np.linalg.norm(x - ref["x"]))
    assert gap <= bound * (1 + 1e-6) + 1e-300, (gap, bound)
    return gap, bound


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
@pytest.mark.parametrize("N", [(4, 4, 4), (20, 20, 20), (17, 9, 23)])
def test_cg_matches_oracle(ctx, N, fmt):
    print("cg", N, fmt, flush=True)
    tol, cap = 1e-8, 200
    A = oracle.assemble(*N)
    ref = oracle.cg(A, tol=tol, max_iter=cap, history=True)
    P = mesh_problem(ctx, N)
    x, st = P.cg(tol=tol, max_iter=cap, fmt=fmt, history=True)
    x = np_(x)
    assert ref["status"] == oracle.OK and st["status"] == 0
    assert abs(st["iterations"] - ref["iterations"]) <= 2
    assert st["rel_res_true"] <= tol and st["rel_res_recurrence"] <= tol
    h, hr = st["history"].numpy(), ref["history"]
    k = min(4, len(h), len(hr))
    assert np.all(np.abs(h[:k] - hr[:k]) <= 1e-10 * hr[:k])
    gap, bound = check_solution_gap(x, ref, st, N, A)
    print("cg", N, fmt, "iters", st["iterations"], ref["iterations"], "solution gap", gap, "bound", bound)
    # bitwise reproducible run to run
    x2, st2 = P.cg(tol=tol, max_iter=cap, fmt=fmt)
    assert np.array_equal(np_(x2), x) and st2["iterations"] == st["iterations"]
    P.close()


def test_cg_128_capped_matches_oracle(ctx):
    """128^3, FP64, CSR and 1x3 BCRS, capped at 200 iterations."""
    N = (128, 128, 128)
    A = oracle.assemble(*N)
    ref = oracle.cg(A, tol=1e-8, max_iter=200, history=True)
    P = mesh_problem(ctx, N)
    for fmt in ("csr", "bcrs13"):
        x, st = P.cg(tol=1e-8, max_iter=200, fmt=fmt, history=True)
        assert st["iterations"] == ref["iterations"] == 200
        assert st["status"] == ref["status"] == oracle.NOT_CONVERGED
        h, hr = st["history"].numpy(), ref["history"]
        assert np.all(np.abs(h[:4] - hr[:4]) <= 1e-10 * hr[:4])
        # the residual levels reached agree to within the bump amplitude
        assert 0.1 < st["rel_res_true"] / ref["rel_res_true"] < 10
        gap, bound = check_solution_gap(np_(x), ref, st, N, A)
        print("128^3", fmt, "res", st["rel_res_true"], ref["rel_res_true"], "gap", gap, "bound", bound)
    P.close()


def test_cg_256_properties(ctx):
    """256^3 to 1e-8 in the benchmark's configuration: properties that hold at any size,
    plus sampled residual rows rebuilt by the oracle."""
    N = (256, 256, 256)
    P = mesh_problem(ctx, N, formats=("bcrs13",))
    x, st = P.cg(tol=1e-8, max_iter=5000, fmt="bcrs13")
    assert st["status"] == 0 and st["rel_res_true"] <= 1e-8
    u = x.view(257, 257, 257)
    assert float(u.min()) >= -1e-6 and float(u.max()) <= 1 + 1e-6  # maximum principle
    assert float((u - u.flip(1)).abs().max()) <= 1e-6             # y -> 1-y symmetry
    c = float(u[128, 128, 128])
    assert abs(c - oracle.analytic_u(0.5, 0.5, 0.5)) <= 1e-4      # FE error O(h^2) at the centre
    xs = np_(x)
    rows = np.random.default_rng(9).integers(0, P.m, 2000)
    got, b = oracle.assemble_rows(*N, rows)
    # ||b||: 1 on the (N+1)^2 nodes of x = 1, h on the (N-1)^2 free nodes next to it
    bn = math.sqrt(257 ** 2 + 255 ** 2 / 256 ** 2)
    for (cols, vals), bi in zip(got, b):
        r = bi - sum(v * xs[cc] for cc, v in zip(cols, vals))
        assert abs(r) <= 1e-8 * bn
    P.close()


def test_cg_edge_cases(ctx):
    N = (6, 6, 6)
    P = mesh_problem(ctx, N)
    # max_iter = 0: nothing happens, not converged
    x, st = P.cg(tol=1e-8, max_iter=0)
    assert st["iterations"] == 0 and st["status"] == 1 and float(x.abs().max()) == 0.0
    # loose tolerance met at the start
    x, st = P.cg(tol=2.0, max_iter=10)
    assert st["iterations"] == 0 and st["status"] == 0
    # b = 0: x = 0 whatever x0
    Z = mesh_problem(ctx, N, face_vals=[0.0] * 6)
    x0 = torch.ones(Z.m, dtype=torch.float64, device=ctx.device)
    x, st = Z.cg(x=x0, tol=1e-8, max_iter=10)
    assert st["status"] == 0 and float(x.abs().max()) == 0.0
    # warm start at the solution: converged at k = 0
    A = oracle.assemble(*N)
    xs = torch.tensor(oracle.cg(A, tol=1e-14, max_iter=500)["x"], device=ctx.device)
    x, st = P.cg(x=xs.clone(), tol=1e-8, max_iter=10)
    assert st["iterations"] == 0
    # capped run: same count and status as the oracle's capped run
    ref = oracle.cg(A, tol=1e-12, max_iter=7, history=True)
    x, st = P.cg(tol=1e-12, max_iter=7, history=True)
    assert st["status"] == 1 and st["iterations"] == 7 and ref["status"] == oracle.NOT_CONVERGED
    h, hr = st["history"].numpy(), ref["history"]
    assert np.all(np.abs(h[:4] - hr[:4]) <= 1e-10 * hr[:4])
    check_solution_gap(np_(x), ref, st, N, A)


def test_mesh_size_limit(ctx):
    """The structural count nnz = (3 Nx + 1)(3 Ny + 1)(3 Nz + 1) must stay below
    2^31 for the 32-bit row pointers: 429^3 elements is the largest cube
    (1288^3 entries) and one more per axis is refused with EUNSUPPORTED before
    anything is allocated, as is a flat mesh whose rows would fit but whose
    entries would not; the context stays usable."""
    from paper_1505_08023_amd._lib import MfeError
    assert (3 * 429 + 1) ** 3 < 2 ** 31 - 1 < (3 * 430 + 1) ** 3
    for N in [(430, 430, 430), (2000, 2000, 60)]:
        print("refused", N, flush=True)
        with pytest.raises(MfeError, match="EUNSUPPORTED"):
            mesh_problem(ctx, N)
    P = mesh_problem(ctx, (4, 4, 4))
    _, st = P.cg(tol=1e-10, max_iter=200)
    assert st["status"] == 0
    P.close()


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
def test_cg_warm_start(ctx, fmt):
    """mfe_cg_warm keeps a guess closer than x0 = 0 and otherwise solves from
    zero, bitwise as mfe_cg from zero (the same kernels see r0 = b)."""
    N = (20, 20, 20)
    A = oracle.assemble(*N)
    ref = oracle.cg(A, tol=1e-12, max_iter=1000)
    P = mesh_problem(ctx, N)
    x_zero, st_zero = P.cg(tol=1e-8, max_iter=500, fmt=fmt, history=True)
    # a guess near the solution: kept, fewer iterations, same stopping rule
    rng = np.random.default_rng(4)
    guess = ref["x"] + 1e-4 * rng.standard_normal(P.m)
    dirichlet = oracle.boundary(*N)[0] != 0
    guess[dirichlet] = ref["x"][dirichlet]  # Dirichlet values exact, as a predicted guess keeps them
    g = torch.tensor(guess, device=ctx.device)
    x, st = P.cg(x=g, tol=1e-8, max_iter=500, fmt=fmt, warm=True, history=True)
    assert st["guess_rejected"] == 0 and st["status"] == 0
    assert st["iterations"] < st_zero["iterations"]
    assert st["rel_res_true"] <= 1e-8
    r0 = A.b - oracle.csr_spmv(A, guess)
    assert abs(float(st["history"][0]) - np.linalg.norm(r0) / np.linalg.norm(A.b)) <= 1e-12
    check_solution_gap(np_(x), ref, st, N, A)
    # a poor guess: rejected, then identical to the zero start
    bad = torch.tensor(10.0 * rng.standard_normal(P.m), device=ctx.device)
    x, st = P.cg(x=bad, tol=1e-8, max_iter=500, fmt=fmt, warm=True, history=True)
    assert st["guess_rejected"] == 1
    assert st["iterations"] == st_zero["iterations"]
    assert np.array_equal(np_(x), np_(x_zero))
    assert np.array_equal(st["history"].numpy(), st_zero["history"].numpy())
    # the plain entry point never rejects
    x, st = P.cg(x=torch.tensor(10.0 * rng.standard_normal(P.m), device=ctx.device), tol=1e-8, max_iter=500,
                 fmt=fmt)
    assert st["guess_rejected"] == 0
    # x0 = 0 itself (||r0|| = ||b||) counts as rejected and changes nothing
    x, st = P.cg(x=torch.zeros(P.m, dtype=torch.float64, device=ctx.device), tol=1e-8, max_iter=500, fmt=fmt,
                 warm=True)
    assert st["guess_rejected"] == 1 and np.array_equal(np_(x), np_(x_zero))
    P.close()


def test_cg_many_solution_buffers(ctx):
    """Solves into 20 different x buffers (more than the per-problem graph
    cache keeps): every solve is right, the old graphs are dropped safely."""
    N = (12, 12, 12)
    P = mesh_problem(ctx, N)
    xs = [torch.full((P.m,), float(i), dtype=torch.float64, device=ctx.device) for i in range(20)]
    x_ref, st_ref = P.cg(tol=1e-8, max_iter=500)
    for x in xs + xs[:3]:
        x.zero_()
        _, st = P.cg(x, tol=1e-8, max_iter=500)
        assert st["status"] == 0 and st["iterations"] == st_ref["iterations"]
        assert torch.equal(x, x_ref)
    P.close()


def test_cg_breakdown_on_indefinite_matrix(ctx):
    from paper_1505_08023_amd.mfe import Problem
    d = ctx.device
    # diag(1, -1): p.Ap = 0 for b = (1, 1)
    ptr = torch.tensor([0, 1, 2], dtype=torch.int32, device=d)
    col = torch.tensor([0, 1], dtype=torch.int32, device=d)
    val = torch.tensor([1.0, -1.0], dtype=torch.float64, device=d)
    b = torch.tensor([1.0, 1.0], dtype=torch.float64, device=d)
    P = Problem.from_csr(ctx, ptr, col, val, b)
    x, st = P.cg(tol=1e-10, max_iter=10, fmt="csr", raise_on_breakdown=False)
    assert st["status"] == -4 and st["iterations"] == 0


def test_context_destroy_releases_attached_objects():
    """mfe_ctx_destroy destroys the problems, batches and networks still
    attached to the context (C callers need not destroy them first)."""
    import ctypes
    from paper_1505_08023_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    _lib.check(lib.mfe_ctx_create(0, None, _lib.mfe_alloc_fn(), _lib.mfe_free_fn(), None, ctypes.byref(h)),
               "mfe_ctx_create")
    p, b, n = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    _lib.check(lib.mfe_problem_create(h, 4, 4, 4, None, None, 3, 1, ctypes.byref(p)), "mfe_problem_create")
    sizes = (ctypes.c_int32 * 6)(3, 4, 5, 4, 4, 4)
    _lib.check(lib.mfe_batch_create(h, 2, sizes, None, 3, 1, ctypes.byref(b)), "mfe_batch_create")
    _lib.check(lib.mfe_net_create(h, 9, 1, ctypes.byref(n)), "mfe_net_create")
    assert lib.mfe_ctx_destroy(h) == 0
