"""CG parity at the full bar, from a start on which it is well posed.

After the symmetric elimination of the Dirichlet values (Sec. 1 boundary
conditions) the matrix has A_DF = A_FD = 0 and A_DD = I.  Starting from
x0 = g on the Dirichlet nodes and 0 on the free ones makes the residual
vanish exactly on the Dirichlet rows (r_D = b_D - x0_D = g - g = 0), and no
later step brings it back, since A p keeps that block zero.  The isolated
eigenvalue 1 of the identity rows then never enters the Krylov space, and
the rounding differences of two correct implementations stay at the level
of the summation order instead of being amplified there (from x0 = 0 they
part ways after a few iterations; see test_gpu_core).  From this start the
GPU must match the oracle's implementation of the same recurrence to:

  iteration counts within 1;
  the first 20 recurrence residuals ||r_k||/||b|| within 1e-10 relative,
  and every later common entry within 1e-8 relative;
  both reach the tolerance; solutions within the lambda_min bound.

Plain CG, single-reduction CG and Jacobi-preconditioned CG at 20^3,
17 x 9 x 23 and 64^3 in both formats, 128^3 capped at 200 iterations, and a
batch of uneven meshes with random face values (each system against its own
oracle solve).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1505_08023_amd import inputs
from test_gpu_core import check_solution_gap, mesh_problem, np_

pytestmark = pytest.mark.gpu

VARIANTS = {"cg": oracle.cg, "single_reduction": oracle.cg_single_reduction, "jacobi": oracle.cg_jacobi}


@pytest.fixture(scope="module")
def ctx():
    from paper_1505_08023_amd.mfe import Context
    c = Context(0)
    yield c
    c.close()


def boundary_start(N, face_vals=None):
    d, g = oracle.boundary(*N, face_vals=face_vals)
    return np.where(d, g, 0.0)


def check_history(h, hr, first=20):
    n = min(len(h), len(hr))
    k = min(first + 1, n)  # k = 0..first
    rel = np.abs(h[:n] - hr[:n]) / hr[:n]
    assert np.all(rel[:k] <= 1e-10), (int(np.argmax(rel[:k])), float(rel[:k].max()))
    assert np.all(rel <= 1e-8), (int(np.argmax(rel)), float(rel.max()))
    return float(rel.max())


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
@pytest.mark.parametrize("N", [(20, 20, 20), (17, 9, 23), (24, 24, 24), (64, 64, 64)])
def test_cg_from_boundary_start_matches_oracle(ctx, N, fmt, variant):
    print("boundary start", variant, N, fmt, flush=True)
    tol, cap = 1e-8, 1000
    A = oracle.assemble(*N)
    x0 = boundary_start(N)
    ref = VARIANTS[variant](A, x0=x0, tol=tol, max_iter=cap, history=True)
    P = mesh_problem(ctx, N)
    x, st = P.cg(x=torch.tensor(x0, device=ctx.device), tol=tol, max_iter=cap, fmt=fmt, history=True,
                 variant=variant)
    assert ref["status"] == oracle.OK and st["status"] == 0
    assert abs(st["iterations"] - ref["iterations"]) <= 1, (st["iterations"], ref["iterations"])
    assert st["rel_res_true"] <= tol and st["rel_res_recurrence"] <= tol
    worst = check_history(st["history"].numpy(), ref["history"])
    gap, bound = check_solution_gap(np_(x), ref, st, N, A)
    print(variant, N, fmt, "its", st["iterations"], ref["iterations"], "worst history gap", worst,
          "solution gap", gap, "bound", bound)
    P.close()


def test_cg_128_capped_from_boundary_start(ctx):
    """128^3, FP64, both formats, capped at 200 iterations, from x0 = g (it
    reaches 1e-8 in 187): the whole residual history and the final true
    residual against the oracle's."""
    N = (128, 128, 128)
    A = oracle.assemble(*N)
    x0 = boundary_start(N)
    ref = oracle.cg(A, x0=x0, tol=1e-8, max_iter=200, history=True)
    assert ref["status"] == oracle.OK and ref["iterations"] < 200
    P = mesh_problem(ctx, N)
    for fmt in ("csr", "bcrs13"):
        print("128^3 boundary start", fmt, flush=True)
        x, st = P.cg(x=torch.tensor(x0, device=ctx.device), tol=1e-8, max_iter=200, fmt=fmt, history=True)
        assert abs(st["iterations"] - ref["iterations"]) <= 1 and st["status"] == 0
        worst = check_history(st["history"].numpy(), ref["history"])
        if st["iterations"] == ref["iterations"]:
            assert abs(st["rel_res_true"] / ref["rel_res_true"] - 1) <= 1e-6, (st["rel_res_true"], ref["rel_res_true"])
        gap, bound = check_solution_gap(np_(x), ref, st, N, A)
        print("128^3", fmt, "worst history gap", worst, "true res", st["rel_res_true"], ref["rel_res_true"],
              "gap", gap, "bound", bound)
    P.close()


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
def test_batch_cg_from_boundary_start(ctx, fmt):
    """Each system of a batch of uneven meshes with random face values, from
    its own x0 = g, against its own oracle solve from the same start: counts
    within 1 (the batch reports no residual history)."""
    from paper_1505_08023_amd.mfe import Batch
    sizes, faces = inputs.batched_meshes(nsys=9, lo=3, hi=24, seed=4)
    B = Batch(ctx, sizes, faces)
    off = B.row_offsets
    x0 = np.zeros(off[-1])
    refs = []
    for j, (N, fv) in enumerate(zip(sizes, faces)):
        N = tuple(int(n) for n in N)
        xs = boundary_start(N, fv)
        x0[off[j]:off[j + 1]] = xs
        A = oracle.assemble(*N, face_vals=fv)
        refs.append((N, A, oracle.cg(A, x0=xs, tol=1e-8, max_iter=5000)))
    x, stats = B.cg(x=torch.tensor(x0, device=ctx.device), tol=1e-8, max_iter=5000, fmt=fmt)
    x = np_(x)
    for j, (N, A, ref) in enumerate(refs):
        st = stats[j]
        assert st["status"] == 0 and st["rel_res_true"] <= 1e-8, (j, st)
        assert abs(st["iterations"] - ref["iterations"]) <= 1, (j, N, st["iterations"], ref["iterations"])
        check_solution_gap(x[off[j]:off[j + 1]], ref, st, N, A)
    B.close()
