"""GPU parity of the CG variants against the oracle's implementations of
the same recurrences: single-reduction (Chronopoulos-Gear) CG and
Jacobi-preconditioned CG.

Like plain CG, two correct implementations of the recurrence part ways at
the residual bumps caused by the isolated eigenvalue 1 of the Dirichlet
identity rows, so the bar is: both converge under the same stopping rule,
iteration counts within 2, the first residual-history entries within 1e-10
relative, and ||x_gpu - x_oracle|| within the bound set by both true
residuals and the smallest eigenvalue (see test_gpu_core.check_solution_gap).
"""
import numpy as np
import pytest
import torch

import oracle
from test_gpu_core import check_solution_gap, mesh_problem, np_

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1505_08023_amd.mfe import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
@pytest.mark.parametrize("N", [(4, 4, 4), (20, 20, 20), (17, 9, 23)])
def test_single_reduction_matches_oracle(ctx, N, fmt):
    print("single-reduction cg", N, fmt, flush=True)
    tol, cap = 1e-8, 300
    A = oracle.assemble(*N)
    ref = oracle.cg_single_reduction(A, tol=tol, max_iter=cap, history=True)
    P = mesh_problem(ctx, N)
    x, st = P.cg(tol=tol, max_iter=cap, fmt=fmt, history=True, variant="single_reduction")
    x = np_(x)
    assert ref["status"] == oracle.OK and st["status"] == 0
    assert abs(st["iterations"] - ref["iterations"]) <= 2
    assert st["rel_res_true"] <= tol and st["rel_res_recurrence"] <= tol
    assert st["spmv_count"] == st["iterations"] + 3  # start residual, loop (its + 1), true residual
    h, hr = st["history"].numpy(), ref["history"]
    k = min(4, len(h), len(hr))
    assert np.all(np.abs(h[:k] - hr[:k]) <= 1e-10 * hr[:k])
    check_solution_gap(x, ref, st, N, A)
    x2, st2 = P.cg(tol=tol, max_iter=cap, fmt=fmt, variant="single_reduction")
    assert np.array_equal(np_(x2), x) and st2["iterations"] == st["iterations"]
    P.close()


def test_single_reduction_edge_cases(ctx):
    N = (6, 6, 6)
    P = mesh_problem(ctx, N)
    sr = dict(variant="single_reduction")
    x, st = P.cg(tol=1e-8, max_iter=0, **sr)
    assert st["iterations"] == 0 and st["status"] == 1 and float(x.abs().max()) == 0.0
    x, st = P.cg(tol=2.0, max_iter=10, **sr)
    assert st["iterations"] == 0 and st["status"] == 0
    Z = mesh_problem(ctx, N, face_vals=[0.0] * 6)
    x, st = Z.cg(x=torch.ones(Z.m, dtype=torch.float64, device=ctx.device), tol=1e-8, max_iter=10, **sr)
    assert st["status"] == 0 and float(x.abs().max()) == 0.0
    A = oracle.assemble(*N)
    ref = oracle.cg_single_reduction(A, tol=1e-12, max_iter=7, history=True)
    x, st = P.cg(tol=1e-12, max_iter=7, history=True, **sr)
    assert st["status"] == 1 and st["iterations"] == 7 and ref["status"] == oracle.NOT_CONVERGED
    h, hr = st["history"].numpy(), ref["history"]
    assert len(h) == 8 and np.all(np.abs(h[:4] - hr[:4]) <= 1e-10 * hr[:4])
    check_solution_gap(np_(x), ref, st, N, A)
    # a nonzero start: the same stopping rule on ||b - A x0||
    x0 = torch.tensor(np.random.default_rng(2).uniform(0, 1, P.m), device=ctx.device)
    ref0 = oracle.cg_single_reduction(A, x0=np_(x0), tol=1e-8, max_iter=300)
    x, st = P.cg(x=x0, tol=1e-8, max_iter=300, **sr)
    assert st["status"] == 0 and abs(st["iterations"] - ref0["iterations"]) <= 2
    P.close()
    Z.close()


def test_single_reduction_breakdown(ctx):
    from paper_1505_08023_amd.mfe import Problem
    d = ctx.device
    # diag(1, -1), b = (1, 1): r.Ar = 0 at the first update
    P = Problem.from_csr(ctx, torch.tensor([0, 1, 2], dtype=torch.int32, device=d),
                         torch.tensor([0, 1], dtype=torch.int32, device=d),
                         torch.tensor([1.0, -1.0], dtype=torch.float64, device=d),
                         torch.tensor([1.0, 1.0], dtype=torch.float64, device=d))
    x, st = P.cg(tol=1e-10, max_iter=10, fmt="csr", raise_on_breakdown=False, variant="single_reduction")
    assert st["status"] == -4 and st["iterations"] == 0
    P.close()


def test_single_reduction_256_properties(ctx):
    """256^3 to 1e-8 in the benchmark's configuration."""
    N = (256, 256, 256)
    P = mesh_problem(ctx, N, formats=("bcrs13",))
    x, st = P.cg(tol=1e-8, max_iter=5000, fmt="bcrs13", variant="single_reduction")
    assert st["status"] == 0 and st["rel_res_true"] <= 1e-8
    _, st_cg = P.cg(tol=1e-8, max_iter=5000, fmt="bcrs13")
    assert abs(st["iterations"] - st_cg["iterations"]) <= 0.02 * st_cg["iterations"] + 2
    u = x.view(257, 257, 257)
    assert float(u.min()) >= -1e-6 and float(u.max()) <= 1 + 1e-6
    assert abs(float(u[128, 128, 128]) - oracle.analytic_u(0.5, 0.5, 0.5)) <= 1e-4
    print("256^3 single reduction", st["iterations"], "its vs", st_cg["iterations"], flush=True)
    P.close()


# ---------------------------------------------------------------- Jacobi-preconditioned CG

@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
@pytest.mark.parametrize("N", [(4, 4, 4), (20, 20, 20), (17, 9, 23)])
def test_jacobi_matches_oracle(ctx, N, fmt):
    print("jacobi cg", N, fmt, flush=True)
    tol, cap = 1e-8, 300
    A = oracle.assemble(*N)
    ref = oracle.cg_jacobi(A, tol=tol, max_iter=cap, history=True)
    P = mesh_problem(ctx, N)
    x, st = P.cg(tol=tol, max_iter=cap, fmt=fmt, history=True, variant="jacobi")
    x = np_(x)
    assert ref["status"] == oracle.OK and st["status"] == 0
    assert abs(st["iterations"] - ref["iterations"]) <= 2
    assert st["rel_res_true"] <= tol and st["rel_res_recurrence"] <= tol
    h, hr = st["history"].numpy(), ref["history"]
    k = min(4, len(h), len(hr))
    assert np.all(np.abs(h[:k] - hr[:k]) <= 1e-10 * hr[:k])
    check_solution_gap(x, ref, st, N, A)
    x2, st2 = P.cg(tol=tol, max_iter=cap, fmt=fmt, variant="jacobi")
    assert np.array_equal(np_(x2), x) and st2["iterations"] == st["iterations"]
    P.close()


def test_jacobi_edge_cases(ctx):
    from paper_1505_08023_amd._lib import MfeError
    from paper_1505_08023_amd.mfe import Problem
    N = (6, 6, 6)
    P = mesh_problem(ctx, N)
    jac = dict(variant="jacobi")
    x, st = P.cg(tol=1e-8, max_iter=0, **jac)
    assert st["iterations"] == 0 and st["status"] == 1 and float(x.abs().max()) == 0.0
    x, st = P.cg(tol=2.0, max_iter=10, **jac)
    assert st["iterations"] == 0 and st["status"] == 0
    Z = mesh_problem(ctx, N, face_vals=[0.0] * 6)
    x, st = Z.cg(x=torch.ones(Z.m, dtype=torch.float64, device=ctx.device), tol=1e-8, max_iter=10, **jac)
    assert st["status"] == 0 and float(x.abs().max()) == 0.0
    A = oracle.assemble(*N)
    ref = oracle.cg_jacobi(A, tol=1e-12, max_iter=5, history=True)
    x, st = P.cg(tol=1e-12, max_iter=5, history=True, **jac)
    assert st["status"] == 1 and st["iterations"] == 5 and ref["status"] == oracle.NOT_CONVERGED
    h, hr = st["history"].numpy(), ref["history"]
    assert np.all(np.abs(h[:4] - hr[:4]) <= 1e-10 * hr[:4])
    # a diagonal system is solved in one step
    d = ctx.device
    D = Problem.from_csr(ctx, torch.arange(5, dtype=torch.int32, device=d), torch.arange(4, dtype=torch.int32, device=d),
                         torch.tensor([2.0, 5.0, 0.5, 7.0], dtype=torch.float64, device=d),
                         torch.tensor([1.0, -2.0, 3.0, 0.5], dtype=torch.float64, device=d))
    x, st = D.cg(tol=1e-14, max_iter=5, fmt="csr", **jac)
    assert st["status"] == 0 and st["iterations"] == 1
    assert np.allclose(np_(x), [0.5, -0.4, 6.0, 0.5 / 7.0], rtol=1e-15, atol=0)
    # a zero diagonal entry is rejected before any iteration
    B = Problem.from_csr(ctx, torch.tensor([0, 1, 2], dtype=torch.int32, device=d),
                         torch.tensor([1, 0], dtype=torch.int32, device=d),
                         torch.tensor([1.0, 1.0], dtype=torch.float64, device=d),
                         torch.tensor([1.0, 1.0], dtype=torch.float64, device=d))
    with pytest.raises(MfeError):
        B.cg(tol=1e-8, max_iter=5, fmt="csr", **jac)
    for Q in (P, Z, D, B):
        Q.close()
