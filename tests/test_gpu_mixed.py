"""GPU parity of the FP32 SpMV and the FP32-inner / FP64-refinement CG.

  FP32 SpMV   against the FP64 product of the FP32-rounded matrix and vector
              (the exact-input reference for an FP32 kernel): per row
              |d_i| <= 32 eps32 sum_j |A32_ij x32_j| (27 rounded FMAs).
  mixed CG    final FP64 true residual <= tol (1e-10), the oracle's mixed
              solve reaches the same, and the solution is within the
              residual bound of the oracle's FP64 CG solution:
              ||x - x_ref|| <= (||r|| + ||r_ref||) / lambda_min(A).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1505_08023_amd import inputs

pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def ctx():
    from paper_1505_08023_amd.mfe import Context
    c = Context(0)
    yield c
    c.close()


def lam_min(N):
    def s(h):
        return (2 - 2 * math.cos(math.pi * h)) / h

    def m(h):
        return h * (4 + 2 * math.cos(math.pi * h)) / 6
    hx, hy, hz = (1.0 / n for n in N)
    return min(s(hx) * m(hy) * m(hz) + m(hx) * s(hy) * m(hz) + m(hx) * m(hy) * s(hz), 1.0)


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
@pytest.mark.parametrize("N", [(2, 3, 4), (20, 20, 20), (33, 17, 9), (64, 64, 64)])
def test_spmv_f32(ctx, N, fmt):
    from paper_1505_08023_amd.mfe import Problem
    A = oracle.assemble(*N)
    P = Problem.mesh(ctx, *N, precisions=("f64", "f32"))
    x32 = inputs.spmv_vector(A.m, seed=3, dtype=np.float32)
    a32 = A.val.astype(np.float32).astype(np.float64)
    ref = np.add.reduceat(a32 * x32.astype(np.float64)[A.col], A.ptr[:-1])
    scale = np.add.reduceat(np.abs(a32) * np.abs(x32.astype(np.float64))[A.col], A.ptr[:-1])
    y = P.spmv(torch.tensor(x32, device=ctx.device), fmt=fmt).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(y - ref) <= 32 * EPS32 * scale + 1e-38)
    P.close()


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
@pytest.mark.parametrize("N", [(2, 3, 4), (33, 17, 9), (128, 128, 128)])
def test_spmv_dot_f32(ctx, N, fmt):
    """The fused FP32 product of the inner solves: q row by row as the FP32
    SpMV bar, and p.q (FP64 accumulation) against the FP64 dot of the FP32
    vectors within the rounding of the FP32 rows."""
    from paper_1505_08023_amd.mfe import Problem
    A = oracle.assemble(*N)
    P = Problem.mesh(ctx, *N, precisions=("f64", "f32"))
    x32 = inputs.spmv_vector(A.m, seed=5, dtype=np.float32)
    a32 = A.val.astype(np.float32).astype(np.float64)
    x64 = x32.astype(np.float64)
    ref = np.add.reduceat(a32 * x64[A.col], A.ptr[:-1])
    scale = np.add.reduceat(np.abs(a32) * np.abs(x64)[A.col], A.ptr[:-1])
    q, pq = P.spmv_dot(torch.tensor(x32, device=ctx.device), fmt=fmt)
    assert q.dtype == torch.float32
    q = q.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(q - ref) <= 32 * EPS32 * scale + 1e-38)
    dot_ref = float(x64 @ q)  # the GPU's own FP32 rows, dotted in FP64
    assert abs(float(pq.cpu()) - dot_ref) <= 1e-12 * float(np.abs(x64) @ np.abs(q))
    P.close()


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
@pytest.mark.parametrize("N", [(20, 20, 20), (17, 9, 23)])
def test_mixed_cg_matches_oracle(ctx, N, fmt):
    from paper_1505_08023_amd.mfe import Problem
    tol = 1e-10
    A = oracle.assemble(*N)
    ref64 = oracle.cg(A, tol=1e-13, max_iter=5000)
    refmx = oracle.cg_mixed(A, tol=tol, inner_tol=1e-4)
    assert refmx["status"] == oracle.OK and refmx["rel_res_true"] <= tol
    P = Problem.mesh(ctx, *N, precisions=("f64", "f32"))
    x, st = P.cg_mixed(tol=tol, inner_tol=1e-4, fmt=fmt)
    print("mixed", N, fmt, st, "oracle outer/inner", refmx["outer"], refmx["inner_iterations"])
    assert st["status"] == 0 and st["rel_res_true"] <= tol
    assert st["outer"] >= 2
    bnorm = np.linalg.norm(A.b)
    gap = np.linalg.norm(x.cpu().numpy() - ref64["x"])
    bound = (st["rel_res_true"] + ref64["rel_res_true"]) * bnorm / lam_min(N) + 1e-12
    assert gap <= bound, (gap, bound)
    P.close()


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
@pytest.mark.parametrize("N", [(20, 20, 20), (17, 9, 23)])
def test_mixed_keep_direction_matches_oracle(ctx, N, fmt):
    """The refinement that keeps the inner direction (mfe_cg_mixed_ex):
    reaches 1e-10 as the oracle's form of it does, within the residual bound
    of the FP64 solution, with no more inner iterations than the oracle's
    (up to rounding: the library also loosens the last inner solve to what
    the outer tolerance needs, the oracle keeps inner_tol) and fewer than
    the restarting solve's."""
    from paper_1505_08023_amd.mfe import Problem
    tol = 1e-10
    A = oracle.assemble(*N)
    ref64 = oracle.cg(A, tol=1e-13, max_iter=5000)
    refk = oracle.cg_mixed(A, tol=tol, inner_tol=1e-2, keep_direction=True)
    assert refk["status"] == oracle.OK and refk["rel_res_true"] <= tol
    P = Problem.mesh(ctx, *N, precisions=("f64", "f32"))
    x, st = P.cg_mixed(tol=tol, inner_tol=1e-2, fmt=fmt, keep_direction=True)
    _, sr = P.cg_mixed(tol=tol, inner_tol=1e-2, fmt=fmt)
    print("keep", N, fmt, st, "oracle outer/inner", refk["outer"], refk["inner_iterations"], "restart", sr)
    assert st["status"] == 0 and st["rel_res_true"] <= tol and st["outer"] >= 2
    assert st["iterations"] <= refk["inner_iterations"] + max(4, 0.1 * refk["inner_iterations"])
    assert st["iterations"] < sr["iterations"]
    bnorm = np.linalg.norm(A.b)
    gap = np.linalg.norm(x.cpu().numpy() - ref64["x"])
    bound = (st["rel_res_true"] + ref64["rel_res_true"]) * bnorm / lam_min(N) + 1e-12
    assert gap <= bound, (gap, bound)
    P.close()


def test_mixed_keep_direction_warm_and_flags(ctx):
    """MFE_MIXED_WARM with the kept direction: a guess closer than zero is
    kept and saves inner iterations; a poor one is rejected and the solve is
    bitwise the zero-start one; unknown flag bits are refused."""
    import ctypes
    from paper_1505_08023_amd._lib import MFE_EINVAL, mfe_cg_stats
    from paper_1505_08023_amd.mfe import Problem, _ptr
    N = (24, 24, 24)
    P = Problem.mesh(ctx, *N, precisions=("f64", "f32"))
    x_zero, st_zero = P.cg_mixed(tol=1e-8, inner_tol=1e-2, keep_direction=True)
    ref = oracle.cg(oracle.assemble(*N), tol=1e-12, max_iter=1000)["x"]
    rng = np.random.default_rng(11)
    guess = ref + 1e-4 * rng.standard_normal(P.m)
    dirichlet = oracle.boundary(*N)[0] != 0
    guess[dirichlet] = ref[dirichlet]
    x, st = P.cg_mixed(x=torch.tensor(guess, device=ctx.device), tol=1e-8, inner_tol=1e-2, warm=True,
                       keep_direction=True)
    assert st["guess_rejected"] == 0 and st["rel_res_true"] <= 1e-8
    assert st["iterations"] < st_zero["iterations"]
    bad = torch.tensor(1e3 * rng.standard_normal(P.m), device=ctx.device)
    x, st = P.cg_mixed(x=bad, tol=1e-8, inner_tol=1e-2, warm=True, keep_direction=True)
    assert st["guess_rejected"] == 1 and st["iterations"] == st_zero["iterations"]
    assert torch.equal(x, x_zero)
    xs = torch.zeros(P.m, dtype=torch.float64, device=ctx.device)
    stt = mfe_cg_stats()
    rc = ctx.lib.mfe_cg_mixed_ex(P.handle, 2, _ptr(xs, torch.float64, P.m, "x"), 1e-8, 1e-2, 10, 100, 4,
                                 ctypes.byref(stt))
    assert rc == MFE_EINVAL
    P.close()


def test_mixed_keep_direction_after_capped_inner_solves(ctx):
    """An inner solve that stops at max_inner is restarted, not continued:
    with every inner solve capped the direction-keeping refinement is bitwise
    the restarting one."""
    from paper_1505_08023_amd.mfe import Problem
    P = Problem.mesh(ctx, 16, 16, 16, precisions=("f64", "f32"))
    # 8 inner iterations gain about two decades here, short of 1e-6: every inner solve is capped
    xa, sa = P.cg_mixed(tol=1e-8, inner_tol=1e-6, max_inner=8, max_outer=200)
    xb, sb = P.cg_mixed(tol=1e-8, inner_tol=1e-6, max_inner=8, max_outer=200, keep_direction=True)
    assert sa["outer"] == sb["outer"] >= 2 and sa["iterations"] == sb["iterations"]
    assert torch.equal(xa, xb)
    P.close()


def test_mixed_cg_128_against_fp64(ctx):
    """128^3: mixed to 1e-10 and FP64 CG to 1e-10 reach the same solution."""
    from paper_1505_08023_amd.mfe import Problem
    N = (128, 128, 128)
    P = Problem.mesh(ctx, *N, precisions=("f64", "f32"))
    xm, sm = P.cg_mixed(tol=1e-10, inner_tol=1e-4)
    xd, sd = P.cg(tol=1e-10, max_iter=20000)
    print("128^3 mixed", sm, "fp64", sd)
    assert sm["status"] == 0 and sm["rel_res_true"] <= 1e-10 and sd["rel_res_true"] <= 1e-10
    bnorm = math.sqrt(129 ** 2 + 127 ** 2 / 128 ** 2)  # ones on x = 1, h next to it
    gap = float(torch.linalg.norm(xm - xd))
    assert gap <= (sm["rel_res_true"] + sd["rel_res_true"]) * bnorm / lam_min(N)
    P.close()


def test_mixed_zero_rhs_and_bad_args(ctx):
    from paper_1505_08023_amd._lib import MfeError
    from paper_1505_08023_amd.mfe import Problem
    P = Problem.mesh(ctx, 6, 6, 6, face_vals=[0.0] * 6, precisions=("f64", "f32"))
    x0 = torch.ones(P.m, dtype=torch.float64, device=ctx.device)
    x, st = P.cg_mixed(x=x0, tol=1e-10)
    assert st["status"] == 0 and float(x.abs().max()) == 0.0
    with pytest.raises(MfeError, match="EINVAL"):
        P.cg_mixed(tol=1e-10, inner_tol=2.0)
    Q = Problem.mesh(ctx, 6, 6, 6)  # no FP32 values built
    with pytest.raises(MfeError, match="EUNSUPPORTED"):
        Q.cg_mixed(tol=1e-10)


@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
def test_mixed_warm_start(ctx, fmt):
    """mfe_cg_mixed_warm keeps a guess closer than x0 = 0 (fewer inner
    iterations, same accuracy) and otherwise solves from zero, bitwise as the
    mixed solve from zero; mfe_cg_mixed never rejects."""
    from paper_1505_08023_amd.mfe import Problem
    N = (20, 20, 20)
    A = oracle.assemble(*N)
    ref = oracle.cg(A, tol=1e-12, max_iter=1000)
    P = Problem.mesh(ctx, *N, precisions=("f64", "f32"))
    x_zero, st_zero = P.cg_mixed(tol=1e-8, fmt=fmt)
    rng = np.random.default_rng(12)
    guess = ref["x"] + 1e-4 * rng.standard_normal(P.m)
    dirichlet = oracle.boundary(*N)[0] != 0
    guess[dirichlet] = ref["x"][dirichlet]
    x, st = P.cg_mixed(x=torch.tensor(guess, device=ctx.device), tol=1e-8, fmt=fmt, warm=True)
    assert st["guess_rejected"] == 0 and st["status"] == 0 and st["rel_res_true"] <= 1e-8
    assert st["iterations"] < st_zero["iterations"]
    bnorm = np.linalg.norm(A.b)
    gap = np.linalg.norm(x.cpu().numpy() - ref["x"])
    assert gap <= (st["rel_res_true"] + ref["rel_res_true"]) * bnorm / lam_min(N) + 1e-12
    bad = torch.tensor(10.0 * rng.standard_normal(P.m), device=ctx.device)
    x, st = P.cg_mixed(x=bad, tol=1e-8, fmt=fmt, warm=True)
    assert st["guess_rejected"] == 1 and st["iterations"] == st_zero["iterations"]
    assert torch.equal(x, x_zero)
    x, st = P.cg_mixed(x=torch.tensor(10.0 * rng.standard_normal(P.m), device=ctx.device), tol=1e-8, fmt=fmt)
    assert st["guess_rejected"] == 0 and st["status"] == 0 and st["rel_res_true"] <= 1e-8
    P.close()
