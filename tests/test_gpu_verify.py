"""Device-side result verification (Sec. 1) against the oracle's series
solution: the series values node by node, the reduced error norms, and the
finite-element error decreasing under refinement."""
import numpy as np
import pytest
import torch

import oracle
from test_gpu_core import mesh_problem, np_

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1505_08023_amd.mfe import Context
    c = Context(0)
    yield c
    c.close()


def node_coords(N):
    Nx, Ny, Nz = N
    n = np.arange(oracle.num_rows(*N))
    return (n % (Nx + 1)) / Nx, ((n // (Nx + 1)) % (Ny + 1)) / Ny, (n // ((Nx + 1) * (Ny + 1))) / Nz


@pytest.mark.parametrize("N,x_max", [((16, 16, 16), 0.75), ((12, 8, 10), 0.5)])
def test_series_values_and_norms_match_oracle(ctx, N, x_max):
    P = mesh_problem(ctx, N)
    x, st = P.cg(tol=1e-12, max_iter=2000)
    v = P.verify_series(x, x_max=x_max, want_u=True)
    u = np_(v["u"])
    X, Y, Z = node_coords(N)
    sel = X <= x_max
    assert np.all(np.isnan(u[~sel])) and not np.any(np.isnan(u[sel]))
    ref = np.array([oracle.analytic_u(a, b, c) for a, b, c in zip(X[sel], Y[sel], Z[sel])])
    assert np.abs(u[sel] - ref).max() <= 1e-13
    e = np_(x)[sel] - ref
    assert v["count"] == sel.sum()
    assert abs(v["max_err"] - np.abs(e).max()) <= 1e-13
    assert abs(v["rms_err"] - np.sqrt(np.mean(e ** 2))) <= 1e-13
    P.close()


def test_fe_error_decreases_under_refinement(ctx):
    errs = []
    for n in (8, 16, 32, 64):
        P = mesh_problem(ctx, (n, n, n), formats=("bcrs13",))
        x, st = P.cg(tol=1e-12, max_iter=5000)
        errs.append(P.verify_series(x, x_max=0.75)["max_err"])
        P.close()
    orders = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    print("max nodal error (x <= 3/4):", errs, "observed orders:", orders)
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_verify_rejects_bad_input(ctx):
    from paper_1505_08023_amd._lib import MfeError
    from paper_1505_08023_amd.mfe import Problem
    P = mesh_problem(ctx, (4, 4, 4))
    x = torch.zeros(P.m, dtype=torch.float64, device=ctx.device)
    for bad in (0.0, 1.0, -0.5):
        with pytest.raises(MfeError):
            P.verify_series(x, x_max=bad)
    d = ctx.device
    Q = Problem.from_csr(ctx, torch.tensor([0, 1], dtype=torch.int32, device=d),
                         torch.tensor([0], dtype=torch.int32, device=d),
                         torch.tensor([1.0], dtype=torch.float64, device=d),
                         torch.tensor([1.0], dtype=torch.float64, device=d))
    with pytest.raises(MfeError):
        Q.verify_series(torch.zeros(1, dtype=torch.float64, device=d))
    P.close()
    Q.close()
