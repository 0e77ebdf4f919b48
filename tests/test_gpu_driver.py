"""The host's graph replay does not change results.

The CG drivers replay captured graphs of 16 iterations and, once a forecast
of the remaining iterations (fitted to the polled residual and seeded with
the rate of the previous solve on the same problem) puts the end near,
graphs of 4.  The stopping test stays on the device, so the iteration count
and every value must be the same whatever lengths the host chose.  A first
solve on a fresh problem runs without a prior rate and a second one with
it, so the two switch to the short graphs at different points (and a solve
capped below one long graph uses only short ones): both must agree bitwise.
"""
import numpy as np
import pytest
import torch

from paper_1505_08023_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1505_08023_amd.mfe import Context
    c = Context(0)
    yield c
    c.close()


def same(a, b):
    return np.array_equal(a.detach().cpu().numpy().view(np.uint64), b.detach().cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("variant", ["cg", "single_reduction", "jacobi"])
@pytest.mark.parametrize("fmt", ["csr", "bcrs13"])
def test_repeated_solves_agree_bitwise(ctx, fmt, variant):
    from paper_1505_08023_amd.mfe import Problem
    print("repeat", variant, fmt, flush=True)
    P = Problem.mesh(ctx, 24, 20, 28)
    runs = []
    for _ in range(3):
        x, st = P.cg(tol=1e-9, max_iter=5000, fmt=fmt, variant=variant, history=True)
        runs.append((x, st))
    (x0, s0), rest = runs[0], runs[1:]
    assert s0["status"] == 0 and s0["rel_res_true"] <= 1e-9
    for x, st in rest:
        assert st["iterations"] == s0["iterations"] and st["spmv_count"] == s0["spmv_count"]
        assert same(x, x0)
        assert np.array_equal(st["history"].numpy(), s0["history"].numpy())
    P.close()


@pytest.mark.parametrize("cap", [1, 3, 4, 5, 17, 33])
def test_capped_solves_stop_at_the_cap(ctx, cap):
    """Caps below, at and just above the short and the long graph length:
    the solve stops at exactly cap iterations, with the same iterate as a
    longer solve's cap-th."""
    from paper_1505_08023_amd.mfe import Problem
    print("cap", cap, flush=True)
    P = Problem.mesh(ctx, 20, 20, 20)
    _, full = P.cg(tol=1e-12, max_iter=5000, history=True)
    assert full["iterations"] > cap
    x, st = P.cg(tol=1e-12, max_iter=cap, history=True, raise_on_breakdown=False)
    assert st["iterations"] == cap
    assert np.array_equal(st["history"].numpy()[:cap + 1], full["history"].numpy()[:cap + 1])
    P.close()


@pytest.mark.parametrize("keep", [False, True])
def test_repeated_mixed_solves_agree_bitwise(ctx, keep):
    from paper_1505_08023_amd.mfe import Problem
    print("mixed repeat", keep, flush=True)
    P = Problem.mesh(ctx, 30, 26, 22, precisions=("f64", "f32"))
    runs = [P.cg_mixed(tol=1e-10, inner_tol=1e-2 if keep else 1e-4, keep_direction=keep) for _ in range(3)]
    (x0, s0) = runs[0]
    assert s0["status"] == 0 and s0["rel_res_true"] <= 1e-10
    for x, st in runs[1:]:
        assert (st["iterations"], st["outer"]) == (s0["iterations"], s0["outer"])
        assert same(x, x0)
    P.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_repeated_batched_solves_agree_bitwise(ctx, mixed):
    """Uneven meshes, so that the small systems stop early and the grid is
    spread over the remaining ones (the batched driver does that at
    multiples of the long graph length only, whatever graphs it launches)."""
    from paper_1505_08023_amd.mfe import Batch
    print("batched repeat", mixed, flush=True)
    sizes, faces = inputs.batched_meshes(nsys=9, lo=3, hi=36, seed=11)
    B = Batch(ctx, sizes, faces, precisions=("f64", "f32") if mixed else ("f64",))
    runs = [(B.cg_mixed(tol=1e-9) if mixed else B.cg(tol=1e-9)) for _ in range(3)]
    x0, s0 = runs[0]
    assert all(s["status"] == 0 for s in s0)
    for x, st in runs[1:]:
        assert [s["iterations"] for s in st] == [s["iterations"] for s in s0]
        assert same(x, x0)
    B.close()
