"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own arithmetic: the element matrix is
computed by Gauss quadrature in the oracle and checked against the
tensor-product closed form here; the assembled matrix against the stencil
and counting formulas; the solver against dense LAPACK solves, the
finite-element patch test, linearity, symmetry, the maximum principle and
the separation-of-variables series.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def closed_form_element(hx, hy, hz):
    """K_ab = (hy hz/hx) s_x m_y m_z + (hx hz/hy) m_x s_y m_z + (hx hy/hz) m_x m_y s_z,
    with 1-D stiffness s = +1 (same node) / -1 and 1-D mass m = 1/3 / 1/6."""
    K = np.zeros((8, 8))
    for a, b in itertools.product(range(8), range(8)):
        f = [(a >> d) & 1 == (b >> d) & 1 for d in range(3)]
        s = [1.0 if e else -1.0 for e in f]
        mm = [1 / 3 if e else 1 / 6 for e in f]
        K[a, b] = (hy * hz / hx) * s[0] * mm[1] * mm[2] + (hx * hz / hy) * mm[0] * s[1] * mm[2] \
            + (hx * hy / hz) * mm[0] * mm[1] * s[2]
    return K


# ---------------------------------------------------------------- element operator (Sec. 1)

@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (0.05, 0.05, 0.05), (0.1, 0.25, 1 / 3), (1 / 96, 1 / 16, 1 / 50)])
def test_element_matrix_closed_form(h):
    K = oracle.element_matrix(*h)
    Kc = closed_form_element(*h)
    assert np.allclose(K, Kc, rtol=0, atol=1e-15 * np.abs(Kc).max())
    assert np.array_equal(K, K.T)
    assert np.abs(K.sum(axis=1)).max() <= 1e-14 * np.abs(K).max()


def test_element_matrix_cube_values():
    h = 0.125
    K = oracle.element_matrix(h, h, h)
    for a, b in itertools.product(range(8), range(8)):
        nd = bin(a ^ b).count("1")  # 0 same node, 1 edge, 2 face diagonal, 3 body diagonal
        want = {0: h / 3, 1: 0.0, 2: -h / 12, 3: -h / 12}[nd]
        assert abs(K[a, b] - want) <= 1e-16, (a, b)
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-15 and ev[1] > 1e-3  # PSD, only constants in the null space


# ---------------------------------------------------------------- structure (Fig 3.6) and formats (Sec. 3.1)

def sizes(Nx, Ny, Nz):
    nx, ny, nz = Nx + 1, Ny + 1, Nz + 1
    return dict(m=nx * ny * nz, nnz=(3 * nx - 2) * (3 * ny - 2) * (3 * nz - 2),
                nns=nx * (3 * ny - 2) * (3 * nz - 2))


@pytest.mark.parametrize("N", [(1, 1, 1), (2, 3, 4), (3, 3, 3), (7, 5, 6), (20, 20, 20)])
def test_counts(N):
    s = sizes(*N)
    assert oracle.num_rows(*N) == s["m"]
    assert oracle.count_nnz(*N) == s["nnz"]
    A = oracle.assemble(*N, apply_bc=False)
    assert A.ptr[-1] == s["nnz"] and A.ptr[0] == 0 and np.all(np.diff(A.ptr) > 0)
    for i in range(A.m):  # ascending, distinct, in range
        c = A.col[A.ptr[i]:A.ptr[i + 1]]
        assert np.all(np.diff(c) > 0) and c[0] >= 0 and c[-1] < A.m
    jas, offs, bptr = oracle.bcrsvar(A)
    assert bptr[-1] == len(jas) and offs[-1] == A.nnz  # ptr[m] = nns, offsets[nns] = nnz
    lengths = np.diff(offs)
    if N[0] >= 3:
        # one segment per (dy, dz) line; length 3 inside in x, 2 on the x faces
        assert len(jas) == s["nns"]
        nx, ny, nz = N[0] + 1, N[1] + 1, N[2] + 1
        assert np.sum(lengths == 2) == 2 * (3 * ny - 2) * (3 * nz - 2)
        assert np.sum(lengths == 3) == (nx - 2) * (3 * ny - 2) * (3 * nz - 2)
    bptr13, bcol13, bval13 = oracle.bcrs13(A)
    if N[0] >= 2:
        assert len(bcol13) == s["nns"]


def test_golden_sizes():
    """Sizes of the paper-problem meshes used throughout (tests/golden/sizes.json)."""
    with open(os.path.join(GOLDEN, "sizes.json")) as f:
        gold = json.load(f)
    for key, row in gold["meshes"].items():
        N = tuple(row["N"])
        want = sizes(*N)
        assert all(want[k] == row[k] for k in ("m", "nnz", "nns") if k in row)
        if row["m"] < 3_000_000:
            assert oracle.count_nnz(*N) == row["nnz"]


def test_interior_stencil_and_symmetry():
    N = 6
    h = 1.0 / N
    A = oracle.assemble(N, N, N, apply_bc=False)
    D = A.dense()
    assert np.array_equal(D, D.T)
    assert np.abs(D.sum(axis=1)).max() <= 1e-14 * np.abs(np.diag(D)).max()
    n = N + 1
    for (ix, iy, iz) in [(3, 3, 3), (1, 2, 4), (5, 5, 1)]:
        i = ix + n * (iy + n * iz)
        for sx, sy, sz in itertools.product((-1, 0, 1), repeat=3):
            j = (ix + sx) + n * ((iy + sy) + n * (iz + sz))
            nz_ = abs(sx) + abs(sy) + abs(sz)
            want = {0: 32, 1: 0, 2: -2, 3: -1}[nz_] * h / 12
            assert abs(D[i, j] - want) <= 1e-15, (i, j)


# ---------------------------------------------------------------- Dirichlet faces (Sec. 1)

@pytest.mark.parametrize("N", [4, 9])
def test_dirichlet_rhs_and_identity_rows(N):
    h = 1.0 / N
    A = oracle.assemble(N, N, N)
    dirm, g = oracle.boundary(N, N, N)
    n = N + 1
    ix = np.arange(A.m) % n
    free = ~dirm
    # paper BCs: 1 on every node with x = 1 (edges included), 0 on the rest of the surface
    assert np.all(g[dirm & (ix == N)] == 1.0) and np.all(g[dirm & (ix < N)] == 0.0)
    assert np.allclose(A.b[free & (ix == N - 1)], h, rtol=0, atol=1e-15)
    assert np.all(A.b[free & (ix < N - 1)] == 0.0)
    D = A.dense()
    assert np.array_equal(D, D.T)
    for i in np.nonzero(dirm)[0]:
        assert D[i, i] == 1.0 and np.count_nonzero(D[i]) == 1 and A.b[i] == g[i]
    # rows whose whole neighbourhood is free keep a zero row sum
    iy = (np.arange(A.m) // n) % n
    iz = np.arange(A.m) // (n * n)
    deep = (ix >= 2) & (ix <= N - 2) & (iy >= 2) & (iy <= N - 2) & (iz >= 2) & (iz <= N - 2)
    assert np.abs(D[deep].sum(axis=1)).max() <= 1e-15


@pytest.mark.parametrize("N", [(1, 1, 1), (3, 5, 4), (8, 8, 8)])
def test_row_assembly_matches_full_assembly(N):
    m = oracle.num_rows(*N)
    rng = np.random.default_rng(3)
    for kw in (dict(), dict(face_vals=rng.uniform(0, 1, 6)), dict(node_g=rng.uniform(0, 1, m))):
        A = oracle.assemble(*N, **kw)
        rows = np.arange(m)
        got, b = oracle.assemble_rows(*N, rows, **kw)
        assert np.array_equal(b, A.b)
        for i, (c, v) in enumerate(got):
            assert np.array_equal(c, A.col[A.ptr[i]:A.ptr[i + 1]])
            assert np.array_equal(v, A.val[A.ptr[i]:A.ptr[i + 1]])


# ---------------------------------------------------------------- SpMV (Figs 3.1-3.3)

@pytest.mark.parametrize("N", [(1, 1, 1), (2, 2, 2), (3, 4, 2), (4, 4, 4), (2, 5, 3)])
def test_spmv_formats_against_dense(N):
    A = oracle.assemble(*N)
    x = np.random.default_rng(1).uniform(-1, 1, A.m)
    y = oracle.csr_spmv(A, x)
    yd = A.dense() @ x
    scale = np.abs(A.dense()) @ np.abs(x)
    assert np.all(np.abs(y - yd) <= 1e-14 * scale + 1e-300)
    fmt = oracle.bcrsvar(A)
    assert np.array_equal(oracle.bcrsvar_spmv(A, fmt, x), y)
    assert np.array_equal(oracle.bcrsvar_spmv(A, fmt, x, switch=True), y)
    f13 = oracle.bcrs13(A)
    y13 = oracle.bcrs13_spmv(A, f13, x)
    # same columns, same order, padding adds +-0 products only
    assert np.all(y13 == y)
    # every stored entry lands in exactly one slot
    bptr, bcol, bval = f13
    assert np.count_nonzero(bval) == np.count_nonzero(A.val)
    assert np.isclose(bval.sum(), A.val.sum(), rtol=0, atol=1e-12)


# ---------------------------------------------------------------- CG (Sec. 1 CG module)

@pytest.mark.parametrize("N", [(1, 1, 1), (2, 2, 2), (3, 2, 4), (4, 4, 4)])
def test_cg_matches_dense_solve(N):
    A = oracle.assemble(*N)
    r = oracle.cg(A, tol=1e-14, max_iter=500)
    assert r["status"] == oracle.OK
    xs = np.linalg.solve(A.dense(), A.b)
    assert np.linalg.norm(r["x"] - xs) <= 1e-10 * np.linalg.norm(xs)
    assert r["rel_res_true"] <= 1e-13


def test_cg_history_and_stop_rule():
    A = oracle.assemble(20, 20, 20)
    r = oracle.cg(A, tol=1e-8, max_iter=200, history=True)
    h = r["history"]
    assert r["status"] == oracle.OK
    assert h[0] == 1.0  # x0 = 0 so r0 = b
    assert h[-1] <= 1e-8 and np.all(h[:-1] > 1e-8)
    assert len(h) == r["iterations"] + 1
    assert abs(r["rel_res_true"] - r["rel_res_rec"]) <= 1e-10
    capped = oracle.cg(A, tol=1e-8, max_iter=10)
    assert capped["status"] == oracle.NOT_CONVERGED and capped["iterations"] == 10
    zero = oracle.cg(A, tol=1e-8, max_iter=0)
    assert zero["iterations"] == 0 and np.all(zero["x"] == 0)


def krylov_minimiser(A, x0, k):
    """x0 + V y minimising the energy norm of the error over the Krylov space
    K_k(A, r0): the iterate that CG defines after k steps (textbook
    optimality), computed by brute force with a dense orthonormal basis."""
    M = A.dense()
    r0 = A.b - M @ x0
    K = np.empty((A.m, k))
    v = r0 / np.linalg.norm(r0)
    for j in range(k):
        K[:, j] = v
        v = M @ v
        v /= np.linalg.norm(v)
    V, _ = np.linalg.qr(K)
    y = np.linalg.solve(V.T @ M @ V, V.T @ r0)
    return x0 + V @ y


@pytest.mark.parametrize("solver", ["cg", "cg_single_reduction"])
@pytest.mark.parametrize("N", [(2, 2, 2), (3, 2, 4)])
def test_cg_iterates_are_krylov_minimisers(solver, N):
    A = oracle.assemble(*N)
    x0 = np.random.default_rng(1).uniform(-1, 1, A.m)
    for k in (1, 2, 3, 4):
        r = getattr(oracle, solver)(A, x0=x0, tol=0.0, max_iter=k)
        assert r["iterations"] == k and r["status"] == oracle.NOT_CONVERGED
        ref = krylov_minimiser(A, x0, k)
        assert np.linalg.norm(r["x"] - ref) <= 1e-9 * np.linalg.norm(ref), (solver, k)


@pytest.mark.parametrize("N", [(3, 4, 3), (4, 4, 5)])
def test_jacobi_cg_iterates_are_preconditioned_krylov_minimisers(N):
    """Preconditioned CG with M = D: x_k minimises the energy norm of the
    error over x0 + K_k(D^-1 A, D^-1 r0) (brute force, dense basis).  The
    meshes have several free nodes: with one (2^3 elements) D^-1 A = I."""
    A = oracle.assemble(*N)
    M = A.dense()
    dinv = 1.0 / np.diag(M)
    x0 = np.random.default_rng(3).uniform(-1, 1, A.m)
    r0 = A.b - M @ x0
    for k in (1, 2, 3, 4):
        r = oracle.cg_jacobi(A, x0=x0, tol=0.0, max_iter=k)
        assert r["iterations"] == k and r["status"] == oracle.NOT_CONVERGED
        K = np.empty((A.m, k))
        v = dinv * r0
        for j in range(k):
            K[:, j] = v / np.linalg.norm(v)
            v = dinv * (M @ K[:, j])
        V, _ = np.linalg.qr(K)
        ref = x0 + V @ np.linalg.solve(V.T @ M @ V, V.T @ r0)
        assert np.linalg.norm(r["x"] - ref) <= 1e-9 * np.linalg.norm(ref), k


def test_jacobi_cg_special_cases():
    # a diagonal matrix is solved exactly in one step
    d = np.array([2.0, 5.0, 0.5, 7.0])
    D = oracle.CSR(np.arange(5, dtype=np.int64), np.arange(4, dtype=np.int32), d, np.array([1.0, -2.0, 3.0, 0.5]))
    r = oracle.cg_jacobi(D, tol=1e-15, max_iter=5)
    assert r["status"] == oracle.OK and r["iterations"] == 1
    assert np.allclose(r["x"], D.b / d, rtol=1e-15, atol=0)
    # dense solve, patch test, and the Dirichlet outlier gone: fewer iterations than CG
    for N in [(3, 2, 4), (4, 4, 4)]:
        A = oracle.assemble(*N)
        xs = np.linalg.solve(A.dense(), A.b)
        r = oracle.cg_jacobi(A, tol=1e-14, max_iter=500)
        assert r["status"] == oracle.OK and np.linalg.norm(r["x"] - xs) <= 1e-10 * np.linalg.norm(xs)
    Nx, Ny, Nz = 6, 5, 7
    n = np.arange(oracle.num_rows(Nx, Ny, Nz))
    u = 0.1 + 0.5 * (n % (Nx + 1)) / Nx + 0.3 * ((n // (Nx + 1)) % (Ny + 1)) / Ny \
        - 0.4 * (n // ((Nx + 1) * (Ny + 1))) / Nz
    A = oracle.assemble(Nx, Ny, Nz, node_g=u)
    r = oracle.cg_jacobi(A, tol=1e-13, max_iter=2000)
    assert r["status"] == oracle.OK and np.abs(r["x"] - u).max() <= 1e-9
    A = oracle.assemble(20, 20, 20)
    rj = oracle.cg_jacobi(A, tol=1e-8, max_iter=500, history=True)
    rc = oracle.cg(A, tol=1e-8, max_iter=500)
    assert rj["status"] == oracle.OK and rj["history"][0] == 1.0 and rj["rel_res_true"] <= 1e-8
    assert rj["iterations"] <= rc["iterations"]
    # a zero diagonal entry is rejected
    Z = oracle.CSR(np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.array([1.0, 1.0]),
                   np.array([1.0, 1.0]))
    assert oracle.cg_jacobi(Z, tol=1e-8, max_iter=5)["status"] == oracle.EINVAL


@pytest.mark.parametrize("N", [(1, 1, 1), (2, 2, 2), (3, 2, 4), (4, 4, 4)])
def test_single_reduction_cg_matches_dense_solve(N):
    A = oracle.assemble(*N)
    r = oracle.cg_single_reduction(A, tol=1e-14, max_iter=500)
    assert r["status"] == oracle.OK
    xs = np.linalg.solve(A.dense(), A.b)
    assert np.linalg.norm(r["x"] - xs) <= 1e-10 * np.linalg.norm(xs)
    assert r["rel_res_true"] <= 1e-13


def test_single_reduction_cg_stop_rule_and_breakdown():
    A = oracle.assemble(20, 20, 20)
    r = oracle.cg_single_reduction(A, tol=1e-8, max_iter=200, history=True)
    ref = oracle.cg(A, tol=1e-8, max_iter=200, history=True)
    h = r["history"]
    assert r["status"] == oracle.OK and h[0] == 1.0
    assert h[-1] <= 1e-8 and np.all(h[:-1] > 1e-8) and len(h) == r["iterations"] + 1
    # the same Krylov iterates as CG: residual histories agree until rounding separates them
    assert np.all(np.abs(h[:6] - ref["history"][:6]) <= 1e-10 * ref["history"][:6])
    assert abs(r["iterations"] - ref["iterations"]) <= 2
    capped = oracle.cg_single_reduction(A, tol=1e-8, max_iter=10)
    assert capped["status"] == oracle.NOT_CONVERGED and capped["iterations"] == 10
    zero = oracle.cg_single_reduction(A, tol=1e-8, max_iter=0)
    assert zero["iterations"] == 0 and np.all(zero["x"] == 0)
    # diag(1, -1), b = (1, 1): r.Ar = 0 at the first step
    D = oracle.CSR(np.array([0, 1, 2], np.int64), np.array([0, 1], np.int32), np.array([1.0, -1.0]),
                   np.array([1.0, 1.0]))
    assert oracle.cg_single_reduction(D, tol=1e-8, max_iter=5)["status"] == oracle.BREAKDOWN


@pytest.mark.parametrize("N", [(6, 6, 6), (5, 3, 7)])
def test_single_reduction_cg_patch_test(N):
    Nx, Ny, Nz = N
    n = np.arange(oracle.num_rows(*N))
    u = 0.3 + 0.7 * (n % (Nx + 1)) / Nx - 0.2 * ((n // (Nx + 1)) % (Ny + 1)) / Ny \
        + 0.45 * (n // ((Nx + 1) * (Ny + 1))) / Nz
    A = oracle.assemble(*N, node_g=u)
    r = oracle.cg_single_reduction(A, tol=1e-13, max_iter=2000)
    assert r["status"] == oracle.OK and np.abs(r["x"] - u).max() <= 1e-9


@pytest.mark.parametrize("N", [(6, 6, 6), (5, 3, 7), (9, 4, 4)])
def test_patch_test_affine_exact(N):
    """Trilinear elements reproduce affine fields exactly (Galerkin is exact on the FE space)."""
    Nx, Ny, Nz = N
    m = oracle.num_rows(*N)
    n = np.arange(m)
    x = (n % (Nx + 1)) / Nx
    y = ((n // (Nx + 1)) % (Ny + 1)) / Ny
    z = (n // ((Nx + 1) * (Ny + 1))) / Nz
    u = 0.3 + 0.7 * x - 0.2 * y + 0.45 * z
    A = oracle.assemble(*N, node_g=u)
    r = oracle.cg(A, tol=1e-13, max_iter=2000)
    assert r["status"] == oracle.OK
    assert np.abs(r["x"] - u).max() <= 1e-9


def test_constant_and_superposition():
    N = 8
    c = 0.37
    A = oracle.assemble(N, N, N, face_vals=[c] * 6)
    r = oracle.cg(A, tol=1e-13, max_iter=1000)
    assert np.abs(r["x"] - c).max() <= 1e-10
    total = np.zeros(A.m)
    for f in range(6):
        fv = [0.0] * 6
        fv[f] = 1.0
        total += oracle.cg(oracle.assemble(N, N, N, face_vals=fv), tol=1e-13, max_iter=1000)["x"]
    assert np.abs(total - 1.0).max() <= 1e-10


def test_maximum_principle_and_symmetry():
    N = 12
    A = oracle.assemble(N, N, N)
    u = oracle.cg(A, tol=1e-13, max_iter=1000)["x"].reshape(N + 1, N + 1, N + 1)  # [z, y, x]
    assert u.min() >= -1e-12 and u.max() <= 1 + 1e-12
    assert np.abs(u - u[:, ::-1, :]).max() <= 1e-10  # y -> 1 - y
    assert np.abs(u - u[::-1, :, :]).max() <= 1e-10  # z -> 1 - z
    assert np.abs(u - u.transpose(1, 0, 2)).max() <= 1e-10  # y <-> z
    assert np.all(np.diff(u[N // 2, N // 2, :]) > 0)  # increases towards x = 1


# ---------------------------------------------------------------- analytic solution (Sec. 1 verification)

def test_series_identities():
    # superposing the six single-face problems gives 1, and at the centre all six are equal
    assert abs(oracle.analytic_u(0.5, 0.5, 0.5) - 1 / 6) <= 1e-13
    assert oracle.analytic_u(0.0, 0.3, 0.6) == 0.0
    assert abs(oracle.analytic_u(0.4, 0.0, 0.6)) <= 1e-15
    assert abs(oracle.analytic_u(0.4, 0.2, 0.7) - oracle.analytic_u(0.4, 0.8, 0.3)) <= 1e-13
    assert abs(oracle.analytic_u(0.4, 0.2, 0.7) - oracle.analytic_u(0.4, 0.7, 0.2)) <= 1e-13
    # near the x = 1 face the series approaches the face value 1
    assert abs(oracle.analytic_u(0.999, 0.5, 0.5) - 1.0) < 0.01


def test_fe_converges_to_series():
    errs = []
    for N in (8, 16, 32):
        A = oracle.assemble(N, N, N)
        u = oracle.cg(A, tol=1e-12, max_iter=2000)["x"].reshape(N + 1, N + 1, N + 1)
        e = 0.0
        for a, b, c in itertools.product((N // 4, N // 2, 3 * N // 4), repeat=3):
            e = max(e, abs(u[c, b, a] - oracle.analytic_u(a / N, b / N, c / N)))
        errs.append(e)
    assert errs[0] < 0.05
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3  # second order in h


# ---------------------------------------------------------------- mixed precision extension

def test_mixed_keep_direction_fp64_inner_is_cg():
    """Keeping the inner direction across refinement steps, with the inner
    steps in FP64, is one uninterrupted CG in exact arithmetic (the FP64
    residual equals the recursive one).  So after K inner iterations in all
    its iterate is CG's K-th iterate, up to rounding, while the restarting
    form needs more iterations to the same tolerance; a wrong carry of the
    direction (scale s/s_old instead of s_old/s, beta dropped) breaks the
    equality."""
    N = 16
    A = oracle.assemble(N, N, N)
    for inner_tol in (1e-1, 1e-2):
        keep = oracle.cg_mixed(A, tol=1e-10, inner_tol=inner_tol, keep_direction=True, inner_f32=False)
        assert keep["status"] == oracle.OK and keep["outer"] >= 5
        K = keep["inner_iterations"]
        cgk = oracle.cg(A, tol=0.0, max_iter=K)
        assert cgk["iterations"] == K
        scale = np.linalg.norm(cgk["x"])
        assert np.linalg.norm(keep["x"] - cgk["x"]) <= 1e-9 * scale
        restart = oracle.cg_mixed(A, tol=1e-10, inner_tol=inner_tol, inner_f32=False)
        assert restart["status"] == oracle.OK and restart["inner_iterations"] > K


def test_mixed_emulated_fp32_matches_native():
    """orc_cg_mixed_keep's FP32 emulation (FP64 operations on FP32 values,
    each rounded to FP32) gives, with keep_direction off, bitwise the
    restarting solve computed in native FP32."""
    for N in ((8, 8, 8), (9, 5, 7)):
        A = oracle.assemble(*N)
        a = oracle.cg_mixed(A, tol=1e-10)
        b = oracle.cg_mixed(A, tol=1e-10, emulated=True)
        assert np.array_equal(a["x"], b["x"]) and a["inner_iterations"] == b["inner_iterations"]


def test_mixed_keep_direction_fp32_reaches_tolerance_in_fewer_iterations():
    N = 24
    A = oracle.assemble(N, N, N)
    ref = oracle.cg(A, tol=1e-13, max_iter=2000)["x"]
    keep = oracle.cg_mixed(A, tol=1e-10, inner_tol=1e-2, keep_direction=True)
    restart = oracle.cg_mixed(A, tol=1e-10, inner_tol=1e-2)
    assert keep["status"] == oracle.OK and keep["rel_res_true"] <= 1e-10
    assert keep["inner_iterations"] < restart["inner_iterations"]
    assert np.linalg.norm(keep["x"] - ref) <= 1e-8 * np.linalg.norm(ref)


def test_mixed_precision_reaches_fp64_accuracy():
    N = 16
    A = oracle.assemble(N, N, N)
    ref = oracle.cg(A, tol=1e-13, max_iter=2000)["x"]
    r = oracle.cg_mixed(A, tol=1e-10, inner_tol=1e-4)
    assert r["status"] == oracle.OK and r["rel_res_true"] <= 1e-10
    assert r["outer"] >= 2  # FP32 alone cannot reach 1e-10
    assert np.linalg.norm(r["x"] - ref) <= 1e-8 * np.linalg.norm(ref)


def test_mixed_safeguard_last_inner_tolerance_reduces_to_cg():
    """The last-step inner tolerance: with the inner steps in FP64, a zero
    start (s = ||b||) and an inner tolerance tighter than the target, the
    first inner solve only has to reach tol ||b|| / (2 s) = tol / 2, so it
    is plain CG on b / ||b|| to tol / 2: one refinement step of exactly CG's
    iteration count to tol / 2.  On these meshes CG to tol stops one
    iteration earlier, so a target off by the factor 2 fails the count; no
    residual of the history lies within rounding of tol / 2.  Without the
    safeguard the inner solve goes on to the tighter inner tolerance."""
    for N in ((12, 12, 12), (9, 14, 7)):
        A = oracle.assemble(*N)
        tol = 1e-8
        r = oracle.cg_mixed(A, tol=tol, inner_tol=1e-13, inner_f32=False, safeguards=True)
        plain = oracle.cg(A, tol=tol / 2, max_iter=2000, history=True)
        assert oracle.cg(A, tol=tol, max_iter=2000)["iterations"] < plain["iterations"]
        assert np.all(np.abs(plain["history"] / (tol / 2) - 1) > 1e-6)
        assert r["status"] == oracle.OK and r["outer"] == 1 and r["fallback_iterations"] == 0
        assert r["inner_iterations"] == plain["iterations"], (r["inner_iterations"], plain["iterations"])
        assert r["rel_res_true"] <= tol
        tight = oracle.cg_mixed(A, tol=tol, inner_tol=1e-13, inner_f32=False)
        assert tight["inner_iterations"] > r["inner_iterations"] + 5


def test_mixed_safeguard_fallback_is_fp64_cg_from_the_refined_iterate():
    """The FP64 fallback: with one inner iteration per refinement step and
    FP64 inner steps, each step is one steepest-descent step on A x = b
    (x += (r.r / r.Ar) r from the current residual r).  At 14^3 the first
    such step cuts the residual to 5 % of ||b|| and the second leaves 59 % of
    it (ratios computed here independently, both far from the halving
    threshold), so the refinement hands over after two steps, and the rest is
    plain CG from the second steepest-descent iterate: the same iteration
    count within 1 and the same solution within the tolerance bound.  With
    the default inner tolerance the fallback does not run."""
    N = (14, 14, 14)
    A = oracle.assemble(*N)
    M = A.dense()
    b = A.b
    x = np.zeros(A.m)
    ratios = []
    for _ in range(2):
        r = b - M @ x
        x = x + (r @ r) / (r @ (M @ r)) * r
        ratios.append(np.linalg.norm(b - M @ x) / np.linalg.norm(r))
    assert ratios[0] < 0.4 and ratios[1] > 0.55, ratios
    tol = 1e-8
    res = oracle.cg_mixed(A, tol=tol, inner_tol=1e-4, max_outer=50, max_inner=1, inner_f32=False, safeguards=True)
    assert res["outer"] == 2 and res["inner_iterations"] == 2 and res["fallback_iterations"] > 0
    ref = oracle.cg(A, x0=x, tol=tol, max_iter=50)
    assert res["status"] == ref["status"] == oracle.OK
    assert abs(res["fallback_iterations"] - ref["iterations"]) <= 1
    assert res["rel_res_true"] <= tol
    assert np.linalg.norm(res["x"] - ref["x"]) <= 4 * tol * np.linalg.norm(b) / min(np.linalg.eigvalsh(M))
    # the same with FP32 inner steps hands over at the same step and still meets the tolerance
    r32 = oracle.cg_mixed(A, tol=tol, inner_tol=1e-4, max_inner=1, safeguards=True)
    assert r32["outer"] == 2 and r32["fallback_iterations"] > 0 and r32["rel_res_true"] <= tol
    # the cap of the fallback is max_inner * max_outer
    capped = oracle.cg_mixed(A, tol=tol, max_outer=3, max_inner=1, inner_f32=False, safeguards=True)
    assert capped["status"] == oracle.NOT_CONVERGED and capped["fallback_iterations"] == 3
    # the default inner tolerance halves the residual at every step: no fallback
    d = oracle.cg_mixed(A, tol=1e-10, safeguards=True)
    assert d["status"] == oracle.OK and d["fallback_iterations"] == 0 and d["outer"] >= 2
