"""mfe_spmv_dot_noalloc, the entry point that allocates no device memory,
against mfe_spmv_dot (the same kernels with context-allocated scratch):
q and p.q bitwise equal, through the C ABI, in both formats, on two calls in
a row with the second on a smaller mesh (the static scratch keeps the first
call's contents), and the FP64 product against the oracle's per-row bar."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1505_08023_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _dp(t):
    return ctypes.c_void_p(t.data_ptr())


def test_spmv_dot_noalloc_matches_spmv_dot():
    from paper_1505_08023_amd.mfe import Context, Problem
    lib = _lib.load()
    ctx = Context(0)
    try:
        for fmt, code in (("bcrs13", _lib.MFE_BCRS13), ("csr", _lib.MFE_CSR)):
            for N in ((24, 20, 22), (9, 7, 5)):  # the second call on a smaller mesh
                print("noalloc", fmt, N, flush=True)
                P = Problem.mesh(ctx, *N)
                A = oracle.assemble(*N)
                x = inputs.spmv_vector(A.m, seed=sum(N))
                p = torch.tensor(x, device=ctx.device)
                q_ref = torch.full_like(p, np.nan)
                q_new = torch.full_like(p, np.nan)
                pq_ref = torch.full((1,), np.nan, dtype=torch.float64, device=ctx.device)
                pq_new = torch.full((1,), np.nan, dtype=torch.float64, device=ctx.device)
                torch.cuda.synchronize()
                _lib.check(lib.mfe_spmv_dot(P.handle, code, _dp(p), _dp(q_ref), _dp(pq_ref), None, None),
                           "mfe_spmv_dot")
                _lib.check(lib.mfe_spmv_dot_noalloc(P.handle, code, _dp(p), _dp(q_new), _dp(pq_new)),
                           "mfe_spmv_dot_noalloc")
                ctx.stream.synchronize()
                qa, qb = q_ref.cpu().numpy(), q_new.cpu().numpy()
                assert np.array_equal(qa.view(np.int64), qb.view(np.int64))
                assert pq_ref.item() == pq_new.item()
                y = oracle.csr_spmv(A, x)
                scale = np.add.reduceat(np.abs(A.val) * np.abs(x[A.col]), A.ptr[:-1])
                assert np.all(np.abs(qb - y) <= 1e-12 * scale + 1e-300)
                assert abs(pq_new.item() - float(np.dot(x, y))) <= 1e-12 * float(np.dot(np.abs(x), scale))
                P.close()
        # argument checks
        assert lib.mfe_spmv_dot_noalloc(None, 1, None, None, None) == _lib.MFE_EINVAL
    finally:
        ctx.close()


def test_spmv_dot_noalloc_python_binding():
    from paper_1505_08023_amd.mfe import Context, Problem
    ctx = Context(0)
    try:
        P = Problem.mesh(ctx, 5, 6, 7)
        x = torch.tensor(inputs.spmv_vector(P.m, seed=3), device=ctx.device)
        q_ref, pq_ref = P.spmv_dot(x)
        q = torch.empty_like(x)
        pq = torch.empty(1, dtype=torch.float64, device=ctx.device)
        P.spmv_dot_noalloc(x, q, pq)
        torch.cuda.synchronize()
        assert torch.equal(q, q_ref) and pq.item() == pq_ref.item()
        P.close()
    finally:
        ctx.close()
