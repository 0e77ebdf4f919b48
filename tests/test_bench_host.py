"""Host-side logic of the benchmark: the algorithmic byte counts against the
structure the oracle builds (nnz, 1x3 blocks) and the closed forms."""
import numpy as np
import pytest

import bench
import oracle


def test_spmv_bytes_at_256_cubed():
    # closed forms at 256^3: m = 257^3, nnz = (3*257-2)^3, nb = 257 (3*257-2)^2
    m, nnz, nb = 257 ** 3, 769 ** 3, 257 * 769 ** 2
    assert bench.spmv_bytes("csr", m, nnz, nb) == 5_796_571_172
    assert bench.spmv_bytes("bcrs13", m, nnz, nb) == 4_594_925_620
    assert oracle.num_rows(256, 256, 256) == m and oracle.count_nnz(256, 256, 256) == nnz


@pytest.mark.parametrize("N", [(4, 4, 4), (7, 5, 6), (20, 20, 20)])
def test_block_count_matches_oracle_conversion(N):
    """The 1x3 block count used in the byte formula is the number of blocks
    the oracle's greedy conversion produces: n_x (3 n_y - 2)(3 n_z - 2)."""
    A = oracle.assemble(*N)
    bptr, bcol, bval = oracle.bcrs13(A)
    nx, ny, nz = (n + 1 for n in N)
    assert bptr[-1] == nx * (3 * ny - 2) * (3 * nz - 2)
    by = bench.spmv_bytes("bcrs13", A.m, A.nnz, int(bptr[-1]))
    assert by == 28 * int(bptr[-1]) + 4 * (A.m + 1) + 16 * A.m


def test_multi_gpu_request_is_refused(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
