"""Host-side logic of the benchmark: the algorithmic byte counts against the
structure the oracle builds (nnz, 1x3 blocks) and the closed forms."""
import os

import numpy as np
import pytest

import b13_model
import bench
import oracle


def test_spmv_bytes_at_256_cubed():
    # closed forms at 256^3: m = 257^3, nnz = (3*257-2)^3, nb = 257 (3*257-2)^2
    m, nnz, nb = 257 ** 3, 769 ** 3, 257 * 769 ** 2
    assert bench.spmv_bytes("csr", m, nnz, nb) == 5_796_571_172
    slices = (m + 63) // 64
    assert bench.spmv_bytes("bcrs13", m, nnz, nb) == 28 * nb + 4 * (slices + 1) + 16 * m
    cs = b13_model.descriptor_slices_closed_form(256, 256, 256)
    assert cs == 260_865
    lay = dict(slices=slices, compressed_slices=cs, compressed_blocks=576 * cs)
    # the descriptor slices drop 576 x 4 index bytes for 48 descriptor bytes each
    assert bench.spmv_bytes("bcrs13", m, nnz, nb, layout=lay) == 24 * nb + 4 * (nb - 576 * cs) + 48 * cs \
        + 4 * (slices + 1) + 16 * m == 3_939_576_724
    assert oracle.num_rows(256, 256, 256) == m and oracle.count_nnz(256, 256, 256) == nnz


@pytest.mark.parametrize("N", [(4, 4, 4), (7, 5, 6), (20, 20, 20)])
def test_block_count_matches_oracle_conversion(N):
    """The 1x3 block count used in the byte formula is the number of blocks
    the oracle's greedy conversion produces: n_x (3 n_y - 2)(3 n_z - 2)."""
    A = oracle.assemble(*N)
    bptr, _, _ = oracle.bcrs13(A)
    nx, ny, nz = (n + 1 for n in N)
    assert bptr[-1] == nx * (3 * ny - 2) * (3 * nz - 2)


def test_csr_bytes_with_tile_descriptors_at_256_cubed():
    m, nnz = 257 ** 3, 769 ** 3
    tiles = (m + 15) // 16
    ct = b13_model.csr_descriptor_tiles_closed_form(256, 256, 256)
    assert ct == 975_375
    lay = dict(tile_rows=16, tiles=tiles, compressed_tiles=ct)
    by = bench.spmv_bytes("csr", m, nnz, 0, layout=lay)
    # values; indices of the 85,538 indexed tiles; descriptors; bounds; x, y
    assert by == 8 * nnz + 4 * (nnz - 432 * ct) + 112 * ct + 4 * (tiles + 1) + 4 * (m - 16 * ct) + 16 * m
    assert by < bench.spmv_bytes("csr", m, nnz, 0)


def test_csr_tile_closed_form_matches_assembly():
    """The closed-form count of CRS descriptor tiles against the direct model
    over the oracle's CRS, on meshes with every alignment of x-lines to the
    16-row tiles."""
    rng = np.random.default_rng(3)
    meshes = [(20, 20, 20), (33, 33, 33), (40, 9, 6), (63, 5, 5), (17, 17, 17), (2, 3, 4)] + \
        [tuple(int(v) for v in rng.integers(1, 40, 3)) for _ in range(12)]
    for N in meshes:
        A = oracle.assemble(*N)
        assert b13_model.csr_descriptor_tiles(A.ptr, A.col, A.m) == b13_model.csr_descriptor_tiles_closed_form(*N), N


def test_descriptor_slice_closed_form_matches_blocking():
    """The closed-form count of descriptor slices (used for the 256^3 byte
    count and its GPU check) against the direct model over the oracle's 1x3
    blocking, on meshes with every alignment of lines and planes to the
    64-row slices (including one where a slice ends on the last interior
    row)."""
    rng = np.random.default_rng(1)
    meshes = [(63, 5, 5), (20, 20, 20), (33, 33, 33), (40, 9, 6), (1, 30, 30), (2, 25, 25), (64, 4, 9),
              (7, 40, 3), (127, 3, 3)] + [tuple(int(v) for v in rng.integers(1, 40, 3)) for _ in range(20)]
    for N in meshes:
        A = oracle.assemble(*N)
        bptr, bcol, _ = oracle.bcrs13(A)
        count, blocks = b13_model.descriptor_slices(bptr, bcol, A.m)
        assert count == b13_model.descriptor_slices_closed_form(*N), N
        assert blocks == 576 * count


def test_multi_gpu_request_is_refused(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


def test_algorithmic_bytes_at_256_cubed():
    """The roofline's bytes: every index read, row pointers counted as for
    CRS (12 nnz + 4 (m+1) + 16 m for CRS FP64; 28 nb + 4 (m+1) + 16 m for the
    1x3 BCRS FP64; values at 4 bytes for FP32)."""
    m, nnz, nb = 257 ** 3, 769 ** 3, 257 * 769 ** 2
    assert bench.algorithmic_bytes("bcrs13", m, nnz, nb) == 28 * nb + 4 * (m + 1) + 16 * m == 4_594_925_620
    assert bench.algorithmic_bytes("csr", m, nnz, nb) == 5_796_571_172
    assert bench.algorithmic_bytes("csr", m, nnz, nb, fp=4) == 8 * nnz + 4 * (m + 1) + 8 * m
    assert bench.algorithmic_bytes("bcrs13", m, nnz, nb, fp=4) == 16 * nb + 4 * (m + 1) + 8 * m


def test_csr_group_walk_bytes_and_closed_form():
    """The CRS group walk's moved bytes at 256^3 (every value, 8 bytes per
    work item, 4 per group, 12 per other row and 4 per entry of the other
    rows, x and y once), with the group counts of the closed form checked
    against the model over the oracle's CRS on small meshes."""
    for N in ((20, 20, 20), (33, 33, 33), (40, 9, 6), (70, 3, 4), (65, 5, 5)):
        A = oracle.assemble(*N)
        items, groups, grows, other = b13_model.csr_groups(A.ptr, A.col, A.m, N)
        assert (groups, grows) == b13_model.csr_groups_closed_form(*N), N
        assert grows + other == A.m
    m, nnz = 257 ** 3, 769 ** 3
    groups, grows = b13_model.csr_groups_closed_form(256, 256, 256)
    assert (groups, grows) == (255 * 255 * 4, 255 ** 3)
    other = m - grows
    lay = dict(items=groups + (other + 15) // 16, groups=groups, group_rows=grows, other_rows=other)
    by = bench.spmv_bytes("csr", m, nnz, 0, layout=lay)
    assert by == 8 * nnz + 8 * lay["items"] + 4 * groups + 12 * other + 4 * (nnz - 27 * grows) + 16 * m
    assert by < bench.spmv_bytes("csr", m, nnz, 0)


def test_cpu_baseline_fields_at_a_small_mesh():
    """The CPU baseline as the bench computes it, on a 28^3 mesh (whose CG
    needs more than the 30 iterations timed, so the timed difference of two
    capped solves is 28 iterations): the oracle's own build, the two native
    builds, both products' times and the extrapolation from the GPU solve's
    iteration count."""
    import glob
    import tempfile

    import bench
    before = set(glob.glob(os.path.join(tempfile.gettempdir(), "oracle_timing_*")))
    out = bench.cpu_baseline(28, 57, its=(2, 30), its_omp=(2, 30))
    assert out["kind"] == "oracle" and out["value"] > 0 and out["cores"] == 1
    assert out.get("native_builds_error") is None, out.get("native_builds_error")
    for key in ("native_O3_one_core", "native_O3_all_cores"):
        o = out[key]
        assert o["value"] > 0 and o["spmv_ms"] > 0 and o["bcrs13_spmv_ms"] > 0
        assert abs(o["bcrs13_over_csr_spmv"] - o["spmv_ms"] / o["bcrs13_spmv_ms"]) < 1e-12
    allc = out["native_O3_all_cores"]
    assert abs(allc["time_to_1e-8_s_extrapolated"] - 57 / allc["value"]) < 1e-9
    assert allc["extrapolation"].startswith("57 iterations")
    # the timing builds' temporary directory is removed
    assert set(glob.glob(os.path.join(tempfile.gettempdir(), "oracle_timing_*"))) <= before
