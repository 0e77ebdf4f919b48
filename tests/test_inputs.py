"""Host-side input generators: the vectorised boundary field against a
per-node evaluation of the same recipe (face priority x=1, x=0, y=1, y=0,
z=1, z=0 at edges and corners; interior nodes zero)."""
import numpy as np

from paper_1505_08023_amd import inputs


def per_node(Nx, Ny, Nz, prm):
    def face(f, s, t):
        return prm["c"][f] + float(np.sum(prm["a"][f] * np.sin(prm["p"][f] * np.pi * s) *
                                          np.sin(prm["q"][f] * np.pi * t)))

    out = np.zeros((Nz + 1) * (Ny + 1) * (Nx + 1))
    for iz in range(Nz + 1):
        for iy in range(Ny + 1):
            for ix in range(Nx + 1):
                x, y, z = ix / Nx, iy / Ny, iz / Nz
                if ix == Nx:
                    v = face(1, y, z)
                elif ix == 0:
                    v = face(0, y, z)
                elif iy == Ny:
                    v = face(3, x, z)
                elif iy == 0:
                    v = face(2, x, z)
                elif iz == Nz:
                    v = face(5, x, y)
                elif iz == 0:
                    v = face(4, x, y)
                else:
                    v = 0.0
                out[ix + (Nx + 1) * (iy + (Ny + 1) * iz)] = v
    return out


def test_node_field_matches_per_node_recipe():
    for seed, (Nx, Ny, Nz) in enumerate([(3, 4, 5), (6, 2, 3), (1, 1, 1)]):
        prm = inputs.smooth_faces(seed)
        assert np.allclose(inputs.node_field(Nx, Ny, Nz, prm), per_node(Nx, Ny, Nz, prm), rtol=0, atol=1e-13)


def test_generators_are_seeded():
    assert np.array_equal(inputs.spmv_vector(100, 3), inputs.spmv_vector(100, 3))
    s1, f1 = inputs.batched_meshes(seed=5)
    s2, f2 = inputs.batched_meshes(seed=5)
    assert np.array_equal(s1, s2) and np.array_equal(f1, f2)
    assert s1.shape == (64, 3) and s1.min() >= 16 and s1.max() <= 96


def test_boundary_mask_marks_the_six_faces():
    """The boundary-node mask of the learned evaluation and the benchmark's
    boundary-only start: against a direct loop over (ix, iy, iz), and the
    count (n+1)^3 - (n-1)^3."""
    from paper_1505_08023_amd.learned import boundary_mask
    for n in (1, 2, 3, 6):
        G = n + 1
        m = boundary_mask(n)
        assert m.shape == (G ** 3,) and m.dtype == bool
        want = [ix in (0, n) or iy in (0, n) or iz in (0, n) for iz in range(G) for iy in range(G) for ix in range(G)]
        assert m.tolist() == want
        assert int(m.sum()) == G ** 3 - max(n - 1, 0) ** 3
