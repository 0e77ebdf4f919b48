"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the oracle.

This module holds no arithmetic of the method: it only draws the random
numbers and boundary data that both sides receive as explicit inputs.

Recipes
-------
spmv_vector      x ~ U[-1, 1), numpy default_rng(seed), float64.
batched_meshes   element counts Nx, Ny, Nz i.i.d. uniform integers in [lo, hi]
                 and six face constants uniform in [0, 1) per mesh
                 (order x=0, x=1, y=0, y=1, z=0, z=1), one default_rng(seed).
smooth_faces     per face f: g_f(s,t) = c_f + sum_{k<8} a_fk sin(p_fk pi s) sin(q_fk pi t),
                 p, q uniform integers in {1..4}, a ~ U[0, 0.25], c ~ U[0, 1),
                 (s, t) the face's two in-plane coordinates in axis order.
                 node_field() evaluates those fields on the boundary nodes of
                 a box mesh, a node on several faces taking the first face in
                 the order x=1, x=0, y=1, y=0, z=1, z=0; interior nodes get 0.
"""
import numpy as np

# face order used by every face-indexed array in this package
FACES = ("x0", "x1", "y0", "y1", "z0", "z1")


def spmv_vector(m, seed=0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=m).astype(dtype)


def batched_meshes(nsys=64, lo=16, hi=96, seed=0):
    """Returns (sizes int32[nsys,3], face_vals float64[nsys,6])."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=(nsys, 3)).astype(np.int32)
    faces = rng.uniform(0.0, 1.0, size=(nsys, 6))
    return sizes, faces


def smooth_faces(seed, modes=8):
    """Parameters of the six smooth face fields: dict of arrays, face-major."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, size=6)
    a = rng.uniform(0.0, 0.25, size=(6, modes))
    p = rng.integers(1, 5, size=(6, modes))
    q = rng.integers(1, 5, size=(6, modes))
    return dict(c=c, a=a, p=p, q=q)


def _face_grid(prm, f, s, t):
    """g_f on the tensor grid s (len S) x t (len T), returned as [T, S]."""
    a = prm["a"][f]
    S = np.sin(np.pi * np.outer(prm["p"][f], s))  # [modes, S]
    Tm = np.sin(np.pi * np.outer(prm["q"][f], t))  # [modes, T]
    return prm["c"][f] + (Tm * a[:, None]).T @ S


def node_field(Nx, Ny, Nz, prm):
    """Boundary values on every node of the (Nx+1)(Ny+1)(Nz+1) mesh, x fastest
    (interior nodes 0).  Faces are written in reverse priority order so that a
    node on several faces ends with the first of x=1, x=0, y=1, y=0, z=1, z=0."""
    x = np.arange(Nx + 1) / Nx
    y = np.arange(Ny + 1) / Ny
    z = np.arange(Nz + 1) / Nz
    g = np.zeros((Nz + 1, Ny + 1, Nx + 1))
    g[0, :, :] = _face_grid(prm, 4, x, y)        # z = 0, (s, t) = (x, y)
    g[Nz, :, :] = _face_grid(prm, 5, x, y)       # z = 1
    g[:, 0, :] = _face_grid(prm, 2, x, z)        # y = 0, (s, t) = (x, z)
    g[:, Ny, :] = _face_grid(prm, 3, x, z)       # y = 1
    g[:, :, 0] = _face_grid(prm, 0, y, z)        # x = 0, (s, t) = (y, z)
    g[:, :, Nx] = _face_grid(prm, 1, y, z)       # x = 1
    return g.reshape(-1)
