"""Host models of the 1x3 BCRS slice descriptors (test helpers).

The library forms the column indices of a 64-row slice from a descriptor
when, for every block slot k and row i of the slice, the first column of the
block is i + e_i + d_k with e_i in {0, 1}.  Two independent counts of such
slices are kept here: a direct model over the oracle's 1x3 blocking, and a
closed form for the box mesh.
"""
import numpy as np


def descriptor_slices(bptr, bcol, m):
    """Direct model from the oracle's blocking: a full slice whose longest row
    has 9 blocks (shorter rows padded with their last block's column, as the
    library pads them) in which column(k, row i) - i - e_i is one value per
    slot k.  Returns (slices, their real blocks)."""
    nblk = np.diff(bptr)
    count = blocks = 0
    for s in range(m // 64):
        rows = np.arange(64 * s, 64 * s + 64)
        if nblk[rows].max() != 9:
            continue
        c = np.zeros((64, 9), dtype=np.int64)
        for l, i in enumerate(rows):
            own = bcol[bptr[i]:bptr[i + 1]]
            c[l, :len(own)] = own
            c[l, len(own):] = own[-1] if len(own) else 0
        d = c - rows[:, None]
        e = d[:, 0] - d[:, 0].min()
        if np.all((e == 0) | (e == 1)) and np.all(d - e[:, None] == (d - e[:, None])[0]):
            count += 1
            blocks += int(nblk[rows].sum())
    return count, blocks


def descriptor_slices_closed_form(Nx, Ny, Nz):
    """Box mesh: a row i with 1 <= iy <= Ny-1 and 1 <= iz <= Nz-1 has the
    full 9 blocks, block (dy, dz) starting at i - 1 + dy (Nx+1) + dz (Nx+1)(Ny+1)
    (one column later when ix = 0: shift e = 1).  In plane iz these rows are
    one contiguous range, and every full slice inside it qualifies except
    one ending at the last interior row of the mesh, whose top block is
    moved back by the end-of-matrix rule (a block starts at m - 3 at the
    latest)."""
    nx, nxny = Nx + 1, (Nx + 1) * (Ny + 1)
    count = 0
    for iz in range(1, Nz):
        lo, hi = iz * nxny + nx, iz * nxny + Ny * nx
        if iz == Nz - 1:
            hi -= 1
        count += max(0, hi // 64 - (lo + 63) // 64)
    return count


def csr_descriptor_tiles(ptr, col, m, R=16):
    """CRS wavefront tiles of R rows whose columns the library may form from a
    descriptor, modelled directly on the oracle's CRS: a full tile whose rows
    each hold 27 entries, with column - row per entry the same in every row."""
    count = 0
    for t in range(m // R):
        r0 = t * R
        lo, hi = ptr[r0], ptr[r0 + R]
        if hi - lo != 27 * R or np.any(np.diff(ptr[r0:r0 + R + 1]) != 27):
            continue
        d = col[lo:hi].astype(np.int64).reshape(R, 27) - np.arange(r0, r0 + R)[:, None]
        if np.all(d == d[0]):
            count += 1
    return count


def csr_descriptor_tiles_closed_form(Nx, Ny, Nz, R=16):
    """Box mesh: the rows with all 27 neighbours (1 <= ix <= Nx-1 and the same
    for y and z) form one run of Nx-1 consecutive rows per interior x-line;
    every R-row tile inside such a run qualifies and no other tile does."""
    nx, nxny = Nx + 1, (Nx + 1) * (Ny + 1)
    count = 0
    for iz in range(1, Nz):
        for iy in range(1, Ny):
            lo = iz * nxny + iy * nx + 1
            hi = lo + Nx - 1
            count += max(0, hi // R - (lo + R - 1) // R)
    return count


def csr_groups(ptr, col, m, N):
    """The CRS product's group walk of a mesh problem, modelled on the
    oracle's CRS: full rows (27 entries, column - row = the mesh's 27
    neighbour offsets in ascending order) in runs of consecutive rows, each
    run cut into groups of at most 64; the other rows packed 16 to an item in
    row order, an item closed when 16 rows are pending before the next run
    (or at the end).  Returns (items, groups, group_rows, other_rows), all 0
    when no row is full."""
    Nx, Ny, Nz = N
    nx, nxy = Nx + 1, (Nx + 1) * (Ny + 1)
    off = np.array([dx + nx * dy + nxy * dz for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    full = np.zeros(m, bool)
    cnt = np.diff(ptr)
    for i in np.nonzero(cnt == 27)[0]:
        full[i] = np.array_equal(col[ptr[i]:ptr[i] + 27].astype(np.int64) - i, off)
    items = groups = grows = pending = 0
    i = 0
    while i < m:
        if full[i]:
            j = i
            while j < m and full[j]:
                j += 1
            items += pending // 16
            pending %= 16
            g = (j - i + 63) // 64
            items += g
            groups += g
            grows += j - i
            i = j
        else:
            pending += 1
            i += 1
    items += (pending + 15) // 16
    if grows == 0:
        return 0, 0, 0, 0  # no full rows: the product walks wavefront tiles instead
    return items, groups, grows, m - grows


def csr_groups_closed_form(Nx, Ny, Nz):
    """Box mesh: one run of Nx - 1 full rows per interior x-line, so
    ceil((Nx - 1) / 64) groups each and (Nx-1)(Ny-1)(Nz-1) group rows."""
    if min(Nx, Ny, Nz) < 2:
        return 0, 0
    return (Ny - 1) * (Nz - 1) * ((Nx - 1 + 63) // 64), (Nx - 1) * (Ny - 1) * (Nz - 1)
