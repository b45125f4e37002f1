"""Shock measurements on a reflecting-wall run: test harness, not the method.

The mirror sits at x = L and the flow enters at x = 0 moving in +x; the
shock the mirror launches runs back toward x = 0.  Densities come from ion
counts (ions per slab over the inflow's ions per slab), the field from the
cell-centred B averaged over the same slabs, so that the GPU run and the
oracle run are measured by the same code from the same kind of data.
"""

import numpy as np


def slab_profiles(x_cells, by, p, slab=8):
    """Density (in units of the inflow density) and mean B_y per slab of
    `slab` cells along x.  x_cells: ion positions in cells; by: B_y at the
    cell centres, x fastest."""
    nx = int(p["nx"])
    ntr = int(np.asarray(by).size // nx)
    nsl = nx // slab
    cnt = np.bincount(np.minimum((np.asarray(x_cells) // slab).astype(np.int64), nsl - 1), minlength=nsl)
    dens = cnt / float(p["ppc"] * slab * ntr)
    b = np.asarray(by, dtype=np.float64).reshape(ntr, nx)[:, : nsl * slab]
    return dens, b.reshape(ntr, nsl, slab).mean(axis=(0, 2))


def shock_state(x_cells, by, p, slab=8, level=2.0, wall_skip=16.0):
    """(front, n2, by2): the distance in d_i from the mirror to the upstream
    edge of the first slab, counted from the inflow, whose density exceeds
    `level`; and the mean density and B_y over the slabs between that front
    and the mirror, leaving out the `wall_skip` d_i next to the mirror."""
    dens, bys = slab_profiles(x_cells, by, p, slab)
    above = np.nonzero(dens > level)[0]
    if above.size == 0:
        return 0.0, float("nan"), float("nan")
    k = int(above[0])
    width = slab * float(p["dx"])
    front = (len(dens) - k) * width
    skip = int(round(wall_skip / width))
    down = slice(k + 1, len(dens) - skip)
    return front, float(dens[down].mean()), float(bys[down].mean())


def by_of(B):
    """B_y at the centres from an (n, 3) array."""
    return np.asarray(B)[:, 1]


def ion_x(parts):
    """Ion x positions in cells from a particle dict (cell + offset)."""
    return parts["cell"][:, 0] + parts["off"][:, 0]
