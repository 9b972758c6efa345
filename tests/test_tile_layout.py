"""Host logic: the decoder of tiled list entries used by the GPU tests.

`tests/gpu_util.tile_slots` maps a tiled entry (16 x the partner's index in
the staged neighbourhood of the key's tile) back to a slot from the layout the
C header states.  Here it is checked against an independent enumeration: for
every key cell and each of its 27 neighbour cells, the staged indices of that
neighbour's particles are found by walking the tile's columns and runs cell
by cell, and decoding them must give the neighbour's slots in order.  Random
cell occupancies (with empty cells), runs that wrap the box in z at either
end, 3-cell axes and tile lengths from 1 to nz - 2 are covered.
"""

import itertools

import numpy as np
import pytest

from tests import gpu_util as G


def _staged_index(start, count, nc, tc, key_cell, neighbour):
    """Index of the neighbour cell's first particle in the staged copy of the
    key cell's tile, by walking the runs cell by cell."""
    nx, ny, nz = nc
    cx, cy, cz = key_cell
    z0 = (cz // tc) * tc
    z1 = min(z0 + tc, nz)
    idx = 0
    for col in range(9):
        X, Y = (cx + col // 3 - 1) % nx, (cy + col % 3 - 1) % ny
        for z in range(z0 - 1, z1 + 1):
            cell = (X * ny + Y) * nz + z % nz
            # the run position of the neighbour is its unwrapped z
            if col == neighbour[0] and z == neighbour[1]:
                return idx
            idx += int(count[cell])
    raise AssertionError("neighbour not in the tile's runs")


@pytest.mark.parametrize("nc,tc_req,mean,seed", [
    ((3, 3, 3), 5, 3.0, 0), ((4, 3, 5), 2, 2.0, 1), ((3, 4, 7), 3, 5.0, 2), ((5, 5, 9), 4, 1.0, 3),
    ((3, 3, 12), 5, 4.0, 4), ((6, 5, 13), 20, 2.5, 5), ((7, 3, 4), 1, 6.0, 6),
])
def test_tile_slots_decodes_every_neighbour(nc, tc_req, mean, seed):
    nx, ny, nz = nc
    rng = np.random.default_rng(seed)
    ncell = nx * ny * nz
    count = rng.poisson(mean, ncell).astype(np.int64)
    count[rng.random(ncell) < 0.15] = 0
    start = np.concatenate([[0], np.cumsum(count)[:-1]])
    tc = max(1, min(tc_req, nz - 2))
    keys, entries, want = [], [], []
    for cx, cy, cz in itertools.product(range(nx), range(ny), range(nz)):
        packed = cx | (cy << 10) | (cz << 20)
        for sx, sy, sz in itertools.product((-1, 0, 1), repeat=3):
            X, Y, Z = (cx + sx) % nx, (cy + sy) % ny, (cz + sz) % nz
            nb = (X * ny + Y) * nz + Z
            col = (sx + 1) * 3 + (sy + 1)
            first = _staged_index(start, count, nc, tc, (cx, cy, cz), (col, cz + sz))
            for i in range(int(count[nb])):
                keys.append(packed)
                entries.append(16 * (first + i))
                want.append(int(start[nb]) + i)
    got = G.tile_slots(start, count, nc, tc, np.asarray(keys), np.asarray(entries))
    assert np.array_equal(got, np.asarray(want))
