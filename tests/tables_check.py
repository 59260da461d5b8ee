"""Bit-exact comparison of the library's index tables with the oracle's
(shared by the GPU parity tests)."""
import numpy as np

import oracle


def _morton_key(cells, M):
    x, y, z = cells % M, (cells // M) % M, cells // (M * M)
    key = np.zeros_like(cells)
    for b in range(max(1, int(M - 1).bit_length())):
        key |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return key


def assert_tables_equal(t, ref: oracle.Tables):
    assert np.array_equal(t["cell_pkg"].view(np.uint32), ref.cell_pkg)
    assert np.array_equal(t["pkg_cell"].view(np.uint32), ref.pkg_cell)
    assert np.array_equal(t["pkg_type"], ref.pkg_type)
    assert np.array_equal(t["pkg_nbr"].view(np.uint32), ref.nbr)
    core = np.nonzero(ref.pkg_type == 1)[0].astype(np.uint32)
    assert np.array_equal(t["core_list"].view(np.uint32), core)
    # sweep order: every activated package once, in Morton order of its cell
    cells = ref.pkg_cell[2:].astype(np.int64)
    order = np.argsort(_morton_key(cells, ref.M), kind="stable") + 2
    assert np.array_equal(t["sweep_order"].view(np.uint32), order.astype(np.uint32))
