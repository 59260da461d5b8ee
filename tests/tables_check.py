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

    # the rank map: cell_pkg of every cell in compact form
    assert np.array_equal(decode_rank_map(t["rank_map"].view(np.uint32), ref.M), ref.cell_pkg)


def _popcount32(v):
    v = v - ((v >> np.uint32(1)) & np.uint32(0x55555555))
    v = (v & np.uint32(0x33333333)) + ((v >> np.uint32(2)) & np.uint32(0x33333333))
    v = (v + (v >> np.uint32(4))) & np.uint32(0x0F0F0F0F)
    return (v * np.uint32(0x01010101)) >> np.uint32(24)


def decode_rank_map(rm, M, rows_per_chunk=2048):
    """cell_pkg [M^3] from the rank map [M*M, ceil(M/32), 4] (uint32)."""
    x = np.arange(M)
    bit = (np.uint32(1) << (x & 31).astype(np.uint32))[None, :]
    out = np.empty(M * M * M, dtype=np.uint32)
    for r0 in range(0, M * M, rows_per_chunk):
        e = rm[r0:r0 + rows_per_chunk][:, x >> 5, :]
        act = (e[..., 0] & bit) != 0
        pop = _popcount32(e[..., 0] & (bit - np.uint32(1)))
        neg = (e[..., 1] & bit) != 0
        ids = np.where(act, np.uint32(2) + e[..., 2] + pop, np.where(neg, np.uint32(0), np.uint32(1)))
        out[r0 * M:(r0 + e.shape[0]) * M] = ids.reshape(-1)
    return out
