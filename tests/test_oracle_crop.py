"""The oracle's crop harness (used where the full grid is too large for a
dense FP64 oracle): the coarse distances of a sub-box equal the matching
slice of the whole grid, and after n iterations every crop point farther than
n + 5 cells from the crop faces holds exactly the full-grid value (updates
read face neighbours only; activation reaches one coarse cell)."""
import numpy as np

import oracle
import synth


def test_crop_coarse_slice():
    s = synth.displaced_torus(7)
    M, E, o = 64, 20, (30, 12, 25)
    full = synth.coarse_sdf(s, M).reshape(M, M, M)
    crop = synth.coarse_sdf(s, M, origin=o, extent=E).reshape(E, E, E)
    assert np.array_equal(crop, full[o[2]:o[2] + E, o[1]:o[1] + E, o[0]:o[0] + E])


def test_crop_interior_matches_full_grid():
    N, n_iter = 128, 10
    s = synth.sphere((0.5, 0.5, 0.5), 0.3)
    full = oracle.setup(s, N, 0.1, 9)
    oracle.run_plain(full, n_iter)
    o, E = (16, 8, 6), 16
    crop = oracle.setup_crop(s, N, o, E, 0.1, 9)
    oracle.run_plain(crop, n_iter)
    n = 4 * E
    m = n_iter + 5
    r = np.arange(m, n - m)
    i, j, k = np.meshgrid(r, r, r, indexing="ij")
    loc = (i + n * (j + n * k)).ravel()
    glob = (i + 4 * o[0] + N * ((j + 4 * o[1]) + N * (k + 4 * o[2]))).ravel()
    band = np.abs(full.phi[glob]) < 16 * full.h - 1e-12
    assert band.sum() > 1000                      # the surface crosses the interior
    assert np.array_equal(crop.phi[loc], full.phi[glob])
    assert np.array_equal(crop.grad[:, loc], full.grad[:, glob])
    # integral windows reach four more points
    ri = np.arange(m + 4, n - m - 4)
    i, j, k = np.meshgrid(ri, ri, ri, indexing="ij")
    loc = (i + n * (j + n * k)).ravel()
    glob = (i + 4 * o[0] + N * ((j + 4 * o[1]) + N * (k + 4 * o[2]))).ravel()
    core_full = np.isin(glob, oracle.active_points(full.tab, (1,)))
    assert core_full.sum() > 500
    a = oracle.integrals(n, crop.h, crop.B, crop.phi, loc[core_full])
    b = oracle.integrals(N, full.h, full.B, full.phi, glob[core_full])
    assert np.array_equal(a, b)
