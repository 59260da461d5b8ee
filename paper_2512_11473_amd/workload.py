"""Set up a named workload on the GPU path: coarse distances, package tables,
initial field in package layout, fields and particle buffers, all resident in
device memory.  The inputs come from the seeded generators in ``synth``; every
step of the method itself runs in the library."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np
import torch

import synth

from . import Grid, build_packages, fill_far_field

_LOCAL = np.arange(64, dtype=np.int64)
_LX, _LY, _LZ = _LOCAL % 4, (_LOCAL // 4) % 4, _LOCAL // 16


def package_points(pkg_cell: np.ndarray, M: int) -> np.ndarray:
    """Fine linear indices [P, 64] of the data points of packages 2.. (the
    package's coarse cell times 4 plus the local index i + 4j + 16k)."""
    N = 4 * M
    c = np.asarray(pkg_cell[2:], dtype=np.int64)
    cx, cy, cz = c % M, (c // M) % M, c // (M * M)
    i = (4 * cx)[:, None] + _LX[None, :]
    j = (4 * cy)[:, None] + _LY[None, :]
    k = (4 * cz)[:, None] + _LZ[None, :]
    return i + N * (j + N * k)


@dataclass
class Workload:
    shape: Dict
    N: int
    h: float
    dtype: torch.dtype
    grid: Grid
    coarse: torch.Tensor          # float32 [M^3] on the device
    phi0: torch.Tensor            # [P+2, 64] initial field (kept to reset)
    phi: torch.Tensor             # [P+2, 64]
    scratch: torch.Tensor         # [P+2, 64]
    grad: torch.Tensor            # [3, P+2, 64]
    points: Optional[np.ndarray] = None    # fine indices [P, 64] (host)
    pos: Optional[torch.Tensor] = None
    phi_p: Optional[torch.Tensor] = None
    nrm_p: Optional[torch.Tensor] = None
    extra: Dict = field(default_factory=dict)

    @property
    def n_updates_per_iter(self) -> int:
        return 64 * self.grid.n_packages

    def reset(self):
        self.phi.copy_(self.phi0)


def setup(shape: Dict, N: int, noise_amp: float, noise_seed: int, dtype=torch.float32,
          particles: Optional[np.ndarray] = None) -> Workload:
    assert N % 4 == 0
    M = N // 4
    h = 1.0 / N
    coarse = torch.from_numpy(synth.coarse_sdf(shape, M)).cuda()
    grid = build_packages(coarse, h)
    pkg_cell = grid.tables()["pkg_cell"].cpu().numpy().view(np.uint32)
    pts = package_points(pkg_cell, M)
    vals = synth.phi0_at(shape, N, pts.ravel(), noise_amp, noise_seed)
    np_dtype = np.float32 if dtype == torch.float32 else np.float64
    phi0 = torch.empty((grid.n_total, 64), dtype=dtype, device="cuda")
    phi0[2:] = torch.from_numpy(vals.astype(np_dtype).reshape(-1, 64)).cuda()
    fill_far_field(grid, phi0)
    wl = Workload(shape, N, h, dtype, grid, coarse, phi0, phi0.clone(), torch.empty_like(phi0),
                  torch.empty((3, grid.n_total, 64), dtype=dtype, device="cuda"), pts)
    if particles is not None:
        p = torch.from_numpy(np.ascontiguousarray(particles, dtype=np_dtype)).cuda()
        wl.pos = p
        wl.phi_p = torch.empty(p.shape[0], dtype=dtype, device="cuda")
        wl.nrm_p = torch.empty((p.shape[0], 3), dtype=dtype, device="cuda")
    torch.cuda.synchronize()
    return wl


@dataclass
class BatchWorkload:
    parts: list                   # per-shape Workload (their own phi0 kept for checks)
    batch: object                 # paper_2512_11473_amd.Batch
    phi0: torch.Tensor            # [n_total, 64] concatenated initial fields
    phi: torch.Tensor
    scratch: torch.Tensor

    @property
    def n_updates_per_iter(self) -> int:
        return 64 * self.batch.n_work

    def reset(self):
        self.phi.copy_(self.phi0)

    def slice(self, k: int, t: torch.Tensor) -> torch.Tensor:
        b = int(self.batch.bases[k])
        return t[b:b + self.parts[k].grid.n_total]


def setup_batch(specs, noise_amp: float) -> BatchWorkload:
    """Grids of several shapes (dicts with shape, N, noise_seed) in one batch."""
    from . import Batch
    parts = [setup(s["shape"], s["N"], noise_amp, s["noise_seed"]) for s in specs]
    batch = Batch([p.grid for p in parts])
    phi0 = torch.cat([p.phi0 for p in parts], dim=0).contiguous()
    assert phi0.shape[0] == batch.n_total
    return BatchWorkload(parts, batch, phi0, phi0.clone(), torch.empty_like(phi0))
