"""Synthetic workloads (stand-ins for the paper's experiments; see workloads.py).

Common to every workload: GMRES restart 10 and relative tolerance 1e-8,
interface degree 1, smoothing overlap 2.  Boundary set-up and source: the
small, batched and serving workloads have no flow on all four sides with the
pressure fixed by its mean, a point injector +1 in cell (0, 0) and a producer
-1 in the last cell.  The channel, large and incl-* workloads use the
paper's set-up for its heterogeneous fields (Section 4): pressure 1 on the
left side and 0 on the right, no flow on the others, no source.  (With no
flow on all sides and point sources, the 1e6 and 1e8 contrast fields are not
solvable to 1e-8 in FP64: a sparse direct solve stops near 1e-6 relative
residual, because regions of floor permeability are nearly disconnected.)
Field recipes and seeds:

* small   64 x 64, log-normal K (sigma 2, correlation 8, seed 1), 4 x 4
          subdomains of 16 x 16, oversampling 2, alpha 1 with L = h, one
          smoothing sweep; FP64.
* channel 220 x 60 channelised facies (Gaussian threshold, correlation 20 x 3
          cells, seed 2; K = 1 in channels, 1e-6 in shale), 11 x 3 subdomains
          of 20 x 20 (the shape of the paper's SPE10 layers), alpha 10 with
          L = H, oversampling in {0, 2, 4}, sweeps in {0, 1, 2}; FP64.
* batched 1024 x 1024, log-normal K (sigma 3, correlation 16, seed 3), 4096
          subdomains of 16 x 16, oversampling 4, one sweep, alpha 10, L = H;
          local and smoothing factors stored in FP32 and applied in FP64
          arithmetic, FP64 factorisation, interface solve and GMRES.
* large   4096 x 4096 (16.8 M cells), channel / log-normal mixture with
          contrast 1e8 (seeds 5, 6), 16384 subdomains of 32 x 32, oversampling
          4, two sweeps, alpha 10, L = H; local and smoothing solves applied
          in FP32 (factors computed in FP64), FP64 interface solve and GMRES
          (FP64 and FP32-stored factors for comparison).
* incl-high, incl-low, incl-both
          160 x 160 thin inclusions (seed 11): 24 segments of K = 1e4, of
          K = 1e-4, or both (contrast 1e8) on K = 1, the stand-ins for the
          paper's inclusion experiments (Section 4.3); 8 x 8 subdomains of
          20 x 20 (4 x 4 of 40 x 40 for comparison), oversampling 2, two
          sweeps, alpha 10, L = H; FP64.

3-D (the model problem of Section 2 with d = 3; the paper reports no 3-D
experiment, so this workload is a stand-in of the same construction):

* cube    96 x 96 x 96 (884 736 cells), log-normal K (sigma 2, correlation
          6, seed 21), 12 x 12 x 12 subdomains of 8 x 8 x 8, oversampling 2
          (12 x 12 x 12 boxes), tensor Legendre degree 1 on every face (4
          functions per face and unknown, 38 016 interface dofs), one
          smoothing sweep with overlap 2, alpha 10, L = H; no flow on all six
          sides with the pressure fixed by its mean, injector +1 in cell
          (0, 0, 0) and producer -1 in the opposite corner; FP64.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import workloads as wl


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    s: int
    oversample: int
    alpha: float
    beta_len: int  # 0: L = H, 1: L = h
    sweeps: int
    overlap: int
    degree: int
    precision: int
    field: str
    bc: tuple = (0, 0, 0, 0)

    def permeability(self) -> np.ndarray:
        if self.field == "small":
            return wl.lognormal_K(self.nx, self.ny, 2.0, 8.0, 1)
        if self.field == "channel":
            return wl.channel_K(self.nx, self.ny, 20.0, 3.0, 2)
        if self.field == "batched":
            return wl.lognormal_K(self.nx, self.ny, 3.0, 16.0, 3)
        if self.field == "large":
            return wl.mixture_K(self.nx, self.ny, 5, 6)
        if self.field.startswith("incl-"):
            return wl.inclusions_K(self.nx, self.ny, self.field[5:], 11)
        raise ValueError(self.field)

    def rhs(self) -> np.ndarray:
        """Algebraic right-hand side of the no-flow workloads."""
        if any(self.bc):
            raise ValueError(f"{self.name}: Dirichlet workload; its right-hand side is "
                             "assembled from boundary_data() by each implementation")
        return wl.corner_sources(self.nx, self.ny)

    def boundary_data(self):
        """(f, g) of the Dirichlet left/right workloads (the right-hand side
        is assembled from them by each implementation)."""
        return wl.dirichlet_left_right(self.nx, self.ny)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)

    def binding_config(self):
        from .binding import Config
        return Config(self.nx, self.ny, tuple(self.bc), self.s, self.s, self.oversample,
                      self.alpha, self.beta_len, self.sweeps, self.overlap, self.degree,
                      self.precision)

    def oracle_args(self):
        """Positional/keyword arguments of oracle.mrcm.MRCM (without K)."""
        return dict(nx=self.nx, ny=self.ny, bc=tuple(self.bc), sx=self.s, sy=self.s,
                    oversample=self.oversample, alpha=self.alpha,
                    beta_len="h" if self.beta_len else "H", sweeps=self.sweeps,
                    overlap=self.overlap, degree=self.degree)

    @property
    def cells(self) -> int:
        return self.nx * self.ny


WORKLOADS = {
    "small": Workload("small", 64, 64, 16, 2, 1.0, 1, 1, 2, 1, 0, "small"),
    "channel": Workload("channel", 220, 60, 20, 2, 10.0, 0, 1, 2, 1, 0, "channel", (1, 1, 0, 0)),
    "batched": Workload("batched", 1024, 1024, 16, 4, 10.0, 0, 1, 2, 1, 2, "batched"),
    "large": Workload("large", 4096, 4096, 32, 4, 10.0, 0, 2, 2, 1, 1, "large", (1, 1, 0, 0)),
}
for _kind in ("high", "low", "both"):
    WORKLOADS[f"incl-{_kind}"] = Workload(f"incl-{_kind}", 160, 160, 20, 2, 10.0, 0, 2, 2, 1, 0,
                                          f"incl-{_kind}", (1, 1, 0, 0))


@dataclass(frozen=True)
class Workload3:
    name: str
    nx: int
    ny: int
    nz: int
    s: int
    oversample: int
    alpha: float
    beta_len: int
    sweeps: int
    overlap: int
    degree: int
    sigma: float
    ell: float
    seed: int
    bc: tuple = (0, 0, 0, 0, 0, 0)
    precision: int = 0  # 0 FP64; 2 FP32-stored plane blocks, FP64 arithmetic

    def permeability(self) -> np.ndarray:
        return wl.lognormal_K3(self.nx, self.ny, self.nz, self.sigma, self.ell, self.seed)

    def with_(self, **kw) -> "Workload3":
        return replace(self, **kw)

    def rhs(self) -> np.ndarray:
        return wl.corner_sources3(self.nx, self.ny, self.nz)

    def binding_config(self):
        from .binding import Config3
        return Config3(self.nx, self.ny, self.nz, tuple(self.bc), self.s, self.s, self.s,
                       self.oversample, self.alpha, self.beta_len, self.sweeps, self.overlap,
                       self.degree, self.precision)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


WORKLOADS3 = {
    "cube": Workload3("cube", 96, 96, 96, 8, 2, 10.0, 0, 1, 2, 1, 2.0, 6.0, 21),
}
