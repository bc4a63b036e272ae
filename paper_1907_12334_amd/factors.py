"""Convergence factors of standard multigrid and MSG on the paper's
anisotropic Matern fields, the robustness comparison of Section 2 (its
residual norms after 50 W(2,2) cycles over the anisotropic ratio eta and the
rotation theta, and its expected convergence factors over cycle shapes and
grid sizes).

Every sample runs plain cycles from v = 0 with h = 1 on its finest grid
(msg_cycles, all samples of a setting in one call) on a lognormal field with
Matern covariance, lambda = 1/4, nu = 1/2 and the setting's eta and theta
(msg_sample_matern).  A sample's averaged convergence factor is
(||r_k|| / ||r_0||)^(1/k) at the last cycle k whose residual ratio is still
above a floor near FP64 rounding, so the rounding plateau does not enter the
average.  A sample whose ratio ends above one, or turns non-finite, has not
converged; the expected factor of a setting is the mean over its samples,
reported as None when any sample did not converge (the paper leaves such
points out).  Nothing here computes any part of the method; the fields and
the cycles run in the library.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

from . import inputs as I
from . import msg

FLOOR = 1e-10
LAMBDA, NU = 0.25, 0.5


def averaged_factors(ratios: np.ndarray, floor: float = FLOOR) -> np.ndarray:
    """Per-sample averaged convergence factor from residual-ratio histories
    (rows: samples, columns: cycles 0..n with ratio[0] = 1); inf where a
    sample did not converge."""
    r = np.atleast_2d(np.asarray(ratios, dtype=float))
    out = np.empty(r.shape[0])
    for s, row in enumerate(r):
        if not np.all(np.isfinite(row)) or row[-1] > row[0]:
            out[s] = math.inf
            continue
        above = np.nonzero(row >= floor)[0]
        k = int(above[-1]) if above.size else 0
        if k == 0:
            # converged below the floor within one cycle
            k = 1
        out[s] = (row[k] / row[0]) ** (1.0 / k)
    return out


def expected_factor(ratios: np.ndarray, floor: float = FLOOR) -> Optional[float]:
    f = averaged_factors(ratios, floor)
    if not np.all(np.isfinite(f)) or np.any(f >= 1.0):
        return None
    return float(f.mean())


class Experiment:
    """Runs settings of (eta, theta, grid, nu, method) on one GPU."""

    def __init__(self, handle: msg.Handle, c: int = 2, samples: int = 100, cycles: int = 50,
                 seed: int = I.BASE_SEED + 7):
        self.h, self.c, self.S, self.n, self.seed = handle, c, samples, cycles, seed
        self.min_eig_ratio = math.inf
        self.field_seconds = 0.0
        self.field_samples = 0

    def fields(self, P: int, eta: float, theta_deg: float):
        """Matern fields of the setting's samples (ids 0..S-1) on the device."""
        import torch
        b = msg.Batch(self.c, [P] * self.S, [P] * self.S)
        lay = b.layout()
        dev = f"cuda:{self.h.device}"
        kx = torch.empty(int(lay["xface"][-1]), dtype=torch.float64, device=dev)
        ky = torch.empty(int(lay["yface"][-1]), dtype=torch.float64, device=dev)
        ratio = torch.empty(self.S, dtype=torch.float64, device=dev)
        spec = msg.MaternSpec(LAMBDA, NU, [eta] * self.S, [math.radians(theta_deg)] * self.S, None, self.seed)
        n = msg.matern_workspace_size(b, spec)
        ws = torch.empty((n + 7) // 8, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.h.sample_matern(spec, b, kx, ky, ratio=ratio, ws=ws)
        torch.cuda.synchronize()
        self.field_seconds += time.perf_counter() - t0
        self.field_samples += self.S
        self.min_eig_ratio = min(self.min_eig_ratio, float(ratio.min()))
        return b, kx, ky

    def ratios(self, b: msg.Batch, kx, ky, P: int, kind: int, nu: int, mu: int = 2) -> np.ndarray:
        import torch
        opts = msg.SolveOpts(mu=mu, nu1=nu, nu2=nu)
        dev = kx.device
        n = (self.c << P) ** 2
        u = torch.empty(self.S * n, dtype=torch.float64, device=dev)
        r = torch.empty(self.S * (self.n + 1), dtype=torch.float64, device=dev)
        nbytes = msg.cycles_workspace_size(b, opts, kind)
        ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
        self.h.cycles(b, opts, kind, self.n, kx, ky, None, u, r, ws)
        return r.cpu().numpy().reshape(self.S, self.n + 1)

    def table(self, etas: Iterable[float], thetas: Iterable[float], Ps: Sequence[int],
              nus: Sequence[int]) -> List[dict]:
        rows = []
        for eta in etas:
            for theta in thetas:
                for P in Ps:
                    b, kx, ky = self.fields(P, eta, theta)
                    for nu in nus:
                        row: Dict[str, object] = {"eta": eta, "theta": theta, "cells": f"{self.c << P}x{self.c << P}",
                                                  "nu": nu}
                        for name, kind in (("MG", msg.CYCLES_MG), ("MSG", msg.CYCLES_MSG)):
                            r = self.ratios(b, kx, ky, P, kind, nu)
                            f = averaged_factors(r)
                            row[name] = expected_factor(r)
                            row[name + "_converged"] = float(np.mean(np.isfinite(f) & (f < 1.0)))
                            row[name + "_median_r10"] = float(np.median(r[:, min(10, self.n)]))
                        rows.append(row)
        return rows
