"""Convergence factors of standard multigrid and MSG on anisotropic
lognormal coefficients, the robustness comparison of Section 2 (its study of
W(nu,nu) cycles on samples of an anisotropic random field).

Every sample runs plain cycles from v = 0 with h = 1 on its finest grid
(msg_cycles, all samples of a setting in one call), and its averaged
convergence factor is (||r_k|| / ||r_0||)^(1/k) at the last cycle k whose
residual ratio is still above a floor near FP64 rounding, so that the
rounding plateau does not enter the average.  A sample whose ratio ends above
one, or turns non-finite, has not converged; the expected factor of a
setting is the mean over its samples, reported as None when any sample did
not converge (the paper leaves such points out).

Fields: lognormal, separable squared-exponential covariance (the field
library's 'separable' kind), correlation length 1/4 in x and eta/4 in y, so
eta plays the role of the anisotropic ratio with the anisotropy aligned to
the grid (rotation 0).  Nothing here computes any part of the method; the
cycles run in the library.
"""
from __future__ import annotations

import math
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

from . import inputs as I
from . import msg

FLOOR = 1e-10


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


def field(eta: float, sigma2: float = 1.0, mx: int = 16, my: int = 64) -> I.FieldSpec:
    return I.FieldSpec(kind="separable", mx=mx, my=my, lx=0.25, ly=0.25 * eta, sigma2=sigma2)


class Experiment:
    """Runs settings of (eta, grid, nu, method) on one GPU."""

    def __init__(self, handle: msg.Handle, c: int = 2, samples: int = 100, cycles: int = 50,
                 seed: int = I.BASE_SEED + 7):
        self.h, self.c, self.S, self.n, self.seed = handle, c, samples, cycles, seed

    def _fields(self, spec: I.FieldSpec, P: int):
        import torch
        b = msg.Batch(self.c, [P] * self.S, [P] * self.S)
        lay = b.layout()
        dev = f"cuda:{self.h.device}"
        kx = torch.empty(int(lay["xface"][-1]), dtype=torch.float64, device=dev)
        ky = torch.empty(int(lay["yface"][-1]), dtype=torch.float64, device=dev)
        xi = torch.tensor(I.draw_xi(spec.n_terms, range(self.S), self.seed), dtype=torch.float64, device=dev)
        self.h.sample_field(msg.FieldSpec(spec), b, xi, kx, ky)
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

    def table(self, etas: Iterable[float], Ps: Sequence[int], nus: Sequence[int]) -> List[dict]:
        rows = []
        for eta in etas:
            spec = field(eta)
            for P in Ps:
                b, kx, ky = self._fields(spec, P)
                for nu in nus:
                    row: Dict[str, object] = {"eta": eta, "cells": f"{self.c << P}x{self.c << P}", "nu": nu}
                    for name, kind in (("MG", msg.CYCLES_MG), ("MSG", msg.CYCLES_MSG)):
                        r = self.ratios(b, kx, ky, P, kind, nu)
                        f = averaged_factors(r)
                        row[name] = expected_factor(r)
                        row[name + "_converged"] = float(np.mean(np.isfinite(f) & (f < 1.0)))
                    rows.append(row)
        return rows
