"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds none of the method's arithmetic: it only draws the standard
normal KL coefficients xi from seeded numpy generators, fixes the workload
presets (grid rectangles, field parameters, sample counts) and draws request
traces for the serving loop.  Both the product and the checker read their
inputs from here and nowhere else.

Each sample draws its xi from its own generator keyed by (base seed, sample
id), so a sample's coefficients do not depend on the batch it is solved in.
"""
from __future__ import annotations

import dataclasses
from typing import Tuple, List, Optional, Sequence

import numpy as np

BASE_SEED = 20190726

# Ten cosine-product KL terms for the "10-term KL sum" fields: frequency pairs
# (a_j, b_j) with a, b >= 0 and a + b <= 3, ordered by a + b, then by a
# descending; amplitude of term j (1-based) is sqrt(j^-2) = 1/j.
KL10_A = (0, 1, 0, 2, 1, 0, 3, 2, 1, 0)
KL10_B = (0, 0, 1, 0, 1, 2, 0, 1, 2, 3)
KL10_AMP = tuple(1.0 / j for j in range(1, 11))


@dataclasses.dataclass(frozen=True)
class FieldSpec:
    """k = exp(Z).  kind 'cos': Z = sum_t amp_t xi_t cos(pi a_t x) cos(pi b_t y).
    kind 'separable': separable squared-exponential KL with mx*my terms,
    correlation lengths lx, ly and variance sigma2.  face_rule 0: k at every
    face midpoint of every grid; 1: k at the finest grid's face midpoints and,
    on every coarser face, the mean of those lying on it."""
    kind: str
    a: Sequence[int] = ()
    b: Sequence[int] = ()
    amp: Sequence[float] = ()
    mx: int = 0
    my: int = 0
    lx: float = 0.0
    ly: float = 0.0
    sigma2: float = 0.0
    face_rule: int = 0

    @property
    def n_terms(self) -> int:
        return len(self.a) if self.kind == "cos" else self.mx * self.my

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


KL10 = FieldSpec(kind="cos", a=KL10_A, b=KL10_B, amp=KL10_AMP)


def separable(lx: float, ly: float, sigma2: float, m: int = 50, face_rule: int = 0) -> FieldSpec:
    return FieldSpec(kind="separable", mx=m, my=m, lx=lx, ly=ly, sigma2=sigma2, face_rule=face_rule)


def constant_field(n_terms: int = 1) -> FieldSpec:
    """k = 1 everywhere (a cosine sum with zero amplitudes)."""
    return FieldSpec(kind="cos", a=(0,) * n_terms, b=(0,) * n_terms, amp=(0.0,) * n_terms)


def draw_xi(n_terms: int, sample_ids: Sequence[int], base_seed: int = BASE_SEED) -> np.ndarray:
    """xi[s, t] ~ N(0,1), one independent generator per (base_seed, sample id)."""
    out = np.empty((len(sample_ids), n_terms), dtype=np.float64)
    for k, sid in enumerate(sample_ids):
        out[k] = np.random.default_rng([int(base_seed), int(sid)]).standard_normal(n_terms)
    return out


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    c: int                      # coarsest cells per direction
    P: List[int]                # finest x index per sample
    Q: List[int]                # finest y index per sample
    field: FieldSpec
    tol: float = 1e-10
    precision: str = "fp64"     # "fp64" or "mixed"
    ir_tol: float = 1e-8
    seed: int = BASE_SEED
    max_cycles: int = 50        # cap per grid; strongly anisotropic fields need more on tiny coarse grids

    @property
    def n_samples(self) -> int:
        return len(self.P)

    def xi(self, sample_ids: Optional[Sequence[int]] = None) -> np.ndarray:
        ids = range(self.n_samples) if sample_ids is None else sample_ids
        return draw_xi(self.field.n_terms, list(ids), self.seed)

    def subset(self, n: int) -> "Workload":
        return dataclasses.replace(self, name=f"{self.name}[:{n}]", P=self.P[:n], Q=self.Q[:n])


def uniform(name, c, P, Q, S, field, **kw) -> Workload:
    return Workload(name=name, c=c, P=[P] * S, Q=[Q] * S, field=field, **kw)


def config(k: int) -> Workload:
    """The five workload presets (sizes, fields, tolerances)."""
    if k == 1:   # 16 samples, finest 32x32 with 4x4 coarsest, KL-10, FP64, W(2,2) to 1e-10
        return uniform("kl10-32x32-s16", 4, 3, 3, 16, KL10, seed=BASE_SEED + 1)
    if k == 2:   # 4096 samples, finest 256x256, 2x2 coarsest (64 grids), separable SE 50x50
        return uniform("se-256x256-s4096", 2, 7, 7, 4096, separable(0.3, 0.03, 1.0, face_rule=1),
                       seed=BASE_SEED + 2,
                       max_cycles=1000)
    if k == 3:   # ragged MIMC index set l1+l2 <= 8, N_l = 8192 * 2^-(l1+l2), at least 16
        P, Q = [], []
        for l1 in range(9):
            for l2 in range(9 - l1):
                n = max(16, 8192 >> (l1 + l2))
                P += [l1] * n
                Q += [l2] * n
        return Workload("kl10-ragged-l1+l2<=8", 4, P, Q, KL10, seed=BASE_SEED + 3)
    if k == 4:   # 1024 samples, finest 1024x64, strong anisotropy, mixed precision
        return uniform("se-1024x64-s1024-mixed", 4, 8, 4, 1024, separable(1.0, 0.01, 2.0, face_rule=1),
                       precision="mixed", ir_tol=1e-8, seed=BASE_SEED + 4, max_cycles=1000)
    raise ValueError(f"no workload preset {k}")


@dataclasses.dataclass(frozen=True)
class MaternPrior:
    """The paper's random coefficient of its multi-index experiments: Matern
    covariance with length scale lam and smoothness nu, the anisotropic ratio
    eta and the rotation theta drawn per sample, uniform on the given ranges
    (theta in degrees), and the embedding factor pad (0: the paper's)."""
    lam: float = 0.25
    nu: float = 0.5
    eta: Tuple[float, float] = (1.0 / 16, 1.0 / 4)
    theta_deg: Tuple[float, float] = (-30.0, 30.0)
    pad: int = 0

    def hyperparameters(self, u: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        """(eta, theta in radians) per sample from rows of two uniforms."""
        eta = self.eta[0] + (self.eta[1] - self.eta[0]) * u[:, 0]
        theta = np.radians(self.theta_deg[0] + (self.theta_deg[1] - self.theta_deg[0]) * u[:, 1])
        return eta, theta


MATERN_PAPER = MaternPrior()


def mimc_uniforms(n: int, batch: int = 0, seed: int = BASE_SEED + 6, d: int = 2) -> np.ndarray:
    """U(0,1] draws, one row per Monte Carlo sample of batch `batch` of the
    multi-index estimator, from which each side draws its random index L."""
    return 1.0 - np.random.default_rng([int(seed), int(batch)]).random((n, d))


def request_trace(n: int, rate: float, seed: int = BASE_SEED + 5, lmax: int = 9):
    """Poisson arrivals (exponential gaps at `rate`/s) of requests whose finest
    index per direction is l in 1..lmax with probability proportional to
    2^-(l-1) (finest sides 8 ... 4*2^lmax).  Returns (t_arrival, P, Q, sample_id)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    ls = np.arange(1, lmax + 1)
    pr = 2.0 ** -(ls - 1)
    pr /= pr.sum()
    P = rng.choice(ls, size=n, p=pr)
    Q = rng.choice(ls, size=n, p=pr)
    return t, P.astype(np.int32), Q.astype(np.int32), np.arange(n, dtype=np.int64)
