"""Multi-index Monte Carlo with sample reuse (Section 3, Algorithm MSG-MIMC)
on top of the batched full-MSG solver.

Every Monte Carlo sample draws a random index L = (L1, L2) from a product of
geometric distributions, and ONE full-MSG solve on the rectangle [0..L1] x
[0..L2] returns the quantity of interest on every grid tau <= L, hence every
multi-index difference Delta Q_tau of the sample at once.  The sample's
contribution is Y = sum_{tau <= L} Delta Q_tau / p_tau with p_tau = P(L >= tau)
(componentwise), so that E[Y] = E[Q] (unbiased, no truncation of the index
set), and the estimator is the mean of the Y's with variance estimate
V = sum (Y - E)^2 / (N (N - 1)).  Samples are drawn, solved and reduced in
batches: a batch is one ragged call of the library (samples of different
rectangles), its quantities come from msg_quantity and its differences from
mimc_delta_q, all on the device; only the per-grid Delta Q return.

The distribution starts at the paper's GEOMETRIC(log(2)(1 + 4)/2) in each
direction (beta = 4, gamma = 1) and is re-fitted after every batch from the
data: per direction, beta_j from a least-squares fit of log2 of the sample
variance of Delta Q_tau against tau, gamma_j from a least-squares fit of log2
of the mean measured work of a sample against its index L, and r_j = log(2)
(beta_j + gamma_j) / 2, as in the paper's derivation of the optimal sample
sizes (Section 3, rates of assumptions A2 and A3).  A sample's work is what
its solve did: the cycles run on each grid tau <= L (returned by the library)
times the cell visits of one W-cycle on that grid's rectangle,
(tau1+1)(tau2+1) c^2 2^(tau1+tau2); samples of one batch share a ragged
launch, so their times cannot be taken one by one.  Each sample keeps the
p_tau of the distribution it was drawn from.  Indices are capped at `lmax`
per direction (tail mass exp(-r (lmax+1))).

A batch in which any sample's solve failed (cycle cap hit, non-finite
residual) or any difference is not finite raises MIMCFailure and adds
nothing to the estimator: dropping the sample would bias the estimate, and
keeping an unconverged difference would add an error nobody controls.

Random numbers are inputs (inputs.mimc_uniforms): L_j = floor(-log(U_j) / r_j).

Two field models.  The default draws the coefficient from a truncated
expansion (inputs.FieldSpec), its normals drawn on the device from the
counter-based streams (estimator seed, sample counter).  With a Matern
prior (inputs.MaternPrior) every sample is the paper's Section 5 setting: a
lognormal field with Matern covariance whose anisotropic ratio eta and
rotation theta are themselves uniform random hyperparameters, drawn per
sample from a second stream of uniforms (inputs.mimc_uniforms with seed + 1),
and sampled exactly by circulant embedding on the device (msg_sample_matern,
the Philox stream keyed by the estimator's seed, the sample counter as id), so
every sample recomputes its embedding's eigenvalues.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import inputs as I
from . import msg

LOG2 = math.log(2.0)


def initial_rates(beta=(4.0, 4.0), gamma=(1.0, 1.0)) -> np.ndarray:
    return LOG2 * (np.asarray(beta, float) + np.asarray(gamma, float)) / 2.0


def draw_indices(u: np.ndarray, r: np.ndarray, lmax: int) -> np.ndarray:
    """Random indices from uniforms in (0,1]: L_j = floor(-log(U_j) / r_j), capped."""
    L = np.floor(-np.log(u) / r[None, :]).astype(np.int64)
    return np.minimum(L, lmax)


def reuse_weights(P: int, Q: int, r: np.ndarray) -> np.ndarray:
    """1 / p_tau on the grids of rectangle (P, Q) in packed order (p-major)."""
    t1 = np.arange(P + 1)[:, None]
    t2 = np.arange(Q + 1)[None, :]
    return np.exp(r[0] * t1 + r[1] * t2).ravel()


class MIMCFailure(RuntimeError):
    """A batch contained samples whose solve did not converge."""

    def __init__(self, failed):
        self.failed = failed          # [(sample id, (L1, L2), status)]
        super().__init__(f"{len(failed)} sample(s) of the batch not solved to tolerance "
                         f"(sample id, index, status): {failed[:8]}")


def sample_work(c: int, P: int, Q: int, cycles: np.ndarray) -> float:
    """Cell visits of one solve: cycles run on each grid times the cell
    visits of one W-cycle on that grid's rectangle."""
    w = 0.0
    for a in range(P + 1):
        for b in range(Q + 1):
            w += float(cycles[a * (Q + 1) + b]) * (a + 1) * (b + 1) * c * c * 2.0 ** (a + b)
    return w


@dataclasses.dataclass
class Estimate:
    E: float
    V: float
    N: int
    rates: Tuple[float, float]
    batches: int
    seconds: float
    index_counts: Dict[Tuple[int, int], int]
    gamma: Tuple[float, float] = (1.0, 1.0)     # work growth rates fitted from the solves

    @property
    def rmse(self) -> float:
        return math.sqrt(self.V)


class MSGMIMC:
    """Algorithm MSG-MIMC driven in batches on one GPU."""

    def __init__(self, handle: msg.Handle, field: I.FieldSpec = I.KL10, c: int = 4,
                 kind: int = msg.QOI_POINT, opts: Optional[msg.SolveOpts] = None, lmax: int = 9,
                 r0: Optional[np.ndarray] = None, seed: int = I.BASE_SEED + 6, learn: bool = True,
                 prior: Optional[I.MaternPrior] = None):
        self.h, self.field, self.c, self.kind = handle, field, c, kind
        self.prior = prior
        self.min_eig_ratio = math.inf
        self.opts = opts or msg.SolveOpts(tol=1e-8, max_cycles=200, precision=msg.MIXED)
        self.lmax, self.seed, self.learn = lmax, seed, learn
        self.r = np.array(initial_rates() if r0 is None else r0, dtype=float)
        self.ys: List[float] = []
        self.dq: Dict[Tuple[int, int], List[float]] = {}
        self.counts: Dict[Tuple[int, int], int] = {}
        self.work: Dict[Tuple[int, int], List[float]] = {}
        self.gamma = np.array([1.0, 1.0])
        self.batches = 0
        self.next_sample_id = 0

    # -------------------------------------------------------------- one batch
    def hyperparameters(self, n: int, batch: int) -> Tuple[np.ndarray, np.ndarray]:
        """(eta, theta in radians) of the n samples of a batch under the prior."""
        return self.prior.hyperparameters(I.mimc_uniforms(n, batch, self.seed + 1))

    def solve_batch(self, L: np.ndarray):
        """One ragged library call: per-grid Delta Q of every sample (host arrays)."""
        import torch
        P, Q = L[:, 0].astype(np.int32), L[:, 1].astype(np.int32)
        batch = msg.Batch(self.c, P, Q)
        ids = np.arange(self.next_sample_id, self.next_sample_id + len(P), dtype=np.int64)
        self.next_sample_id += len(P)
        bufs = msg.Buffers(batch, self.opts)
        if self.prior is None:
            # normals drawn on the device from the streams (seed, sample id)
            msg.run(self.h, self.field, batch, self.opts, None, bufs, seed=self.seed, sample_id=ids)
        else:
            pr = self.prior
            eta, theta = self.hyperparameters(len(P), self.batches)
            spec = msg.MaternSpec(pr.lam, pr.nu, eta, theta, ids, self.seed, pr.pad)
            ratio = torch.empty(len(P), dtype=torch.float64, device="cuda:0")
            self.h.sample_matern(spec, batch, bufs.kx, bufs.ky, bufs.kx32, bufs.ky32, ratio=ratio)
            msg.run(self.h, None, batch, self.opts, None, bufs, field=False)
            self.min_eig_ratio = min(self.min_eig_ratio, float(ratio.min()))
        if self.kind != msg.QOI_MEAN:
            msg.quantity(batch, self.kind, bufs.kx, bufs.u, bufs.q)
            msg.delta_q(batch, bufs.q, bufs.dq)
        lay = bufs.layout
        dq = bufs.dq.cpu().numpy()
        status = bufs.status.cpu().numpy()
        cyc = bufs.cycles.cpu().numpy()
        g = lay["grid"]
        return ([dq[g[k]:g[k + 1]] for k in range(len(P))], status, [cyc[g[k]:g[k + 1]] for k in range(len(P))],
                ids)

    def add_batch(self, n: int) -> None:
        u = I.mimc_uniforms(n, self.batches, self.seed)
        L = draw_indices(u, self.r, self.lmax)
        dqs, status, cycles, ids = self.solve_batch(L)
        failed = [(int(i), (int(l[0]), int(l[1])), int(st)) for i, l, st, d in zip(ids, L, status, dqs)
                  if st != msg.SAMPLE_CONVERGED or not np.all(np.isfinite(d))]
        if failed:
            raise MIMCFailure(failed)
        for (P, Q), d, cy in zip(L, dqs, cycles):
            w = reuse_weights(int(P), int(Q), self.r)
            self.ys.append(float(np.dot(d, w)))
            for a in range(P + 1):
                for b in range(Q + 1):
                    self.dq.setdefault((a, b), []).append(float(d[a * (Q + 1) + b]))
            self.counts[(int(P), int(Q))] = self.counts.get((int(P), int(Q)), 0) + 1
            self.work.setdefault((int(P), int(Q)), []).append(sample_work(self.c, int(P), int(Q), cy))
        self.batches += 1
        if self.learn:
            self.refit()

    # -------------------------------------------------------------- learning
    def refit(self, min_samples: int = 8) -> None:
        """Re-fit the geometric rates from the sample variances of Delta Q."""
        rows, vals = [], []
        for (a, b), xs in self.dq.items():
            if len(xs) >= min_samples:
                v = float(np.var(xs, ddof=1))
                if v > 0.0:
                    rows.append((1.0, a, b))
                    vals.append(math.log2(v))
        if len(rows) < 4:
            return
        A = np.array(rows)
        if np.linalg.matrix_rank(A) < 3:
            return
        coef, *_ = np.linalg.lstsq(A, np.array(vals), rcond=None)
        beta = np.clip(-coef[1:], 0.5, 8.0)
        self.gamma = self.fit_gamma(min_samples)
        self.r = LOG2 * (beta + self.gamma) / 2.0

    def fit_gamma(self, min_samples: int = 8) -> np.ndarray:
        """gamma_j from log2 of the mean measured work of a sample at L
        against L (least squares), or the previous value while fewer than
        three independent indices have enough samples."""
        rows, vals = [], []
        for (a, b), ws in self.work.items():
            if len(ws) >= min_samples:
                rows.append((1.0, a, b))
                vals.append(math.log2(float(np.mean(ws))))
        if len(rows) < 3 or np.linalg.matrix_rank(np.array(rows)) < 3:
            return self.gamma
        coef, *_ = np.linalg.lstsq(np.array(rows), np.array(vals), rcond=None)
        return np.clip(coef[1:], 0.5, 4.0)

    def estimate(self) -> Tuple[float, float]:
        y = np.asarray(self.ys)
        n = len(y)
        e = float(y.mean())
        v = float(((y - e) ** 2).sum() / (n * (n - 1))) if n > 1 else float("inf")
        return e, v

    def run(self, tol: float, batch: int = 256, max_samples: int = 1 << 20) -> Estimate:
        """Draw batches until sqrt(V) <= tol (Algorithm MSG-MIMC)."""
        t0 = time.perf_counter()
        while True:
            self.add_batch(batch)
            e, v = self.estimate()
            if math.sqrt(v) <= tol or len(self.ys) >= max_samples:
                break
        return Estimate(e, v, len(self.ys), (float(self.r[0]), float(self.r[1])), self.batches,
                        time.perf_counter() - t0, dict(self.counts), (float(self.gamma[0]), float(self.gamma[1])))
