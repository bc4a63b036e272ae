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

With pmf="learned" the indices come instead from the learned distribution
of the paper's experiments (Section 3, eq. Nell): sample sizes N_tau
proportional to sqrt(V_tau / C_tau), with V_tau the sample variance of
Delta Q_tau and C_tau the mean measured work of a solve on rectangle tau where
an index has enough samples, and the fitted laws 2^(v0 - beta.tau) and
2^(w0 + gamma.tau) elsewhere.  The tail p_tau = min(1, N_tau / N_0) becomes a
pmf on the box [0..lmax]^2 by inclusion-exclusion, its negative masses are
dropped, and it is renormalised and mixed with weight eps with the geometric
pmf of the current rates, so that every index of the box keeps a positive
probability and the estimator stays unbiased; the weights 1/p_tau use the
tail of that mixture.  A draw takes one uniform and inverts the cumulative
mass over the indices in p-major order.

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
MATERN_WS_BYTES = 16 << 30      # cap of the Matern sampler's workspace per batch


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


def geometric_tail(r: np.ndarray, lmax: int) -> np.ndarray:
    """p_tau = exp(-r_1 tau_1) exp(-r_2 tau_2) on the box [0..lmax]^2."""
    t = np.arange(lmax + 1, dtype=float)
    return np.exp(-r[0] * t)[:, None] * np.exp(-r[1] * t)[None, :]


def pmf_from_tail(p: np.ndarray) -> np.ndarray:
    """pi(l) = P(L = l) from p(tau) = P(L >= tau) on a box (zero outside)."""
    n = p.shape[0]
    z = np.zeros((n + 1, n + 1))
    z[:n, :n] = p
    return z[:-1, :-1] - z[1:, :-1] - z[:-1, 1:] + z[1:, 1:]


def tail_from_pmf(pi: np.ndarray) -> np.ndarray:
    """p(tau) = sum of pi over l >= tau in both directions."""
    return pi[::-1, ::-1].cumsum(0).cumsum(1)[::-1, ::-1].copy()


def learned_distribution(V: np.ndarray, C: np.ndarray, r: np.ndarray, eps: float) -> Tuple[np.ndarray, np.ndarray]:
    """(pi, p) on the box from per-index variances V and costs C (eq. Nell)."""
    n0 = math.sqrt(V[0, 0] / C[0, 0])
    raw = np.maximum(pmf_from_tail(np.minimum(1.0, np.sqrt(V / C) / n0)), 0.0)
    raw /= raw.sum()
    pi = (1.0 - eps) * raw + eps * pmf_from_tail(geometric_tail(r, V.shape[0] - 1))
    return pi, tail_from_pmf(pi)


def draw_indices_pmf(u: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """Indices from uniforms in (0,1]: the first index, in p-major order,
    whose cumulative mass reaches u."""
    n = pi.shape[0]
    k = np.minimum(np.searchsorted(np.cumsum(pi.ravel()), u, side="left"), n * n - 1)
    return np.stack([k // n, k % n], axis=1).astype(np.int64)


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
    pmf: str = "geometric"                       # index distribution: geometric or learned

    @property
    def rmse(self) -> float:
        return math.sqrt(self.V)


class MSGMIMC:
    """Algorithm MSG-MIMC driven in batches on one GPU."""

    def __init__(self, handle: msg.Handle, field: I.FieldSpec = I.KL10, c: int = 4,
                 kind: int = msg.QOI_POINT, opts: Optional[msg.SolveOpts] = None, lmax: int = 9,
                 r0: Optional[np.ndarray] = None, seed: int = I.BASE_SEED + 6, learn: bool = True,
                 prior: Optional[I.MaternPrior] = None, pmf: str = "geometric", eps: float = 0.1):
        if pmf not in ("geometric", "learned"):
            raise ValueError(f"pmf must be 'geometric' or 'learned', not {pmf!r}")
        self.h, self.field, self.c, self.kind = handle, field, c, kind
        self.prior = prior
        self.min_eig_ratio = math.inf
        # batches of a few hundred samples spread over many rectangles: 64 KB
        # on-chip tails (fewer host level visits) suit them better than the
        # library's default sized for thousands of problems per class
        self.opts = opts or msg.SolveOpts(tol=1e-8, max_cycles=200, precision=msg.MIXED, tail_budget=65536)
        self.lmax, self.seed, self.learn = lmax, seed, learn
        self.r = np.array(initial_rates() if r0 is None else r0, dtype=float)
        self.ys: List[float] = []
        self.ystat: Tuple[int, float, float] = (0, 0.0, 0.0)         # count, mean, M2 of the Y's
        self.dq: Dict[Tuple[int, int], Tuple[int, float, float]] = {}     # index -> (count, mean, M2)
        self.counts: Dict[Tuple[int, int], int] = {}
        self.work: Dict[Tuple[int, int], Tuple[int, float]] = {}          # L -> (count, summed work)
        self.gamma = np.array([1.0, 1.0])
        self.pmf, self.eps = pmf, eps
        self.vfit: Optional[Tuple[float, np.ndarray]] = None     # (v0, beta): log2 V = v0 - beta.tau
        self.wfit: Optional[Tuple[float, np.ndarray]] = None     # (w0, gamma): log2 C = w0 + gamma.tau
        self.tail = geometric_tail(self.r, lmax)
        self.pi = pmf_from_tail(self.tail)
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
            # a workspace of at most MATERN_WS_BYTES (but one sample of the
            # largest embedding at least): the library then fields fewer
            # samples per chunk
            k = int(np.argmax(P.astype(np.int64) + Q.astype(np.int64)))
            one = msg.matern_workspace_size(msg.Batch(self.c, [int(P[k])], [int(Q[k])]),
                                            msg.MaternSpec(pr.lam, pr.nu, [1.0], [0.0], None, self.seed, pr.pad))
            n = max(one, min(msg.matern_workspace_size(batch, spec), MATERN_WS_BYTES))
            ws = torch.empty((n + 7) // 8, dtype=torch.float64, device="cuda:0")
            self.h.sample_matern(spec, batch, bufs.kx, bufs.ky, bufs.kx32, bufs.ky32, ratio=ratio, ws=ws)
            del ws
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
        if self.pmf == "learned":
            L = draw_indices_pmf(u[:, 0], self.pi)
            tail = self.tail
        else:
            L = draw_indices(u, self.r, self.lmax)
            tail = None
        dqs, status, cycles, ids = self.solve_batch(L)
        failed = [(int(i), (int(l[0]), int(l[1])), int(st)) for i, l, st, d in zip(ids, L, status, dqs)
                  if st != msg.SAMPLE_CONVERGED or not np.all(np.isfinite(d))]
        if failed:
            raise MIMCFailure(failed)
        ybatch = np.empty(len(L))
        groups: Dict[Tuple[int, int], List[int]] = {}
        for k, (P, Q) in enumerate(L):
            groups.setdefault((int(P), int(Q)), []).append(k)
        for (P, Q), ks in groups.items():
            D = np.stack([dqs[k] for k in ks])                    # samples x grids of rectangle (P, Q)
            w = reuse_weights(P, Q, self.r) if tail is None else 1.0 / tail[:P + 1, :Q + 1].ravel()
            ybatch[ks] = D @ w
            self.merge_stats(P, Q, D)
            work = np.array([sample_work(self.c, P, Q, cycles[k]) for k in ks])
            n0, s0 = self.work.get((P, Q), (0, 0.0))
            self.work[(P, Q)] = (n0 + len(ks), s0 + float(work.sum()))
            self.counts[(P, Q)] = self.counts.get((P, Q), 0) + len(ks)
        self.ys.extend(ybatch.tolist())
        n0, m0, s0 = self.ystat
        nb, mb = len(ybatch), float(ybatch.mean())
        n1, delta = n0 + nb, mb - m0
        self.ystat = (n1, m0 + delta * nb / n1, s0 + float(((ybatch - mb) ** 2).sum()) + delta * delta * n0 * nb / n1)
        self.batches += 1
        if self.learn:
            self.refit()

    # -------------------------------------------------------------- learning
    def merge_stats(self, P: int, Q: int, D: np.ndarray) -> None:
        """Fold the columns of D (Delta Q of a group of samples on rectangle
        (P, Q)) into the per-index count, mean and sum of squared deviations
        (pairwise merge of two samples' statistics)."""
        nb = D.shape[0]
        mb = D.mean(axis=0)
        m2b = ((D - mb) ** 2).sum(axis=0)
        for a in range(P + 1):
            for b in range(Q + 1):
                j = a * (Q + 1) + b
                n0, m0, s0 = self.dq.get((a, b), (0, 0.0, 0.0))
                n1 = n0 + nb
                delta = float(mb[j]) - m0
                self.dq[(a, b)] = (n1, m0 + delta * nb / n1, s0 + float(m2b[j]) + delta * delta * n0 * nb / n1)

    def variance(self, key: Tuple[int, int], min_samples: int) -> float:
        """Sample variance of Delta Q at an index, or 0 with fewer than min_samples samples."""
        n, _, m2 = self.dq.get(key, (0, 0.0, 0.0))
        return m2 / (n - 1) if n >= min_samples else 0.0

    def refit(self, min_samples: int = 8) -> None:
        """Re-fit the geometric rates from the sample variances of Delta Q."""
        rows, vals = [], []
        for (a, b) in self.dq:
            v = self.variance((a, b), min_samples)
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
        self.vfit = (float(coef[0]), beta)
        self.gamma = self.fit_gamma(min_samples)
        self.r = LOG2 * (beta + self.gamma) / 2.0
        if self.pmf == "learned" and self.wfit is not None:
            V, C = self.index_tables(min_samples)
            self.pi, self.tail = learned_distribution(V, C, self.r, self.eps)
        else:
            self.tail = geometric_tail(self.r, self.lmax)
            self.pi = pmf_from_tail(self.tail)

    def index_tables(self, min_samples: int = 8) -> Tuple[np.ndarray, np.ndarray]:
        """V_tau and C_tau on the box: sample variance of Delta Q_tau and mean
        measured work of a solve on rectangle tau where an index has at least
        min_samples samples, the fitted laws elsewhere."""
        n = self.lmax + 1
        t = np.arange(n, dtype=float)
        v0, beta = self.vfit
        w0, gamma = self.wfit
        V = 2.0 ** (v0 - beta[0] * t[:, None] - beta[1] * t[None, :])
        C = 2.0 ** (w0 + gamma[0] * t[:, None] + gamma[1] * t[None, :])
        for (a, b) in self.dq:
            v = self.variance((a, b), min_samples)
            if a < n and b < n and v > 0.0:
                V[a, b] = v
        for (a, b), (cnt, total) in self.work.items():
            if a < n and b < n and cnt >= min_samples:
                C[a, b] = total / cnt
        return V, C

    def fit_gamma(self, min_samples: int = 8) -> np.ndarray:
        """gamma_j from log2 of the mean measured work of a sample at L
        against L (least squares), or the previous value while fewer than
        three independent indices have enough samples."""
        rows, vals = [], []
        for (a, b), (cnt, total) in self.work.items():
            if cnt >= min_samples:
                rows.append((1.0, a, b))
                vals.append(math.log2(total / cnt))
        if len(rows) < 3 or np.linalg.matrix_rank(np.array(rows)) < 3:
            return self.gamma
        coef, *_ = np.linalg.lstsq(np.array(rows), np.array(vals), rcond=None)
        gamma = np.clip(coef[1:], 0.5, 4.0)
        self.wfit = (float(coef[0]), gamma)
        return gamma

    def estimate(self) -> Tuple[float, float]:
        """E = mean of Y and V = sum (Y - E)^2 / (N (N - 1)), from the running
        count, mean and sum of squared deviations of the Y's."""
        n, e, m2 = self.ystat
        return e, (m2 / (n * (n - 1)) if n > 1 else float("inf"))

    def run(self, tol: float, batch: int = 256, max_samples: int = 1 << 20) -> Estimate:
        """Draw batches until sqrt(V) <= tol (Algorithm MSG-MIMC)."""
        t0 = time.perf_counter()
        while True:
            self.add_batch(batch)
            e, v = self.estimate()
            if math.sqrt(v) <= tol or len(self.ys) >= max_samples:
                break
        return Estimate(e, v, len(self.ys), (float(self.r[0]), float(self.r[1])), self.batches,
                        time.perf_counter() - t0, dict(self.counts), (float(self.gamma[0]), float(self.gamma[1])),
                        self.pmf)
