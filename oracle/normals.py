"""Standard normal KL coefficients from the counter-based stream (seed,
sample id) -- the oracle's side of the device draw.

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg use it.  It shares no code with the HIP path, which draws the
same stream on the device from its own Philox.

The coefficient xi[t] of a sample is normal t of the stream: Philox4x64-10
(Salmon et al. 2011) at counter (t // 4, sample id, 0, 0) under key
(seed, KEY_KL); words (0, 1) give normals 4n and 4n+1 (the cosine and sine of
one Box-Muller pair), words (2, 3) normals 4n+2 and 4n+3.  Uniforms are
u = ((w >> 12) + 1/2) 2^-52.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .matern_oracle import box_muller, philox4x64

KEY_KL = 0x4B4C2D7869


def kl_normals(n_terms: int, sample_ids: Sequence[int], seed: int) -> np.ndarray:
    """xi[s, t] for every listed sample id (rows) and term t < n_terms."""
    groups = (n_terms + 3) // 4
    out = np.empty((len(sample_ids), 4 * groups))
    n = np.arange(groups, dtype=np.uint64)
    zero = np.zeros_like(n)
    for k, sid in enumerate(sample_ids):
        w = philox4x64(n, np.full_like(n, int(sid)), zero, zero, int(seed), KEY_KL)
        out[k, 0::4], out[k, 1::4] = box_muller(w[0], w[1])
        out[k, 2::4], out[k, 3::4] = box_muller(w[2], w[3])
    return out[:, :n_terms]
