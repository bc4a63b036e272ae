"""Matern Gaussian random fields by circulant embedding -- the oracle.

TEST INFRASTRUCTURE.  Plain FP64 numpy, slow and direct; only tests/,
__graft_entry__.smoke() and bench.py's CPU-baseline leg may use it.  It shares
no code with the HIP path.

What it computes (the paper's random coefficient, Section 1 and Section 5):

* Covariance, eq. matern: C(r) = 2^(1-nu) / Gamma(nu) (2 sqrt(nu) r)^nu
  K_nu(2 sqrt(nu) r), C(0) = 1, with r = ||T (x1 - x2)||_2 and T = S R, S the
  scaling diag(1/sqrt(eta lambda), 1/sqrt(lambda)) and R the rotation by
  theta; lambda is the length scale, eta the anisotropic ratio.
* Sampling, Section 5: exact samples by circulant embedding on a periodic
  domain larger than the unit square by the factor
  m = 1 + 2 ceil(sqrt(nu) log2(n)) per direction.  Reading: n is the number
  of cells per direction of the finest grid the field is sampled for
  (max(c 2^P, c 2^Q)); the embedding lattice is then rounded up to a power of
  two per direction.
* The points: every face midpoint of every grid (p,q) <= (P,Q) lies on the
  lattice of half the finest mesh width, (a / (2 Nx), b / (2 Ny)),
  0 <= a <= 2 Nx, 0 <= b <= 2 Ny with Nx = c 2^P, Ny = c 2^Q; one sample of Z
  on that lattice serves every grid of the sample (the same realisation on
  every grid, as the multi-index differences of Section 3 need).
* Embedding: the first row of the block-circulant matrix holds
  C(dx hx, dy hy) at the wrapped displacements (dx, dy); on the half-period
  lines both signs of the displacement are averaged, which keeps the matrix
  symmetric (C(v) = C(-v) but C(vx, vy) != C(vx, -vy) once rotated).  Its
  eigenvalues are the 2D DFT of that row; Y = DFT(sqrt(Lambda / M) xi) with
  complex standard normal xi gives Re(Y) ~ N(0, C) on the lattice.  The
  smallest eigenvalue over the largest is returned: below zero the
  embedding is not positive semi-definite (negative eigenvalues are then
  clamped to zero, and the sample is only approximate).
* Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel
  random numbers: as easy as 1, 2, 3", SC 2011) with counter
  (n, sample id, 0, 0) and key (seed, KEY1) for the pair n of embedding
  points l = 2n, 2n+1 (row-major, x fastest); its four words give, through
  u = ((w >> 12) + 1/2) 2^-52 (exact in FP64, strictly inside (0,1)) and the
  Box-Muller transform (Box and Muller 1958), the real and imaginary normals
  of point 2n (words 0, 1) and of point 2n + 1 (words 2, 3).
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np
from scipy import special

KEY1 = 0x6D617465726E  # second key word of the field's random stream

_M0, _M1 = np.uint64(0xD2E7470EE14C6C93), np.uint64(0xCA5A826395121157)
_W0, _W1 = np.uint64(0x9E3779B97F4A7C15), np.uint64(0xBB67AE8584CAA73B)
_LO = np.uint64(0xFFFFFFFF)
_32 = np.uint64(32)


def _mulhilo(a, b):
    """(high, low) 64-bit halves of the 128-bit product, by 32-bit limbs."""
    a0, a1 = a & _LO, a >> _32
    b0, b1 = b & _LO, b >> _32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _32) + (p01 & _LO) + (p10 & _LO)
    hi = p11 + (p01 >> _32) + (p10 >> _32) + (mid >> _32)
    return hi, a * b


def philox4x64(c0, c1, c2, c3, k0, k1):
    """Philox4x64-10 of counters (arrays) under key (k0, k1)."""
    c = [np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3)]
    k0, k1 = np.uint64(k0), np.uint64(k1)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0, k1 = k0 + _W0, k1 + _W1
            hi0, lo0 = _mulhilo(_M0, c[0])
            hi1, lo1 = _mulhilo(_M1, c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def uniform52(w):
    """(0,1) uniform from the top 52 bits of a 64-bit word (exact: k + 1/2
    with k < 2^52 needs 53 significant bits)."""
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def box_muller(wa, wb):
    ua, ub = uniform52(wa), uniform52(wb)
    rho = np.sqrt(-2.0 * np.log(ua))
    return rho * np.cos(2.0 * math.pi * ub), rho * np.sin(2.0 * math.pi * ub)


def embedding_normals(Mx: int, My: int, sample_id: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Real and imaginary standard normals on the My x Mx embedding lattice."""
    M = Mx * My
    n = np.arange(M // 2, dtype=np.uint64)
    zero = np.zeros_like(n)
    w = philox4x64(n, np.full_like(n, sample_id), zero, zero, seed, KEY1)
    re0, im0 = box_muller(w[0], w[1])
    re1, im1 = box_muller(w[2], w[3])
    re = np.empty(M)
    im = np.empty(M)
    re[0::2], re[1::2] = re0, re1
    im[0::2], im[1::2] = im0, im1
    return re.reshape(My, Mx), im.reshape(My, Mx)


# ---------------------------------------------------------------- covariance
def matern(r, nu: float):
    """eq. matern as a function of the transformed distance r."""
    r = np.asarray(r, dtype=np.float64)
    z = 2.0 * math.sqrt(nu) * r
    out = np.ones_like(z)
    pos = z > 0
    out[pos] = 2.0 ** (1.0 - nu) / math.gamma(nu) * z[pos] ** nu * special.kv(nu, z[pos])
    return out


def transform(lam: float, eta: float, theta: float) -> np.ndarray:
    """T = S R (theta in radians)."""
    S = np.diag([1.0 / math.sqrt(eta * lam), 1.0 / math.sqrt(lam)])
    R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    return S @ R


def covariance(dx, dy, lam: float, nu: float, eta: float, theta: float):
    """C between points displaced by (dx, dy) in the unit square."""
    T = transform(lam, eta, theta)
    dx, dy = np.asarray(dx, dtype=np.float64), np.asarray(dy, dtype=np.float64)
    tx = T[0, 0] * dx + T[0, 1] * dy
    ty = T[1, 0] * dx + T[1, 1] * dy
    return matern(np.sqrt(tx * tx + ty * ty), nu)


# ---------------------------------------------------------------- embedding
def pad_factor(nu: float, n: int) -> int:
    return 1 + 2 * math.ceil(math.sqrt(nu) * math.log2(n))


def _pow2(x: int) -> int:
    return 1 << max(0, int(x - 1).bit_length())


def embedding_shape(Nx: int, Ny: int, nu: float, pad: int = 0) -> Tuple[int, int]:
    """(Mx, My) of the embedding of the (2Nx+1) x (2Ny+1) half-step lattice."""
    m = pad if pad > 0 else pad_factor(nu, max(Nx, Ny))
    m = max(m, 2)                     # at least the minimal embedding, 2 (2N) points
    return _pow2(m * 2 * Nx), _pow2(m * 2 * Ny)


def _wrapped(M: int):
    i = np.arange(M)
    d = np.where(i <= M // 2, i, i - M)
    d_alt = np.where(i == M // 2, -d, d)      # the other sign on the half-period line
    return d, d_alt


def first_row(Mx: int, My: int, hx: float, hy: float, lam: float, nu: float, eta: float, theta: float):
    """Block-circulant first row c[iy, ix] (x fastest)."""
    dx, dxa = _wrapped(Mx)
    dy, dya = _wrapped(My)
    acc = np.zeros((My, Mx))
    for X in (dx, dxa):
        for Y in (dy, dya):
            acc += covariance(X[None, :] * hx, Y[:, None] * hy, lam, nu, eta, theta)
    return acc / 4.0


def sample_embedding(c: np.ndarray, re: np.ndarray, im: np.ndarray) -> Tuple[np.ndarray, float]:
    """Re(DFT(sqrt(Lambda / M) (re + i im))) and min(Lambda) / max(Lambda)."""
    lam = np.fft.fft2(c).real
    ratio = float(lam.min() / lam.max())
    s = np.sqrt(np.maximum(lam, 0.0) / c.size)
    return np.fft.fft2(s * (re + 1j * im)).real, ratio


def lattice_field(c: int, P: int, Q: int, lam: float, nu: float, eta: float, theta: float, sample_id: int,
                  seed: int, pad: int = 0) -> Tuple[np.ndarray, float]:
    """Z on the half-step lattice of the finest grid, [b, a] = (y, x); and
    the embedding's smallest eigenvalue ratio."""
    Nx, Ny = c << P, c << Q
    Mx, My = embedding_shape(Nx, Ny, nu, pad)
    row = first_row(Mx, My, 1.0 / (2 * Nx), 1.0 / (2 * Ny), lam, nu, eta, theta)
    re, im = embedding_normals(Mx, My, sample_id, seed)
    Y, ratio = sample_embedding(row, re, im)
    return Y[:2 * Ny + 1, :2 * Nx + 1], ratio


def hierarchy_field(c: int, P: int, Q: int, lam: float, nu: float, eta: float, theta: float, sample_id: int,
                    seed: int, pad: int = 0):
    """k = exp(Z) at the x- and y-face midpoints of every grid (p,q) of the
    rectangle, packed p-major, q-minor, row-major with x fastest; and the
    embedding's smallest eigenvalue ratio."""
    Z, ratio = lattice_field(c, P, Q, lam, nu, eta, theta, sample_id, seed, pad)
    kxs, kys = [], []
    for p in range(P + 1):
        for q in range(Q + 1):
            nx, ny = c << p, c << q
            i = np.arange(nx + 1)[None, :]
            j = np.arange(ny)[:, None]
            kxs.append(np.exp(Z[(2 * j + 1) << (Q - q), i << (P - p + 1)]).ravel())
            i = np.arange(nx)[None, :]
            j = np.arange(ny + 1)[:, None]
            kys.append(np.exp(Z[j << (Q - q + 1), (2 * i + 1) << (P - p)]).ravel())
    return np.concatenate(kxs), np.concatenate(kys), ratio
