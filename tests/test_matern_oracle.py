"""Pins of the Matern circulant-embedding oracle (oracle/matern_oracle.py)
against facts outside itself: an independent Philox implementation, closed
forms of the Matern covariance, the geometry of the transformation T = S R,
the defining property of an exact sampler (its linear map B from the normals
to the lattice values satisfies B B^T = C), positive definiteness of the
embedding at the paper's parameters, and the nesting of the grids' faces."""
import math

import numpy as np
import pytest

from oracle import matern_oracle as MO

PAPER = dict(lam=0.25, nu=0.5)


def test_philox_matches_numpy_bit_generator():
    """numpy's Philox is Philox4x64-10 and advances its counter before each
    block: its first four raw words are philox(counter + 1, key)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2)
        raw = np.random.Philox(counter=ctr, key=key).random_raw(4)
        with np.errstate(over="ignore"):
            c0 = ctr[0] + np.uint64(1)
        mine = MO.philox4x64(c0, ctr[1], ctr[2], ctr[3], key[0], key[1])
        assert [int(x) for x in mine] == [int(x) for x in raw]


def test_box_muller_values_and_moments():
    wa = np.array([0, 2 ** 63, 2 ** 64 - 1], dtype=np.uint64)
    ua = MO.uniform52(wa)
    assert ua[0] == 0.5 * 2.0 ** -52 and ua[1] == 0.5 + 0.5 * 2.0 ** -52 and ua[2] == 1.0 - 0.5 * 2.0 ** -52
    z0, z1 = MO.box_muller(np.array([2 ** 63], dtype=np.uint64), np.array([2 ** 62], dtype=np.uint64))
    rho = math.sqrt(-2.0 * math.log(0.5 + 0.5 * 2.0 ** -52))
    u = 0.25 + 0.5 * 2.0 ** -52
    assert math.isclose(z0[0], rho * math.cos(2 * math.pi * u), abs_tol=1e-15)
    assert math.isclose(z1[0], rho * math.sin(2 * math.pi * u), rel_tol=1e-15)
    re, im = MO.embedding_normals(512, 512, 3, 11)
    n = re.size
    for x in (re, im):
        assert abs(x.mean()) < 5 / math.sqrt(n) and abs(x.var() - 1) < 5 * math.sqrt(2 / n)
        assert abs(np.mean(x ** 4) - 3) < 0.05
    assert abs(np.mean(re * im)) < 5 / math.sqrt(n)
    assert abs(np.mean(re[:, 1:] * re[:, :-1])) < 5 / math.sqrt(n)   # neighbours (pairs) independent
    # different samples draw different streams
    re2, _ = MO.embedding_normals(512, 512, 4, 11)
    assert abs(np.mean(re * re2)) < 5 / math.sqrt(n)


@pytest.mark.parametrize("r", [0.0, 1e-9, 0.01, 0.3, 1.0, 4.0])
def test_matern_closed_forms(r):
    assert math.isclose(MO.matern(r, 0.5), math.exp(-math.sqrt(2) * r), rel_tol=1e-12)
    s6, s10 = math.sqrt(6) * r, math.sqrt(10) * r
    assert math.isclose(MO.matern(r, 1.5), (1 + s6) * math.exp(-s6), rel_tol=1e-12)
    assert math.isclose(MO.matern(r, 2.5), (1 + s10 + s10 * s10 / 3) * math.exp(-s10), rel_tol=1e-12)


def test_transformation_geometry():
    lam, nu, eta = 0.25, 0.5, 1 / 16
    d = 0.07
    # theta = 0: x is scaled by 1/sqrt(eta lam), y by 1/sqrt(lam)
    assert math.isclose(MO.covariance(d, 0.0, lam, nu, eta, 0.0), math.exp(-math.sqrt(2) * d / math.sqrt(eta * lam)))
    assert math.isclose(MO.covariance(0.0, d, lam, nu, eta, 0.0), math.exp(-math.sqrt(2) * d / math.sqrt(lam)))
    rng = np.random.default_rng(0)
    dx, dy = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50)
    th = 0.3
    c = MO.covariance(dx, dy, lam, nu, eta, th)
    assert np.allclose(c, MO.covariance(-dx, -dy, lam, nu, eta, th), rtol=1e-14)          # stationary, even
    assert np.allclose(c, MO.covariance(dx, dy, lam, nu, eta, th + math.pi), rtol=1e-13)  # half turn
    assert np.allclose(MO.covariance(dx, dy, lam, nu, eta, math.pi / 2),
                       MO.covariance(dy, dx, lam, nu, eta, 0.0), rtol=1e-13)              # quarter turn swaps axes
    assert not np.allclose(c, MO.covariance(dx, -dy, lam, nu, eta, th), rtol=1e-3)          # rotated: not mirror-even
    # isotropic (eta = 1): every rotation gives the same covariance
    assert np.allclose(MO.covariance(dx, dy, lam, nu, 1.0, 0.0), MO.covariance(dx, dy, lam, nu, 1.0, 1.1), rtol=1e-13)


def _sampler_matrix(c, P, Q, lam, nu, eta, theta, pad=0):
    Nx, Ny = c << P, c << Q
    Mx, My = MO.embedding_shape(Nx, Ny, nu, pad)
    row = MO.first_row(Mx, My, 1 / (2 * Nx), 1 / (2 * Ny), lam, nu, eta, theta)
    cols = []
    for part in ("re", "im"):
        for q in range(Mx * My):
            e = np.zeros((My, Mx))
            e.flat[q] = 1.0
            z = np.zeros((My, Mx))
            Y, ratio = MO.sample_embedding(row, *((e, z) if part == "re" else (z, e)))
            cols.append(Y[:2 * Ny + 1, :2 * Nx + 1].ravel())
    return np.array(cols).T, ratio


@pytest.mark.parametrize("c,P,Q,eta,theta", [(1, 1, 1, 1 / 16, math.radians(20)), (1, 2, 1, 1 / 4, math.radians(-30)),
                                             (2, 0, 1, 1 / 8, math.radians(10))])
def test_embedding_is_an_exact_sampler(c, P, Q, eta, theta):
    """B B^T equals the covariance matrix of the lattice points, evaluated
    from the definition at their physical displacements."""
    lam, nu = PAPER["lam"], PAPER["nu"]
    Nx, Ny = c << P, c << Q
    B, ratio = _sampler_matrix(c, P, Q, lam, nu, eta, theta)
    assert ratio > -1e-12
    a, b = np.meshgrid(np.arange(2 * Nx + 1) / (2 * Nx), np.arange(2 * Ny + 1) / (2 * Ny))
    x, y = a.ravel(), b.ravel()
    C = MO.covariance(x[:, None] - x[None, :], y[:, None] - y[None, :], lam, nu, eta, theta)
    assert np.max(np.abs(B @ B.T - C)) < 1e-12


@pytest.mark.parametrize("cells", [8, 32, 64])
@pytest.mark.parametrize("eta,theta_deg", [(1 / 16, 0), (1 / 16, 30), (1 / 16, -30), (1 / 4, 10), (1 / 4, 0), (1.0, 0)])
def test_paper_parameters_embed_positive_definite(cells, eta, theta_deg):
    lam, nu = PAPER["lam"], PAPER["nu"]
    Mx, My = MO.embedding_shape(cells, cells, nu)
    row = MO.first_row(Mx, My, 1 / (2 * cells), 1 / (2 * cells), lam, nu, eta, math.radians(theta_deg))
    lam_ = np.fft.fft2(row)
    assert np.max(np.abs(lam_.imag)) < 1e-9 * np.max(lam_.real)    # symmetric first row
    assert lam_.real.min() / lam_.real.max() > -1e-12


def test_too_small_embedding_is_detected():
    """A long correlation on the minimal embedding is indefinite: the ratio
    reports it (the paper's padding exists for this reason)."""
    Mx, My = MO.embedding_shape(8, 8, 0.5, pad=1)
    row = MO.first_row(Mx, My, 1 / 16, 1 / 16, 4.0, 2.5, 1.0, 0.0)
    _, ratio = MO.sample_embedding(row, np.zeros((My, Mx)), np.zeros((My, Mx)))
    assert ratio < -1e-6


def test_pad_factor_and_shape():
    assert MO.pad_factor(0.5, 64) == 1 + 2 * math.ceil(math.sqrt(0.5) * 6) == 11
    assert MO.pad_factor(0.5, 2) == 3
    assert MO.embedding_shape(64, 64, 0.5) == (2048, 2048)
    assert MO.embedding_shape(64, 16, 0.5) == (2048, 512)
    assert MO.embedding_shape(4, 4, 0.5, pad=1) == (16, 16)


def test_faces_shared_between_grids_coincide():
    c, P, Q = 2, 3, 2
    kx, ky, ratio = MO.hierarchy_field(c, P, Q, 0.25, 0.5, 1 / 16, 0.4, 7, 99)
    assert ratio > -1e-12
    off_x, off_y, g = 0, 0, {}
    for p in range(P + 1):
        for q in range(Q + 1):
            nx, ny = c << p, c << q
            g[(p, q)] = (kx[off_x:off_x + (nx + 1) * ny].reshape(ny, nx + 1),
                         ky[off_y:off_y + nx * (ny + 1)].reshape(ny + 1, nx))
            off_x += (nx + 1) * ny
            off_y += nx * (ny + 1)
    assert off_x == kx.size and off_y == ky.size
    # x-faces of (p,q) at even i are x-faces of (p-1,q) (same x, same y rows)
    for p in range(1, P + 1):
        for q in range(Q + 1):
            assert np.array_equal(g[(p, q)][0][:, ::2], g[(p - 1, q)][0])
    # y-faces of (p,q) at even j are y-faces of (p,q-1)
    for p in range(P + 1):
        for q in range(1, Q + 1):
            assert np.array_equal(g[(p, q)][1][::2, :], g[(p, q - 1)][1])
    assert np.all(kx > 0) and np.all(ky > 0)


def test_samples_are_reproducible_and_distinct():
    a = MO.lattice_field(2, 2, 2, 0.25, 0.5, 0.1, 0.2, 5, 123)[0]
    b = MO.lattice_field(2, 2, 2, 0.25, 0.5, 0.1, 0.2, 5, 123)[0]
    d = MO.lattice_field(2, 2, 2, 0.25, 0.5, 0.1, 0.2, 6, 123)[0]
    assert np.array_equal(a, b) and not np.allclose(a, d)
