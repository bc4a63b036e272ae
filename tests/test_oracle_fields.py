"""Pins of the oracle's coefficient fields against facts outside itself.

* The separable squared-exponential expansion: its exact covariance, built
  from the field's linear dependence on the normals (unit vectors fed through
  the oracle), against the closed form that Poisson summation gives for a
  cosine series with eigenvalues proportional to exp(-pi^2 l^2 k^2 / 2): the
  squared-exponential shape exp(-d^2 / (2 l^2)) plus wall images, with
  variance (s / l) / (1 + s / l), s = sqrt(2 / pi), at interior points.
* The face-mean rule: closed forms of midpoint sums of cosines, and the
  Galerkin identities that make its coarse operators consistent with the
  fine ones (R A P with the oracle's own restriction and prolongation).
* The counter-based normals: numpy's independent Philox bit generator and
  the Box-Muller map.
* Why the face-mean reading exists: on strongly anisotropic fields the
  pointwise rule diverges on grids too coarse for the field, the face mean
  converges (residual histories of the oracle).
"""
import math

import numpy as np
import pytest

from paper_1907_12334_amd import inputs as I

S2PI = math.sqrt(2.0 / math.pi)


def _linear_map(oracle, nx, ny, mx, my, lx, ly, sigma2, which):
    """Z at every face (which = 0: x-faces, 1: y-faces) for each unit normal:
    rows are terms, columns faces.  Z is linear in xi, so Cov = A^T A."""
    rows = []
    for t in range(mx * my):
        e = np.zeros(mx * my)
        e[t] = 1.0
        kx, ky = oracle.field_separable(nx, ny, mx, my, lx, ly, sigma2, e)
        rows.append(np.log(kx if which == 0 else ky))
    return np.array(rows)


def _se_1d(x1, x2, l):
    """Exact covariance of the infinite cosine series in one direction
    (Poisson summation over the images of the reflected kernel), normalised
    so that its eigenvalues sum to one."""
    tot = 0.0
    for n in range(-3, 4):
        tot += math.exp(-((x1 - x2 - 2 * n) ** 2) / (2 * l * l)) + math.exp(-((x1 + x2 - 2 * n) ** 2) / (2 * l * l))
    norm = 1.0 + (S2PI / l) * sum(math.exp(-((2 * n) ** 2) / (2 * l * l)) for n in range(-3, 4))
    return (S2PI / l) * tot / 2.0 / (norm / 2.0)


@pytest.mark.parametrize("l", [0.1, 0.2])
def test_separable_decay_law_gives_the_squared_exponential_covariance(oracle, l):
    """One direction at a time (the other has one mode, phi_0 = 1): the
    50-term expansion's covariance between x-faces equals sigma^2 times the
    reflected squared-exponential kernel of length l, to 1e-12; away from
    the walls the correlation is exp(-d^2 / (2 l^2)).  Dropping the /2 of
    the decay law (length sqrt(2) l) fails this by far."""
    sigma2 = 1.7
    nx = 40
    A = _linear_map(oracle, nx, 2, 50, 1, l, 0.5, sigma2, 0)
    C = A.T @ A                                             # x-faces (nx+1) * 2 rows
    xs = np.arange(nx + 1) / nx
    for i in range(nx + 1):
        for j in range(nx + 1):
            want = sigma2 * _se_1d(xs[i], xs[j], l)
            assert abs(C[i, j] - want) <= 1e-12 * sigma2, (i, j, C[i, j], want)
    # interior: pure squared-exponential shape and the closed-form variance
    mid = [i for i in range(nx + 1) if 5 * l <= xs[i] <= 1 - 5 * l]
    for i in mid:
        assert abs(C[i, i] - sigma2 * (S2PI / l) / (1 + S2PI / l)) <= 1e-12 * sigma2
        for j in mid:
            assert abs(C[i, j] / C[i, i] - math.exp(-((xs[i] - xs[j]) ** 2) / (2 * l * l))) <= 1e-12


def test_separable_decay_law_in_y_and_the_mode_pairing(oracle):
    """Both directions with different lengths: the covariance is the product
    of the two one-dimensional kernels, which pins the pairing of xi index
    m*my + n with x-mode m and y-mode n."""
    lx, ly, sigma2 = 0.5, 0.35, 0.8
    nx, ny, mx, my = 6, 5, 9, 12
    A = _linear_map(oracle, nx, ny, mx, my, lx, ly, sigma2, 1)   # y-faces
    C = A.T @ A
    pts = [((i + 0.5) / nx, j / ny) for j in range(ny + 1) for i in range(nx)]
    # truncation at 9 and 12 modes leaves exp(-pi^2 l^2 m^2 / 2) < 1e-12 relative
    for a, (x1, y1) in enumerate(pts):
        for b, (x2, y2) in enumerate(pts):
            want = sigma2 * _se_1d(x1, x2, lx) * _se_1d(y1, y2, ly)
            assert abs(C[a, b] - want) <= 1e-11 * sigma2, (a, b)


# ---------------------------------------------------------------- face mean
def _cos_mean(b, y0, m, h):
    """(1/m) sum_t cos(pi b (y0 + (t + 1/2) h)) in closed form (a Dirichlet sum)."""
    if b == 0:
        return 1.0
    return math.cos(math.pi * b * (y0 + m * h / 2)) * math.sin(m * math.pi * b * h / 2) / (
        m * math.sin(math.pi * b * h / 2))


@pytest.mark.parametrize("c,P,Q,p,q", [(4, 3, 2, 1, 0), (2, 4, 4, 2, 3), (4, 2, 3, 2, 1), (2, 3, 1, 0, 1)])
def test_face_mean_of_separable_cosines(oracle, c, P, Q, p, q):
    """Finest faces carrying g(x) h(y) with cosines: every coarse x-face
    takes g at its own x (it lies on a finest face column) and the midpoint
    mean of h along it in closed form; y-faces likewise."""
    nxF, nyF, nx, ny = c << P, c << Q, c << p, c << q
    a, b = 3, 5
    g = lambda x: 2.0 + math.cos(math.pi * a * x)
    h = lambda y: 2.0 + math.cos(math.pi * b * y)
    kxF = np.array([[g(i / nxF) * h((j + 0.5) / nyF) for i in range(nxF + 1)] for j in range(nyF)]).ravel()
    kyF = np.array([[g((i + 0.5) / nxF) * h(j / nyF) for i in range(nxF)] for j in range(nyF + 1)]).ravel()
    kx, ky = oracle.face_mean(c, P, Q, kxF, kyF, p, q)
    m = 1 << (Q - q)
    for j in range(ny):
        for i in range(nx + 1):
            want = g(i / nx) * (2.0 + _cos_mean(b, j / ny, m, 1.0 / nyF))
            assert abs(kx[j * (nx + 1) + i] - want) <= 1e-14 * abs(want)
    m = 1 << (P - p)
    for j in range(ny + 1):
        for i in range(nx):
            want = (2.0 + _cos_mean(a, i / nx, m, 1.0 / nxF)) * h(j / ny)
            assert abs(ky[j * nx + i] - want) <= 1e-14 * abs(want)


def test_face_mean_leaves_the_finest_grid_pointwise(oracle):
    w = I.config(4)
    spec = w.field.as_dict()
    xi = w.xi([3])[0]
    kx, ky = oracle.hierarchy_field(4, 2, 1, spec, xi)
    fx, fy = oracle.field_separable(16, 8, 50, 50, spec["lx"], spec["ly"], spec["sigma2"], xi)
    nfx, nfy = 17 * 8, 16 * 9
    assert np.array_equal(kx[-nfx:], fx) and np.array_equal(ky[-nfy:], fy)


def _dense(oracle, nx, ny, kx, ky):
    n = nx * ny
    A = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = oracle.apply(nx, ny, kx, ky, e)
    return A


def _transfers(oracle, nx, ny, direction):
    """R (average of two fine cells) and P (linear, odd reflection) between a
    fine grid and its coarsening in one direction, as matrices."""
    if direction == "y":
        nc, n = nx * (ny // 2), nx * ny
        R = np.column_stack([oracle.restrict_y(nx, ny // 2, np.eye(n)[:, k]) for k in range(n)])
        Pm = np.column_stack([oracle.prolong_y(nx, ny // 2, np.eye(nc)[:, k]) for k in range(nc)])
    else:
        nc, n = (nx // 2) * ny, nx * ny
        R = np.column_stack([oracle.restrict_x(nx // 2, ny, np.eye(n)[:, k]) for k in range(n)])
        Pm = np.column_stack([oracle.prolong_x(nx // 2, ny, np.eye(nc)[:, k]) for k in range(nc)])
    return R, Pm


@pytest.mark.parametrize("direction", ["x", "y"])
def test_face_mean_normal_coefficients_are_galerkin(oracle, direction):
    """Only the faces normal to the coarsening direction conduct (the other
    faces carry k = 0): the grid lines then decouple into one-dimensional
    chains, and R A_fine P equals the coarse operator of the face-mean rule
    exactly, walls included (the coarse face takes the conductance of the
    fine face it lies on)."""
    rng = np.random.default_rng(11)
    c = 2
    P, Q = (2, 1) if direction == "x" else (1, 2)
    nxF, nyF = c << P, c << Q
    kxF = np.exp(rng.normal(0, 1.5, (nxF + 1) * nyF))
    kyF = np.exp(rng.normal(0, 1.5, nxF * (nyF + 1)))
    if direction == "x":
        kyF[:] = 0.0
        p, q = P - 1, Q
    else:
        kxF[:] = 0.0
        p, q = P, Q - 1
    kx, ky = oracle.face_mean(c, P, Q, kxF, kyF, p, q)
    Af = _dense(oracle, nxF, nyF, kxF, kyF)
    Ac = _dense(oracle, c << p, c << q, kx, ky)
    R, Pm = _transfers(oracle, nxF, nyF, direction)
    G = R @ Af @ Pm
    assert np.allclose(G, Ac, rtol=0, atol=1e-12 * np.abs(Ac).max())


@pytest.mark.parametrize("direction", ["x", "y"])
def test_face_mean_along_the_face_is_lumped_galerkin(oracle, direction):
    """Only the faces parallel to the coarsening direction conduct: R A P then
    couples neighbouring coarse lines through P's spread, and summing those
    couplings (lumping) over the coarsened direction gives the coarse
    operator of the face-mean rule on every interior coarse line (the mean
    along the face); an arithmetic mean, not a harmonic one."""
    rng = np.random.default_rng(12)
    c = 2
    P, Q = (3, 1) if direction == "x" else (1, 3)
    nxF, nyF = c << P, c << Q
    kxF = np.exp(rng.normal(0, 1.5, (nxF + 1) * nyF))
    kyF = np.exp(rng.normal(0, 1.5, nxF * (nyF + 1)))
    if direction == "x":
        kxF[:] = 0.0
        p, q = P - 1, Q
    else:
        kyF[:] = 0.0
        p, q = P, Q - 1
    kx, ky = oracle.face_mean(c, P, Q, kxF, kyF, p, q)
    nx, ny = c << p, c << q
    Af = _dense(oracle, nxF, nyF, kxF, kyF)
    Ac = _dense(oracle, nx, ny, kx, ky)
    R, Pm = _transfers(oracle, nxF, nyF, direction)
    G = R @ Af @ Pm
    checked = 0
    for J in range(ny):
        for I_ in range(nx):
            line = I_ if direction == "x" else J
            nlines = nx if direction == "x" else ny
            if line == 0 or line == nlines - 1:
                continue                                       # P's rows sum to 1/2 at the walls
            row = J * nx + I_
            for d in (-1, 0, 1):                               # neighbours along the conducting direction
                if direction == "x":
                    if not 0 <= J + d < ny:
                        continue
                    cols = [(J + d) * nx + a for a in range(nx)]
                    want = Ac[row, (J + d) * nx + I_]
                else:
                    if not 0 <= I_ + d < nx:
                        continue
                    cols = [b * nx + I_ + d for b in range(ny)]
                    want = Ac[row, J * nx + I_ + d]
                got = G[row, cols].sum()
                assert abs(got - want) <= 1e-12 * np.abs(Ac).max()
                checked += 1
    assert checked > 10


# ---------------------------------------------------------------- normals
def test_kl_normals_follow_numpy_philox():
    """The stream (seed, id) is numpy's Philox4x64-10 started one before the
    256-bit counter (n, id, 0, 0) (numpy advances it before each block), key
    (seed, KEY_KL), mapped by Box-Muller to four normals per block."""
    from oracle import normals as N
    from oracle import matern_oracle as MO
    seed, ids = 20190726, [0, 5, 1 << 40]
    xi = N.kl_normals(23, ids, seed)
    for row, sid in enumerate(ids):
        for n in range(6):
            v = (n + (sid << 64) - 1) % (1 << 256)              # the 256-bit counter minus one
            ctr = np.array([(v >> (64 * k)) & ((1 << 64) - 1) for k in range(4)], dtype=np.uint64)
            key = np.array([seed, N.KEY_KL], dtype=np.uint64)
            w = np.random.Philox(counter=ctr, key=key).random_raw(4)
            z = MO.box_muller(w[0:1], w[1:2]) + MO.box_muller(w[2:3], w[3:4])
            for h in range(4):
                if 4 * n + h < 23:
                    assert xi[row, 4 * n + h] == z[h][0]


def test_kl_normals_moments_and_independence():
    from oracle import normals as N
    xi = N.kl_normals(2500, range(80), 7)                   # 200 000 draws
    n = xi.size
    assert abs(xi.mean()) <= 4 / math.sqrt(n)
    assert abs(xi.var() - 1.0) <= 4 * math.sqrt(2.0 / n)
    assert abs(np.mean(xi[:, 0::2] * xi[:, 1::2])) <= 4 / math.sqrt(n / 2)   # cosine and sine of a pair
    assert abs(np.mean(xi[0] * xi[1])) <= 4 / math.sqrt(2500)                 # streams of two ids


# ---------------------------------------------------------------- why the face mean
@pytest.mark.parametrize("sid", [5, 48])
def test_face_mean_converges_where_pointwise_diverges(oracle, sid):
    """Samples of the 1024x64 preset (ly = 0.01, sigma^2 = 2): with k taken
    pointwise on every grid, some grid's cycles grow the residual (the
    coarse operators of grids that do not resolve the field are unrelated to
    their fine grids); with the face mean, every grid converges."""
    w = I.config(4)
    spec = dict(w.field.as_dict())
    xi = w.xi([sid])[0]
    kx, ky = oracle.hierarchy_field(4, 8, 4, spec, xi)
    r1 = oracle.fmsg_solve(4, 8, 4, kx, ky, oracle.opts(max_cycles=150, tol=1e-10))
    assert r1["status"] == 0 and r1["cycles"].max() < 150
    o = oracle.opts(max_cycles=60, tol=1e-10)
    spec["face_rule"] = 0
    kx, ky = oracle.hierarchy_field(4, 8, 4, spec, xi)
    r0 = oracle.fmsg_solve(4, 8, 4, kx, ky, o, want_hist=True)
    h = r0["hist"]
    grows = [g for g in range(h.shape[0])
             if np.sum(~np.isnan(h[g])) > 10 and h[g][10] > 10 * h[g][2]]
    assert r0["status"] != 0 and grows
