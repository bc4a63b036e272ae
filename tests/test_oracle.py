"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks a closed form, an
identity, a library routine or a property that a plausible mistake in the
oracle (a dropped wall factor, a swapped direction, a wrong colour order, a
wrong restriction case, a wrong sign in the multi-index difference) breaks.
"""
import fractions
import math
import os

import numpy as np
import pytest

from paper_1907_12334_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def kl10_faces(O, nx, ny, sid=3):
    xi = I.draw_xi(10, [sid])[0]
    return O.field_cos(nx, ny, I.KL10_A, I.KL10_B, I.KL10_AMP, xi)


def const_faces(nx, ny, K=1.0):
    return np.full((nx + 1) * ny, K), np.full(nx * (ny + 1), K)


def cell_centres(nx, ny):
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    return np.meshgrid(x, y)          # (ny, nx) arrays


def dense(O, nx, ny, kx, ky):
    n = nx * ny
    A = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = O.apply(nx, ny, kx, ky, e)
    return A


# ---------------------------------------------------------------- operator
@pytest.mark.parametrize("nx,ny", [(2, 2), (4, 4), (8, 32), (64, 4), (16, 8)])
@pytest.mark.parametrize("m,n", [(1, 1), (2, 3)])
def test_sine_modes_are_exact_eigenvectors(oracle, nx, ny, m, n):
    """Cell-centred sine modes satisfy A s = K lambda_h s exactly (odd
    reflection at the Dirichlet walls), lambda_h = sum 4/h^2 sin^2(m pi h/2)."""
    K = 1.7
    kx, ky = const_faces(nx, ny, K)
    X, Y = cell_centres(nx, ny)
    s = (np.sin(m * np.pi * X) * np.sin(n * np.pi * Y)).ravel()
    hx, hy = 1.0 / nx, 1.0 / ny
    lam = 4 / hx**2 * np.sin(m * np.pi * hx / 2) ** 2 + 4 / hy**2 * np.sin(n * np.pi * hy / 2) ** 2
    As = oracle.apply(nx, ny, kx, ky, s)
    assert np.max(np.abs(As - K * lam * s)) <= 1e-12 * K * lam


@pytest.mark.parametrize("nx,ny", [(4, 8), (16, 4), (8, 8)])
def test_energy_identity_and_symmetry(oracle, nx, ny):
    """u.Au equals the sum over faces of conductance times squared jump (wall
    faces: twice the conductance, jump to zero); v.Au = u.Av."""
    kx, ky = kl10_faces(oracle, nx, ny)
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal(nx * ny), rng.standard_normal(nx * ny)
    U = u.reshape(ny, nx)
    KX = kx.reshape(ny, nx + 1)
    KY = ky.reshape(ny + 1, nx)
    hx2, hy2 = (1.0 / nx) ** 2, (1.0 / ny) ** 2
    Upad = np.pad(U, 1)                                      # zero outside the domain
    jx = Upad[1:-1, 1:] - Upad[1:-1, :-1]                    # (ny, nx+1) jumps across x-faces
    jy = Upad[1:, 1:-1] - Upad[:-1, 1:-1]                    # (ny+1, nx) jumps across y-faces
    wx = KX / hx2
    wx[:, 0] *= 2
    wx[:, -1] *= 2
    wy = KY / hy2
    wy[0, :] *= 2
    wy[-1, :] *= 2
    energy = np.sum(wx * jx**2) + np.sum(wy * jy**2)
    Au = oracle.apply(nx, ny, kx, ky, u)
    Av = oracle.apply(nx, ny, kx, ky, v)
    assert abs(u @ Au - energy) <= 1e-12 * energy
    assert abs(v @ Au - u @ Av) <= 1e-12 * np.linalg.norm(Au) * np.linalg.norm(v)


def test_operator_spd_and_interior_row_sums(oracle):
    nx, ny = 8, 4
    kx, ky = kl10_faces(oracle, nx, ny)
    A = dense(oracle, nx, ny, kx, ky)
    np.linalg.cholesky(A)                                    # raises unless SPD
    rows = A.sum(axis=1).reshape(ny, nx)
    assert np.max(np.abs(rows[1:-1, 1:-1])) <= 1e-10 * np.abs(A).max()


# ---------------------------------------------------------------- smoother
def test_rbgs_colour_order_and_fixed_point(oracle):
    """After one red-then-black sweep every black equation holds exactly while
    red ones do not; the exact solution is a fixed point."""
    nx, ny = 8, 8
    kx, ky = kl10_faces(oracle, nx, ny)
    b = np.ones(nx * ny)
    u = oracle.rbgs(nx, ny, kx, ky, b, np.zeros(nx * ny), 1)
    r = oracle.residual(nx, ny, kx, ky, b, u).reshape(ny, nx)
    J, Ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    red = (Ii + J) % 2 == 0
    scale = np.abs(b).max()
    assert np.max(np.abs(r[~red])) <= 1e-12 * scale
    assert np.max(np.abs(r[red])) > 1e-3 * scale
    A = dense(oracle, nx, ny, kx, ky)
    ustar = np.linalg.solve(A, b)
    u2 = oracle.rbgs(nx, ny, kx, ky, b, ustar, 2)
    assert np.max(np.abs(u2 - ustar)) <= 1e-12 * np.abs(ustar).max()


# ---------------------------------------------------------------- weights
@pytest.mark.parametrize("nx,ny", [(8, 8), (16, 8), (8, 32)])
def test_weights_constant_coefficient(oracle, nx, ny):
    """Interior weight for constant k: kappa_x = hy^4/(hx^4+hy^4) (1/2 for
    hx = hy, Mulder's choice; 16/17 when hx = hy/2)."""
    kx, ky = const_faces(nx, ny, 3.0)
    ka, kb = oracle.weights(nx, ny, kx, ky)
    ka, kb = ka.reshape(ny, nx), kb.reshape(ny, nx)
    hx, hy = 1.0 / nx, 1.0 / ny
    want = hy**4 / (hx**4 + hy**4)
    assert np.allclose(ka[1:-1, 1:-1], want, rtol=0, atol=1e-14)
    assert np.allclose(ka + kb, 1.0, rtol=0, atol=1e-14)
    if nx == 16 and ny == 8:
        assert np.allclose(ka[1:-1, 1:-1], 16.0 / 17.0, atol=1e-14)


def test_weights_variable_coefficient_closed_form(oracle):
    """|A f| = 2(k_W + k_E)/hx^2 plus 2 k_wall/hy^2 on cells touching a y-wall
    (f = (-1)^i; a wall face counts twice its conductance against zero)."""
    nx, ny = 8, 16
    kx, ky = kl10_faces(oracle, nx, ny)
    KX, KY = kx.reshape(ny, nx + 1), ky.reshape(ny + 1, nx)
    hx2, hy2 = (1.0 / nx) ** 2, (1.0 / ny) ** 2
    lx = 2 * (KX[:, :-1] + KX[:, 1:]) / hx2
    lx[0, :] += 2 * KY[0, :] / hy2
    lx[-1, :] += 2 * KY[-1, :] / hy2
    ly = 2 * (KY[:-1, :] + KY[1:, :]) / hy2
    ly[:, 0] += 2 * KX[:, 0] / hx2
    ly[:, -1] += 2 * KX[:, -1] / hx2
    ka, kb = oracle.weights(nx, ny, kx, ky)
    want = lx**2 / (lx**2 + ly**2)
    assert np.max(np.abs(ka.reshape(ny, nx) - want)) <= 1e-13
    assert np.max(np.abs(ka + kb - 1)) <= 1e-14


# ---------------------------------------------------------------- transfers
def test_restriction_row_sums_and_sines(oracle):
    nxc, ny = 8, 4
    assert np.allclose(oracle.restrict_x(nxc, ny, np.ones(2 * nxc * ny)), 1.0, atol=0)
    assert np.allclose(oracle.restrict_y(ny, nxc, np.ones(ny * 2 * nxc)), 1.0, atol=0)
    # averaging two sampled sines a fine cell apart gives cos(pi hf/2) sin(pi X)
    nxf = 2 * nxc
    X, _ = cell_centres(nxf, ny)
    s = np.sin(np.pi * X).ravel()
    Xc, _ = cell_centres(nxc, ny)
    want = np.cos(np.pi / nxf / 2) * np.sin(np.pi * Xc).ravel()
    assert np.max(np.abs(oracle.restrict_x(nxc, ny, s) - want)) <= 1e-15
    _, Yf = cell_centres(ny, nxf)
    s = np.sin(np.pi * Yf).ravel()
    _, Yc = cell_centres(ny, nxc)
    want = np.cos(np.pi / nxf / 2) * np.sin(np.pi * Yc).ravel()
    assert np.max(np.abs(oracle.restrict_y(ny, nxc, s) - want)) <= 1e-15


def _line_values(f, n):
    return f((np.arange(n) + 0.5) / n)


def test_linear_prolongation_reproduces_linears(oracle):
    n, ny = 8, 3
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal(2)
    for f, keep in [(lambda x: a * x + b, slice(2, -2)),       # interior
                    (lambda x: a * x, slice(0, 8)),             # vanishes on the left wall
                    (lambda x: a * (1 - x), slice(8, 16))]:     # vanishes on the right wall
        c = np.tile(_line_values(f, n), (ny, 1)).ravel()
        fine = oracle.prolong_x(n, ny, c, cubic=False).reshape(ny, 2 * n)
        want = _line_values(f, 2 * n)
        assert np.max(np.abs(fine[:, keep] - want[keep])) <= 1e-14
        cy = np.tile(_line_values(f, n)[:, None], (1, ny)).ravel()
        finey = oracle.prolong_y(ny, n, cy, cubic=False).reshape(2 * n, ny)
        assert np.max(np.abs(finey[keep, :] - want[keep, None])) <= 1e-14


def test_cubic_weights_and_reproduction(oracle):
    """Lagrange weights at t = -1/4 on nodes -2..1 are (-5,35,105,-7)/128 (exact
    rationals); the cubic FMG interpolation reproduces cubics in the interior
    and odd cubics at the left wall."""
    F = fractions.Fraction
    nodes = [-2, -1, 0, 1]
    t = F(-1, 4)
    w = []
    for k in nodes:
        v = F(1)
        for m in nodes:
            if m != k:
                v *= (t - m) / F(k - m)
        w.append(v)
    assert w == [F(-5, 128), F(35, 128), F(105, 128), F(-7, 128)]
    # the oracle applies exactly those weights: interpolate unit impulses
    n = 8
    e = np.zeros(n)
    e[4] = 1.0
    fine = oracle.prolong_x(n, 1, e, cubic=True)
    assert np.allclose(fine[[8, 10, 12, 14]], [105 / 128, 35 / 128, -5 / 128, 0.0], atol=1e-16)
    assert np.allclose(fine[[5, 7, 9, 11]], [-5 / 128, 35 / 128, 105 / 128, -7 / 128], atol=1e-16)
    rng = np.random.default_rng(4)
    cf = rng.standard_normal(4)
    poly = lambda x: cf[0] + cf[1] * x + cf[2] * x**2 + cf[3] * x**3
    odd = lambda x: cf[1] * x + cf[3] * x**3
    n = 16
    for f, keep in [(poly, slice(4, -4)), (odd, slice(0, 8))]:
        fine = oracle.prolong_y(1, n, _line_values(f, n), cubic=True)
        want = _line_values(f, 2 * n)
        assert np.max(np.abs(fine[keep] - want[keep])) <= 1e-13


# ---------------------------------------------------------------- full MSG
def _hier(O, c, P, Q, spec, sid=0):
    xi = I.draw_xi(spec.n_terms, [sid])[0]
    return O.hierarchy_field(c, P, Q, spec.as_dict(), xi)


@pytest.mark.parametrize("c,P,Q", [(2, 2, 1), (4, 1, 1), (2, 0, 3), (2, 3, 0), (4, 0, 0), (2, 2, 2)])
def test_every_grid_matches_dense_solve(oracle, c, P, Q):
    """Each returned grid solution is A^{-1} b of that grid (b = 1 on every
    grid, since the restriction of h = 1 is 1), within ||A^{-1}|| ||r|| with
    ||r|| <= tol ||b||."""
    kx, ky = _hier(oracle, c, P, Q, I.KL10, sid=5)
    tol = 1e-10
    res = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(tol=tol))
    assert res["status"] == 0
    U = oracle.split_cells(res["u"], c, P, Q)
    ox = oy = 0
    for p, q, nx, ny in oracle.grid_shapes(c, P, Q):
        gkx = kx[ox:ox + (nx + 1) * ny]
        gky = ky[oy:oy + nx * (ny + 1)]
        ox += (nx + 1) * ny
        oy += nx * (ny + 1)
        A = dense(oracle, nx, ny, gkx, gky)
        b = np.ones(nx * ny)
        ustar = np.linalg.solve(A, b)
        bound = np.linalg.norm(np.linalg.inv(A), 2) * tol * np.linalg.norm(b)
        err = np.linalg.norm(U[(p, q)].ravel() - ustar)
        assert err <= bound + 1e-13 * np.linalg.norm(ustar), (p, q, err, bound)
        if P == 0 and Q == 0:
            assert err <= 1e-13 * np.linalg.norm(ustar)        # direct coarsest solve


def _restriction_factors(c, P, Q):
    """c_{p,q} of the sine right-hand side pushed down by eq. restriction:
    restricting in a direction multiplies sin by cos(pi h_fine / 2)."""
    fac = {(P, Q): 1.0}
    for L in range(P + Q - 1, -1, -1):
        for p in range(P + 1):
            q = L - p
            if not 0 <= q <= Q:
                continue
            parts = []
            if p + 1 <= P:
                parts.append(fac[(p + 1, q)] * math.cos(math.pi / (c << (p + 1)) / 2))
            if q + 1 <= Q:
                parts.append(fac[(p, q + 1)] * math.cos(math.pi / (c << (q + 1)) / 2))
            fac[(p, q)] = sum(parts) / len(parts)
    return fac


@pytest.mark.parametrize("c,P,Q", [(4, 3, 2), (2, 1, 4)])
def test_manufactured_sine_on_every_grid(oracle, c, P, Q):
    """Constant k, b = 2 pi^2 sin sin on the finest grid: the F-cycle's
    right-hand side on (p,q) is c_pq 2 pi^2 s, so its solution is
    c_pq (2 pi^2 / lambda_h) s; the discretisation error 2pi^2/lambda_h - 1
    is O(h^2)."""
    kx, ky = _hier(oracle, c, P, Q, I.constant_field())
    nxT, nyT = c << P, c << Q
    X, Y = cell_centres(nxT, nyT)
    rhs = (2 * np.pi**2 * np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()
    res = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(tol=1e-12), rhs_top=rhs)
    U = oracle.split_cells(res["u"], c, P, Q)
    fac = _restriction_factors(c, P, Q)
    for p, q, nx, ny in oracle.grid_shapes(c, P, Q):
        hx, hy = 1.0 / nx, 1.0 / ny
        lam = 4 / hx**2 * np.sin(np.pi * hx / 2) ** 2 + 4 / hy**2 * np.sin(np.pi * hy / 2) ** 2
        Xg, Yg = cell_centres(nx, ny)
        s = np.sin(np.pi * Xg) * np.sin(np.pi * Yg)
        want = fac[(p, q)] * 2 * np.pi**2 / lam * s
        assert np.max(np.abs(U[(p, q)] - want)) <= 1e-10 * np.abs(want).max(), (p, q)
        assert abs(2 * np.pi**2 / lam - 1) <= 0.5 * (np.pi**2 / 12) * (hx**2 + hy**2) * 2
        # Q = mean over cells; sum_i sin(pi (i+1/2)/n) = 1 / sin(pi/(2n))
        qmean = fac[(p, q)] * 2 * np.pi**2 / lam / (nx * np.sin(np.pi / (2 * nx))) / (ny * np.sin(np.pi / (2 * ny)))
        assert res["q"][p * (Q + 1) + q] == pytest.approx(qmean, rel=1e-10)


def test_transposed_problem_gives_transposed_solution(oracle):
    """Swapping x and y (field, rectangle) transposes every grid's solution."""
    c, P, Q = 2, 3, 1
    kx, ky = _hier(oracle, c, P, Q, I.KL10, sid=9)
    res = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts())
    # build the transposed packing: grid (q,p) of the transposed problem
    kxg, kyg = {}, {}
    ox = oy = 0
    for p, q, nx, ny in oracle.grid_shapes(c, P, Q):
        kxg[(p, q)] = kx[ox:ox + (nx + 1) * ny].reshape(ny, nx + 1)
        kyg[(p, q)] = ky[oy:oy + nx * (ny + 1)].reshape(ny + 1, nx)
        ox += (nx + 1) * ny
        oy += nx * (ny + 1)
    tkx, tky = [], []
    for p, q, nx, ny in oracle.grid_shapes(c, Q, P):
        tkx.append(kyg[(q, p)].T.ravel())      # x-faces of the transposed grid are y-faces
        tky.append(kxg[(q, p)].T.ravel())
    rt = oracle.fmsg_solve(c, Q, P, np.concatenate(tkx), np.concatenate(tky), oracle.opts())
    U = oracle.split_cells(res["u"], c, P, Q)
    UT = oracle.split_cells(rt["u"], c, Q, P)
    for (p, q), u in U.items():
        assert np.max(np.abs(UT[(q, p)].T - u)) <= 1e-12 * np.abs(u).max()
        assert res["cycles"][p * (Q + 1) + q] == rt["cycles"][q * (P + 1) + p]


# ---------------------------------------------------------------- convergence
@pytest.mark.parametrize("c,P,Q,spec,bound", [
    (4, 3, 3, I.constant_field(), 0.25),
    (4, 3, 3, I.KL10, 0.5),
    (2, 4, 4, I.separable(0.3, 0.03, 1.0, m=10), 0.5),
    (4, 4, 1, I.separable(1.0, 0.01, 2.0, m=10), 0.5),
])
def test_wcycle_reduction_per_cycle_is_bounded(oracle, c, P, Q, spec, bound):
    """W(2,2) residual reduction per cycle after the first stays below the
    fixed bound, until the round-off floor is reached."""
    kx, ky = _hier(oracle, c, P, Q, spec, sid=11)
    _, ratios = oracle.msg_cycles(c, P, Q, kx, ky, 12)
    for k in range(2, len(ratios)):
        if ratios[k - 1] < 1e-12:
            break
        assert ratios[k] / ratios[k - 1] <= bound, (k, ratios)
    res = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(), want_hist=True)
    assert res["status"] == 0
    for g in range((P + 1) * (Q + 1)):
        h = res["hist"][g][: res["cycles"][g] + 1]
        for k in range(2, len(h)):
            if h[k - 1] < 1e-12:
                break
            assert h[k] / h[k - 1] <= bound, (g, h)


def test_joint_lower_stages_converge_slowly(oracle):
    """Evidence for solving each grid of an F-cycle level over its own
    rectangle: cycling all grids of a lower level together (coarse grids
    shared by two independent finest grids, residuals averaged) converges
    slowly even for constant k, while the per-grid form meets the bound."""
    c, P, Q = 4, 3, 3
    kx, ky = _hier(oracle, c, P, Q, I.constant_field())
    joint = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(joint_stages=True, max_cycles=30), want_hist=True)
    g = 2 * (Q + 1) + 2                                            # grid (2,2), level 4
    h = joint["hist"][g][: joint["cycles"][g] + 1]
    assert (h[-1] / h[1]) ** (1.0 / (len(h) - 2)) > 0.5
    per = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(), want_hist=True)
    assert per["status"] == 0 and per["cycles"].max() <= 10


def test_status_codes(oracle):
    c, P, Q = 4, 1, 1
    kx, ky = _hier(oracle, c, P, Q, I.KL10)
    assert oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(max_cycles=1))["status"] == 1
    bad = kx.copy()
    bad[3] = np.nan
    res = oracle.fmsg_solve(c, P, Q, bad, ky, oracle.opts())
    assert res["status"] == 2 and np.all(np.isnan(res["u"])) and np.all(np.isnan(res["q"]))
    # forced counts are honoured regardless of the tolerance
    forced = np.array([1, 2, 3, 4], dtype=np.int32)
    res = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(), forced_cycles=forced)
    assert list(res["cycles"]) == [1, 2, 3, 4]


# ---------------------------------------------------------------- multi-index differences
def test_delta_q_worked_example_from_paper(oracle):
    lines = [ln.split() for ln in open(os.path.join(GOLDEN, "delta_q_worked_example.txt"))
             if ln.strip() and not ln.startswith("#")]
    tp, tq = int(lines[0][1]), int(lines[0][2])
    terms = [(int(s), int(p), int(q)) for s, p, q in lines[1:]]
    P, Q = 5, 6
    rng = np.random.default_rng(7)
    q = rng.standard_normal((P + 1) * (Q + 1))
    dq = oracle.delta_q(P, Q, q)
    want = sum(s * q[p * (Q + 1) + r] for s, p, r in terms)
    assert dq[tp * (Q + 1) + tq] == pytest.approx(want, abs=1e-15)


def test_delta_q_telescopes(oracle):
    """sum_{tau <= l} Delta Q_tau = Q_l for every l (the identity behind the
    unbiasedness proof of Section 3)."""
    P, Q = 4, 3
    rng = np.random.default_rng(8)
    q = rng.standard_normal((P + 1) * (Q + 1))
    dq = oracle.delta_q(P, Q, q).reshape(P + 1, Q + 1)
    Qm = q.reshape(P + 1, Q + 1)
    for p in range(P + 1):
        for s in range(Q + 1):
            assert dq[: p + 1, : s + 1].sum() == pytest.approx(Qm[p, s], abs=1e-13)


# ---------------------------------------------------------------- fields
def test_field_zero_coefficients_and_face_coincidence(oracle):
    """xi = 0 gives k = 1; faces that coincide on two grids get equal k (the
    x-faces of the x-coarsened grid sit on every other fine x-face)."""
    kx, ky = oracle.field_cos(8, 4, I.KL10_A, I.KL10_B, I.KL10_AMP, np.zeros(10))
    assert np.all(kx == 1.0) and np.all(ky == 1.0)
    xi = I.draw_xi(10, [2])[0]
    fkx, fky = oracle.field_cos(16, 8, I.KL10_A, I.KL10_B, I.KL10_AMP, xi)
    ckx, cky = oracle.field_cos(8, 8, I.KL10_A, I.KL10_B, I.KL10_AMP, xi)
    assert np.array_equal(fkx.reshape(8, 17)[:, ::2], ckx.reshape(8, 9))
    ykx, yky = oracle.field_cos(16, 4, I.KL10_A, I.KL10_B, I.KL10_AMP, xi)
    assert np.array_equal(fky.reshape(9, 16)[::2, :], yky.reshape(5, 16))
    sx, sy = oracle.field_separable(16, 8, 5, 5, 0.3, 0.1, 1.0, I.draw_xi(25, [2])[0])
    tx, ty = oracle.field_separable(8, 8, 5, 5, 0.3, 0.1, 1.0, I.draw_xi(25, [2])[0])
    assert np.array_equal(sx.reshape(8, 17)[:, ::2], tx.reshape(8, 9))


def test_kl10_pointwise_variance(oracle):
    """Var Z at the corner face (0, h/2) tends to sum_j j^-2 cos^2(pi b_j h/2)
    (about 1.5498 for the ten terms); empirical over 4000 draws."""
    nd = 4000
    xi = I.draw_xi(10, range(nd), base_seed=123)
    z = np.empty(nd)
    for k in range(nd):
        kx, _ = oracle.field_cos(64, 64, I.KL10_A, I.KL10_B, I.KL10_AMP, xi[k])
        z[k] = np.log(kx[0])
    y = 0.5 / 64
    want = sum((1.0 / j) ** 2 * np.cos(np.pi * b * y) ** 2 for j, b in zip(range(1, 11), I.KL10_B))
    assert abs(want - 1.549768) < 2e-3
    assert abs(z.var() - want) <= 4 * want * math.sqrt(2.0 / nd)


def test_separable_domain_variance_is_sigma2(oracle):
    """The separable KL basis is orthonormal and its eigenvalues sum to one, so
    the domain average of Var Z is sigma^2; with lx != ly the pointwise
    variance along x differs from that along y (direction pairing)."""
    nd, n = 600, 32
    sigma2 = 2.0
    xi = I.draw_xi(36, range(nd), base_seed=321)
    zs = []
    for k in range(nd):
        _, ky = oracle.field_separable(n, n, 6, 6, 1.0, 0.05, sigma2, xi[k])
        zs.append(np.log(ky.reshape(n + 1, n))[1:-1])          # interior y-faces
    z = np.array(zs)
    avg_var = (z**2).mean()
    assert abs(avg_var - sigma2) <= 0.12 * sigma2
    # long correlation in x: Z barely varies along x; short in y: varies along y
    dzx = np.mean((z[:, :, 1:] - z[:, :, :-1]) ** 2)
    dzy = np.mean((z[:, 1:, :] - z[:, :-1, :]) ** 2)
    assert dzy > 5 * dzx


# ---------------------------------------------------------------- correction pairing
@pytest.mark.parametrize("cubic", [False, True])
def test_correction_pairs_weights_with_directions(oracle, cubic):
    """eq. interpolation: the x-coarsened grid's interpolant is weighted by
    kappa_x, the y-coarsened one's by kappa_y; one-sided on p = 0 or q = 0.
    A constant coarse iterate interpolates to that constant away from walls."""
    c, p, q = 4, 2, 2
    nx, ny = c << p, c << q
    kx, ky = kl10_faces(oracle, nx, ny, sid=13)
    ka, kb = oracle.weights(nx, ny, kx, ky)
    ones_x = np.ones((nx // 2) * ny)
    ones_y = np.ones(nx * (ny // 2))
    w = 4 if cubic else 2                      # cells whose stencil stays off the walls
    inner = (slice(w, -w), slice(w, -w))
    out = oracle.correction(c, p, q, kx, ky, ones_x, 0 * ones_y, cubic).reshape(ny, nx)
    assert np.max(np.abs(out[inner] - ka.reshape(ny, nx)[inner])) <= 1e-14
    out = oracle.correction(c, p, q, kx, ky, 0 * ones_x, ones_y, cubic).reshape(ny, nx)
    assert np.max(np.abs(out[inner] - kb.reshape(ny, nx)[inner])) <= 1e-14
    # q = 0: only P_x, unweighted
    kx0, ky0 = kl10_faces(oracle, nx, c, sid=13)
    out = oracle.correction(c, p, 0, kx0, ky0, np.ones((nx // 2) * c), None, cubic).reshape(c, nx)
    assert np.max(np.abs(out[:, w:-w] - 1.0)) <= 1e-14
    # p = 0: only P_y, unweighted
    kx1, ky1 = kl10_faces(oracle, c, ny, sid=13)
    out = oracle.correction(c, 0, q, kx1, ky1, None, np.ones(c * (ny // 2)), cubic).reshape(ny, c)
    assert np.max(np.abs(out[w:-w, :] - 1.0)) <= 1e-14


def test_fmg_initial_guess_is_accurate(oracle):
    """With zero cycles forced on the finest grid, the returned solution is the
    nested-iteration guess: cubic interpolation of converged coarse solutions
    of the sine problem, within a small multiple of h^2 of the exact solution."""
    c, P, Q = 4, 3, 2
    kx, ky = _hier(oracle, c, P, Q, I.constant_field())
    nxT, nyT = c << P, c << Q
    X, Y = cell_centres(nxT, nyT)
    rhs = (2 * np.pi**2 * np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()
    free = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(tol=1e-13), rhs_top=rhs)
    forced = free["cycles"].copy()
    forced[-1] = 0
    res = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts(tol=1e-13), rhs_top=rhs, forced_cycles=forced)
    exact = oracle.split_cells(free["u"], c, P, Q)[(P, Q)]
    guess = oracle.split_cells(res["u"], c, P, Q)[(P, Q)]
    h2 = (1.0 / nxT) ** 2 + (1.0 / nyT) ** 2
    err = np.abs(guess - exact).max() / np.abs(exact).max()
    assert 0 < err <= 2.0 * h2
    # and it is the weighted cubic interpolation of the returned coarse solutions
    U = oracle.split_cells(res["u"], c, P, Q)
    ktop = oracle.hierarchy_field(c, P, Q, I.constant_field().as_dict(), np.zeros(1))
    kxT = ktop[0][-(nxT + 1) * nyT:]
    kyT = ktop[1][-nxT * (nyT + 1):]
    want = oracle.correction(c, P, Q, kxT, kyT, U[(P - 1, Q)].ravel(), U[(P, Q - 1)].ravel(), cubic=True)
    assert np.max(np.abs(guess.ravel() - want)) <= 1e-14 * np.abs(want).max()
    lin = oracle.correction(c, P, Q, kxT, kyT, U[(P - 1, Q)].ravel(), U[(P, Q - 1)].ravel(), cubic=False)
    assert np.max(np.abs(lin - want)) > 1e-6 * np.abs(want).max()


def test_kl10_variance_separates_directions(oracle):
    """Var Z at (0, 1/2) sums j^-2 over even b_j; at (1/2, 0) over even a_j
    (1.3729 vs 1.2270 for the ten-term table); empirical over 6000 draws on
    the 1x1 grid whose faces sit exactly there."""
    nd = 6000
    xi = I.draw_xi(10, range(nd), base_seed=77)
    zx = np.empty(nd)
    zy = np.empty(nd)
    for k in range(nd):
        kx, ky = oracle.field_cos(1, 1, I.KL10_A, I.KL10_B, I.KL10_AMP, xi[k])
        zx[k], zy[k] = np.log(kx[0]), np.log(ky[0])
    wx = sum(1.0 / j**2 for j, b in zip(range(1, 11), I.KL10_B) if b % 2 == 0)
    wy = sum(1.0 / j**2 for j, a in zip(range(1, 11), I.KL10_A) if a % 2 == 0)
    assert abs(wx - 1.3729) < 1e-3 and abs(wy - 1.2270) < 1e-3
    tol = 3.5 * math.sqrt(2.0 / nd)
    assert abs(zx.var() / wx - 1) <= tol and abs(zy.var() / wy - 1) <= tol


# ---------------------------------------------------------------- paper QoIs (Section 5)
@pytest.mark.parametrize("nx,ny", [(2, 2), (4, 8), (3, 6), (12, 5)])
def test_point_value_reproduces_bilinear_fields(oracle, nx, ny):
    """Q1 = u(1/2,1/2) from cell centres: exact for any bilinear field, whether
    the point is a cell centre (odd sizes) or lies between four centres."""
    X, Y = cell_centres(nx, ny)
    u = 1.0 + 2.0 * X + 3.0 * Y + 4.0 * X * Y
    assert abs(oracle.qoi_grid(u, None, oracle.QOI_POINT) - 4.5) <= 1e-13


@pytest.mark.parametrize("nx,ny", [(8, 8), (2, 2), (4, 16), (6, 10), (3, 3)])
def test_subdomain_average_of_piecewise_constant_field(oracle, nx, ny):
    """Q2: average over [1/4,1/2]^2 of the cell-wise constant solution.  A
    constant averages to itself; u = x averages to the overlap-weighted mean
    of the covered cell centres, checked against the exact integral of the
    piecewise-constant function computed on a fine lattice of sub-cells."""
    assert abs(oracle.qoi_grid(np.full((ny, nx), 2.5), None, oracle.QOI_SUBDOMAIN) - 2.5) <= 1e-14
    X, Y = cell_centres(nx, ny)
    rng = np.random.default_rng(nx * 31 + ny)
    u = rng.standard_normal((ny, nx))
    f = 16 * math.lcm(nx, ny, 4)                      # sub-cells per unit length: every face is a lattice line
    xs = (np.arange(f) + 0.5) / f
    inside = (xs >= 0.25) & (xs <= 0.5)
    ii = np.minimum((xs * nx).astype(int), nx - 1)
    jj = np.minimum((xs * ny).astype(int), ny - 1)
    brute = u[np.ix_(jj[inside], ii[inside])].mean()
    assert abs(oracle.qoi_grid(u, None, oracle.QOI_SUBDOMAIN) - brute) <= 1e-12
    if nx % 4 == 0 and ny % 4 == 0:                   # faces on 1/4 and 1/2: mean of covered centres
        assert abs(oracle.qoi_grid(X, None, oracle.QOI_SUBDOMAIN) - 0.375) <= 1e-14


@pytest.mark.parametrize("n", [4, 8, 16])
def test_flux_of_symmetric_problem_is_a_quarter_of_the_source(oracle, n):
    """Q3 through x = 1: with k = 1 and h = 1 on an n x n grid, the discrete
    solution has the square's symmetry, so the four walls carry equal flux;
    the scheme is conservative, so together they carry int h = 1."""
    kx, ky = const_faces(n, n)
    A = dense(oracle, n, n, kx, ky)
    u = np.linalg.solve(A, np.ones(n * n)).reshape(n, n)
    q3 = oracle.qoi_grid(u, kx.reshape(n, n + 1), oracle.QOI_FLUX)
    assert abs(q3 - 0.25) <= 1e-12
    # the wall flux scales with the wall coefficient and is blind to the others
    kx2 = kx.reshape(n, n + 1).copy()
    kx2[:, n] *= 3.0
    kx2[:, 0] *= 7.0
    assert abs(oracle.qoi_grid(u, kx2, oracle.QOI_FLUX) - 0.75) <= 1e-12


def test_flux_balances_the_source_with_a_variable_field(oracle):
    """Conservation with a KL-10 field: the flux through x = 1, plus the same
    functional on the solution mirrored in x, y and the transpose (the other
    three walls), sums to int h = 1."""
    n = 8
    kx, ky = kl10_faces(oracle, n, n)
    A = dense(oracle, n, n, kx, ky)
    u = np.linalg.solve(A, np.ones(n * n)).reshape(n, n)
    KX, KY = kx.reshape(n, n + 1), ky.reshape(n + 1, n)
    east = oracle.qoi_grid(u, KX, oracle.QOI_FLUX)
    west = oracle.qoi_grid(u[:, ::-1].copy(), KX[:, ::-1].copy(), oracle.QOI_FLUX)
    north = oracle.qoi_grid(u.T.copy(), KY.T.copy(), oracle.QOI_FLUX)
    south = oracle.qoi_grid(u.T[:, ::-1].copy(), KY.T[:, ::-1].copy(), oracle.QOI_FLUX)
    assert abs(east + west + north + south - 1.0) <= 1e-12
    assert min(east, west, north, south) > 0.0


def test_mean_quantity_matches_the_solver_q(oracle):
    """kind 0 is the Q the solver returns per grid."""
    c, P, Q = 4, 2, 1
    kx, ky = oracle.hierarchy_field(c, P, Q, I.KL10.as_dict(), I.draw_xi(10, [5])[0])
    r = oracle.fmsg_solve(c, P, Q, kx, ky, oracle.opts())
    assert np.allclose(oracle.qoi(c, P, Q, r["u"], kx, oracle.QOI_MEAN), r["q"], rtol=1e-14, atol=0)


# ---------------------------------------------------------------- standard multigrid (comparison)
def aniso_faces(O, c, P, Q, ex, ey):
    kx, ky = [], []
    for p, q, nx, ny in O.grid_shapes(c, P, Q):
        kx.append(np.full((nx + 1) * ny, ex))
        ky.append(np.full(nx * (ny + 1), ey))
    return np.concatenate(kx), np.concatenate(ky)


def test_mg_on_the_coarsest_grid_is_a_direct_solve(oracle):
    kx, ky = aniso_faces(oracle, 4, 0, 0, 1.0, 1.0)
    _, r = oracle.mg_cycles(4, 0, 0, kx, ky, 1)
    assert r[0] == 1.0 and r[1] <= 1e-14


@pytest.mark.parametrize("P,Q", [(3, 3), (4, 2)])
def test_mg_converges_to_the_dense_solution(oracle, P, Q):
    """Square and rectangular (coarsest 16x4) hierarchies with a KL-10 field:
    the cycles converge to numpy's dense solve of the finest system."""
    c = 2
    kx, ky = oracle.hierarchy_field(c, P, Q, I.KL10.as_dict(), I.draw_xi(10, [11])[0])
    nx, ny = c << P, c << Q
    fx = sum((a + 1) * b for _, _, a, b in oracle.grid_shapes(c, P, Q)[:-1])
    fy = sum(a * (b + 1) for _, _, a, b in oracle.grid_shapes(c, P, Q)[:-1])
    A = dense(oracle, nx, ny, kx[fx:], ky[fy:])
    exact = np.linalg.solve(A, np.ones(nx * ny))
    u, r = oracle.mg_cycles(c, P, Q, kx, ky, 40)
    assert r[-1] <= 1e-11
    assert np.linalg.norm(u - exact) <= 1e-9 * np.linalg.norm(exact)


def test_mg_isotropic_factor_and_anisotropic_breakdown(oracle):
    """Point-smoothed standard multigrid converges fast for an isotropic
    coefficient and stalls as the coefficient becomes anisotropic, while MSG
    keeps its factor (the robustness Section 2 claims for MSG)."""
    c, P, Q = 2, 5, 5
    o = oracle.opts(nu1=2, nu2=2)

    def factor(fn, ex, ey):
        kx, ky = aniso_faces(oracle, c, P, Q, ex, ey)
        _, r = fn(c, P, Q, kx, ky, 12, o)
        return (r[-1] / r[2]) ** (1 / 10)

    assert factor(oracle.mg_cycles, 1.0, 1.0) <= 0.2
    assert factor(oracle.mg_cycles, 1.0, 1e-3) >= 0.8
    assert factor(oracle.msg_cycles, 1.0, 1e-3) <= 0.2
