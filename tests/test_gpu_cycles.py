"""Plain cycles from zero on the GPU (msg_cycles, through the C-ABI) against
the oracle's msg_cycles / mg_cycles: the residual-ratio history of every
cycle and the final iterate, for MSG and standard multigrid, on lognormal
fields and on constant anisotropic coefficients (the comparison of
Section 2).

Both sides take the same face conductances, computed by the oracle and
uploaded, so that only the cycles are compared.

Tolerances: the iterate to 1e-10 (relative L2, the FP64 bar).  A residual
ratio ||b - A v|| / ||b|| of an iterate that agrees to rounding carries an
absolute error of about eps * ||A|| ||v|| / ||b||, which for these grids
(at most 256 x 256 cells, conductances within e^{+-4}) stays below 1e-11;
so ratios are compared to 1e-10 relative plus 1e-11 absolute."""
import numpy as np
import pytest

from oracle import binding as O
from paper_1907_12334_amd import inputs as I
from paper_1907_12334_amd import msg

pytestmark = pytest.mark.gpu

U_TOL = 1e-10
R_REL, R_ABS = 1e-10, 1e-11


@pytest.fixture(scope="module")
def handle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return msg.Handle(0)


def _fields(c, P, Q, field, S, seed):
    """Per-sample packed conductances of every grid (host arrays)."""
    if field == "kl10":
        xi = I.draw_xi(I.KL10.n_terms, range(S), seed)
        return [O.hierarchy_field(c, P, Q, I.KL10.as_dict(), xi[s]) for s in range(S)]
    if field == "se_aniso":
        spec = I.separable(0.25, 0.25 / 16, 1.0, m=24)
        xi = I.draw_xi(spec.n_terms, range(S), seed)
        return [O.hierarchy_field(c, P, Q, spec.as_dict(), xi[s]) for s in range(S)]
    assert field.startswith("const")
    eps = float(field.split("_")[1])
    out = []
    for s in range(S):
        kx = [np.full((c << b) * ((c << a) + 1), 1.0 + s) for a in range(P + 1) for b in range(Q + 1)]
        ky = [np.full((c << a) * ((c << b) + 1), eps * (1.0 + s)) for a in range(P + 1) for b in range(Q + 1)]
        out.append((np.concatenate(kx), np.concatenate(ky)))
    return out


def _run(handle, c, P, Q, S, kind, fields, opts, ncycles, rhs=None):
    import torch
    b = msg.Batch(c, [P] * S, [Q] * S)
    dev = "cuda:0"
    kx = torch.tensor(np.concatenate([f[0] for f in fields]), dtype=torch.float64, device=dev)
    ky = torch.tensor(np.concatenate([f[1] for f in fields]), dtype=torch.float64, device=dev)
    n = (c << P) * (c << Q)
    u = torch.full((S * n,), float("nan"), dtype=torch.float64, device=dev)
    ratios = torch.full((S * (ncycles + 1),), float("nan"), dtype=torch.float64, device=dev)
    nbytes = msg.cycles_workspace_size(b, opts, kind)
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
    rhs_d = torch.tensor(rhs, dtype=torch.float64, device=dev) if rhs is not None else None
    handle.cycles(b, opts, kind, ncycles, kx, ky, rhs_d, u, ratios, ws)
    torch.cuda.synchronize()
    return u.cpu().numpy().reshape(S, n), ratios.cpu().numpy().reshape(S, ncycles + 1)


def _compare(c, P, Q, kind, fields, opts, ncycles, u, ratios, rhs=None):
    o = O.opts(mu=opts.mu, nu1=opts.nu1, nu2=opts.nu2, omega=opts.omega)
    f = O.mg_cycles if kind == msg.CYCLES_MG else O.msg_cycles
    n = (c << P) * (c << Q)
    worst_u = worst_r = 0.0
    for s, (kx, ky) in enumerate(fields):
        r_top = None if rhs is None else rhs[s * n:(s + 1) * n]
        u_o, r_o = f(c, P, Q, kx, ky, ncycles, o, rhs_top=r_top)
        eu = np.linalg.norm(u[s] - u_o) / max(np.linalg.norm(u_o), 1e-300)
        assert np.all(np.abs(ratios[s] - r_o) <= R_REL * r_o + R_ABS), (s, ratios[s], r_o)
        assert eu <= U_TOL, (s, eu)
        worst_u = max(worst_u, eu)
        worst_r = max(worst_r, float(np.max(np.abs(ratios[s] - r_o))))
    return worst_u, worst_r


@pytest.mark.parametrize("kind", [msg.CYCLES_MSG, msg.CYCLES_MG])
@pytest.mark.parametrize("field", ["kl10", "se_aniso", "const_0.01"])
def test_cycles_match_oracle(handle, kind, field):
    c, P, Q, S, ncyc = 2, 4, 4, 5, 6
    print(f"cycles kind={kind} field={field} c={c} P={P} Q={Q} S={S}", flush=True)
    fields = _fields(c, P, Q, field, S, I.BASE_SEED + 11)
    opts = msg.SolveOpts()
    u, r = _run(handle, c, P, Q, S, kind, fields, opts, ncyc)
    assert np.all(r[:, 0] == 1.0)
    _compare(c, P, Q, kind, fields, opts, ncyc, u, r)


@pytest.mark.parametrize("kind", [msg.CYCLES_MSG, msg.CYCLES_MG])
@pytest.mark.parametrize("mu,nu1,nu2,omega", [(1, 3, 1, 1.0), (2, 1, 0, 1.0), (2, 5, 5, 0.9), (3, 2, 2, 1.0)])
def test_cycle_kinds_sweeps_and_damping(handle, kind, mu, nu1, nu2, omega):
    c, P, Q, S, ncyc = 4, 3, 3, 3, 4
    print(f"cycles kind={kind} mu={mu} nu=({nu1},{nu2}) omega={omega}", flush=True)
    fields = _fields(c, P, Q, "kl10", S, I.BASE_SEED + 12)
    opts = msg.SolveOpts(mu=mu, nu1=nu1, nu2=nu2, omega=omega)
    u, r = _run(handle, c, P, Q, S, kind, fields, opts, ncyc)
    _compare(c, P, Q, kind, fields, opts, ncyc, u, r)


@pytest.mark.parametrize("kind,P,Q", [(msg.CYCLES_MSG, 0, 0), (msg.CYCLES_MG, 0, 0), (msg.CYCLES_MSG, 1, 1),
                                      (msg.CYCLES_MG, 1, 1), (msg.CYCLES_MSG, 2, 5), (msg.CYCLES_MSG, 6, 1)])
def test_small_and_rectangular_grids(handle, kind, P, Q):
    c, S, ncyc = 3, 4, 3
    print(f"cycles kind={kind} c={c} P={P} Q={Q}", flush=True)
    fields = _fields(c, P, Q, "kl10", S, I.BASE_SEED + 13)
    opts = msg.SolveOpts()
    u, r = _run(handle, c, P, Q, S, kind, fields, opts, ncyc)
    if P + Q == 0:
        # the coarsest grid is solved exactly by either method
        assert np.all(r[:, 1:] < 1e-12)
    _compare(c, P, Q, kind, fields, opts, ncyc, u, r)


def test_zero_cycles_and_rhs_argument(handle):
    c, P, Q, S = 2, 3, 3, 3
    fields = _fields(c, P, Q, "kl10", S, I.BASE_SEED + 14)
    opts = msg.SolveOpts()
    u, r = _run(handle, c, P, Q, S, msg.CYCLES_MG, fields, opts, 0)
    assert np.all(u == 0.0) and np.all(r == 1.0)
    n = (c << P) * (c << Q)
    rhs = np.random.default_rng(3).standard_normal(S * n)
    for kind in (msg.CYCLES_MSG, msg.CYCLES_MG):
        u, r = _run(handle, c, P, Q, S, kind, fields, opts, 3, rhs=rhs)
        _compare(c, P, Q, kind, fields, opts, 3, u, r, rhs=rhs)


def test_full_size_grid_two_cycles(handle):
    """256 x 256 cells (several smoother tiles per grid, a deep hierarchy)."""
    c, P, Q, S, ncyc = 2, 7, 7, 2, 2
    fields = _fields(c, P, Q, "kl10", S, I.BASE_SEED + 15)
    opts = msg.SolveOpts()
    for kind in (msg.CYCLES_MSG, msg.CYCLES_MG):
        print(f"cycles kind={kind} c={c} P={P} Q={Q}", flush=True)
        u, r = _run(handle, c, P, Q, S, kind, fields, opts, ncyc)
        _compare(c, P, Q, kind, fields, opts, ncyc, u, r)


def test_anisotropy_contrast(handle):
    """Standard multigrid degrades with the anisotropy of the coefficients,
    MSG does not (the robustness claim of Section 2), on the GPU path."""
    c, P, Q, S, ncyc = 2, 5, 5, 2, 12
    opts = msg.SolveOpts()
    fac = {}
    for field in ("const_1", "const_0.001"):
        fields = _fields(c, P, Q, field, S, 0)
        for kind in (msg.CYCLES_MSG, msg.CYCLES_MG):
            _, r = _run(handle, c, P, Q, S, kind, fields, opts, ncyc)
            fac[(field, kind)] = float(np.mean((r[:, ncyc] / r[:, 2]) ** (1.0 / (ncyc - 2))))
    assert fac[("const_0.001", msg.CYCLES_MG)] > 0.8
    assert fac[("const_0.001", msg.CYCLES_MSG)] < 0.2
    assert fac[("const_1", msg.CYCLES_MG)] < 0.2 and fac[("const_1", msg.CYCLES_MSG)] < 0.2
