"""HIP path (through the C-ABI) against the oracle on the same seeded inputs.

FP64 bar: per grid ||u_gpu - u_oracle||_2 / ||u_oracle||_2 <= 1e-10, Q within
1e-10 relative, Delta Q within 1e-10 of the largest |Q| it combines, with the
oracle run at the GPU's per-grid cycle counts (a tie at the tolerance may
change a count by one; the iterates are then compared at equal counts).
Mixed precision: the same quantities within 1e-8 of the FP64 oracle run to
1e-10.
"""
import dataclasses

import numpy as np
import pytest

from oracle import binding as O
from paper_1907_12334_amd import inputs as I
from paper_1907_12334_amd import msg

from . import parity as PR

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-8


@pytest.fixture(scope="module")
def handle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return msg.Handle(0)


def _check_batch(handle, c, P, Q, spec, opts, seed=I.BASE_SEED, tol=FP64_TOL, ids=None, xi=None):
    xi = I.draw_xi(spec.n_terms, range(len(P)), seed) if xi is None else xi
    out = PR.gpu_solve(c, P, Q, spec, xi, opts, handle=handle)
    ids = range(len(P)) if ids is None else ids
    worst = 0.0
    for s in ids:
        g = PR.per_sample(out, s)
        eu, eq, edq, ora = PR.compare_sample(c, int(P[s]), int(Q[s]), spec, xi[s], g, tol=opts.tol,
                                             max_cycles=opts.max_cycles, omega=opts.omega, mu=opts.mu,
                                             nu1=opts.nu1, nu2=opts.nu2)
        assert g["status"] == ora["status"], (s, g["status"], ora["status"])
        assert eu <= tol and eq <= tol and edq <= tol, (s, eu, eq, edq)
        worst = max(worst, eu)
    return out, worst


def test_field_matches_oracle(handle):
    for spec, c, P, Q in [(I.KL10, 4, 3, 2), (I.separable(0.3, 0.03, 1.0, m=20), 2, 4, 5)]:
        xi = I.draw_xi(spec.n_terms, range(3))
        out = PR.gpu_solve(c, [P] * 3, [Q] * 3, spec, xi, msg.SolveOpts(max_cycles=0), handle=handle)
        for s in range(3):
            g = PR.per_sample(out, s)
            kx, ky = O.hierarchy_field(c, P, Q, spec.as_dict(), xi[s])
            assert np.max(np.abs(g["kx"] / kx - 1)) <= 1e-13
            assert np.max(np.abs(g["ky"] / ky - 1)) <= 1e-13


def test_config1_all_samples(handle):
    w = I.config(1)
    out, worst = _check_batch(handle, w.c, w.P, w.Q, w.field, msg.SolveOpts(), seed=w.seed)
    assert np.all(out["status"] == 0)


@pytest.mark.parametrize("handoff", [0, -1])
@pytest.mark.parametrize("max_cycles", [0, 1, 2])
def test_unconverged_iterates_match_step_by_step(handle, max_cycles, handoff):
    """Cycle caps of 0, 1, 2 stop every grid early, so the returned iterates
    expose the nested-iteration guess and single cycles, not just the
    converged solution (with the host loop alone, and with the handoff of
    the last cycling problems to one kernel)."""
    opts = msg.SolveOpts(max_cycles=max_cycles, handoff=handoff)
    for c, P, Q, spec in [(4, 3, 3, I.KL10), (2, 4, 3, I.separable(0.3, 0.03, 1.0, m=10))]:
        _check_batch(handle, c, [P] * 3, [Q] * 3, spec, opts, tol=1e-12)


@pytest.mark.parametrize("fields", ["kl10", "se"])
def test_multi_tile_grids_step_by_step(handle, fields):
    """Grids wider and taller than one smoother tile (128x64 and 16x256 finest
    grids, every level on the batched kernels with tail_levels = 0, then with
    the automatic tail) after one and two cycles."""
    spec = I.KL10 if fields == "kl10" else I.separable(0.3, 0.03, 1.0, m=10)
    for tail in (0, -1):
        for mc in (1, 2, 3):
            for handoff in (0, -1):
                opts = msg.SolveOpts(max_cycles=mc, tail_levels=tail, handoff=handoff)
                _check_batch(handle, 4, [5, 2], [4, 6], spec, opts, tol=1e-12)


@pytest.mark.parametrize("tail", [0, 1, 3, -1])
def test_tail_depth_does_not_change_results(handle, tail):
    c, P, Q, spec = 2, 4, 4, I.KL10
    opts = msg.SolveOpts(tail_levels=tail, max_cycles=2)
    _check_batch(handle, c, [P] * 2, [Q] * 2, spec, opts, tol=1e-12)


@pytest.mark.parametrize("precision", [msg.FP64, msg.MIXED])
@pytest.mark.parametrize("max_cycles", [1, 2, 400])
def test_wide_tails_for_few_large_samples(handle, precision, max_cycles):
    """A tail budget of 150 KB per problem (the request loop's large-request
    lane): deeper tails on four wavefronts and larger rectangles solved whole
    in one kernel.  Unconverged iterates match the oracle step by step, and
    converged ones within the bar (FP64: 1e-10; mixed: 1e-8 against the FP64
    oracle)."""
    c, P, Q = 4, [6, 5, 7], [5, 6, 1]
    spec = I.separable(0.3, 0.03, 1.0, m=20, face_rule=1)
    xi = I.draw_xi(spec.n_terms, range(3), base_seed=31)
    if precision == msg.FP64:
        opts = msg.SolveOpts(max_cycles=max_cycles, tail_budget=150 * 1024)
        _check_batch(handle, c, P, Q, spec, opts, xi=xi, tol=1e-12 if max_cycles < 400 else FP64_TOL)
        return
    if max_cycles < 400:
        pytest.skip("mixed precision is compared converged")
    opts = msg.SolveOpts(precision=msg.MIXED, tol=1e-8, max_cycles=max_cycles, tail_budget=150 * 1024)
    out = PR.gpu_solve(c, P, Q, spec, xi, opts, handle=handle)
    for s in range(3):
        g = PR.per_sample(out, s)
        ora = PR.oracle_solve(c, P[s], Q[s], spec, xi[s], tol=1e-10, max_cycles=max_cycles)
        assert g["status"] == 0 and ora["status"] == 0
        eu, eq, edq = PR.errors(c, P[s], Q[s], g, ora)
        assert max(eu, eq, edq) <= MIXED_TOL, (s, eu, eq, edq)


@pytest.mark.parametrize("handoff", [0, 1, -1])
def test_converged_with_and_without_handoff(handle, handoff):
    """Converged solves through the host loop only, with a handoff once a
    single problem of a class is left, and with the default threshold."""
    c, P, Q, spec = 2, 5, 4, I.separable(0.3, 0.03, 1.0, m=20)
    _check_batch(handle, c, [P] * 6, [Q] * 6, spec, msg.SolveOpts(max_cycles=1000, handoff=handoff))


@pytest.mark.parametrize("mu,nu1,nu2", [(2, 3, 2), (2, 1, 0), (1, 2, 2), (2, 1, 1)])
def test_cycle_kinds_and_sweep_counts(handle, mu, nu1, nu2):
    """V- and W-cycles, odd and even smoothing counts (odd totals take the
    stage level through an odd number of buffer swaps per cycle), with
    problems of one class stopping at different cycles; host loop only."""
    c, P, Q, spec = 2, 5, 4, I.separable(0.3, 0.03, 1.0, m=20)
    opts = msg.SolveOpts(mu=mu, nu1=nu1, nu2=nu2, max_cycles=400, handoff=0)
    out, _ = _check_batch(handle, c, [P] * 6, [Q] * 6, spec, opts)
    cyc = out["cycles"].reshape(6, -1)
    assert len({tuple(r) for r in cyc}) > 1        # the samples stopped at different counts


def test_overlap_modes_give_identical_results(handle):
    """Every launch on the caller's stream, classes over two streams, and
    concurrently solved parts of the batch: bitwise the same answers."""
    c, spec = 2, I.separable(0.3, 0.03, 1.0, m=20)
    P, Q = [5] * 520 + [4] * 8, [4] * 520 + [5] * 8          # the parts get different rectangles
    xi = I.draw_xi(spec.n_terms, range(len(P)))
    outs = [PR.gpu_solve(c, P, Q, spec, xi, msg.SolveOpts(max_cycles=400, overlap=ov), handle=handle)
            for ov in (0, 1, 2)]
    for o in outs[1:]:
        for k in ("u", "q", "dq", "cycles", "status"):
            assert np.array_equal(o[k], outs[0][k]), k
    g = PR.per_sample(outs[2], 0)
    eu, eq, edq, ora = PR.compare_sample(c, P[0], Q[0], spec, xi[0], g, max_cycles=400)
    assert g["status"] == ora["status"] and max(eu, eq, edq) <= FP64_TOL


def test_autotuned_plan_gives_the_same_answers(handle, tmp_path):
    """The autotuner's choice and every candidate plan solve the same problem:
    same cycle counts, iterates equal to rounding; the choice is cached."""
    from paper_1907_12334_amd import autotune as AT
    import dataclasses
    w = dataclasses.replace(I.config(2).subset(24), P=[5] * 24, Q=[4] * 24)
    base = msg.SolveOpts(tol=1e-10, max_cycles=400)
    cache = str(tmp_path / "tune.json")
    tuned, rep = AT.autotune(handle, w, base, samples=24, cycles=2, reps=1, cache=cache)
    assert len(rep["trials"]) == len(AT.TILES) + len(AT.TAIL_BUDGETS) - 1 and not rep["cached"]
    again, rep2 = AT.autotune(handle, w, base, samples=24, cycles=2, reps=1, cache=cache)
    assert rep2["cached"] and again == tuned
    xi = w.xi()
    ref = PR.gpu_solve(w.c, w.P, w.Q, w.field, xi, base, handle=handle)
    for params in [tuned] + [dataclasses.replace(base, tile_width=t[0], tile_cells=t[1], tile_lds=t[2])
                             for t in AT.TILES[1:]] + [dataclasses.replace(base, tail_budget=b)
                                                        for b in AT.TAIL_BUDGETS[1:]]:
        out = PR.gpu_solve(w.c, w.P, w.Q, w.field, xi, params, handle=handle)
        assert np.array_equal(out["cycles"], ref["cycles"]) and np.array_equal(out["status"], ref["status"])
        for s in range(0, 24, 5):
            a, b = PR.per_sample(out, s), PR.per_sample(ref, s)
            assert PR.grid_errors(w.c, w.P[s], w.Q[s], a["u"], b["u"]) <= 1e-12


@pytest.mark.parametrize("precision,overlap", [(msg.FP64, 0), (msg.FP64, 2), (msg.MIXED, 0)])
def test_graph_replay_matches_launches(handle, precision, overlap):
    """Each class's W-cycle captured once per stage and replayed every later
    cycle (with the convergence checks and host synchronisation between
    replays): the same bits as launching every kernel, over many replays."""
    c, spec = 2, I.separable(0.3, 0.03, 1.0, m=20)
    P, Q = [5] * 6 + [4] * 4 + [3] * 2, [4] * 6 + [5] * 4 + [3] * 2
    xi = I.draw_xi(spec.n_terms, range(len(P)))
    tol = 1e-10 if precision == msg.FP64 else 1e-8
    base = msg.SolveOpts(tol=tol, max_cycles=400, precision=precision, overlap=overlap, handoff=0, tail_levels=2)
    ref = PR.gpu_solve(c, P, Q, spec, xi, base, handle=handle)
    out = PR.gpu_solve(c, P, Q, spec, xi, dataclasses.replace(base, graphs=1), handle=handle)
    assert ref["cycles"].max() >= 10                    # many replays per stage
    for k in ("u", "q", "dq", "cycles", "status"):
        assert np.array_equal(out[k], ref[k]), k


@pytest.mark.parametrize("precision,cycle", [(msg.FP64, (2, 2, 2)), (msg.FP64, (1, 1, 3)), (msg.MIXED, (2, 2, 2))])
def test_fused_passes_match_split_sweeps_bitwise(handle, monkeypatch, precision, cycle):
    """The fused smoothing passes (tiles with recomputed halos in LDS, the
    correction applied in the load, the residual restricted in the
    pre-smoothing pass) against the debug mode that runs every step on its
    own: the correction kernel, then one in-place launch per colour of every
    half-sweep over whole grids, then the plain restriction kernel.  Same
    bits, on a batch whose levels above the tail are several tiles wide."""
    mu, nu1, nu2 = cycle
    c, spec = 2, I.separable(0.3, 0.03, 1.0, m=20)
    P, Q = [6] * 3 + [5] * 3 + [3] * 2, [5] * 3 + [6] * 3 + [3] * 2
    xi = I.draw_xi(spec.n_terms, range(len(P)))
    tol = 1e-10 if precision == msg.FP64 else 1e-8
    opts = msg.SolveOpts(mu=mu, nu1=nu1, nu2=nu2, tol=tol, max_cycles=400, precision=precision, handoff=0,
                         tail_levels=2)
    monkeypatch.delenv("MSG_DEBUG_SPLIT_SWEEPS", raising=False)
    ref = PR.gpu_solve(c, P, Q, spec, xi, opts, handle=handle)
    monkeypatch.setenv("MSG_DEBUG_SPLIT_SWEEPS", "1")
    out = PR.gpu_solve(c, P, Q, spec, xi, opts, handle=handle)
    monkeypatch.delenv("MSG_DEBUG_SPLIT_SWEEPS")
    assert np.all(ref["status"] == 0) and ref["cycles"].max() >= 3
    for k in ("u", "q", "dq", "cycles", "status"):
        assert np.array_equal(out[k], ref[k]), k


def test_ragged_batch_and_batch_invariance(handle):
    rng = np.random.default_rng(5)
    P = rng.integers(0, 5, size=12)
    Q = rng.integers(0, 5, size=12)
    P[0], Q[0] = 0, 0
    P[1], Q[1] = 5, 0
    P[2], Q[2] = 0, 5
    spec = I.KL10
    xi = I.draw_xi(10, range(12))
    out, _ = _check_batch(handle, 4, P, Q, spec, msg.SolveOpts(), xi=xi)
    # the same sample alone gives the same bits
    for s in (0, 3, 7):
        alone = PR.gpu_solve(4, [P[s]], [Q[s]], spec, xi[s:s + 1], msg.SolveOpts(), handle=handle)
        a = PR.per_sample(alone, 0)
        b = PR.per_sample(out, s)
        assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["q"], b["q"])
        assert np.array_equal(a["cycles"], b["cycles"])


def test_mixed_precision_against_fp64_oracle(handle):
    c, P, Q = 4, 5, 2
    spec = I.separable(1.0, 0.01, 2.0, m=20)
    xi = I.draw_xi(spec.n_terms, range(4))
    opts = msg.SolveOpts(precision=msg.MIXED, tol=1e-8, max_cycles=1000)
    out = PR.gpu_solve(c, [P] * 4, [Q] * 4, spec, xi, opts, handle=handle)
    for s in range(4):
        g = PR.per_sample(out, s)
        ora = PR.oracle_solve(c, P, Q, spec, xi[s], tol=1e-10, max_cycles=1000)
        assert g["status"] == 0 and ora["status"] == 0
        # coefficients in FP64 match; solutions within the mixed bar
        assert PR.grid_errors(c, P, Q, g["u"], ora["u"]) <= MIXED_TOL
        assert np.max(np.abs(g["q"] - ora["q"]) / np.abs(ora["q"])) <= MIXED_TOL


def test_mixed_precision_at_the_1024x64_shape(handle):
    """The 1024x64 preset's own shape and field ((P,Q) = (8,4), c = 4, 45
    grids, ly = 0.01, sigma^2 = 2, face means): mixed precision refined to
    1e-8 against the FP64 oracle run to 1e-10 on a seeded subset; per grid
    u, Q and Delta Q within 1e-8.  Most levels cycle on the host in FP32
    here and hand over to the FP64 on-chip solves below them."""
    w = I.config(4)
    ids = [1, 2, 3, 5]
    xi = w.xi(ids)
    opts = msg.SolveOpts(precision=msg.MIXED, tol=w.ir_tol, max_cycles=w.max_cycles)
    out = PR.gpu_solve(w.c, [8] * 4, [4] * 4, w.field, xi, opts, handle=handle)
    for s in range(4):
        g = PR.per_sample(out, s)
        print(f"sample {ids[s]}: oracle at 1e-10", flush=True)
        ora = PR.oracle_solve(w.c, 8, 4, w.field, xi[s], tol=1e-10, max_cycles=w.max_cycles)
        ora["dq"] = O.delta_q(8, 4, ora["q"])
        assert g["status"] == 0 and ora["status"] == 0
        eu, eq, edq = PR.errors(w.c, 8, 4, g, ora)
        print(f"sample {ids[s]}: u {eu:.2e} Q {eq:.2e} dQ {edq:.2e}", flush=True)
        assert max(eu, eq, edq) <= MIXED_TOL, (ids[s], eu, eq, edq)


def test_delta_q_on_device(handle):
    import torch
    b = msg.Batch(4, [2, 3, 0], [3, 1, 4])
    n = int(b.layout()["grid"][-1])
    q = torch.tensor(np.random.default_rng(3).standard_normal(n), dtype=torch.float64, device="cuda:0")
    dq = torch.empty_like(q)
    msg.delta_q(b, q, dq)
    torch.cuda.synchronize()
    qh, dqh = q.cpu().numpy(), dq.cpu().numpy()
    lay = b.layout()["grid"]
    for s, (P, Q) in enumerate(zip(b.P, b.Q)):
        want = O.delta_q(int(P), int(Q), qh[lay[s]:lay[s + 1]])
        assert np.allclose(dqh[lay[s]:lay[s + 1]], want, rtol=0, atol=1e-15)


def test_failure_paths_are_per_sample(handle):
    c, P, Q, spec = 4, 2, 2, I.KL10
    xi = I.draw_xi(10, range(3))
    xi[1, 4] = np.nan
    out = PR.gpu_solve(c, [P] * 3, [Q] * 3, spec, xi, msg.SolveOpts(), handle=handle)
    assert list(out["status"]) == [0, 2, 0]
    bad = PR.per_sample(out, 1)
    assert np.all(np.isnan(bad["u"])) and np.all(np.isnan(bad["q"]))
    for s in (0, 2):
        alone = PR.gpu_solve(c, [P], [Q], spec, xi[s:s + 1], msg.SolveOpts(), handle=handle)
        assert np.array_equal(PR.per_sample(alone, 0)["u"], PR.per_sample(out, s)["u"])
    capped = PR.gpu_solve(c, [P], [Q], spec, xi[:1], msg.SolveOpts(max_cycles=1), handle=handle)
    assert int(capped["status"][0]) == 1


def test_rhs_argument_manufactured_sine(handle):
    """A caller right-hand side on the finest grid (sine, constant k): every
    returned grid matches the oracle."""
    c, P, Q = 4, 2, 3
    spec = I.constant_field()
    nx, ny = c << P, c << Q
    X, Y = np.meshgrid((np.arange(nx) + 0.5) / nx, (np.arange(ny) + 0.5) / ny)
    rhs = (2 * np.pi**2 * np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()
    xi = np.zeros((1, 1))
    out = PR.gpu_solve(c, [P], [Q], spec, xi, msg.SolveOpts(), rhs=rhs, handle=handle)
    g = PR.per_sample(out, 0)
    eu, eq, edq, _ = PR.compare_sample(c, P, Q, spec, xi[0], g, rhs=rhs)
    assert eu <= FP64_TOL and eq <= FP64_TOL


def test_full_size_config2_sampled(handle):
    """The 256x256 (c = 2, 64 grids) separable field at full size in the
    benchmark's launch shape, on a 32-sample slice: every sample converges,
    and two sampled solves match the oracle grid by grid."""
    w = I.config(2).subset(32)
    xi = w.xi()
    out = PR.gpu_solve(w.c, w.P, w.Q, w.field, xi, msg.SolveOpts(max_cycles=w.max_cycles), handle=handle)
    assert np.all(out["status"] == 0)
    for s in (0, 31):
        g = PR.per_sample(out, s)
        eu, eq, edq, _ = PR.compare_sample(w.c, 7, 7, w.field, xi[s], g, max_cycles=w.max_cycles)
        assert eu <= FP64_TOL and eq <= FP64_TOL and edq <= FP64_TOL, (s, eu, eq, edq)


def test_full_size_config2_whole_batch(handle):
    """The whole 4096-sample 256x256 batch in the benchmark's launch
    configuration (automatic overlap: three concurrently solved parts, the
    shared passes of consecutive visits, lockstep tails): every sample
    converges, and samples at both ends of every part match the oracle
    grid by grid."""
    import torch
    w = I.config(2)
    xi = w.xi()
    print("config 2, 4096 samples", flush=True)
    opts = msg.SolveOpts(tol=w.tol, max_cycles=w.max_cycles)
    b = msg.Batch(w.c, w.P, w.Q)
    bufs = msg.Buffers(b, opts)
    msg.run(handle, w.field, b, opts, torch.tensor(xi, dtype=torch.float64, device="cuda:0"), bufs)
    torch.cuda.synchronize()
    assert np.all(bufs.status.cpu().numpy() == 0)
    lay = bufs.layout
    for s in (0, 1365, 1366, 4095):
        c0, c1, g0, g1 = (int(x) for x in (lay["cell"][s], lay["cell"][s + 1], lay["grid"][s], lay["grid"][s + 1]))
        g = {"u": bufs.u[c0:c1].cpu().numpy(), "q": bufs.q[g0:g1].cpu().numpy(),
             "dq": bufs.dq[g0:g1].cpu().numpy(), "cycles": bufs.cycles[g0:g1].cpu().numpy()}
        eu, eq, edq, _ = PR.compare_sample(w.c, 7, 7, w.field, xi[s], g, max_cycles=w.max_cycles)
        assert eu <= FP64_TOL and eq <= FP64_TOL and edq <= FP64_TOL, (s, eu, eq, edq)
    del bufs
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", [msg.QOI_MEAN, msg.QOI_POINT, msg.QOI_SUBDOMAIN, msg.QOI_FLUX])
def test_quantities_of_interest_match_oracle(handle, kind):
    """Section 5's quantities on every grid: from the GPU's own solutions they
    equal the oracle's functional to rounding; end to end (oracle solution)
    within the FP64 bar; their differences follow as for Q."""
    import torch
    c, P, Q = 3, [2, 1, 3, 0], [1, 2, 0, 2]                     # odd sizes: the point is a cell centre on some grids
    spec = I.KL10
    xi = I.draw_xi(spec.n_terms, range(len(P)))
    out = PR.gpu_solve(c, P, Q, spec, xi, msg.SolveOpts(), handle=handle)
    b = msg.Batch(c, P, Q)
    dev = lambda a, dt=torch.float64: torch.tensor(a, dtype=dt, device="cuda:0")
    q = torch.empty(int(out["layout"]["grid"][-1]), dtype=torch.float64, device="cuda:0")
    msg.quantity(b, kind, dev(out["kx"]), dev(out["u"]), q)
    qg = q.cpu().numpy()
    lay = out["layout"]
    for s in range(len(P)):
        g = PR.per_sample(out, s)
        mine = qg[lay["grid"][s]:lay["grid"][s + 1]]
        same_u = O.qoi(c, P[s], Q[s], g["u"], g["kx"], kind)
        assert np.allclose(mine, same_u, rtol=1e-13, atol=1e-15), (s, mine, same_u)
        ora = PR.oracle_solve(c, P[s], Q[s], spec, xi[s])
        ref = O.qoi(c, P[s], Q[s], ora["u"], ora["kx"], kind)
        assert np.max(np.abs(mine - ref) / np.abs(ref)) <= FP64_TOL
        if kind == msg.QOI_MEAN:
            assert np.allclose(mine, g["q"], rtol=1e-14, atol=0)
    assert np.all(qg > 0)                                          # h = 1 > 0: u > 0 and outward flux


def test_quantity_argument_errors(handle):
    b = msg.Batch(4, [1], [1])
    with pytest.raises(msg.MsgError):
        msg.quantity(b, 7, None, None, None)
    import torch
    u = torch.zeros(int(b.layout()["cell"][-1]), dtype=torch.float64, device="cuda:0")
    q = torch.zeros(int(b.layout()["grid"][-1]), dtype=torch.float64, device="cuda:0")
    with pytest.raises(msg.MsgError):
        msg.quantity(b, msg.QOI_FLUX, None, u, q)                  # the flux needs kx


def test_sampled_event_timing_counts_every_launch(handle):
    """Event timing of one launch in 8: every launch is still counted (the
    same counts as with every launch timed), the byte totals scaled from the
    timed launches estimate the full ones, and the results do not change.  A
    negative rate is refused."""
    c, S = 2, 8
    xi = I.draw_xi(I.KL10.n_terms, range(S))
    opts = msg.SolveOpts()
    runs = {}
    for every in (1, 8):
        print(f"profiling every {every}", flush=True)
        handle.set_profiling(True, every=every)
        out = PR.gpu_solve(c, [5] * S, [5] * S, I.KL10, xi, opts, handle=handle)
        runs[every] = (out, handle.profile())
        handle.set_profiling(False)
    (o1, p1), (o8, p8) = runs[1], runs[8]
    assert np.array_equal(o1["u"], o8["u"]) and np.array_equal(o1["cycles"], o8["cycles"])
    for k in p1:
        assert p1[k][0] == p8[k][0], k
    n, b1, b8 = p1["smooth"][0], p1["smooth"][2], p8["smooth"][2]
    print("smooth launches", n, "bytes", b1, b8, flush=True)
    assert n > 100 and 0.7 * b1 <= b8 <= 1.4 * b1
    assert p8["smooth"][1] > 0.0
    assert msg.lib().msg_set_profiling(handle.h, -1) == msg.MSG_ERR_ARG
