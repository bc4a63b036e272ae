"""Host-side checks of the C-ABI: the library loads, exports every function
include/msg.h declares, computes the documented layout, and rejects bad
arguments before touching a device.  No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1907_12334_amd import msg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "msg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msg_[a-z_]+|mimc_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function():
    names = declared_functions()
    assert set(names) == set(msg.EXPORTS)
    L = msg.lib()
    for n in names:
        assert hasattr(L, n), n


def _independent_layout(c, P, Q):
    cell = [0]
    xf = [0]
    yf = [0]
    grid = [0]
    for p_, q_ in zip(P, Q):
        ncell = nxf = nyf = 0
        for a in range(p_ + 1):
            for b in range(q_ + 1):
                nx, ny = c << a, c << b
                ncell += nx * ny
                nxf += (nx + 1) * ny
                nyf += nx * (ny + 1)
        cell.append(cell[-1] + ncell)
        xf.append(xf[-1] + nxf)
        yf.append(yf[-1] + nyf)
        grid.append(grid[-1] + (p_ + 1) * (q_ + 1))
    return cell, xf, yf, grid


@pytest.mark.parametrize("c", [1, 2, 4, 3])
def test_layout_matches_definition(c):
    rng = np.random.default_rng(c)
    P = rng.integers(0, 7, size=23)
    Q = rng.integers(0, 7, size=23)
    lay = msg.Batch(c, P, Q).layout()
    cell, xf, yf, grid = _independent_layout(c, P.tolist(), Q.tolist())
    assert lay["cell"].tolist() == cell
    assert lay["xface"].tolist() == xf
    assert lay["yface"].tolist() == yf
    assert lay["grid"].tolist() == grid


def test_bad_batches_are_rejected():
    for c, P, Q, code in [(0, [1], [1], msg.MSG_ERR_LAYOUT), (9, [1], [1], msg.MSG_ERR_LAYOUT),
                          (4, [15], [0], msg.MSG_ERR_LAYOUT), (4, [-1], [0], msg.MSG_ERR_LAYOUT),
                          (8, [13], [0], msg.MSG_ERR_LAYOUT)]:
        with pytest.raises(msg.MsgError) as e:
            msg.Batch(c, P, Q).layout()
        assert e.value.code == code
        assert msg.last_error()


def test_workspace_size_and_options():
    o = msg.default_opts()
    assert (o.mu, o.nu1, o.nu2, o.max_cycles, o.tol, o.omega, o.precision) == (2, 2, 2, 50, 1e-10, 1.0, msg.FP64)
    b = msg.Batch(4, [3] * 8, [3] * 8)
    n64 = msg.workspace_size(b, o)
    om = msg.SolveOpts(precision=msg.MIXED)
    assert msg.workspace_size(b, om) > n64 > 0
    assert msg.workspace_size(msg.Batch(4, [3] * 16, [3] * 16), o) > n64
    with pytest.raises(msg.MsgError):
        msg.workspace_size(b, msg.SolveOpts(mu=0))
    with pytest.raises(msg.MsgError):
        msg.workspace_size(b, msg.SolveOpts(tail_levels=9))
    assert (o.tail_levels, o.handoff, o.overlap) == (-1, -1, -1)
    assert (o.tail_budget, o.tile_width, o.tile_cells, o.tile_lds) == (0, 0, 0, 0)
    for bad in (-2, 3):
        with pytest.raises(msg.MsgError):
            msg.workspace_size(b, msg.SolveOpts(overlap=bad))
    for bad in (dict(tail_budget=512), dict(tail_budget=160000), dict(tile_width=48), dict(tile_width=512),
                dict(tile_cells=32), dict(tile_lds=9000)):
        with pytest.raises(msg.MsgError):
            msg.workspace_size(b, msg.SolveOpts(**bad))
    # a deeper tail needs a larger per-stage conductance image
    big = msg.Batch(2, [7] * 4, [7] * 4)
    assert msg.workspace_size(big, msg.SolveOpts(tail_budget=40960)) > msg.workspace_size(big, msg.SolveOpts())


def test_entry_points_reject_null_handle_without_device_work():
    b = msg.Batch(4, [1], [1])
    o = msg.SolveOpts().c_struct()
    L = msg.lib()
    code = L.msg_solve_batch(None, ctypes.byref(b.c_struct), ctypes.byref(o), *([None] * 10), 0, None)
    assert code == msg.MSG_ERR_ARG
    spec = msg.FieldSpec(type("S", (), {"kind": "cos", "a": [0], "b": [0], "amp": [1.0]})())
    code = L.msg_sample_field(None, ctypes.byref(spec.c_struct), ctypes.byref(b.c_struct), *([None] * 6))
    assert code == msg.MSG_ERR_ARG
    code = L.msg_sample_field_noalloc(None, ctypes.byref(spec.c_struct), ctypes.byref(b.c_struct), *([None] * 6))
    assert code == msg.MSG_ERR_ARG
    code = L.mimc_delta_q(ctypes.byref(b.c_struct), None, None, None)
    assert code == msg.MSG_ERR_ARG


def test_create_reports_missing_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    code = msg.lib().msg_create(ctypes.byref(h), 0)
    assert code in (msg.MSG_ERR_HIP, msg.MSG_ERR_ARG)
    assert msg.last_error()


def test_plain_cycles_workspace_and_validation():
    o = msg.SolveOpts()
    msg_ws = msg.cycles_workspace_size(msg.Batch(2, [4] * 8, [4] * 8), o, msg.CYCLES_MSG)
    mg_ws = msg.cycles_workspace_size(msg.Batch(2, [4] * 8, [4] * 8), o, msg.CYCLES_MG)
    # standard multigrid holds one grid per level, MSG all (P+1)(Q+1) grids
    assert 0 < mg_ws < msg_ws
    assert msg.cycles_workspace_size(msg.Batch(2, [4] * 16, [4] * 16), o, msg.CYCLES_MG) > mg_ws
    assert msg.cycles_workspace_size(msg.Batch(2, [3] * 4, [5] * 4), o, msg.CYCLES_MSG) > 0
    for batch, opts, kind, code in [
        (msg.Batch(2, [3, 4], [4, 4]), o, msg.CYCLES_MSG, msg.MSG_ERR_UNSUPPORTED),     # ragged
        (msg.Batch(2, [3] * 2, [5] * 2), o, msg.CYCLES_MG, msg.MSG_ERR_UNSUPPORTED),    # P != Q for MG
        (msg.Batch(2, [3] * 2, [3] * 2), msg.SolveOpts(precision=msg.MIXED), msg.CYCLES_MG, msg.MSG_ERR_UNSUPPORTED),
        (msg.Batch(2, [3] * 2, [3] * 2), o, 2, msg.MSG_ERR_ARG),
        (msg.Batch(2, [3] * 2, [3] * 2), msg.SolveOpts(mu=4), msg.CYCLES_MSG, msg.MSG_ERR_ARG),
    ]:
        with pytest.raises(msg.MsgError) as e:
            msg.cycles_workspace_size(batch, opts, kind)
        assert e.value.code == code, (kind, msg.last_error())
    b = msg.Batch(2, [3], [3])
    code = msg.lib().msg_cycles(None, ctypes.byref(b.c_struct), ctypes.byref(o.c_struct()), 0, 2,
                                *([None] * 6), 0, None)
    assert code == msg.MSG_ERR_ARG


def test_matern_workspace_and_validation():
    b = msg.Batch(2, [3, 1, 3], [3, 2, 3])
    spec = msg.MaternSpec(0.25, 0.5, [1 / 16, 0.25, 0.1], [0.0, 0.3, -0.5])
    n = msg.matern_workspace_size(b, spec)
    # three samples (fewer than a chunk); largest embedding: 16 cells, m = 1 + 2 ceil(0.707 * 4) = 7,
    # 7 * 2 * 16 = 224 -> 256 points per direction; two complex buffers
    assert n >= 2 * 3 * 256 * 256 * 16
    assert msg.matern_workspace_size(b, msg.MaternSpec(0.25, 0.5, [0.1] * 3, [0.0] * 3, pad=16)) > n
    bad = [dict(lam=0.0), dict(nu=0.0), dict(nu=9.0), dict(eta=[0.1, -1.0, 0.1]), dict(theta=[0.0, float("nan"), 0.0]),
           dict(pad=65)]
    for kw in bad:
        args = dict(lam=0.25, nu=0.5, eta=[0.1] * 3, theta=[0.0] * 3, pad=0)
        args.update(kw)
        with pytest.raises(msg.MsgError) as e:
            msg.matern_workspace_size(b, msg.MaternSpec(**args))
        assert e.value.code == msg.MSG_ERR_ARG, kw
    # 256 x 256 cells: the paper's factor 13 needs 8192 points per direction (the most one workgroup's row holds)
    assert msg.matern_workspace_size(msg.Batch(2, [7], [7]), msg.MaternSpec(0.25, 0.5, [0.1], [0.0])) >= 2 * 8192 ** 2 * 16
    # 512 x 512 cells (2^18 unknowns, the paper's largest): factor 15 needs 16384, by the four-step FFT
    assert msg.matern_workspace_size(msg.Batch(2, [8], [8]), msg.MaternSpec(0.25, 0.5, [0.1], [0.0])) >= 2 * 16384 ** 2 * 16
    # 2048 x 2048 cells: factor 17 needs 2^17 points per direction, beyond the 32768 supported
    with pytest.raises(msg.MsgError) as e:
        msg.matern_workspace_size(msg.Batch(2, [10], [10]), msg.MaternSpec(0.25, 0.5, [0.1], [0.0]))
    assert e.value.code == msg.MSG_ERR_UNSUPPORTED
    assert msg.matern_workspace_size(msg.Batch(2, [10], [10]), msg.MaternSpec(0.25, 0.5, [0.1], [0.0], pad=3)) > 0
    code = msg.lib().msg_sample_matern(None, ctypes.byref(spec.c_struct), ctypes.byref(b.c_struct),
                                       *([None] * 6), 0, None)
    assert code == msg.MSG_ERR_ARG


def test_empty_batch_is_rejected():
    with pytest.raises(msg.MsgError) as e:
        msg.Batch(4, [], []).layout()
    assert e.value.code == msg.MSG_ERR_ARG
    with pytest.raises(msg.MsgError) as e:
        msg.workspace_size(msg.Batch(4, [], []), msg.SolveOpts())
    assert e.value.code == msg.MSG_ERR_ARG
