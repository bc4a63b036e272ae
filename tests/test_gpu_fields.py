"""Coefficient fields on the device against the oracle: the face-mean rule
(the coarse faces as means of the finest grid's faces), the FP32 copies, and
the standard normals drawn on the device from the streams (seed, sample id)
against the oracle's own Philox stream."""
import numpy as np
import pytest

from oracle import binding as O
from oracle import normals as N
from paper_1907_12334_amd import inputs as I
from paper_1907_12334_amd import msg

from . import parity as PR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return msg.Handle(0)


def _fields(handle, c, P, Q, spec, xi, seed=0, ids=None, mixed=False):
    import torch
    b = msg.Batch(c, P, Q)
    opts = msg.SolveOpts(precision=msg.MIXED if mixed else msg.FP64)
    bufs = msg.Buffers(b, opts)
    xi_d = torch.tensor(np.ascontiguousarray(xi), dtype=torch.float64, device="cuda:0") if xi is not None else None
    handle.sample_field(msg.FieldSpec(spec, seed, ids), b, xi_d, bufs.kx, bufs.ky, bufs.kx32, bufs.ky32)
    torch.cuda.synchronize()
    lay = bufs.layout
    out = []
    for s in range(len(P)):
        fx = slice(int(lay["xface"][s]), int(lay["xface"][s + 1]))
        fy = slice(int(lay["yface"][s]), int(lay["yface"][s + 1]))
        r = {"kx": bufs.kx[fx].cpu().numpy(), "ky": bufs.ky[fy].cpu().numpy()}
        if mixed:
            r["kx32"], r["ky32"] = bufs.kx32[fx].cpu().numpy(), bufs.ky32[fy].cpu().numpy()
        out.append(r)
    return out


@pytest.mark.parametrize("c,P,Q", [(4, 8, 4), (2, 5, 5), (4, 0, 3), (2, 3, 0)])
def test_face_mean_fields_match_oracle(handle, c, P, Q):
    """Every face of every grid: the face-mean rule of the squared-exponential
    presets within 1e-13 of the oracle (the finest faces agree to the last
    bits of exp; the means add nothing beyond rounding)."""
    spec = I.separable(1.0, 0.01, 2.0, face_rule=1)
    xi = I.draw_xi(spec.n_terms, range(3), base_seed=99)
    got = _fields(handle, c, [P] * 3, [Q] * 3, spec, xi, mixed=True)
    for s in range(3):
        kx, ky = O.hierarchy_field(c, P, Q, spec.as_dict(), xi[s])
        assert np.max(np.abs(got[s]["kx"] / kx - 1)) <= 1e-13
        assert np.max(np.abs(got[s]["ky"] / ky - 1)) <= 1e-13
        assert np.array_equal(got[s]["kx32"], got[s]["kx"].astype(np.float32))
        assert np.array_equal(got[s]["ky32"], got[s]["ky"].astype(np.float32))


def test_face_mean_ragged_batch(handle):
    """Samples with different finest grids in one call: each sample's coarse
    faces are means of its own finest grid's faces."""
    spec = I.separable(0.3, 0.03, 1.0, m=20, face_rule=1)
    P, Q = [3, 0, 5, 2], [2, 4, 1, 2]
    xi = I.draw_xi(spec.n_terms, range(4), base_seed=7)
    got = _fields(handle, 2, P, Q, spec, xi)
    for s in range(4):
        kx, ky = O.hierarchy_field(2, P[s], Q[s], spec.as_dict(), xi[s])
        assert np.max(np.abs(got[s]["kx"] / kx - 1)) <= 1e-13
        assert np.max(np.abs(got[s]["ky"] / ky - 1)) <= 1e-13


@pytest.mark.parametrize("spec_name", ["kl10", "se"])
def test_device_normals_follow_the_oracle_stream(handle, spec_name):
    """Normals drawn on the device (d_xi = NULL) from (seed, sample id) give
    the fields the oracle builds from its own Philox stream of the same ids,
    whatever the order of the samples in the batch."""
    spec = I.KL10 if spec_name == "kl10" else I.separable(0.3, 0.03, 1.0, face_rule=1)
    seed, ids = 20190731, np.array([17, 0, 5, 1 << 33], dtype=np.int64)
    c, P, Q = 2, 3, 4
    got = _fields(handle, c, [P] * 4, [Q] * 4, spec, None, seed=seed, ids=ids)
    xi = N.kl_normals(spec.n_terms, ids, seed)
    for s in range(4):
        kx, ky = O.hierarchy_field(c, P, Q, spec.as_dict(), xi[s])
        assert np.max(np.abs(got[s]["kx"] / kx - 1)) <= 1e-13
        assert np.max(np.abs(got[s]["ky"] / ky - 1)) <= 1e-13
    swapped = _fields(handle, c, [P] * 2, [Q] * 2, spec, None, seed=seed, ids=ids[[3, 0]])
    assert np.array_equal(swapped[0]["kx"], got[3]["kx"]) and np.array_equal(swapped[1]["ky"], got[0]["ky"])


def test_device_normals_solve_end_to_end(handle):
    """A solve whose normals are drawn on the device matches the oracle fed
    with the oracle's stream of the same ids (FP64 bar)."""
    spec = I.KL10
    seed, ids = 11, np.arange(40, 44, dtype=np.int64)
    c, P, Q = 4, 3, 2
    out = PR.gpu_solve(c, [P] * 4, [Q] * 4, spec, None, msg.SolveOpts(), handle=handle, seed=seed, sample_id=ids)
    xi = N.kl_normals(spec.n_terms, ids, seed)
    for s in range(4):
        g = PR.per_sample(out, s)
        eu, eq, edq, ora = PR.compare_sample(c, P, Q, spec, xi[s], g)
        assert g["status"] == ora["status"] == 0
        assert max(eu, eq, edq) <= 1e-10, (s, eu, eq, edq)


def test_face_rule_is_validated(handle):
    import ctypes
    import torch
    b = msg.Batch(2, [1], [1])
    spec = msg.FieldSpec(I.KL10)
    spec.c_struct.face_rule = 7
    kx = torch.zeros(int(b.layout()["xface"][-1]), dtype=torch.float64, device="cuda:0")
    ky = torch.zeros(int(b.layout()["yface"][-1]), dtype=torch.float64, device="cuda:0")
    code = msg.lib().msg_sample_field(handle.h, ctypes.byref(spec.c_struct), ctypes.byref(b.c_struct), None,
                                      kx.data_ptr(), ky.data_ptr(), None, None, None)
    assert code == msg.MSG_ERR_ARG
