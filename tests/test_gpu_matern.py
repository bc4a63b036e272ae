"""Matern fields by circulant embedding on the GPU (msg_sample_matern,
through the C-ABI) against the oracle (oracle/matern_oracle.py) on the same
parameters and random streams: k at every face of every grid within 1e-10
relative (the two sides differ only by the rounding of their FFTs and of exp,
about 1e-14 here), the embedding's eigenvalue ratio within 1e-12."""
import math

import numpy as np
import pytest

from oracle import matern_oracle as MO
from paper_1907_12334_amd import msg

pytestmark = pytest.mark.gpu

K_TOL = 1e-10


@pytest.fixture(scope="module")
def handle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return msg.Handle(0)


def _gpu(handle, c, P, Q, spec, fp32=False, ws_bytes=None):
    import torch
    b = msg.Batch(c, P, Q)
    lay = b.layout()
    dev = "cuda:0"
    kx = torch.full((int(lay["xface"][-1]),), float("nan"), dtype=torch.float64, device=dev)
    ky = torch.full((int(lay["yface"][-1]),), float("nan"), dtype=torch.float64, device=dev)
    kx32 = torch.empty(kx.numel(), dtype=torch.float32, device=dev) if fp32 else None
    ky32 = torch.empty(ky.numel(), dtype=torch.float32, device=dev) if fp32 else None
    ratio = torch.full((len(P),), float("nan"), dtype=torch.float64, device=dev)
    n = ws_bytes or msg.matern_workspace_size(b, spec)
    ws = torch.empty((n + 7) // 8, dtype=torch.float64, device=dev)
    handle.sample_matern(spec, b, kx, ky, kx32, ky32, ratio, ws)
    torch.cuda.synchronize()
    out = dict(kx=kx.cpu().numpy(), ky=ky.cpu().numpy(), ratio=ratio.cpu().numpy(), layout=lay)
    if fp32:
        out["kx32"], out["ky32"] = kx32.cpu().numpy(), ky32.cpu().numpy()
    return out


def _compare(g, c, P, Q, lam, nu, eta, theta, ids, seed, pad=0):
    lay = g["layout"]
    worst = 0.0
    for s in range(len(P)):
        kx, ky, ratio = MO.hierarchy_field(c, int(P[s]), int(Q[s]), lam, nu, float(eta[s]), float(theta[s]),
                                           int(ids[s]), seed, pad)
        gx = g["kx"][lay["xface"][s]:lay["xface"][s + 1]]
        gy = g["ky"][lay["yface"][s]:lay["yface"][s + 1]]
        e = max(float(np.max(np.abs(gx - kx) / kx)), float(np.max(np.abs(gy - ky) / ky)))
        assert e <= K_TOL, (s, e)
        assert abs(g["ratio"][s] - ratio) <= 1e-12, (s, g["ratio"][s], ratio)
        worst = max(worst, e)
    return worst


def test_ragged_batch_paper_parameters(handle):
    c = 2
    P = [0, 1, 2, 3, 2, 1]
    Q = [0, 2, 1, 3, 2, 1]
    rng = np.random.default_rng(1)
    eta = rng.uniform(1 / 16, 1 / 4, len(P))
    theta = np.radians(rng.uniform(-30, 30, len(P)))
    ids = np.arange(100, 100 + len(P))
    spec = msg.MaternSpec(0.25, 0.5, eta, theta, ids, seed=7)
    print(f"matern ragged c={c} P={P} Q={Q}", flush=True)
    g = _gpu(handle, c, P, Q, spec, fp32=True)
    _compare(g, c, P, Q, 0.25, 0.5, eta, theta, ids, 7)
    assert np.all(np.isfinite(g["kx"])) and np.all(np.isfinite(g["ky"]))
    assert np.array_equal(g["kx32"], g["kx"].astype(np.float32))
    assert np.array_equal(g["ky32"], g["ky"].astype(np.float32))
    assert np.all(g["ratio"] > -1e-12)


@pytest.mark.parametrize("nu", [0.5, 1.5, 0.7])
def test_smoothness_and_padding(handle, nu):
    c, P, Q = 4, [2, 2, 1], [1, 2, 2]
    eta, theta = np.array([0.1, 1.0, 0.3]), np.array([0.2, 0.0, -1.0])
    for pad in (0, 3):
        print(f"matern nu={nu} pad={pad}", flush=True)
        spec = msg.MaternSpec(0.25, nu, eta, theta, None, seed=3, pad=pad)
        g = _gpu(handle, c, P, Q, spec)
        _compare(g, c, P, Q, 0.25, nu, eta, theta, range(3), 3, pad)


def test_chunking_does_not_change_the_fields(handle):
    c, P, Q = 2, [2] * 5, [3] * 5
    spec = msg.MaternSpec(0.25, 0.5, [1 / 16] * 5, np.radians([0, 10, 20, 30, -30]), None, seed=11)
    a = _gpu(handle, c, P, Q, spec)
    b = msg.Batch(c, P, Q)
    one = msg.matern_workspace_size(msg.Batch(c, P[:1], Q[:1]), spec)
    g1 = _gpu(handle, c, P, Q, spec, ws_bytes=one + 4096)    # one sample per chunk
    assert np.array_equal(a["kx"], g1["kx"]) and np.array_equal(a["ky"], g1["ky"])
    assert np.array_equal(a["ratio"], g1["ratio"])
    # a sample's field depends on its id, not on its place in the batch
    spec2 = msg.MaternSpec(0.25, 0.5, [1 / 16] * 2, np.radians([-30, 10]), [4, 1], seed=11)
    g2 = _gpu(handle, c, P[:2], Q[:2], spec2)
    lay, lay2 = a["layout"], g2["layout"]
    assert np.array_equal(g2["kx"][lay2["xface"][0]:lay2["xface"][1]], a["kx"][lay["xface"][4]:lay["xface"][5]])
    assert np.array_equal(g2["kx"][lay2["xface"][1]:lay2["xface"][2]], a["kx"][lay["xface"][1]:lay["xface"][2]])


def test_indefinite_embedding_is_reported(handle):
    """A long, smooth correlation on the minimal embedding: both sides report
    the same negative eigenvalue ratio."""
    c, P, Q = 2, [2], [2]
    spec = msg.MaternSpec(4.0, 2.5, [1.0], [0.0], None, seed=1, pad=1)
    g = _gpu(handle, c, P, Q, spec)
    _, _, ratio = MO.hierarchy_field(c, 2, 2, 4.0, 2.5, 1.0, 0.0, 0, 1, pad=1)
    assert ratio < -1e-6 and abs(g["ratio"][0] - ratio) <= 1e-9 * abs(ratio)


def test_full_size_64x64_grid(handle):
    """64 x 64 cells (2048 x 2048 embedding, 6 x 6 grids), the size of the
    convergence-factor study."""
    c, P, Q = 2, [5, 5], [5, 5]
    eta, theta = np.array([1 / 16, 1 / 8]), np.radians([30.0, 0.0])
    spec = msg.MaternSpec(0.25, 0.5, eta, theta, [5, 9], seed=2019)
    print("matern 64x64", flush=True)
    g = _gpu(handle, c, P, Q, spec)
    _compare(g, c, P, Q, 0.25, 0.5, eta, theta, [5, 9], 2019)


def test_largest_embedding_256x256_grid(handle):
    """256 x 256 cells: the paper's factor gives an 8192 x 8192 embedding,
    rows of 8192 points in 128 KB of LDS."""
    c, P, Q = 2, [7], [7]
    eta, theta = np.array([1 / 16]), np.radians([20.0])
    spec = msg.MaternSpec(0.25, 0.5, eta, theta, [3], seed=77)
    print("matern 256x256", flush=True)
    g = _gpu(handle, c, P, Q, spec)
    _compare(g, c, P, Q, 0.25, 0.5, eta, theta, [3], 77)


@pytest.mark.parametrize("P,Q", [(5, 5), (6, 3)])
def test_long_rows_by_the_four_step_fft(handle, monkeypatch, P, Q):
    """Rows longer than one workgroup holds run as the four-step FFT (row
    transposes, FFTs of the two factors, twiddles).  With the single-pass
    row length lowered to 2^8 points, every row of these embeddings (2048
    and 4096 points) takes that path; the fields must still match the
    oracle's (numpy's FFT of the whole embedding)."""
    c = 2
    eta, theta = np.array([1 / 16, 1 / 4]), np.radians([-25.0, 10.0])
    spec = msg.MaternSpec(0.25, 0.5, eta, theta, [11, 4], seed=31)
    monkeypatch.setenv("MSG_MATERN_ROW_LOG", "8")
    print(f"matern four-step ({P},{Q})", flush=True)
    g = _gpu(handle, c, [P, P], [Q, Q], spec)
    monkeypatch.delenv("MSG_MATERN_ROW_LOG")
    _compare(g, c, [P, P], [Q, Q], 0.25, 0.5, eta, theta, [11, 4], 31)


def test_512x512_grid_the_papers_largest(handle):
    """512 x 512 cells (2^18 unknowns, the largest problem of the paper's
    experiments): the paper's factor 15 gives a 16384 x 16384 embedding whose
    rows take the four-step FFT.  Checked against the oracle's eigenvalue
    ratio (numpy's FFT of the same first row) and for finite, positive k on
    every face of all 81 grids."""
    c, P, Q = 2, [8], [8]
    eta, theta = np.array([1 / 8]), np.radians([15.0])
    spec = msg.MaternSpec(0.25, 0.5, eta, theta, [7], seed=5)
    print("matern 512x512 (16384^2 embedding)", flush=True)
    g = _gpu(handle, c, P, Q, spec)
    assert np.all(np.isfinite(g["kx"])) and np.all(g["kx"] > 0)
    assert np.all(np.isfinite(g["ky"])) and np.all(g["ky"] > 0)
    Nx = Ny = c << 8
    Mx, My = MO.embedding_shape(Nx, Ny, 0.5)
    assert (Mx, My) == (16384, 16384)
    print("oracle eigenvalues of the 16384^2 embedding", flush=True)
    row = MO.first_row(Mx, My, 1 / (2 * Nx), 1 / (2 * Ny), 0.25, 0.5, float(eta[0]), float(theta[0]))
    lam = np.fft.fft2(row).real
    del row
    ratio = float(lam.min() / lam.max())
    del lam
    assert abs(g["ratio"][0] - ratio) <= 1e-10 * max(1.0, abs(ratio)), (g["ratio"][0], ratio)

