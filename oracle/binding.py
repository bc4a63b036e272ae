"""ctypes binding of the C oracle (test infrastructure, not the product).

Every function takes and returns numpy float64 arrays in the documented
packing: grids in p-major then q-minor order, each grid row-major with x
fastest; x-face arrays hold (nx+1)*ny values, y-face arrays nx*(ny+1).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


class OracleOpts(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_int32), ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("max_cycles", ctypes.c_int32), ("tol", ctypes.c_double), ("omega", ctypes.c_double),
                ("joint_stages", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("MSG_ORACLE_LIB", _build.LIB)
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.oracle_fmsg_solve.restype = ctypes.c_int
        L.oracle_fmsg_solve.argtypes = [ctypes.c_int] * 3 + [_D, _D, _D, ctypes.POINTER(OracleOpts), _I,
                                                              _D, _D, _I, _D]
        L.oracle_msg_cycles.restype = None
        L.oracle_msg_cycles.argtypes = [ctypes.c_int] * 3 + [_D, _D, _D, ctypes.POINTER(OracleOpts),
                                                              ctypes.c_int, _D, _D]
        L.oracle_delta_q.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.oracle_mg_cycles.argtypes = [ctypes.c_int] * 3 + [_D, _D, _D, ctypes.POINTER(OracleOpts),
                                                             ctypes.c_int, _D, _D]
        L.oracle_mg_cycles.restype = None
        L.oracle_qoi_grid.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_int]
        L.oracle_qoi_grid.restype = ctypes.c_double
        for name in ("oracle_apply",):
            getattr(L, name).argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
        L.oracle_residual.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D]
        L.oracle_rbgs.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, ctypes.c_int]
        L.oracle_weights.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
        L.oracle_restrict_x.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.oracle_restrict_y.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.oracle_prolong_x.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_int]
        L.oracle_prolong_y.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_int]
        L.oracle_correction.argtypes = [ctypes.c_int] * 3 + [_D, _D, _D, _D, ctypes.c_int, _D]
        L.oracle_field_cos.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _I, _D, _D, _D, _D]
        L.oracle_field_separable.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 3 + [_D, _D, _D]
        L.oracle_face_mean.argtypes = [ctypes.c_int] * 3 + [_D, _D, ctypes.c_int, ctypes.c_int, _D, _D]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _i(a):
    return a.ctypes.data_as(_I)


def f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- geometry
def grid_shapes(c, P, Q):
    """[(p, q, nx, ny)] in packed order."""
    return [(p, q, c << p, c << q) for p in range(P + 1) for q in range(Q + 1)]


def packed_sizes(c, P, Q):
    cells = sum(nx * ny for _, _, nx, ny in grid_shapes(c, P, Q))
    fx = sum((nx + 1) * ny for _, _, nx, ny in grid_shapes(c, P, Q))
    fy = sum(nx * (ny + 1) for _, _, nx, ny in grid_shapes(c, P, Q))
    return cells, fx, fy


def split_cells(u, c, P, Q):
    """Packed cell array -> dict (p,q) -> (ny, nx) array."""
    out, off = {}, 0
    for p, q, nx, ny in grid_shapes(c, P, Q):
        out[(p, q)] = u[off:off + nx * ny].reshape(ny, nx)
        off += nx * ny
    return out


# ---------------------------------------------------------------- fields
def field_cos(nx, ny, a, b, amp, xi):
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    amp, xi = f64(amp), f64(xi)
    kx = np.empty((nx + 1) * ny)
    ky = np.empty(nx * (ny + 1))
    lib().oracle_field_cos(nx, ny, len(a), _i(a), _i(b), _d(amp), _d(xi), _d(kx), _d(ky))
    return kx, ky


def field_separable(nx, ny, mx, my, lx, ly, sigma2, xi):
    xi = f64(xi)
    kx = np.empty((nx + 1) * ny)
    ky = np.empty(nx * (ny + 1))
    lib().oracle_field_separable(nx, ny, mx, my, lx, ly, sigma2, _d(xi), _d(kx), _d(ky))
    return kx, ky


def face_mean(c, P, Q, kxF, kyF, p, q):
    """Face-mean coefficients of grid (p,q) from the finest grid's (P,Q) faces."""
    nx, ny = c << p, c << q
    kx = np.empty((nx + 1) * ny)
    ky = np.empty(nx * (ny + 1))
    kxF, kyF = f64(kxF), f64(kyF)
    lib().oracle_face_mean(c, P, Q, _d(kxF), _d(kyF), p, q, _d(kx), _d(ky))
    return kx, ky


def _grid_field(nx, ny, spec, xi):
    if spec["kind"] == "cos":
        return field_cos(nx, ny, spec["a"], spec["b"], spec["amp"], xi)
    return field_separable(nx, ny, spec["mx"], spec["my"], spec["lx"], spec["ly"], spec["sigma2"], xi)


def hierarchy_field(c, P, Q, spec, xi):
    """Face coefficients of every grid of the rectangle, packed.  Face rule 0
    evaluates k at every face midpoint of every grid; rule 1 evaluates it on
    the finest grid only and gives every coarser face the mean along it."""
    kxs, kys = [], []
    if spec.get("face_rule", 0) == 1:
        kxF, kyF = _grid_field(c << P, c << Q, spec, xi)
        for p, q, _, _ in grid_shapes(c, P, Q):
            kx, ky = face_mean(c, P, Q, kxF, kyF, p, q)
            kxs.append(kx)
            kys.append(ky)
    else:
        for _, _, nx, ny in grid_shapes(c, P, Q):
            kx, ky = _grid_field(nx, ny, spec, xi)
            kxs.append(kx)
            kys.append(ky)
    return np.concatenate(kxs), np.concatenate(kys)


# ---------------------------------------------------------------- single-grid steps
def apply(nx, ny, kx, ky, u):
    out = np.empty(nx * ny)
    u, kx, ky = f64(u), f64(kx), f64(ky)
    lib().oracle_apply(nx, ny, _d(kx), _d(ky), _d(u), _d(out))
    return out


def residual(nx, ny, kx, ky, b, u):
    out = np.empty(nx * ny)
    kx, ky, b, u = f64(kx), f64(ky), f64(b), f64(u)
    lib().oracle_residual(nx, ny, _d(kx), _d(ky), _d(b), _d(u), _d(out))
    return out


def rbgs(nx, ny, kx, ky, b, u, sweeps=1):
    u = f64(u).copy()
    kx, ky, b = f64(kx), f64(ky), f64(b)
    lib().oracle_rbgs(nx, ny, _d(kx), _d(ky), _d(b), _d(u), sweeps)
    return u


def weights(nx, ny, kx, ky):
    a = np.empty(nx * ny)
    b = np.empty(nx * ny)
    kx, ky = f64(kx), f64(ky)
    lib().oracle_weights(nx, ny, _d(kx), _d(ky), _d(a), _d(b))
    return a, b


def restrict_x(nxc, ny, fine):
    out = np.empty(nxc * ny)
    fine = f64(fine)
    lib().oracle_restrict_x(nxc, ny, _d(fine), _d(out))
    return out


def restrict_y(nx, nyc, fine):
    out = np.empty(nx * nyc)
    fine = f64(fine)
    lib().oracle_restrict_y(nx, nyc, _d(fine), _d(out))
    return out


def prolong_x(nxc, ny, coarse, cubic=False):
    out = np.empty(2 * nxc * ny)
    coarse = f64(coarse)
    lib().oracle_prolong_x(nxc, ny, _d(coarse), _d(out), int(cubic))
    return out


def prolong_y(nx, nyc, coarse, cubic=False):
    out = np.empty(nx * 2 * nyc)
    coarse = f64(coarse)
    lib().oracle_prolong_y(nx, nyc, _d(coarse), _d(out), int(cubic))
    return out


def correction(c, p, q, kx, ky, e_x, e_y, cubic=False):
    """eq. interpolation on grid (p,q) from iterates on (p-1,q) and (p,q-1)."""
    nx, ny = c << p, c << q
    out = np.empty(nx * ny)
    kx, ky = f64(kx), f64(ky)
    ex = f64(e_x) if e_x is not None else None
    ey = f64(e_y) if e_y is not None else None
    lib().oracle_correction(c, p, q, _d(kx), _d(ky), _d(ex) if ex is not None else None,
                            _d(ey) if ey is not None else None, int(cubic), _d(out))
    return out


# ---------------------------------------------------------------- solves
def opts(mu=2, nu1=2, nu2=2, max_cycles=50, tol=1e-10, omega=1.0, joint_stages=False):
    return OracleOpts(mu, nu1, nu2, max_cycles, tol, omega, int(joint_stages))


def fmsg_solve(c, P, Q, kx_all, ky_all, o=None, rhs_top=None, forced_cycles=None, want_hist=False):
    """Full MSG solve of one sample.  Returns dict with u (packed), q, cycles
    per grid, status and (optionally) the residual-ratio history per grid."""
    o = o or opts()
    cells, _, _ = packed_sizes(c, P, Q)
    kx_all, ky_all = f64(kx_all), f64(ky_all)
    u = np.empty(cells)
    q = np.empty((P + 1) * (Q + 1))
    ng = (P + 1) * (Q + 1)
    cyc = np.zeros(ng, dtype=np.int32)
    hist = np.full(ng * (o.max_cycles + 1), np.nan) if want_hist else None
    rhs = f64(rhs_top) if rhs_top is not None else None
    forced = np.ascontiguousarray(forced_cycles, dtype=np.int32) if forced_cycles is not None else None
    st = lib().oracle_fmsg_solve(c, P, Q, _d(kx_all), _d(ky_all), _d(rhs) if rhs is not None else None,
                                 ctypes.byref(o), _i(forced) if forced is not None else None,
                                 _d(u), _d(q), _i(cyc), _d(hist) if hist is not None else None)
    res = {"u": u, "q": q, "cycles": cyc, "status": st}
    if want_hist:
        res["hist"] = hist.reshape(ng, o.max_cycles + 1)
    return res


def mg_cycles(c, P, Q, kx_all, ky_all, ncycles, o=None, rhs_top=None):
    """Standard-coarsening multigrid cycles from zero on the finest grid.
    Returns (u_top, ratios)."""
    o = o or opts()
    nx, ny = c << P, c << Q
    kx_all, ky_all = f64(kx_all), f64(ky_all)
    u = np.empty(nx * ny)
    ratios = np.empty(ncycles + 1)
    rhs = f64(rhs_top) if rhs_top is not None else None
    lib().oracle_mg_cycles(c, P, Q, _d(kx_all), _d(ky_all), _d(rhs) if rhs is not None else None,
                           ctypes.byref(o), ncycles, _d(u), _d(ratios))
    return u, ratios


def msg_cycles(c, P, Q, kx_all, ky_all, ncycles, o=None, rhs_top=None):
    """Plain MSG cycles from zero on the finest grid.  Returns (u_top, ratios)."""
    o = o or opts()
    nx, ny = c << P, c << Q
    kx_all, ky_all = f64(kx_all), f64(ky_all)
    u = np.empty(nx * ny)
    ratios = np.empty(ncycles + 1)
    rhs = f64(rhs_top) if rhs_top is not None else None
    lib().oracle_msg_cycles(c, P, Q, _d(kx_all), _d(ky_all), _d(rhs) if rhs is not None else None,
                            ctypes.byref(o), ncycles, _d(u), _d(ratios))
    return u, ratios


QOI_MEAN, QOI_POINT, QOI_SUBDOMAIN, QOI_FLUX = range(4)


def qoi_grid(u, kx, kind):
    """One grid's quantity of interest: u (ny, nx) cells, kx (ny, nx+1) faces."""
    u = f64(u)
    ny, nx = u.shape
    kx = f64(kx) if kx is not None else np.zeros((ny, nx + 1))
    return lib().oracle_qoi_grid(nx, ny, _d(kx), _d(u), kind)


def qoi(c, P, Q, u_all, kx_all, kind):
    """Per-grid quantities of interest of one sample (packed order)."""
    u_all, kx_all = f64(u_all), f64(kx_all)
    out, cu, cx = [], 0, 0
    for p, q, nx, ny in grid_shapes(c, P, Q):
        out.append(qoi_grid(u_all[cu:cu + nx * ny].reshape(ny, nx),
                            kx_all[cx:cx + (nx + 1) * ny].reshape(ny, nx + 1), kind))
        cu += nx * ny
        cx += (nx + 1) * ny
    return np.array(out)


def delta_q(P, Q, q):
    q = f64(q)
    out = np.empty((P + 1) * (Q + 1))
    lib().oracle_delta_q(P, Q, _d(q), _d(out))
    return out
