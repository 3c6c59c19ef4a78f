"""CPU tests of the native library: it loads, exports every symbol the header
declares, rejects bad arguments, and its host-built ghost map equals the
oracle's fixed point (no device is used)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle.ghost import GhostMap
from paper_2411_19185_amd import _lib
from paper_2411_19185_amd._lib import header_functions, inspect_ghost_map, lib, make_desc


def test_library_exports_every_header_function():
    L = lib()
    names = header_functions()
    assert "hope_grid_create" in names and "hope_tendency_vjp" in names and "hope_rk_step" in names
    for name in names:
        assert hasattr(L, name), name


@pytest.mark.parametrize("n,order,scheme,code", [(12, 4, "tpp", -2), (12, 15, "tpp", -2), (12, 7, "weno", -2),
                                                 (4, 5, "tpp", -2), (4097, 5, "weno", -2), (0, 3, "tpp", -2),
                                                 (-5, 3, "tpp", -2), (12, 1, "tpp", -2)])
def test_inspect_rejects_unsupported(n, order, scheme, code):
    d = make_desc(n, order, scheme)
    rows, nnz = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().hope_inspect_ghost_map(ctypes.byref(d), ctypes.byref(rows), ctypes.byref(nnz), None, None, None,
                                      None, None)
    assert rc == code
    assert lib().hope_last_error().decode()


def test_create_rejects_bad_struct_size():
    d = make_desc(12, 5)
    d.struct_size = 8
    h = ctypes.c_void_p()
    assert lib().hope_grid_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert lib().hope_grid_create(None, ctypes.byref(h)) == -1


def _apply_library_ghost_map(n, k, q, ghost_iters=0):
    dst, ptr, col, val, sweeps = inspect_ghost_map(n, k, ghost_iters=ghost_iters)
    r = (k - 1) // 2
    P = n + 2 * r
    qp = np.zeros((3, 6 * P * P))
    jj, ii = np.meshgrid(np.arange(r, r + n), np.arange(r, r + n), indexing="ij")
    idx = np.concatenate([(A * P * P + jj * P + ii).ravel() for A in range(6)])
    qp[:, idx] = q.reshape(3, -1)
    rows = np.repeat(np.arange(len(dst)), np.diff(ptr))
    qp[0, dst] = np.bincount(rows, val[0] * qp[0, col], len(dst))
    qp[1, dst] = np.bincount(rows, val[1] * qp[1, col] + val[2] * qp[2, col], len(dst))
    qp[2, dst] = np.bincount(rows, val[3] * qp[1, col] + val[4] * qp[2, col], len(dst))
    return qp.reshape(3, 6, P, P), sweeps


@pytest.mark.parametrize("n,k", [(6, 3), (8, 5), (13, 5), (10, 7), (12, 11), (3, 3), (5, 5), (9, 9)])
def test_library_ghost_map_equals_oracle_fixed_point(n, k):
    """The library builds G with its own geometry (3D basis vectors), weights
    (primitive-function Lagrange form) and Gauss-Seidel iteration; applied to
    a random state it reproduces the oracle's Jacobi fixed point."""
    q = np.random.default_rng(n * 31 + k).uniform(0.5, 1.5, (3, 6, n, n))
    a, sweeps = _apply_library_ghost_map(n, k, q)
    b = GhostMap(n, k, 6.371e6).fill(torch.tensor(q)).numpy()
    for v in range(3):
        assert np.abs(a[v] - b[v]).max() / np.abs(b[v]).max() < 1e-14
    assert sweeps < 40


@pytest.mark.parametrize("n,k,iters", [(8, 5, 1), (8, 5, 2), (13, 5, 10), (10, 7, 10), (9, 3, 4)])
def test_library_ghost_map_of_fixed_sweeps_equals_oracle(n, k, iters):
    """With ghost_iters = N the library's map is that of exactly N Jacobi
    sweeps from g = 0 (the fixed sweep count of section 3.3.1's iteration):
    it reproduces the oracle's N-sweep fill, and for small N it differs
    measurably from the fixed point, so the count is really honoured."""
    q = np.random.default_rng(n * 37 + k + iters).uniform(0.5, 1.5, (3, 6, n, n))
    a, sweeps = _apply_library_ghost_map(n, k, q, ghost_iters=iters)
    assert sweeps == iters
    b = GhostMap(n, k, 6.371e6).fill(torch.tensor(q), sweeps=iters).numpy()
    for v in range(3):
        assert np.abs(a[v] - b[v]).max() / np.abs(b[v]).max() < 1e-14
    if iters <= 2:
        c = GhostMap(n, k, 6.371e6).fill(torch.tensor(q)).numpy()
        assert np.abs(a - c).max() > 1e-8


@pytest.mark.parametrize("iters", [-1, 301])
def test_create_rejects_bad_ghost_iters(iters):
    d = make_desc(12, 5, ghost_iters=iters)
    h = ctypes.c_void_p()
    assert lib().hope_grid_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert "ghost_iters" in lib().hope_last_error().decode()


def test_batch_create_rejects_bad_arguments():
    h = ctypes.c_void_p()
    assert lib().hope_batch_create(None, 1, None, ctypes.byref(h)) == -1
    arr = (ctypes.c_void_p * 1)(None)
    assert lib().hope_batch_create(arr, 1, None, ctypes.byref(h)) == -1
    assert lib().hope_batch_create(arr, 0, None, ctypes.byref(h)) == -1
    assert "null" in lib().hope_last_error().decode() or "n_members" in lib().hope_last_error().decode()


def _tangent_basis(p, x, y, h=1e-6):
    """Columns d(point)/dx, d(point)/dy of panel p at angles (x, y) (extended
    coordinates allowed), by central differences of the oracle's panel map."""
    from oracle.geometry import panel_xyz
    ex = (panel_xyz(p, np.tan(x + h), np.tan(y)) - panel_xyz(p, np.tan(x - h), np.tan(y))) / (2 * h)
    ey = (panel_xyz(p, np.tan(x), np.tan(y + h)) - panel_xyz(p, np.tan(x), np.tan(y - h))) / (2 * h)
    return np.stack([ex, ey], axis=-1)


def _rotation_image(R, p, i, j, n):
    """Panel, centred cell indices and 2x2 map of contravariant components of
    the image under the cube rotation R of cell (i, j) of panel p (indices
    in [-r, n+r): ghost cells in p's extended coordinates)."""
    from oracle.geometry import PANEL_AXIS, panel_xyz, xyz_to_XY
    D = np.pi / (2 * n)
    x, y = (i + 0.5 - n / 2) * D, (j + 0.5 - n / 2) * D
    v = R @ panel_xyz(p, np.tan(x), np.tan(y))
    q = int(np.argmin(np.abs(PANEL_AXIS - R @ PANEL_AXIS[p]).sum(axis=1)))
    X2, Y2 = xyz_to_XY(q, v)
    x2, y2 = np.arctan(X2), np.arctan(Y2)
    i2, j2 = x2 / D + n / 2 - 0.5, y2 / D + n / 2 - 0.5
    assert abs(i2 - round(i2)) < 1e-9 and abs(j2 - round(j2)) < 1e-9
    E, E2 = _tangent_basis(p, x, y), _tangent_basis(q, x2, y2)
    Mx = np.linalg.lstsq(E2, R @ E, rcond=None)[0]
    M = np.round(Mx)
    assert np.abs(Mx - M).max() < 1e-6      # a signed permutation
    return q, int(round(i2)), int(round(j2)), M


@pytest.mark.parametrize("n,k", [(7, 3), (8, 5)])
@pytest.mark.parametrize("axis_perm,signs", [((1, 0, 2), (-1, 1, 1)), ((0, 2, 1), (1, -1, 1)), ((2, 0, 1), (1, 1, 1))])
def test_library_ghost_map_commutes_with_cube_rotations(n, k, axis_perm, signs):
    """The ghost map is equivariant under the cube's rotations: the ghosts of a
    rotated field are the rotated ghosts.  Rotations and momentum frames come
    from the oracle's panel maps (independent of the library's frame codes,
    which compress the map by this symmetry)."""
    R = np.zeros((3, 3))
    for a, (b, s) in enumerate(zip(axis_perm, signs)):
        R[a, b] = s
    assert abs(np.linalg.det(R) - 1) < 1e-12
    r = (k - 1) // 2
    P = n + 2 * r
    rng = np.random.default_rng(n * 7 + k)
    q = rng.uniform(0.5, 1.5, (3, 6, n, n))
    rot = np.zeros_like(q)
    for p in range(6):
        for j in range(n):
            for i in range(n):
                p2, i2, j2, M = _rotation_image(R, p, i, j, n)
                rot[0, p2, j2, i2] = q[0, p, j, i]
                rot[1:, p2, j2, i2] = M @ q[1:, p, j, i]
    a, _ = _apply_library_ghost_map(n, k, q)
    b, _ = _apply_library_ghost_map(n, k, rot)
    scale = np.abs(a).max()
    worst = 0.0
    for p in range(6):
        for jj in range(P):
            for ii in range(P):
                if r <= jj < r + n and r <= ii < r + n:
                    continue
                p2, i2, j2, M = _rotation_image(R, p, ii - r, jj - r, n)
                want = np.concatenate([[a[0, p, jj, ii]], M @ a[1:, p, jj, ii]])
                got = b[:, p2, j2 + r, i2 + r]
                worst = max(worst, np.abs(want - got).max() / scale)
    assert worst < 1e-13, worst


def test_entry_points_reject_null_handles_without_a_device():
    """Argument checks come before any device work: null grids and buffers
    are rejected with HOPE_ERR_INVALID and a message."""
    L = lib()
    n_bad = ctypes.c_int64(5)
    assert L.hope_check_state(None, None, ctypes.byref(n_bad), None) == -1
    assert n_bad.value == 0
    assert L.hope_fill_halo(None, None, None) == -1
    assert L.hope_tendency(None, None, None, None, 0, None) == -1
    assert L.hope_rk_step(None, None, 1.0, 0, None, 0, None) == -1
    assert L.hope_grid_profile(None, 1) == -1
    assert L.hope_grid_layout(None, None) == -1
    assert L.hope_last_error().decode()
