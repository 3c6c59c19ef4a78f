"""GPU tests of the on-disk cache of host tables: a grid created from a cache
file gives bitwise the results of a freshly built one (tendency, its adjoint,
an RK step), also for another axis tilt, and a damaged file is rebuilt."""
import os

import pytest
import torch

from cases import STATES, cfl_dt, to_padded

pytestmark = pytest.mark.gpu


def _results(g, q, dt):
    qp = to_padded(q, g.r)
    t = g.tendency(qp.clone())
    w = torch.sin(torch.arange(t.numel(), dtype=torch.float64, device="cuda")).reshape(t.shape)
    v = g.tendency_vjp(qp.clone(), w)
    s = qp.clone()
    g.rk_step(s, dt)
    torch.cuda.synchronize()
    return t.cpu(), v.cpu(), g.interior(s).cpu()


@pytest.mark.parametrize("n,order,scheme,tilt", [(30, 5, "weno", 0.0), (12, 11, "tpp", 0.7)])
def test_cached_grid_is_bitwise_the_built_grid(tmp_path, n, order, scheme, tilt):
    from paper_2411_19185_amd import Grid
    print(f"case n={n} order={order} {scheme} tilt={tilt}", flush=True)
    d = str(tmp_path / "cache")
    _, q = STATES["member"](n, 5)
    dt = cfl_dt(q)
    ref = Grid(n, order, scheme, axis_tilt=tilt)
    assert ref.layout.tables_cached == 0
    want = _results(ref, q, dt)
    g1 = Grid(n, order, scheme, axis_tilt=tilt, cache_dir=d)
    assert g1.layout.tables_cached == 0
    files = os.listdir(d)
    assert len(files) == 1 and files[0].endswith(".bin")
    g2 = Grid(n, order, scheme, axis_tilt=tilt, cache_dir=d)
    assert g2.layout.tables_cached == 1
    assert g2.layout.ghost_sweeps == ref.layout.ghost_sweeps
    assert g2.layout.device_bytes == ref.layout.device_bytes
    for a, b in zip(_results(g2, q, dt), want):
        assert torch.equal(a, b)
    # the axis tilt is not part of the key: the same file serves another tilt
    g3 = Grid(n, order, scheme, axis_tilt=tilt + 0.3, cache_dir=d)
    assert g3.layout.tables_cached == 1
    ref3 = Grid(n, order, scheme, axis_tilt=tilt + 0.3)
    for a, b in zip(_results(g3, q, dt), _results(ref3, q, dt)):
        assert torch.equal(a, b)
    assert len(os.listdir(d)) == 1


def test_damaged_cache_file_is_rebuilt(tmp_path):
    from paper_2411_19185_amd import Grid
    d = str(tmp_path / "cache")
    n = 16
    _, q = STATES["member"](n, 6)
    dt = cfl_dt(q)
    want = _results(Grid(n, 5, "tpp", cache_dir=d), q, dt)
    path = os.path.join(d, os.listdir(d)[0])
    data = bytearray(open(path, "rb").read())
    data[len(data) // 2] ^= 0x10
    open(path, "wb").write(data)
    g = Grid(n, 5, "tpp", cache_dir=d)
    assert g.layout.tables_cached == 0
    for a, b in zip(_results(g, q, dt), want):
        assert torch.equal(a, b)
    open(path, "wb").write(data[:1000])
    g = Grid(n, 5, "tpp", cache_dir=d)
    assert g.layout.tables_cached == 0
    assert Grid(n, 5, "tpp", cache_dir=d).layout.tables_cached == 1
    # another ghost-map setting is another file
    assert Grid(n, 5, "tpp", cache_dir=d, ghost_iters=10).layout.tables_cached == 0
    assert len(os.listdir(d)) == 2
