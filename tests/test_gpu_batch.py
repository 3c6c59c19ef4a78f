"""GPU tests of the batched ensemble: every member of a batch of uneven
resolutions, with its own axis tilt and time step, must equal bitwise what
its own grid gives through the single-grid entry points, whatever the
work-item shapes and grid size, including inside a replayed HIP graph; and a
member is checked against the FP64 oracle at 1e-11."""
import pytest
import torch

import hope_inputs as hi
from cases import STATES, cfl_dt, oracle_grid, rel_err, to_padded
from oracle.rk import ssp_rk3

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _grid(n, order, scheme, alpha=0.0):
    from paper_2411_19185_amd import Grid
    return Grid(n, order, scheme, axis_tilt=alpha)


def _setup(ns, order=5, scheme="weno", seed=0, state="member"):
    """A batch whose members share one grid per resolution, each member with
    its own tilt and state (seeded), plus per-member reference grids."""
    from paper_2411_19185_amd.ensemble import Ensemble
    shared = {n: _grid(n, order, scheme) for n in sorted(set(ns))}
    tilts, states = [], []
    for i, n in enumerate(ns):
        alpha, q = STATES[state](n, seed + i, nq=2)
        tilts.append(alpha)
        states.append(q)
    ens = Ensemble([shared[n] for n in ns], axis_tilt=tilts)
    q_all = ens.new_state()
    for i, q in enumerate(states):
        ens.member_interior(q_all, i).copy_(q.cuda())
    return ens, q_all, tilts, states, shared


def test_batch_tendency_equals_each_member_grid_bitwise():
    ns = [10, 13, 10, 16, 13]
    print("case batch tendency", ns, flush=True)
    ens, q_all, tilts, states, _ = _setup(ns, seed=100)
    assert ens.info.fill_blocks > 0          # WENO5 rows take the LDS-staged batched fill
    out = ens.tendency(q_all)
    for i, n in enumerate(ns):
        g = _grid(n, 5, "weno", tilts[i])
        ref = g.tendency(to_padded(states[i], g.r))
        got = ens.member_field(out, i)
        torch.cuda.synchronize()
        same = torch.equal(got, ref)
        assert same, (i, rel_err(got, ref))
    # and one member against the oracle
    og = oracle_grid(ns[1], 5, "weno", tilts[1])
    err = rel_err(ens.member_field(out, 1), og.tendency(states[1]))
    print("oracle rel err", err, flush=True)
    assert max(err) < TOL, err


@pytest.mark.parametrize("order,scheme,ns", [(3, "tpp", [3, 8, 3, 31]), (3, "weno", [3, 5, 9]),
                                             (11, "tpp", [11, 14, 11]), (5, "tpp", [5, 64, 6])])
def test_batch_of_other_orders_and_smallest_members_equals_member_grids(order, scheme, ns):
    """Other orders and schemes, with members as small as the order allows."""
    print("case batch", order, scheme, ns, flush=True)
    ens, q_all, tilts, states, _ = _setup(ns, order=order, scheme=scheme, seed=200 + order)
    out = ens.tendency(q_all)
    for i, n in enumerate(ns):
        g = _grid(n, order, scheme, tilts[i])
        ref = g.tendency(to_padded(states[i], g.r))
        got = ens.member_field(out, i)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (i, n, rel_err(got, ref))
    og = oracle_grid(ns[0], order, scheme, tilts[0])
    err = rel_err(ens.member_field(out, 0), og.tendency(states[0]))
    print("oracle rel err", err, flush=True)
    assert max(err) < TOL, err


@pytest.mark.parametrize("scheme", ["ssp3", "ws3"])
def test_batch_rk_steps_equal_each_member_grid_bitwise(scheme):
    ns = [12, 9, 12, 15]
    print("case batch rk", scheme, ns, flush=True)
    ens, q_all, tilts, states, _ = _setup(ns, order=5, scheme="tpp", seed=200)
    dts = [cfl_dt(q) * (1.0 + 0.1 * i) for i, q in enumerate(states)]
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    ws = ens.workspace()
    for _ in range(3):
        ens.rk_step(q_all, dt, ws, scheme)
    for i, n in enumerate(ns):
        g = _grid(n, 5, "tpp", tilts[i])
        qp = to_padded(states[i], g.r)
        w = g.workspace()
        for _ in range(3):
            g.rk_step(qp, dts[i], scheme, w)
        torch.cuda.synchronize()
        got = ens.member_interior(q_all, i)
        same = torch.equal(got, g.interior(qp))
        assert same, (i, rel_err(got, g.interior(qp)))


@pytest.mark.parametrize("blocks", [0, 5])
def test_batch_segment_seams_rk_steps_equal_each_member_grid_bitwise(blocks):
    """WENO5 members cut into 2-, 3- and 4-row segments, so that the batched
    segment seams finish the rows beside every boundary (the Runge-Kutta
    combination included), one workgroup per item or persistent."""
    ns = [12, 17, 9]
    print("case batch seams rk", ns, blocks, flush=True)
    ens, q_all, tilts, states, _ = _setup(ns, order=5, scheme="weno", seed=400)
    ens.set_launch([6, 17, 30], [2, 3, 4], blocks)
    dts = [cfl_dt(q) * (1.0 - 0.1 * i) for i, q in enumerate(states)]
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    ws = ens.workspace()
    for _ in range(2):
        ens.rk_step(q_all, dt, ws, "ssp3")
    for i, n in enumerate(ns):
        g = _grid(n, 5, "weno", tilts[i])
        qp = to_padded(states[i], g.r)
        w = g.workspace()
        for _ in range(2):
            g.rk_step(qp, dts[i], "ssp3", w)
        torch.cuda.synchronize()
        got = ens.member_interior(q_all, i)
        assert torch.equal(got, g.interior(qp)), (i, rel_err(got, g.interior(qp)))


def test_batch_launch_shapes_and_persistent_grid_do_not_change_results():
    ns = [16, 11, 16]
    ens, q_all, _, _, _ = _setup(ns, seed=300)
    base = ens.tendency(q_all).clone()
    for sw, sh, blocks in [([5, 11, 7], [3, 2, 16], 0), ([16, 4, 9], [1, 11, 5], 7), ([8, 8, 8], [4, 4, 4], 64)]:
        ens.set_launch(sw, sh, blocks)
        other = ens.tendency(q_all)
        torch.cuda.synchronize()
        same = torch.equal(base, other)
        assert same, (sw, sh, blocks)


def test_batch_graph_replays_equal_eager_steps():
    """One captured RK step replayed three times, with unrelated eager work
    and synchronisations between the replays, equals three eager steps; the
    per-member dt is read at replay time."""
    ns = [10, 14, 10]
    ens, q_all, _, states, _ = _setup(ns, seed=400)
    dts = [cfl_dt(q) for q in states]
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    q_eager = q_all.clone()
    ws_e = ens.workspace()
    graph = ens.capture_step(q_all, dt)
    scratch = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
    for r in range(3):
        if r == 2:
            dt.mul_(0.5)              # new steps without re-capture
        graph.replay()
        scratch.mul_(1.0001).add_(1.0)     # eager work between replays
        torch.cuda.synchronize()
        ens.rk_step(q_eager, dt, ws_e)
        torch.cuda.synchronize()
        for i in range(len(ns)):
            same = torch.equal(ens.member_interior(q_all, i), ens.member_interior(q_eager, i))
            assert same, (r, i)


def test_captured_batch_keeps_its_launch_and_ensemble_alive():
    """A graph captured from a batch refers to its work-item list and member
    table: hope_batch_set_launch refuses afterwards (set_launch before the
    capture works), and the graph keeps the ensemble alive, so a replay after
    the caller drops it still equals eager steps on a separate ensemble."""
    import gc

    from paper_2411_19185_amd._lib import HopeError
    ns = [10, 12]
    ens, q_all, _, states, _ = _setup(ns, seed=410)
    ens.set_launch([7, 6], [3, 4], 0)
    dt = torch.tensor([cfl_dt(q) for q in states], dtype=torch.float64, device="cuda")
    ref, q_ref, _, _, _ = _setup(ns, seed=410)
    graph = ens.capture_step(q_all, dt)
    with pytest.raises(HopeError) as e:
        ens.set_launch([5, 5], [2, 2], 0)
    assert "captured" in str(e.value)
    del ens
    gc.collect()
    for _ in range(2):
        graph.replay()
        ref.rk_step(q_ref, dt)
    torch.cuda.synchronize()
    assert torch.equal(q_all, q_ref)


def test_full_size_uneven_ensemble_against_member_grids_and_oracle():
    """The 64-member ensemble of the benchmark (16 members each at C48, C64,
    C90 and C128, WENO5, own tilt and dt): two graph-replayed steps equal, for
    one member of each resolution, the same steps on that member's own grid;
    the C48 member's first step matches the oracle."""
    from paper_2411_19185_amd.ensemble import Ensemble
    sizes = [48, 64, 90, 128]
    ns = [sizes[i % 4] for i in range(64)]
    print("case C5 ensemble", flush=True)
    shared = {n: _grid(n, 5, "weno") for n in sizes}
    tilts, states = [], []
    for i, n in enumerate(ns):
        f = hi.BalancedFlowWithCap(seed=5000 + i)
        from oracle.ic import cell_average
        tilts.append(f.alpha)
        states.append(cell_average(f, n, hi.EARTH_RADIUS, nq=2))
    ens = Ensemble([shared[n] for n in ns], axis_tilt=tilts)
    q_all = ens.new_state()
    for i, q in enumerate(states):
        ens.member_interior(q_all, i).copy_(q.cuda())
    dts = [cfl_dt(q) for q in states]
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    graph = ens.capture_step(q_all, dt)
    graph.replay()
    torch.cuda.synchronize()
    first = ens.member_interior(q_all, 0).cpu().clone()
    graph.replay()
    torch.cuda.synchronize()
    print("batch done", flush=True)
    for i in range(4):
        n = ns[i]
        g = _grid(n, 5, "weno", tilts[i])
        qp = to_padded(states[i], g.r)
        w = g.workspace()
        g.rk_step(qp, dts[i], "ssp3", w)
        g.rk_step(qp, dts[i], "ssp3", w)
        torch.cuda.synchronize()
        got = ens.member_interior(q_all, i)
        same = torch.equal(got, g.interior(qp))
        assert same, (i, rel_err(got, g.interior(qp)))
    og = oracle_grid(48, 5, "weno", tilts[0])
    ref = ssp_rk3(og.tendency, states[0], dts[0])
    err = rel_err(first, ref)
    print("oracle rel err", err, flush=True)
    assert max(err) < TOL, err


def test_derived_member_grid_equals_a_fresh_grid_and_member_gradient():
    """A member's derived grid (its tilt, the shared ghost map) gives bitwise
    the tendency and adjoint of a grid built from scratch with that tilt, and
    the ensemble's per-member loss gradient matches autograd over the oracle."""
    ns = [10, 12]
    ens, q_all, tilts, states, _ = _setup(ns, seed=500, state="perturbed_member")
    for i, n in enumerate(ns):
        g = ens.member_grid(i)
        fresh = _grid(n, 5, "weno", tilts[i])
        qa = to_padded(states[i], g.r)
        a = g.tendency(qa)
        b = fresh.tendency(to_padded(states[i], g.r))
        w = torch.tensor(hi.normal_array(600 + i, (3, 6, n, n))).cuda()
        va = g.tendency_vjp(to_padded(states[i], g.r), w)
        vb = fresh.tendency_vjp(to_padded(states[i], g.r), w)
        torch.cuda.synchronize()
        same = torch.equal(a, b) and torch.equal(va, vb)
        assert same, i
    # gradient of 0.5 ||q_T||^2 after 2 steps, member 0, against the oracle
    from oracle.rk import ssp_rk3 as oracle_step
    q0 = states[0]
    dt = cfl_dt(q0)
    grad = ens.member_loss_gradient(0, ens.member_interior(q_all, 0).contiguous(), dt, 2, checkpoint_every=1)
    og = oracle_grid(ns[0], 5, "weno", tilts[0])
    qq = q0.clone().requires_grad_(True)
    x = qq
    for _ in range(2):
        x = oracle_step(og.tendency, x, dt)
    (0.5 * (x * x).sum()).backward()
    err = rel_err(grad, qq.grad)
    print("member gradient rel err", err, flush=True)
    assert max(err) < TOL, err


@pytest.mark.parametrize("tilted", [True, False])
def test_member_gradients_on_streams_equal_one_by_one(tilted):
    """Per-member loss gradients computed concurrently on several HIP streams
    equal bitwise those computed one member after another (members with and
    without their own axis tilt, two sharing one grid)."""
    from paper_2411_19185_amd.ensemble import Ensemble
    ns = [10, 12, 10]
    print("case member gradients on streams", tilted, flush=True)
    shared = {n: _grid(n, 5, "weno") for n in sorted(set(ns))}
    tilts, states = [], []
    for i, n in enumerate(ns):
        alpha, q = STATES["perturbed_member"](n, 700 + i, nq=2)
        tilts.append(alpha)
        states.append(q)
    ens = Ensemble([shared[n] for n in ns], axis_tilt=tilts if tilted else None)
    q0s = [q.cuda() for q in states]
    dts = [cfl_dt(q) for q in states]
    conc = ens.member_loss_gradients(q0s, dts, 2, checkpoint_every=1, streams=3)
    torch.cuda.synchronize()
    for i in range(len(ns)):
        one = ens.member_loss_gradient(i, q0s[i], dts[i], 2, checkpoint_every=1)
        torch.cuda.synchronize()
        same = torch.equal(conc[i], one)
        assert same, (i, rel_err(conc[i], one))
