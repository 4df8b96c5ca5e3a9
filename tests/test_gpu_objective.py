"""GPU parity of the low-weight objective (objective_eval, objective_delta) against the checker.

Per-edge values (contractibility, weight) are computed by the same operations in the same order
on both sides, so they are compared bit for bit, as are move statuses. Sums are compared within
the reordering bound of a floating-point sum: |a - b| <= 2 n u sum|terms| for n terms (u = 2^-53),
since each side's sum lies within n u sum|terms| of the exact sum of identical terms.
"""
import math

import numpy as np
import pytest

import helpers
import oracle
import scenegen as sg
from oracle import objective as ob

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"
U = 2.0 ** -53


@pytest.fixture(scope="module")
def ccsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05570_amd as m
    return m


@pytest.fixture(scope="module")
def tiny():
    mesh = helpers.subdivided(sg.make_scene("tiny"))
    return mesh, ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)


def _params(ccsp, p: ob.Params):
    return ccsp.objective_params(p.eps, p.delta, p.eps0, p.mu_angle, p.mu_len, p.polish)


def _clustered(mesh, om, p, seed, n_try=3000):
    """Positions after moves that pull free and constrained vertices next to a neighbour
    (contraction-to-neighbour moves of Sec. 3.2.6), each kept if the checker finds it valid."""
    rng = np.random.default_rng(seed)
    xy = mesh.xy.copy()
    movable = np.nonzero(mesh.kind != sg.ORIGINAL)[0]
    for v in rng.choice(movable, n_try):
        nb = om.nbr[om.nbr_off[v]:om.nbr_off[v + 1]]
        w = nb[rng.integers(0, nb.shape[0])]
        r = 0.3 * p.eps * math.sqrt(rng.random())
        th = 2 * math.pi * rng.random()
        q = xy[w] + r * np.array([math.cos(th), math.sin(th)])
        if mesh.kind[v] == sg.CONSTRAINED:
            a, b = mesh.prim_v[mesh.line[v]]
            e = xy[b] - xy[a]
            q = xy[v] + ((q - xy[v]) @ e) / (e @ e) * e
        if ob.move_status(om, xy, int(v), q) == ob.MOVED:
            xy[v] = q
    return xy


def _check_eval(ccsp, om, xy, p, what):
    ref = ob.objective(om, xy, p)
    with ccsp.MovableMesh(om.tri_v, om.kind, om.line, om.prim_v) as gm:
        assert np.array_equal(gm.edges(), om.edge_v), f"{what}: edge numbering"
        out, con, w = gm.eval(torch.from_numpy(xy).to(DEV), _params(ccsp, p), per_edge=True)
        torch.cuda.synchronize()
        out, con, w = out.cpu().numpy(), con.cpu().numpy(), w.cpu().numpy()
    assert np.array_equal(con.astype(bool), ref["contractible"]), f"{what}: contractibility"
    bad = np.nonzero(w != ref["w"])[0]
    assert bad.size == 0, f"{what}: weights differ at {bad[:5]}: {w[bad[:5]]} vs {ref['w'][bad[:5]]}"
    ne, nc = om.n_edges, ref["angle"].size
    parts = [("wcontr", ref["edge"], ne), ("pangle", ref["angle"], nc), ("plen", ref["short"], ne)]
    for k, (name, t, n) in enumerate(parts, start=1):
        tol = 2 * n * U * np.abs(t).sum()
        assert abs(out[k] - ref[name]) <= tol, f"{what}: {name} {out[k]} vs {ref[name]}"
    scale = (np.abs(ref["edge"]).sum() + p.mu_angle * np.abs(ref["angle"]).sum()
             + p.mu_len * np.abs(ref["short"]).sum())
    assert abs(out[0] - ref["f"]) <= 2 * (ne + nc) * U * scale + 4 * U * abs(ref["f"]), what
    return ref, out


@pytest.mark.parametrize("eps,polish", [(0.02, False), (0.05, False), (1e-300, False),
                                        (1e6, False), (0.05, True)])
def test_tiny_eval(ccsp, tiny, eps, polish):
    mesh, om = tiny
    p = ob.Params(eps, polish=polish)
    ref, _ = _check_eval(ccsp, om, mesh.xy, p, f"eps={eps} polish={polish}")
    if eps == 0.05 and not polish:
        assert 0.1 < ref["contractible"].mean() < 1.0 and (ref["c"] < 1.0).any()


@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_eval_clustered(ccsp, tiny, seed):
    """Clusters of nearly merged vertices: weights of 1/2 and 0 and the 1-hop rule at work."""
    mesh, om = tiny
    p = ob.Params(0.03)
    xy = _clustered(mesh, om, p, seed)
    ref, _ = _check_eval(ccsp, om, xy, p, f"clustered {seed}")
    assert (ref["w"] == 0.0).any() and ((ref["w"] > 0.4) & (ref["w"] < 0.6)).any()
    assert (~one_hop(om, xy, p)).any()


def one_hop(om, xy, p):
    return ob.one_hop_contractible(om, xy, p.eps)


def _gpu_delta(ccsp, om, xy, p, v, q):
    with ccsp.MovableMesh(om.tri_v, om.kind, om.line, om.prim_v) as gm:
        d, st = gm.delta(torch.from_numpy(xy).to(DEV), _params(ccsp, p),
                         torch.from_numpy(np.ascontiguousarray(v, dtype=np.int32)).to(DEV),
                         torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64)).to(DEV))
        torch.cuda.synchronize()
        return d.cpu().numpy(), st.cpu().numpy()


def _check_deltas(om, xy, p, v, q, d, st, what, idx=None):
    base = ob.terms(om, xy, p)
    for i in (range(v.shape[0]) if idx is None else idx):
        rs, rd, bound = ob.delta_f(om, xy, p, v[i], q[i], base=base)
        assert st[i] == rs, f"{what}: move {i} (vertex {v[i]}) status {st[i]} vs {rs}"
        if rs != ob.MOVED:
            assert d[i] == math.inf
            continue
        assert abs(d[i] - rd) <= 1e-12 * bound, f"{what}: move {i}: {d[i]} vs {rd} (bound {bound})"


@pytest.mark.parametrize("state", ["subdivided", "clustered"])
@pytest.mark.parametrize("polish", [False, True])
def test_tiny_delta(ccsp, tiny, state, polish):
    mesh, om = tiny
    p = ob.Params(0.03, polish=polish)
    xy = mesh.xy if state == "subdivided" else _clustered(mesh, om, ob.Params(0.03), 5)
    v1, q1 = sg.vertex_moves(mesh, 300, 11, 0.05)
    v2, q2 = sg.vertex_moves(mesh, 150, 12, 0.6)
    free = int(np.nonzero(mesh.kind == sg.FREE)[0][0])
    fixed = int(np.nonzero(mesh.kind == sg.ORIGINAL)[0][0])
    special_v = np.array([free, free, fixed, mesh.n_vertices, -1, free], dtype=np.int32)
    special_q = np.array([xy[free], [np.nan, 0.0], xy[fixed] + 1e-3, [0.0, 0.0], [0.0, 0.0],
                          [np.inf, 0.0]])
    v = np.concatenate([v1, v2, special_v])
    q = np.concatenate([q1, q2, special_q])
    d, st = _gpu_delta(ccsp, om, xy, p, v, q)
    _check_deltas(om, xy, p, v, q, d, st, f"{state} polish={polish}")
    n = v1.shape[0] + v2.shape[0]
    assert d[n] == 0.0 and st[n] == 1  # null move
    assert list(st[n + 1:]) == [-2, -1, -2, -2, -2]
    assert (st[:n] == 1).sum() > 100 and (st[:n] == 0).sum() > 10


@pytest.mark.parametrize("state", ["subdivided", "clustered"])
def test_joint_moves_equal_checker(ccsp, tiny, state):
    """The second variant of Sec. 3.2.2 (anneal_joint): a random 5% of the movable vertices moved
    together, one decision. Status equal to the checker's joint_move, the change of f within the
    reordering bound of its sums, positions after each step bit for bit; a chain of steps at two
    temperatures and step scales (some accepted, some rejected, some folded), then invalid
    inputs (a repeated, an original and an out-of-range id) that leave the positions alone."""
    mesh, om = tiny
    p = ob.Params(0.03)
    xy = mesh.xy.copy() if state == "subdivided" else _clustered(mesh, om, p, 8)
    rng = np.random.default_rng(61)
    movable = np.nonzero(mesh.kind != sg.ORIGINAL)[0]
    k = max(2, movable.shape[0] // 20)
    seen = set()
    with ccsp.MovableMesh(om.tri_v, om.kind, om.line, om.prim_v) as gm:
        prm = _params(ccsp, p)
        X = torch.from_numpy(xy.copy()).to(DEV)
        for step in range(24):
            lam, temp = ((0.05, 1e-3), (0.3, 1e-4), (0.01, 0.0))[step % 3]
            vids = rng.choice(movable, k, replace=False).astype(np.int32)
            xi = rng.standard_normal((k, 2))
            uu = float(rng.random())
            d, st = gm.joint(X, prm, temp, lam, torch.from_numpy(vids).to(DEV),
                             torch.from_numpy(xi).to(DEV), uu)
            rs, rd, bound, xy_new, margin = ob.joint_move(om, xy, p, temp, lam, vids, xi, uu)
            assert margin > 1e-10, "a decision lies within rounding of its threshold"
            assert st == rs, (step, st, rs)
            if rs in (ob.ACCEPTED, ob.REJECTED):
                assert abs(d - rd) <= bound, (step, d, rd, bound)
            else:
                assert d == math.inf
            xy = xy_new
            assert np.array_equal(X.cpu().numpy(), xy), step
            seen.add(rs)
        assert seen >= {ob.ACCEPTED, ob.REJECTED, ob.FOLDED}, seen
        orig = int(np.nonzero(mesh.kind == sg.ORIGINAL)[0][0])
        good = movable[:3].astype(np.int32)
        for bad in ([good[0], good[1], good[0]], [good[0], orig, good[1]],
                    [good[0], good[1], mesh.n_vertices]):
            d, st = gm.joint(X, prm, 1e-3, 0.05, torch.tensor(bad, dtype=torch.int32, device=DEV),
                             torch.full((3, 2), 0.1, dtype=torch.float64, device=DEV), 0.5)
            assert st == -2 and d == math.inf
        assert np.array_equal(X.cpu().numpy(), xy)


@pytest.mark.parametrize("eps", [0.03, 0.08])
def test_joint_group_moves_equal_checker(ccsp, tiny, eps):
    """The second variant of Sec. 3.2.3 (anneal_joint_groups): a few random centres' groups moved
    together, one decision, overlapping groups taking the first group's displacement. Status equal
    to the checker's joint_groups, the change of f within the reordering bound, positions after
    each step bit for bit, over a chain of steps; then a centre that is ORIGINAL (BAD, nothing
    moves)."""
    mesh, om = tiny
    p = ob.Params(eps)
    xy = mesh.xy.copy()
    rng = np.random.default_rng(71)
    movable = np.nonzero(mesh.kind != sg.ORIGINAL)[0]
    seen = set()
    with ccsp.MovableMesh(om.tri_v, om.kind, om.line, om.prim_v) as gm:
        prm = _params(ccsp, p)
        X = torch.from_numpy(xy.copy()).to(DEV)
        for step in range(20):
            lam, temp = ((0.005, 1e-3), (0.02, 1e-4), (0.002, 0.0), (0.005, 1e9))[step % 4]
            n = int(rng.integers(1, 6))
            cs = rng.choice(movable, n).astype(np.int32)  # repeats allowed
            draws = np.zeros((n, 4))
            draws[:, :2] = rng.standard_normal((n, 2))
            draws[:, 2] = rng.random(n)
            uu = float(rng.random()) if temp < 1e9 else 0.0
            d, st = gm.joint_groups(X, prm, temp, lam, torch.from_numpy(cs).to(DEV),
                                    torch.from_numpy(draws).to(DEV), uu)
            rs, rd, bound, xy_new, margin = ob.joint_groups(om, xy, p, temp, lam, cs,
                                                            draws[:, :2], draws[:, 2], uu)
            assert margin > 1e-10, "a decision lies within rounding of its threshold"
            assert st == rs, (step, st, rs)
            if rs in (ob.ACCEPTED, ob.REJECTED):
                assert abs(d - rd) <= bound, (step, d, rd, bound)
            else:
                assert d == math.inf
            xy = xy_new
            assert np.array_equal(X.cpu().numpy(), xy), step
            seen.add(rs)
        assert seen >= {ob.ACCEPTED, ob.REJECTED, ob.FOLDED}, seen
        orig = int(np.nonzero(mesh.kind == sg.ORIGINAL)[0][0])
        cs = torch.tensor([int(movable[0]), orig], dtype=torch.int32, device=DEV)
        d, st = gm.joint_groups(X, prm, 1e-3, 0.05, cs,
                                torch.full((2, 4), 0.1, dtype=torch.float64, device=DEV), 0.5)
        assert st == -2 and d == math.inf
        assert np.array_equal(X.cpu().numpy(), xy)


def test_rules_follow_original_positions(ccsp, tiny):
    """The conditioning restriction reads ORIGINAL positions only, so the library keeps its result
    from call to call and recomputes it when an ORIGINAL position changes. One mesh evaluated at
    positions whose ORIGINAL vertices change (a squash that makes triangles near-collinear), then
    at positions where only movable vertices change, then back, equals the checker each time."""
    mesh, om = tiny
    p = ob.Params(0.03)
    xy1 = mesh.xy
    xy2 = mesh.xy.copy()
    xy2[:, 1] *= 0.02
    xy3 = xy2.copy()
    movable = mesh.kind != sg.ORIGINAL
    xy3[movable] = _clustered(mesh, om, p, 9)[movable]
    xy3[:, 1][movable] *= 0.02
    assert (ob.conditioning_contractible(om, xy1) != ob.conditioning_contractible(om, xy2)).sum() > 10
    with ccsp.MovableMesh(om.tri_v, om.kind, om.line, om.prim_v) as gm:
        for k, xy in enumerate((xy1, xy2, xy3, xy1, xy3)):
            ref = ob.objective(om, xy, p)
            out, con, w = gm.eval(torch.from_numpy(xy).to(DEV), _params(ccsp, p), per_edge=True)
            torch.cuda.synchronize()
            assert np.array_equal(con.cpu().numpy().astype(bool), ref["contractible"]), k
            assert np.array_equal(w.cpu().numpy(), ref["w"]), k


def test_large_batches_equal_small_ones(ccsp, tiny):
    """Batches of 4096 moves or more are evaluated in the order of their vertices (a sort inside
    the call); every result equals the same move's result from batches below that size, and a
    sample equals the checker. Bad ids sit among the sorted moves; a larger batch then a smaller
    one run on the same mesh (the sort's scratch grows, then is reused)."""
    mesh, om = tiny
    p = ob.Params(0.03)
    xy = _clustered(mesh, om, p, 5)
    rng = np.random.default_rng(44)
    parts = [sg.vertex_moves(mesh, 3000, 40 + j, (0.05, 0.3, 0.6)[j % 3]) for j in range(6)]
    v = np.concatenate([a for a, _ in parts]).astype(np.int32)
    q = np.concatenate([b for _, b in parts]).astype(np.float64)
    bad = rng.choice(v.shape[0], 40, replace=False)
    v[bad[:20]] = -1 - rng.integers(0, 5, 20)
    v[bad[20:]] = mesh.n_vertices + rng.integers(0, 5, 20)
    X = torch.from_numpy(xy).to(DEV)
    with ccsp.MovableMesh(om.tri_v, om.kind, om.line, om.prim_v) as gm:
        prm = _params(ccsp, p)

        def run(vv, qq):
            d, st = gm.delta(X, prm, torch.from_numpy(np.ascontiguousarray(vv)).to(DEV),
                             torch.from_numpy(np.ascontiguousarray(qq)).to(DEV))
            torch.cuda.synchronize()
            return d.cpu().numpy(), st.cpu().numpy()

        small = [run(v[i:i + 1000], q[i:i + 1000]) for i in range(0, v.shape[0], 1000)]
        ds = np.concatenate([a for a, _ in small])
        ss = np.concatenate([b for _, b in small])
        for n in (v.shape[0], 4096, 9001):
            d, st = run(v[:n], q[:n])
            assert np.array_equal(st, ss[:n]), n
            assert np.array_equal(d.view(np.int64), ds[:n].view(np.int64)), n
    assert (ss[bad] == -2).all()
    assert (ss == 1).sum() > 5000 and (ss == 0).sum() > 500
    ok = np.nonzero(ss == 1)[0]
    idx = np.concatenate([ok[:: ok.size // 6][:6], np.nonzero(ss == 0)[0][:2]])
    _check_deltas(om, xy, p, v, q, ds, ss, "large batch", idx=idx)


def test_move_back_is_exact_negative(ccsp, tiny):
    """Applying a move and proposing the way back gives exactly the opposite change, and the
    change agrees with two full evaluations."""
    mesh, om = tiny
    p = ob.Params(0.03)
    xy = _clustered(mesh, om, p, 7)
    v, q = sg.vertex_moves(mesh, 400, 21, 0.05)
    params = None
    with ccsp.MovableMesh(om.tri_v, om.kind, om.line, om.prim_v) as gm:
        params = _params(ccsp, p)
        X = torch.from_numpy(xy).to(DEV)
        d, st = gm.delta(X, params, torch.from_numpy(v).to(DEV), torch.from_numpy(q).to(DEV))
        d, st = d.cpu().numpy(), st.cpu().numpy()
        done = 0
        for i in np.nonzero(st == 1)[0][:40]:
            f0 = gm.eval(X, params).cpu().numpy()[0]
            old = X[v[i]].clone()
            X[v[i]] = torch.from_numpy(q[i]).to(DEV)
            f1 = gm.eval(X, params).cpu().numpy()[0]
            back, sb = gm.delta(X, params, torch.tensor([v[i]], dtype=torch.int32, device=DEV),
                                old.reshape(1, 2).contiguous())
            fwd, sf = gm.delta(X, params, torch.tensor([v[i]], dtype=torch.int32, device=DEV),
                               torch.from_numpy(q[i:i + 1]).to(DEV))
            assert sb.item() == 1 and sf.item() == 1 and fwd.item() == 0.0
            X[v[i]] = old
            dd = gm.delta(X, params, torch.tensor([v[i]], dtype=torch.int32, device=DEV),
                          torch.from_numpy(q[i:i + 1]).to(DEV))[0].item()
            assert dd == d[i]
            assert back.item() == -d[i]
            assert abs((f1 - f0) - d[i]) <= 1e-10 * abs(f0)
            done += 1
        assert done == 40


@pytest.fixture(scope="module")
def grid():
    mesh = helpers.subdivided(sg.make_scene("grid"))
    return mesh, ob.Mesh(mesh.tri_v, mesh.kind, mesh.line, mesh.prim_v)


def test_grid_eval_and_sampled_deltas(ccsp, grid):
    """The subdivided grid scene (2,088,968 triangles): evaluation in full, and 2^16 moves with a
    sample against the checker."""
    mesh, om = grid
    p = ob.Params(0.2)
    ref, _ = _check_eval(ccsp, om, mesh.xy, p, "grid")
    assert 0.3 < ref["contractible"].mean() < 1.0
    v, q = sg.vertex_moves(mesh, 1 << 16, 31, 0.1)
    d, st = _gpu_delta(ccsp, om, mesh.xy, p, v, q)
    ok = np.nonzero(st == 1)[0]
    folded = np.nonzero(st == 0)[0]
    assert ok.size > 1000 and folded.size > 100
    idx = np.concatenate([ok[:: max(1, ok.size // 5)][:5], folded[:2]])
    _check_deltas(om, mesh.xy, p, v, q, d, st, "grid", idx=idx)
    for i in np.concatenate([ok[:60], folded[:60]]):
        assert st[i] == ob.move_status(om, mesh.xy, int(v[i]), q[i])


HUB_DEGREE = 32  # the library's hubs: ORIGINAL vertices of more neighbours than this


def _is_hub(om, a):
    return om.kind[a] == ob.ORIGINAL and om.nbr_off[a + 1] - om.nbr_off[a] > HUB_DEGREE


def _ball(om, v, r):
    """Vertices within r edges of v along paths that do not pass through hubs (a hub is in the
    ball, but not gone through): the separation the library's classes and group claims keep."""
    seen, front = {v}, [v]
    for _ in range(r):
        nxt = []
        for a in front:
            if _is_hub(om, a):
                continue
            for w in om.nbr[om.nbr_off[a]:om.nbr_off[a + 1]].tolist():
                if w not in seen:
                    seen.add(w)
                    nxt.append(w)
        front = nxt
    return seen


def test_classes_partition_and_separation(ccsp, tiny):
    """Every movable vertex is in exactly one class; members of a class are more than four edges
    apart."""
    mesh, om = tiny
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        cls = gm.classes()
    assert np.array_equal(np.sort(np.concatenate(cls)), np.nonzero(mesh.kind != sg.ORIGINAL)[0])
    for c in cls:
        s = set(c.tolist())
        for v in c.tolist():
            assert not (_ball(om, v, 4) & s) - {v}, f"class members within four edges of {v}"


def _sweep(ccsp, gm, params, xy0, cls, disp, u, temperature):
    X = torch.from_numpy(xy0.copy()).to(DEV)
    sts, dfs, off = [], [], 0
    for c in cls:
        k = c.shape[0]
        d, st = gm.anneal(X, params, temperature, torch.from_numpy(c).to(DEV),
                          torch.from_numpy(disp[off:off + k]).to(DEV),
                          torch.from_numpy(u[off:off + k]).to(DEV))
        sts.append(st.cpu().numpy())
        dfs.append(d.cpu().numpy())
        off += k
    torch.cuda.synchronize()
    return X.cpu().numpy(), np.concatenate(sts), np.concatenate(dfs)


@pytest.mark.parametrize("state,temperature", [("subdivided", 1e-3), ("clustered", 1e-4),
                                               ("subdivided", 0.0), ("clustered", 1e-2)])
def test_anneal_sweep_equals_sequential_chain(ccsp, tiny, state, temperature):
    """One sweep over all classes equals the checker's Metropolis chain over the same moves in the
    same order: positions bit for bit, statuses equal, changes of f within rounding."""
    mesh, om = tiny
    p = ob.Params(0.03)
    xy0 = mesh.xy.copy() if state == "subdivided" else _clustered(mesh, om, p, 9)
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        cls = gm.classes()
        order = np.concatenate(cls)
        disp = sg.vertex_displacements(mesh, order, 3, 0.05)
        u = np.random.default_rng(5).random(order.shape[0])
        xy_gpu, st_gpu, df_gpu = _sweep(ccsp, gm, _params(ccsp, p), xy0, cls, disp, u, temperature)
        X = torch.from_numpy(xy0.copy()).to(DEV)
        d_s, st_s = gm.sweep(X, _params(ccsp, p), temperature, torch.from_numpy(disp).to(DEV),
                             torch.from_numpy(u).to(DEV))
        xy_s, st_s, d_s = X.cpu().numpy(), st_s.cpu().numpy(), d_s.cpu().numpy()
    # the whole sweep in one call equals the class-by-class calls
    assert np.array_equal(xy_s, xy_gpu) and np.array_equal(st_s, st_gpu)
    assert np.array_equal(d_s, df_gpu)
    xy_ref, st_ref, df_ref, margin = ob.metropolis_chain(om, xy0, p, temperature, order, disp, u)
    valid = (st_ref == ob.ACCEPTED) | (st_ref == ob.REJECTED)
    assert (margin[valid] > 1e-10).all(), "a decision lies within rounding of its threshold"
    assert np.array_equal(st_gpu, st_ref), np.nonzero(st_gpu != st_ref)[0][:5]
    assert np.array_equal(xy_gpu, xy_ref)
    fin = np.isfinite(df_ref)
    assert np.array_equal(np.isfinite(df_gpu), fin)
    assert np.allclose(df_gpu[fin], df_ref[fin], rtol=1e-9, atol=1e-13)
    assert (st_ref == ob.ACCEPTED).sum() > 20
    if temperature > 0:
        assert (st_ref == ob.REJECTED).sum() > 0


def test_anneal_class_at_scale(ccsp, grid):
    """Subdivided grid scene: a class applied in one call or in two halves gives the same
    positions; the accepted changes add up to the change of f; a sample agrees with the checker;
    sampled members are more than four edges apart."""
    mesh, om = grid
    p = ob.Params(0.2)
    temperature = 1e-3
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        cls = gm.classes()
        assert len(cls) > 20
        c = max(cls, key=len)
        disp = sg.vertex_displacements(mesh, c, 7, 0.05)
        u = np.random.default_rng(8).random(c.shape[0])
        params = _params(ccsp, p)
        X0 = torch.from_numpy(mesh.xy).to(DEV)
        X1 = X0.clone()
        d1, s1 = gm.anneal(X1, params, temperature, torch.from_numpy(c).to(DEV),
                           torch.from_numpy(disp).to(DEV), torch.from_numpy(u).to(DEV))
        X2 = X0.clone()
        h = c.shape[0] // 2
        for lo, hi in ((0, h), (h, c.shape[0])):
            gm.anneal(X2, params, temperature, torch.from_numpy(c[lo:hi]).to(DEV),
                      torch.from_numpy(disp[lo:hi]).to(DEV), torch.from_numpy(u[lo:hi]).to(DEV))
        assert torch.equal(X1, X2)
        f0 = gm.eval(X0, params).cpu().numpy()[0]
        f1 = gm.eval(X1, params).cpu().numpy()[0]
        d1, s1 = d1.cpu().numpy(), s1.cpu().numpy()
    acc = s1 == 1
    assert acc.sum() > 1000 and (s1 == 2).sum() > 0
    assert abs((f1 - f0) - d1[acc].sum()) <= 1e-9 * abs(f0)
    base = ob.terms(om, mesh.xy, p)
    for i in np.nonzero(acc)[0][:3]:
        q = mesh.xy[c[i]] + ob.project(om, mesh.xy, int(c[i]), disp[i])
        rs, rd, bound = ob.delta_f(om, mesh.xy, p, int(c[i]), q, base=base)
        assert rs == ob.MOVED and abs(rd - d1[i]) <= 1e-12 * bound
    s = set(c.tolist())
    for v in c[:: max(1, c.shape[0] // 40)].tolist():
        assert not (_ball(om, v, 4) & s) - {v}


def test_sweep_at_scale_equals_class_calls(ccsp, grid):
    """Subdivided grid scene: two sweeps in single calls (scratch refreshed in the kernel after each
    accepted move) equal the same moves made class by class with a full recomputation per call."""
    mesh, om = grid
    p = ob.Params(0.2)
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        cls = gm.classes()
        order = np.concatenate(cls)
        params = _params(ccsp, p)
        XA = torch.from_numpy(mesh.xy).to(DEV)
        XB = XA.clone()
        for sweep, temperature in ((0, 1e-2), (1, 1e-3)):
            disp = sg.vertex_displacements(mesh, order, 40 + sweep, 0.05)
            u = np.random.default_rng(50 + sweep).random(order.shape[0])
            dA, sA = gm.sweep(XA, params, temperature, torch.from_numpy(disp).to(DEV),
                              torch.from_numpy(u).to(DEV))
            off = 0
            sB = []
            for c in cls:
                k = c.shape[0]
                _, s = gm.anneal(XB, params, temperature, torch.from_numpy(c).to(DEV),
                                 torch.from_numpy(disp[off:off + k]).to(DEV),
                                 torch.from_numpy(u[off:off + k]).to(DEV))
                sB.append(s)
                off += k
            assert torch.equal(XA, XB), f"sweep {sweep}: positions differ"
            assert torch.equal(sA, torch.cat(sB))
            assert (sA == 1).sum().item() > 10000


def _unit_draws(rng, s, m):
    """Heavy-tailed unit draws of Sec. 3.2.2: a point uniform in the unit disk, its radius scaled by
    a Pareto(1/2) factor (x >= 1)."""
    r = np.sqrt(rng.random((s, m)))
    th = 2 * np.pi * rng.random((s, m))
    f = (1.0 - rng.random((s, m))) ** -2.0
    return np.ascontiguousarray(np.stack([r * f * np.cos(th), r * f * np.sin(th)], -1))


def test_schedule_equals_sequential_annealing(ccsp, tiny):
    """Four sweeps with falling temperature and contraction length and the adaptive step scale
    equal the checker's sequential annealing: positions bit for bit, step scales and accepted
    counts exactly."""
    mesh, om = tiny
    p = ob.Params(0.05)
    temps = [1e-2, 3e-3, 1e-3, 3e-4]
    epss = [0.05, 0.03, 0.02, 0.01]
    rng = np.random.default_rng(17)
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        order = np.concatenate(gm.classes())
        xi = _unit_draws(rng, 4, order.shape[0])
        u = np.ascontiguousarray(rng.random((4, order.shape[0])))
        X = torch.from_numpy(mesh.xy.copy()).to(DEV)
        lam, acc = gm.schedule(X, _params(ccsp, p), temps, epss, 0.05,
                               torch.from_numpy(xi).to(DEV), torch.from_numpy(u).to(DEV))
        xy_gpu = X.cpu().numpy()
    xy_ref, lam_ref, acc_ref, margin = ob.annealing_schedule(om, mesh.xy, p, temps, epss, 0.05,
                                                              0.23, order, xi, u)
    assert margin > 1e-10, "a decision lies within rounding of its threshold"
    assert np.array_equal(acc, acc_ref), (acc, acc_ref)
    assert np.array_equal(lam, lam_ref), (lam, lam_ref)
    assert np.array_equal(xy_gpu, xy_ref)
    assert (acc > 0).all() and len(set(lam.tolist())) > 1


def test_schedule_at_scale(ccsp, grid):
    """Subdivided grid scene: the step scale follows its rule from the accepted counts, and a cold
    schedule lowers f."""
    mesh, om = grid
    p = ob.Params(0.2)
    rng = np.random.default_rng(23)
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        m = gm.n_movable()
        params = _params(ccsp, p)
        X = torch.from_numpy(mesh.xy).to(DEV)
        f0 = gm.eval(X, params).cpu().numpy()[0]
        s = 3
        xi = torch.from_numpy(_unit_draws(rng, s, m)).to(DEV)
        u = torch.from_numpy(rng.random((s, m))).to(DEV)
        lam, acc = gm.schedule(X, params, [1e-6] * s, [0.2] * s, 0.02, xi, u)
        f1 = gm.eval(X, params).cpu().numpy()[0]
    assert f1 < f0
    for k in range(s - 1):
        a = acc[k] / m
        assert lam[k + 1] == lam[k] * min(2.0, max(0.5, 1.0 + (a - 0.23)))


def _submesh(mesh, seeds, rings):
    """The checker's mesh of the triangles touching a vertex within `rings` edges of the seed
    vertices, in their original order, vertices relabelled (original-edge ends outside it become
    -1): enough to evaluate per-edge values of edges between seeds, which read two rings."""
    tv = mesh.tri_v
    near = np.zeros(mesh.n_vertices, dtype=bool)
    near[seeds] = True
    for _ in range(rings):
        hit = near[tv].any(axis=1)
        near[tv[hit].ravel()] = True
    keep = np.nonzero(near[tv].any(axis=1))[0]
    sub = tv[keep]
    verts = np.unique(sub)
    new = -np.ones(mesh.n_vertices, dtype=np.int64)
    new[verts] = np.arange(verts.shape[0])
    pv = np.where(mesh.prim_v >= 0, new[mesh.prim_v], -1)
    return ob.Mesh(new[sub], mesh.kind[verts], mesh.line[verts], pv), new, verts


def test_large_bench_configuration_sampled(ccsp):
    """The objective's bench configuration: the large scene subdivided once (16,000,008 triangles)
    with the bench's parameters. Sampled edges' contractibility and weights equal the checker's,
    computed on the triangles around them, bit for bit; f and its parts equal the sums of terms
    built from the per-edge weights within the reordering bound."""
    sc = sg.make_scene("large")
    mesh = helpers.subdivided(sc)
    size = sc.box[1] - sc.box[0]
    p = ob.Params(1e-3 * size, eps0=1e-10 * size, mu_angle=1.0 * size, mu_len=10.0 * size)
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        ev = gm.edges().astype(np.int64)
        out, con, w = gm.eval(torch.from_numpy(mesh.xy).to(DEV), _params(ccsp, p), per_edge=True)
        torch.cuda.synchronize()
        out, con, w = out.cpu().numpy(), con.cpu().numpy().astype(bool), w.cpu().numpy()
    assert ev.shape[0] == 24_000_016
    rng = np.random.default_rng(12)
    active = np.nonzero(w < 1.0)[0]
    assert active.size > 1000 and (~con).any()
    sample = np.concatenate([rng.choice(ev.shape[0], 1500, replace=False),
                             rng.choice(active, 500, replace=False),
                             np.nonzero(~con)[0][:100]])
    om, new, verts = _submesh(mesh, np.unique(ev[sample]), 2)
    key = new[ev[sample, 0]] * om.nv + new[ev[sample, 1]]
    local = np.searchsorted(om.edge_key, key)
    assert np.array_equal(om.edge_key[local], key), "sampled edges are edges of the mesh"
    k, _, wr = ob.edge_values(om, mesh.xy[verts], p, local)
    assert np.array_equal(con[sample], k)
    assert np.array_equal(w[sample], wr)
    ln = ob.lengths(mesh.xy, ev[:, 0], ev[:, 1])
    edge = w * ln
    tri = type("Triangles", (), {"tri_v": mesh.tri_v.astype(np.int64)})()
    ang = ob.angle_terms(tri, mesh.xy, p)
    short = np.maximum(0.0, p.eps0 - ln) / p.eps0
    for got, terms in ((out[1], edge), (out[2], ang), (out[3], short)):
        assert abs(got - terms.sum()) <= 2 * terms.size * U * np.abs(terms).sum()
    f = edge.sum() + p.mu_angle * ang.sum() + p.mu_len * short.sum()
    scale = np.abs(edge).sum() + p.mu_angle * np.abs(ang).sum() + p.mu_len * np.abs(short).sum()
    assert abs(out[0] - f) <= 2 * (edge.size + ang.size) * U * scale


_KINDS = {"resample": ob.RESAMPLE, "swap": ob.SWAP, "contract": ob.CONTRACT}


def _proposal_draws(rng, m, kind):
    """Four draws per vertex: uniforms, with (r2, r3) a unit-disk point for swaps."""
    r = rng.random((m, 4))
    if kind == "swap":
        rad = np.sqrt(rng.random(m))
        th = 2 * math.pi * rng.random(m)
        r[:, 2], r[:, 3] = rad * np.cos(th), rad * np.sin(th)
    return r


@pytest.mark.parametrize("kind", ["resample", "swap", "contract"])
@pytest.mark.parametrize("state,temperature", [("subdivided", 1e-3), ("clustered", 1e-4),
                                               ("clustered", 0.0)])
def test_propose_sweep_equals_sequential_chain(ccsp, tiny, kind, state, temperature):
    """A sweep of resampling, swap or contraction proposals (Secs. 3.2.4-3.2.6) equals the
    checker's chain over the same draws in the same order: positions bit for bit, statuses
    (skipped ones included) equal, changes of f within rounding."""
    mesh, om = tiny
    p = ob.Params(0.03)
    xy0 = mesh.xy.copy() if state == "subdivided" else _clustered(mesh, om, p, 9)
    rng = np.random.default_rng(11)
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        order = np.concatenate(gm.classes())
        draws = _proposal_draws(rng, order.shape[0], kind)
        u = rng.random(order.shape[0])
        X = torch.from_numpy(xy0.copy()).to(DEV)
        d, st = gm.propose(X, _params(ccsp, p), temperature, kind, torch.from_numpy(draws).to(DEV),
                           torch.from_numpy(u).to(DEV))
        xy_g, st_g, df_g = X.cpu().numpy(), st.cpu().numpy(), d.cpu().numpy()
    xy_r, st_r, df_r, margin = ob.proposal_chain(om, xy0, p, temperature, _KINDS[kind], order,
                                                 draws, u)
    valid = (st_r == ob.ACCEPTED) | (st_r == ob.REJECTED)
    assert (margin[valid] > 1e-10).all(), "a decision lies within rounding of its threshold"
    assert np.array_equal(st_g, st_r), np.nonzero(st_g != st_r)[0][:5]
    assert np.array_equal(xy_g, xy_r)
    fin = np.isfinite(df_r)
    assert np.array_equal(np.isfinite(df_g), fin)
    assert np.allclose(df_g[fin], df_r[fin], rtol=1e-9, atol=1e-13)
    assert (st_r == ob.ACCEPTED).sum() > 0
    if kind != "resample":
        assert (st_r == ob.SKIPPED).sum() > 0


def test_propose_rejects_bad_kind(ccsp, tiny):
    mesh, _ = tiny
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        m = gm.n_movable()
        X = torch.from_numpy(mesh.xy.copy()).to(DEV)
        r = torch.zeros((m, 4), dtype=torch.float64, device=DEV)
        u = torch.zeros(m, dtype=torch.float64, device=DEV)
        with pytest.raises(ValueError):
            gm.propose(X, _params(ccsp, ob.Params(0.03)), 0.0, "jump", r, u)
        from paper_2112_05570_amd import binding as B
        with pytest.raises(B.CcspError, match="unknown proposal kind"):
            B.anneal_propose(gm.handle, X.data_ptr(), _params(ccsp, ob.Params(0.03)), 0.0, 7,
                             r.data_ptr(), u.data_ptr(), u.data_ptr(), u.data_ptr())


@pytest.mark.parametrize("kind", ["resample", "swap", "contract"])
def test_propose_at_scale(ccsp, grid, kind):
    """Subdivided grid scene, one sweep at T = 0: accepted changes are <= 0 and add up to the
    change of f; only accepted vertices move; vertices of the first class (tried against the
    initial positions) match the checker's proposal, status and new position exactly."""
    mesh, om = grid
    p = ob.Params(0.2)
    rng = np.random.default_rng(12)
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        cls = gm.classes()
        order = np.concatenate(cls)
        draws = _proposal_draws(rng, order.shape[0], kind)
        u = rng.random(order.shape[0])
        params = _params(ccsp, p)
        X0 = torch.from_numpy(mesh.xy).to(DEV)
        X = X0.clone()
        d, st = gm.propose(X, params, 0.0, kind, torch.from_numpy(draws).to(DEV),
                           torch.from_numpy(u).to(DEV))
        f0 = gm.eval(X0, params).cpu().numpy()[0]
        f1 = gm.eval(X, params).cpu().numpy()[0]
        xy1, d, st = X.cpu().numpy(), d.cpu().numpy(), st.cpu().numpy()
    acc = st == ob.ACCEPTED
    assert acc.sum() > 100 and (d[acc] <= 0).all()
    assert set(np.unique(st).tolist()) <= {ob.ACCEPTED, ob.REJECTED, ob.SKIPPED, ob.FOLDED}
    assert abs((f1 - f0) - d[acc].sum()) <= 1e-9 * abs(f0)
    moved = np.nonzero((xy1 != mesh.xy).any(axis=1))[0]
    assert np.array_equal(np.sort(moved), np.sort(order[acc]))
    first = cls[0].shape[0]
    for i in range(0, first, max(1, first // 25)):
        v = int(order[i])
        q = ob.propose(om, mesh.xy, p, v, _KINDS[kind], draws[i])
        if q is None:
            assert st[i] == ob.SKIPPED
            continue
        assert st[i] in (ob.ACCEPTED, ob.REJECTED, ob.FOLDED)
        assert (st[i] == ob.FOLDED) == (ob.move_status(om, mesh.xy, v, q) == ob.FOLDED)
        if st[i] == ob.ACCEPTED:
            assert np.array_equal(xy1[v], q)
        else:
            assert np.array_equal(xy1[v], mesh.xy[v])


def _group_sweep_vs_chain(ccsp, gm, om, xy0, p, temperature, lam, draws, u, centres=None):
    """A GPU group sweep against the checker's chain over the centres in the order the GPU made
    the moves, (round, index): positions bit for bit, statuses and group sizes equal, changes of
    f within rounding (the GPU adds the members' changes one by one, the checker differences f as
    a whole). Returns (statuses, sizes, rounds) per centre."""
    X = torch.from_numpy(xy0.copy()).to(DEV)
    d, st, mem, rnd = gm.group_sweep(X, _params(ccsp, p), temperature, lam,
                                     torch.from_numpy(draws).to(DEV), torch.from_numpy(u).to(DEV),
                                     centres=centres)
    xy_g, st_g, df_g, mem_g, rnd_g = (X.cpu().numpy(), st.cpu().numpy(), d.cpu().numpy(),
                                      mem.cpu().numpy(), rnd.cpu().numpy())
    cen = gm.movable if centres is None else np.asarray(centres)
    order = np.lexsort((np.arange(cen.shape[0]), rnd_g))
    assert (rnd_g >= 0).all()
    xy_r, st_r, df_r, margin, size = ob.group_chain(om, xy0, p, temperature, lam, cen[order],
                                                    draws[order, :2], draws[order, 2], u[order])
    st_g, df_g, mem_g = st_g[order], df_g[order], mem_g[order]
    valid = (st_r == ob.ACCEPTED) | (st_r == ob.REJECTED)
    # a decision within rounding of its threshold is only comparable when both sides computed the
    # same change exactly (a cluster whose edges all weigh 0 moves with a change of exactly 0)
    close = valid & (margin <= 1e-10)
    assert (df_g[close] == df_r[close]).all(), "a decision lies within rounding of its threshold"
    assert np.array_equal(mem_g, size)
    assert np.array_equal(st_g, st_r), np.nonzero(st_g != st_r)[0][:5]
    assert np.array_equal(xy_g, xy_r)
    fin = np.isfinite(df_r)
    assert np.array_equal(np.isfinite(df_g), fin)
    assert np.allclose(df_g[fin], df_r[fin], rtol=1e-9, atol=1e-12)
    return st_r, size, rnd_g


@pytest.mark.parametrize("state,temperature,eps", [("subdivided", 1e-3, 0.03),
                                                   ("clustered", 1e-4, 0.03),
                                                   ("clustered", 0.0, 0.1)])
def test_group_sweep_equals_sequential_chain(ccsp, tiny, state, temperature, eps):
    """A sweep of group moves (Sec. 3.2.3, every movable vertex within d of the centre) equals the
    checker's chain over the same centres and draws, in the order the GPU made the moves."""
    mesh, om = tiny
    p = ob.Params(eps)
    xy0 = mesh.xy.copy() if state == "subdivided" else _clustered(mesh, om, ob.Params(0.03), 9)
    rng = np.random.default_rng(13)
    with ccsp.MovableMesh.from_mesh(mesh) as gm:
        M = gm.movable.shape[0]
        draws = np.zeros((M, 4))
        draws[:, :2] = rng.standard_normal((M, 2))
        draws[:, 2] = rng.random(M)
        u = rng.random(M)
        st_r, size, rnd = _group_sweep_vs_chain(ccsp, gm, om, xy0, p, temperature, 0.05, draws, u)
    assert (st_r == ob.ACCEPTED).sum() > 5 and (size > 1).sum() > 20 and rnd.max() >= 1
    # groups that reach past the centre's neighbours occur (the paper's definition)
    far = 0
    for i, c in enumerate(gm.movable[:400]):
        d = (0.5 + 4.5 * draws[i, 2]) * p.eps
        mem = ob.group_members(om, xy0, int(c), d)
        far += any(not om.has_edge(int(c), w) for w in mem[1:])
    assert far > 0 or state == "subdivided"


def _fan_mesh(n_ring, n_outer):
    """A free centre 0 inside a ring of n_ring free vertices at radius 1, with n_outer free
    vertices at radius 1.5 hanging off the ring and an ORIGINAL frame around everything."""
    ring = [[math.cos(2 * math.pi * k / n_ring), math.sin(2 * math.pi * k / n_ring)]
            for k in range(n_ring)]
    step = n_ring // n_outer
    outer = [[1.5 * math.cos(2 * math.pi * (j * step + 0.5) / n_ring),
              1.5 * math.sin(2 * math.pi * (j * step + 0.5) / n_ring)] for j in range(n_outer)]
    frame = [[4.0 * math.cos(2 * math.pi * k / 8), 4.0 * math.sin(2 * math.pi * k / 8)]
             for k in range(8)]
    xy = np.array([[0.0, 0.0]] + ring + outer + frame)
    return xy


def test_large_and_far_reaching_groups(ccsp):
    """Groups of up to thirty-one members, ten of them two edges from their centre (no edge joins
    them to it), repeated centres and a centre that cannot move: the GPU equals the checker's
    chain. The mesh is the Delaunay triangulation of the points (scipy), counter-clockwise, with
    the octagon frame ORIGINAL and every other vertex free."""
    spatial = pytest.importorskip("scipy.spatial")
    xy = _fan_mesh(20, 10)
    n = xy.shape[0]
    frame = list(range(n - 8, n))
    tri = spatial.Delaunay(xy).simplices.astype(np.int32)
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    cw = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]) < 0
    tri[cw] = tri[cw][:, [0, 2, 1]]
    assert all(oracle.orient(*xy[t]) > 0 for t in tri)
    kind = np.full(n, ob.FREE, dtype=np.int32)
    kind[frame] = ob.ORIGINAL
    line = np.zeros(n, dtype=np.int32)
    prim_v = np.array([[frame[k], frame[(k + 1) % 8]] for k in range(8)], dtype=np.int32)
    om = ob.Mesh(tri, kind, line, prim_v)
    p = ob.Params(0.5)  # d up to 2.5: the whole cluster
    rng = np.random.default_rng(21)
    with ccsp.MovableMesh(tri, kind, line, prim_v) as gm:
        M = gm.movable.shape[0]
        for rep in range(3):
            draws = np.zeros((M, 4))
            draws[:, :2] = 0.02 * rng.standard_normal((M, 2))
            draws[:, 2] = rng.random(M)
            draws[0, 2] = 0.99
            u = rng.random(M)
            st_r, size, rnd = _group_sweep_vs_chain(ccsp, gm, om, xy, p, 1e-3, 0.05, draws, u)
            assert size.max() >= 20 and rnd.max() >= 3
        # repeated centres, in any order, and a vertex that is not movable
        cen = np.array([0, 5, 0, frame[0], 3, 0], dtype=np.int32)
        draws = np.zeros((cen.shape[0], 4))
        draws[:, :2] = 0.02 * rng.standard_normal((cen.shape[0], 2))
        draws[:, 2] = 0.9
        u = rng.random(cen.shape[0])
        X = torch.from_numpy(xy.copy()).to(DEV)
        d, st, mem, rnd = gm.group_sweep(X, _params(ccsp, p), 1e-3, 0.05,
                                         torch.from_numpy(draws).to(DEV),
                                         torch.from_numpy(u).to(DEV), centres=cen)
        st, rnd = st.cpu().numpy(), rnd.cpu().numpy()
        assert st[3] == ccsp.binding.CCSP_MOVE_FIXED and rnd[3] == -1
        keep = np.array([0, 1, 2, 4, 5])
        _group_sweep_vs_chain(ccsp, gm, om, xy, p, 1e-3, 0.05, draws[keep], u[keep],
                              centres=cen[keep])


def _hub_mesh(n_ring=40, rings=3):
    """An ORIGINAL hub at the origin whose fan is a ring of n_ring free vertices, further free
    rings (each offset by half a step) and an ORIGINAL frame: the hub's degree is n_ring, above the
    library's hub threshold. Delaunay (scipy), counter-clockwise."""
    spatial = pytest.importorskip("scipy.spatial")
    pts = [[0.0, 0.0]]
    for r in range(rings):
        rad = 1.0 + 0.6 * r
        pts += [[rad * math.cos(2 * math.pi * (k + 0.5 * r) / n_ring),
                 rad * math.sin(2 * math.pi * (k + 0.5 * r) / n_ring)] for k in range(n_ring)]
    frame = [[4.0 * math.cos(2 * math.pi * k / 12), 4.0 * math.sin(2 * math.pi * k / 12)]
             for k in range(12)]
    xy = np.array(pts + frame)
    n = xy.shape[0]
    tri = spatial.Delaunay(xy).simplices.astype(np.int32)
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    cw = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]) < 0
    tri[cw] = tri[cw][:, [0, 2, 1]]
    kind = np.full(n, ob.FREE, dtype=np.int32)
    kind[0] = ob.ORIGINAL
    fr = list(range(n - 12, n))
    kind[fr] = ob.ORIGINAL
    line = np.zeros(n, dtype=np.int32)
    prim_v = np.array([[fr[k], fr[(k + 1) % 12]] for k in range(12)], dtype=np.int32)
    return xy, tri, kind, line, prim_v


@pytest.mark.parametrize("eps,rep", [(0.04, 0), (0.04, 1), (0.12, 2)])
def test_group_moves_around_a_hub(ccsp, eps, rep):
    """Groups around an ORIGINAL vertex of degree 40: claims do not pass through such a hub, so
    groups on different sides of its fan move in the same round, and the sweep still equals the
    checker's sequential chain (positions bit for bit)."""
    xy, tri, kind, line, prim_v = _hub_mesh()
    assert int((tri == 0).any(axis=1).sum()) == 40  # the hub's fan
    om = ob.Mesh(tri, kind, line, prim_v)
    p = ob.Params(eps)
    rng = np.random.default_rng(31 + rep)
    with ccsp.MovableMesh(tri, kind, line, prim_v) as gm:
        M = gm.movable.shape[0]
        draws = np.zeros((M, 4))
        draws[:, :2] = 0.3 * eps * rng.standard_normal((M, 2))
        draws[:, 2] = rng.random(M)
        u = rng.random(M)
        st_r, size, rnd = _group_sweep_vs_chain(ccsp, gm, om, xy, p, 1e-3, 0.05, draws, u)
        assert (st_r == ob.ACCEPTED).sum() > 10
        # the hub's 40 fan vertices alone as centres: claims through the hub would make every two
        # of them conflict (40 rounds); without, each conflicts with about a dozen fan neighbours
        fan = np.arange(1, 41, dtype=np.int32)
        k = np.searchsorted(gm.movable, fan)
        _, _, rnd_f = _group_sweep_vs_chain(ccsp, gm, om, xy, p, 1e-3, 0.05, draws[k], u[k],
                                            centres=fan)
        assert rnd_f.max() + 1 < 35, rnd_f.max()
        # single-vertex sweeps: classes separate the fan vertices along the ring, not through the
        # hub (through it every two of the 40 would conflict), and a sweep equals the chain
        cls = gm.classes()
        assert len(cls) < 35, len(cls)
        order = np.concatenate(cls)
        for c in cls:
            s_c = set(c.tolist())
            for v in c.tolist():
                assert not (_ball(om, v, 4) & s_c) - {v}
        disp = 0.3 * eps * rng.standard_normal((order.shape[0], 2))
        uu = rng.random(order.shape[0])
        X = torch.from_numpy(xy.copy()).to(DEV)
        d_s, st_s = gm.sweep(X, _params(ccsp, p), 1e-3, torch.from_numpy(disp).to(DEV),
                             torch.from_numpy(uu).to(DEV))
        xy_s, st_s = X.cpu().numpy(), st_s.cpu().numpy()
    xy_ref, st_ref, _, margin = ob.metropolis_chain(om, xy, p, 1e-3, order, disp, uu)
    valid = (st_ref == ob.ACCEPTED) | (st_ref == ob.REJECTED)
    assert (margin[valid] > 1e-10).all(), "a decision lies within rounding of its threshold"
    assert np.array_equal(st_s, st_ref) and np.array_equal(xy_s, xy_ref)
    assert (st_ref == ob.ACCEPTED).sum() > 10


@pytest.mark.parametrize("eps,rep", [(0.04, 0), (0.3, 1)])
def test_group_moves_with_a_free_vertex_of_high_degree(ccsp, eps, rep):
    """The hub mesh with its centre made FREE: a movable vertex of 40 neighbours, more than the
    LDS tables of the wave that applies a group hold, so that member's move is taken on one lane
    while the others' are spread over the wave. Group sweeps (at eps = 0.3 the groups near the
    centre hold it and much of its fan) equal the checker's sequential chain."""
    xy, tri, kind, line, prim_v = _hub_mesh()
    kind = kind.copy()
    kind[0] = ob.FREE
    om = ob.Mesh(tri, kind, line, prim_v)
    p = ob.Params(eps)
    rng = np.random.default_rng(71 + rep)
    with ccsp.MovableMesh(tri, kind, line, prim_v) as gm:
        M = gm.movable.shape[0]
        assert gm.movable[0] == 0
        draws = np.zeros((M, 4))
        draws[:, :2] = 0.3 * eps * rng.standard_normal((M, 2))
        draws[:, 2] = rng.random(M)
        u = rng.random(M)
        st_r, size, rnd = _group_sweep_vs_chain(ccsp, gm, om, xy, p, 1e-3, 0.05, draws, u)
        assert (st_r == ob.ACCEPTED).sum() > 5
        if eps > 0.2:
            assert size.max() > 20


@pytest.mark.parametrize("seed,eps", [(0, 0.3), (1, 1.0), (2, 2.0), (3, 0.3)])
def test_conditioning_and_flat_rules_on_gpu(ccsp, seed, eps):
    """Sec. 2.2.2's conditioning and flat-triangle restrictions: on meshes where both fire (the
    checker finds edges that they alone make incontractible), the GPU's evaluation, changes of f,
    a single-vertex sweep and a group sweep equal the checker's."""
    tri, kind, line, prim_v, xy = helpers.rules_mesh(seed)
    om = ob.Mesh(tri, kind, line, prim_v)
    p = ob.Params(eps)
    base = ob.direct_contractible(om) & ob.one_hop_contractible(om, xy, eps)
    cond = ob.conditioning_contractible(om, xy)
    full = ob.contractible(om, xy, eps)
    assert (base & ~cond).sum() > 5, "the conditioning rule does not fire"
    if eps < 1.5:
        assert (base & cond & ~full).sum() > 5, "the flat-triangle rule does not fire"
    _check_eval(ccsp, om, xy, p, f"rules mesh {seed}")
    rng = np.random.default_rng(40 + seed)
    movable = np.nonzero(kind != ob.ORIGINAL)[0]
    v = rng.choice(movable, 400).astype(np.int32)
    q = xy[v] + rng.normal(0.0, 0.2, (400, 2))
    for i in range(400):  # constrained vertices move along their original edge
        if kind[v[i]] == ob.CONSTRAINED:
            q[i] = xy[v[i]] + ob.project(om, xy, int(v[i]), q[i] - xy[v[i]])
    d, st = _gpu_delta(ccsp, om, xy, p, v, q)
    _check_deltas(om, xy, p, v, q, d, st, f"rules mesh {seed}")
    assert (st == 1).sum() > 100
    with ccsp.MovableMesh(tri, kind, line, prim_v) as gm:
        cls = gm.classes()
        order = np.concatenate(cls)
        disp = rng.normal(0.0, 0.3, (order.shape[0], 2))
        u = rng.random(order.shape[0])
        X = torch.from_numpy(xy.copy()).to(DEV)
        d_s, st_s = gm.sweep(X, _params(ccsp, p), 1e-2, torch.from_numpy(disp).to(DEV),
                             torch.from_numpy(u).to(DEV))
        xy_s, st_s, d_s = X.cpu().numpy(), st_s.cpu().numpy(), d_s.cpu().numpy()
        xy_r, st_r, df_r, margin = ob.metropolis_chain(om, xy, p, 1e-2, order, disp, u)
        valid = (st_r == ob.ACCEPTED) | (st_r == ob.REJECTED)
        close = valid & (margin <= 1e-10)
        assert (d_s[close] == df_r[close]).all(), "a decision lies within rounding of its threshold"
        assert np.array_equal(st_s, st_r) and np.array_equal(xy_s, xy_r)
        M = gm.movable.shape[0]
        draws = np.zeros((M, 4))
        draws[:, :2] = rng.standard_normal((M, 2))
        draws[:, 2] = rng.random(M)
        _group_sweep_vs_chain(ccsp, gm, om, xy, p, 1e-2, 0.05, draws, rng.random(M))
