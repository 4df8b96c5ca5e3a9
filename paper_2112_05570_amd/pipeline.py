"""The low-weight triangulation pipeline (paper Secs. 3.1-3.5) composed from the library's pieces.

The annealing sweeps, proposals, greedy flips and objective evaluations run in the GPU library
(``MovableMesh``, ``flip_anneal``); contraction runs in the library's host code (``contract``).
This module only sequences them and converts between a mesh with Steiner vertices and the arrays
the walk loads. Input is a subdivided triangulation (Sec. 3.5.2) as host arrays: positions,
counter-clockwise triangles, vertex kinds (0 original, 1 constrained to original edge line[v],
2 free) and the two original vertices of each original edge (prim_v).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field, replace

import numpy as np

from . import MovableMesh, contract, flip_anneal, objective_params, subdivide

ORIGINAL, CONSTRAINED, FREE = 0, 1, 2


def weight(tri_v, xy) -> float:
    """Total edge length, each edge once."""
    tv = np.asarray(tri_v, dtype=np.int64)
    a, b = tv[:, [1, 2, 0]].ravel(), tv[:, [2, 0, 1]].ravel()
    V = xy.shape[0]
    u = np.unique(np.minimum(a, b) * V + np.maximum(a, b))
    a, b = u // V, u % V
    return float(np.sqrt(((xy[a] - xy[b]) ** 2).sum(1)).sum())


def walk_arrays(tri_v, kind, line, prim_v, xy):
    """Neighbours and primitives for the walk of a triangulation with Steiner vertices. Each
    constrained edge (both ends on one original edge k: its original ends or vertices constrained
    to k) becomes a primitive of its own, the segment between its two vertices, so that it is
    exactly collinear with its primitive as the walk's loader requires; sub_to_orig maps it back
    to k. Returns (tri_nbr, tri_prim, prims, sub_to_orig)."""
    tv = np.asarray(tri_v, dtype=np.int64)
    kind = np.asarray(kind)
    line = np.asarray(line)
    prim_v = np.asarray(prim_v, dtype=np.int64).reshape(-1, 2)
    xy = np.asarray(xy, dtype=np.float64)
    T, V = tv.shape[0], xy.shape[0]
    pa, pb = tv[:, [1, 2, 0]].ravel(), tv[:, [2, 0, 1]].ravel()  # slot 3t + i: (v[i+1], v[i+2])
    key = np.minimum(pa, pb) * V + np.maximum(pa, pb)
    order = np.argsort(key, kind="stable")
    sk = key[order]
    same = np.nonzero(sk[1:] == sk[:-1])[0]
    nbr = -np.ones(3 * T, dtype=np.int64)
    nbr[order[same]] = order[same + 1] // 3
    nbr[order[same + 1]] = order[same] // 3
    k = -np.ones(3 * T, dtype=np.int64)
    ca = kind[pa] == CONSTRAINED
    k[ca] = line[pa[ca]]
    cb = ~ca & (kind[pb] == CONSTRAINED)
    k[cb] = line[pb[cb]]
    oo = (kind[pa] == ORIGINAL) & (kind[pb] == ORIGINAL)
    if prim_v.shape[0] and oo.any():
        pkey = np.minimum(prim_v[:, 0], prim_v[:, 1]) * V + np.maximum(prim_v[:, 0], prim_v[:, 1])
        po = np.argsort(pkey)
        pos = np.clip(np.searchsorted(pkey[po], key[oo]), 0, pkey.shape[0] - 1)
        k[oo] = np.where(pkey[po][pos] == key[oo], po[pos], -1)

    def on(v, kk):
        ok = kk >= 0
        kc = np.where(ok, kk, 0)
        return ok & (((kind[v] == CONSTRAINED) & (line[v] == kc)) |
                     ((kind[v] == ORIGINAL) & ((prim_v[kc, 0] == v) | (prim_v[kc, 1] == v))))
    if prim_v.shape[0]:
        k[~(on(pa, k) & on(pb, k))] = -1
    cons = np.nonzero(k >= 0)[0]
    _, first, inv = np.unique(key[cons], return_index=True, return_inverse=True)
    prim = -np.ones(3 * T, dtype=np.int64)
    prim[cons] = inv
    s0 = cons[first]
    prims = np.concatenate([xy[pa[s0]], xy[pb[s0]]], axis=1).reshape(-1, 4)
    return (nbr.reshape(T, 3).astype(np.int32), prim.reshape(T, 3).astype(np.int32),
            np.ascontiguousarray(prims), k[s0])


@dataclass
class Schedule:
    """Stages of the main optimisation at temperature and contraction length lowered together
    (Sec. 3.3.1), both relative to the box side; weights of the penalties relative to it too."""
    stages: int = 24
    t0_rel: float = 1.5e-4
    t1_rel: float = 3e-6
    e0_rel: float = 1.5e-3
    e1_rel: float = 1.5e-4
    lambda0: float = 0.05
    target: float = 0.23
    mu_angle_rel: float = 1.0
    mu_len_rel: float = 10.0
    eps0_rel: float = 1e-10
    polish_sweeps: int = 4
    polish_step_rel: float = 6e-5
    flip_rounds: int = 64
    outer_max: int = 12
    seed: int = 0
    # group stages move the groups of a random share of the movable vertices: every vertex as a
    # centre costs far more than a single-vertex sweep (groups of tens of members, in rounds), and
    # Sec. 3.3.2 balances the perturbation types by the time they take
    group_share: float = 1.0 / 32
    # > 0: each stage runs this many sweeps whose types (displacement, resampling, contraction,
    # swap, group) are drawn with probability inversely proportional to each type's last measured
    # time, so that every type receives about equal time (Sec. 3.3.2); results then depend on the
    # timings. 0: one displacement sweep and one sweep of the next proposal type in turn
    balance_sweeps: int = 0


@dataclass
class Result:
    tri_v: np.ndarray
    kind: np.ndarray
    line: np.ndarray
    xy: np.ndarray
    log: dict = field(default_factory=dict)


def optimise(tri_v, kind, line, prim_v, xy, size, schedule: Schedule | None = None,
             verbose=False) -> Result:
    """Turn a subdivided triangulation into a low-weight one (Secs. 3.1-3.4):
    1. `stages` stages of annealing: each one displacement sweep with the adaptive step scale
       (Secs. 3.2, 3.2.2) and one sweep of resampling, contraction, swap or group moves in turn
       (Secs. 3.2.3-3.2.6; group moves with the displacement's step scale, centred at a random
       `group_share` of the movable vertices), at the stage's temperature and contraction length;
    2. contraction of the edges shorter than the final length (Sec. 3.4.1);
    3. polishing sweeps without fuzzy contraction alternated with greedy flips (the weight as
       energy, T = 0) (Sec. 3.4.2);
    4. the contraction length raised by 30% at a time, contracting, polishing and flipping again,
       keeping the lightest triangulation, until the weight exceeds 1.1 times the best or
       `outer_max` rounds (Sec. 3.4.2).
    size is the box side the schedule is relative to. Random draws come from a torch generator
    seeded with schedule.seed. Needs a GPU."""
    import torch

    s = schedule or Schedule()
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(s.seed)
    prim_v = np.ascontiguousarray(prim_v, dtype=np.int32).reshape(-1, 2)
    log = {}

    def unit_draws(m):
        r = torch.rand((m, 3), generator=gen, device=dev, dtype=torch.float64)
        rad = torch.sqrt(r[:, 0]) * (1.0 - r[:, 2]) ** -2.0
        th = 2.0 * np.pi * r[:, 1]
        return torch.stack([rad * torch.cos(th), rad * torch.sin(th)], 1).contiguous()

    def proposal_draws(m, kind):
        r = torch.rand((m, 4), generator=gen, device=dev, dtype=torch.float64)
        if kind == "swap":
            rad = torch.sqrt(r[:, 2])
            th = 2.0 * np.pi * r[:, 3]
            r[:, 2], r[:, 3] = rad * torch.cos(th), rad * torch.sin(th)
        return r

    def uniforms(*shape):
        return torch.rand(shape, generator=gen, device=dev, dtype=torch.float64)

    temps = s.t0_rel * size * np.geomspace(1.0, s.t1_rel / s.t0_rel, s.stages)
    epss = s.e0_rel * size * np.geomspace(1.0, s.e1_rel / s.e0_rel, s.stages)
    mu = (s.eps0_rel * size, s.mu_angle_rel * size, s.mu_len_rel * size)
    log["weight_start"] = weight(tri_v, np.asarray(xy))
    t0 = time.perf_counter()
    X = torch.from_numpy(np.array(xy, dtype=np.float64)).to(dev)
    with MovableMesh(tri_v, kind, line, prim_v) as gm:
        m = gm.n_movable()
        movable = torch.from_numpy(np.ascontiguousarray(gm.movable, dtype=np.int32)).to(dev)
        lam, acc = s.lambda0, []
        kinds = ("displace", "resample", "contract", "swap", "group")
        spent = {kd_: 0.0 for kd_ in kinds}
        last = {kd_: 0.0 for kd_ in kinds}
        counts = {kd_: 0 for kd_ in kinds}
        pick_rng = np.random.default_rng(s.seed)

        def run(kind_k, k):
            """One sweep of a perturbation type at stage k; returns the accepted share."""
            nonlocal lam
            p = objective_params(epss[k], None, *mu)
            if kind_k == "displace":
                _, a = gm.schedule(X, p, [temps[k]], [epss[k]], lam, unit_draws(m)[None],
                                   uniforms(1, m), target=s.target)
                frac = int(a[0]) / m
                lam = lam * min(2.0, max(0.5, 1.0 + (frac - s.target)))
                return frac
            if kind_k == "group":
                n_c = max(1, int(m * s.group_share))
                pick = torch.randperm(m, generator=gen, device=dev)[:n_c]
                cen = movable[pick].contiguous()
                r = proposal_draws(n_c, "group")
                r[:, :2] = unit_draws(n_c)
                _, st, _, _ = gm.group_sweep(X, p, temps[k], lam, r, uniforms(n_c), centres=cen)
            else:
                _, st = gm.propose(X, p, temps[k], kind_k, proposal_draws(m, kind_k),
                                   uniforms(m))
            return int((st == 1).sum().item()) / st.shape[0]

        def timed_run(kind_k, k):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = run(kind_k, k)
            torch.cuda.synchronize()
            last[kind_k] = time.perf_counter() - t
            spent[kind_k] += last[kind_k]
            counts[kind_k] += 1
            return r

        for k in range(s.stages):
            if s.balance_sweeps > 0:
                shares = []
                for j in range(s.balance_sweeps):
                    # every type once first, so that each has a measured time
                    untimed = [kd_ for kd_ in kinds if counts[kd_] == 0]
                    if untimed:
                        kind_k = untimed[0]
                    else:
                        w = np.array([1.0 / max(last[kd_], 1e-6) for kd_ in kinds])
                        kind_k = kinds[int(pick_rng.choice(len(kinds), p=w / w.sum()))]
                    shares.append((kind_k, timed_run(kind_k, k)))
                frac = np.mean([sh for kd_, sh in shares if kd_ == "displace"] or [0.0])
                acc.append([float(frac), shares])
            else:
                frac = run("displace", k)
                kind_k = ("resample", "contract", "swap", "group")[k % 4]
                acc.append([frac, run(kind_k, k)])
            if verbose:
                f = gm.eval(X, objective_params(epss[k], None, *mu)).cpu().tolist()
                what = (f"{kind_k} {acc[-1][1]:.3f}" if s.balance_sweeps == 0 else
                        " ".join(f"{kd_}:{sh:.3f}" for kd_, sh in acc[-1][1]))
                print(f"[optimise] stage {k}: T {temps[k]:.3g} eps {epss[k]:.3g} "
                      f"accepted {frac:.2f} / {what}, f {f[0]:.1f}", flush=True)
    xy_opt = X.cpu().numpy()
    log["anneal_s"] = time.perf_counter() - t0
    log["acceptance"] = acc
    if s.balance_sweeps > 0:
        log["balance"] = {"sweeps": counts, "seconds": spent}
    log["weight_annealed"] = weight(tri_v, xy_opt)

    pol = objective_params(epss[-1], None, *mu, polish=True)
    pv_dev = torch.from_numpy(prim_v).to(dev)

    def polish_and_flip(tv, kd, ln, pos, rounds, seed):
        nflips = 0
        for rnd in range(rounds + 1):
            Xp = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
            with MovableMesh(tv, kd, ln, prim_v) as pm:
                mp = pm.n_movable()
                for j in range(s.polish_sweeps):
                    if j % 2 == 0:
                        pm.sweep(Xp, pol, temps[-1],
                                 (s.polish_step_rel * size * unit_draws(mp)).contiguous(),
                                 uniforms(mp))
                    else:
                        pm.propose(Xp, pol, temps[-1], "resample", proposal_draws(mp, "resample"),
                                   uniforms(mp))
            pos = Xp.cpu().numpy()
            if rnd == rounds:
                break
            nbr, prim, _, _ = walk_arrays(tv, kd, ln, prim_v, pos)
            arrs = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (tv, nbr, prim)]
            vline = torch.from_numpy(np.where(kd == CONSTRAINED, ln, -1).astype(np.int32)).to(dev)
            nflips += int(flip_anneal(Xp, *arrs, [0.0] * s.flip_rounds, seed + rnd, vline,
                                      pv_dev).sum())
            tv = arrs[0].cpu().numpy()
        return tv, pos, nflips

    t1 = time.perf_counter()
    c = contract(tri_v, kind, line, prim_v, xy_opt, epss[-1])
    tv, kd, ln, pos = c["tri_v"], c["kind"], c["line"], c["xy"]
    tv, pos, nflips = polish_and_flip(tv, kd, ln, pos, 2, s.seed)
    best = Result(tv, kd, ln, pos)
    best_w = weight(tv, pos)
    hist = [{"eps": float(epss[-1]), "contractions": c["contracted"], "vertices": int(pos.shape[0]),
             "weight": best_w, "greedy_flips": nflips}]
    e = float(epss[-1])
    for r in range(s.outer_max):
        e *= 1.3
        c = contract(tv, kd, ln, prim_v, pos, e)
        tv, kd, ln, pos = c["tri_v"], c["kind"], c["line"], c["xy"]
        tv, pos, nflips = polish_and_flip(tv, kd, ln, pos, 1, s.seed + 10 * (r + 1))
        w = weight(tv, pos)
        hist.append({"eps": e, "contractions": c["contracted"], "vertices": int(pos.shape[0]),
                     "weight": w, "greedy_flips": nflips})
        if verbose:
            print(f"[optimise] contract at eps {e:.3g}: {pos.shape[0]} vertices, weight {w:.1f}",
                  flush=True)
        if w < best_w:
            best, best_w = Result(tv, kd, ln, pos), w
        elif w > 1.1 * best_w:
            break
    log["contract_polish_s"] = time.perf_counter() - t1
    log["contract_polish"] = hist
    log["weight_final"] = best_w
    best.log = log
    return best


def optimise_iterated(tri_v, kind, line, prim_v, xy, size, schedule: Schedule | None = None,
                      rounds: int = 2, verbose=False) -> Result:
    """The iterated strategy of Sec. 3.5.3: `rounds` times, subdivide the current triangulation
    (Sec. 3.5.2; the first round starts from the given one, normally the CDT, whose vertices are
    all ORIGINAL, so that there is nothing to move without it) and run `optimise` on the result.
    Round k uses the schedule's seed + k. Returns the lightest of the rounds' results (keeping the
    lightest, as the contraction rounds of Sec. 3.4.2 do: a later round starts from a subdivision,
    which is heavier, and need not end lighter), with each round's log in log["rounds"]. When a
    later round's subdivision is not valid (a sub-triangle not strictly counter-clockwise after
    rounding), the strategy stops there and log["stopped"] says why."""
    from .binding import CcspError

    s = schedule or Schedule()
    prim_v = np.ascontiguousarray(prim_v, dtype=np.int32).reshape(-1, 2)
    tv, kd, ln, pos = tri_v, kind, line, np.asarray(xy, dtype=np.float64)
    best, logs, stopped = None, [], None
    for k in range(rounds):
        try:
            tv2, kd2, ln2, pv2, pos2 = subdivide(tv, kd, ln, prim_v, pos)
        except CcspError as err:
            # an optimised triangulation can hold slivers (vertices on one original edge up to
            # rounding) whose midpoints round across an edge; the strategy then ends here
            if best is None:
                raise
            stopped = f"round {k}: {err}"
            break
        r = optimise(tv2, kd2, ln2, pv2, pos2, size, replace(s, seed=s.seed + k), verbose)
        logs.append(dict(r.log, subdivided_vertices=int(pos2.shape[0]),
                         vertices=int(r.xy.shape[0])))
        if verbose:
            print(f"[optimise] round {k}: {pos2.shape[0]} vertices subdivided, weight "
                  f"{r.log['weight_final']:.1f}", flush=True)
        if best is None or r.log["weight_final"] < best.log["weight_final"]:
            best = r
        tv, kd, ln, pos = r.tri_v, r.kind, r.line, r.xy
    best.log = dict(best.log, rounds=logs, stopped=stopped)
    return best
