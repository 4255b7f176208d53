"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* brute-force enumeration of every cut (the definition, eq. (1) of Sec. 2);
* hand-derived examples (tests/golden/hand_examples.json);
* closed forms at full workload size (all n-links zero; n-links too strong to cut);
* two independent solvers (push-relabel and Dinic) and the duality certificate;
* the paper's own method (reference P-ARD / S-ARD) with its statements checked
  after every sweep (Sec. 4.2-4.4) and the 2|B|^2+1 sweep bound.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _grid_from_json(ex):
    dims = tuple(ex["dims"])
    return synth.GridInstance(dims=dims, conn=ex["conn"], cs=np.array(ex["cs"], np.int32),
                              ct=np.array(ex["ct"], np.int32),
                              nbr=np.array(ex["nbr"], np.int32))


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


@pytest.mark.parametrize("seed", range(120))
def test_pushrelabel_and_dinic_match_brute_force(seed):
    n = 2 + seed % 15
    pu, pv, cuv, cvu, cs, ct = synth.random_digraph(n, seed)
    bf = oracle.brute_force(n, pu, pv, cuv, cvu, cs, ct)
    for method in ("pr", "dinic"):
        r = oracle.solve_pairs(n, pu, pv, cuv, cvu, cs, ct, method=method)
        assert r["flow"] == bf["flow"]
        assert (r["smin"] == bf["smin"]).all()
        assert (r["smax"] == bf["smax"]).all()
        oracle.certify(n, pu, pv, cuv, cvu, cs, ct, r["r_uv"], r["r_vu"], r["rt"], r["ex"],
                       r["flow"], r["smin"], r["smax"])


def test_brute_force_cut_cost_terms():
    # one vertex, s-link 7, t-link 3: cutting it to the sink side costs 7, to the source side 3
    z = np.zeros(0, np.int32)
    cs = np.array([7], np.int32)
    ct = np.array([3], np.int32)
    assert oracle.cut_cost(np.array([0]), z, z, z, z, cs, ct) == 7
    assert oracle.cut_cost(np.array([1]), z, z, z, z, cs, ct) == 3
    # two vertices, arc 0->1 of 5 and 1->0 of 2: only the arc leaving the source side counts
    pu, pv = np.array([0], np.int32), np.array([1], np.int32)
    cuv, cvu = np.array([5], np.int32), np.array([2], np.int32)
    zero2 = np.zeros(2, np.int32)
    assert oracle.cut_cost(np.array([1, 0]), pu, pv, cuv, cvu, zero2, zero2) == 5
    assert oracle.cut_cost(np.array([0, 1]), pu, pv, cuv, cvu, zero2, zero2) == 2


def test_hand_examples():
    with open(os.path.join(HERE, "golden", "hand_examples.json")) as f:
        data = json.load(f)
    for ex in data["examples"]:
        inst = _grid_from_json(ex)
        for method in ("pr", "dinic"):
            r = oracle.solve_grid(inst, method=method)
            assert r["flow"] == ex["flow"], ex["name"]
            assert r["smin"].tolist() == ex["smin"], ex["name"]
            assert r["smax"].tolist() == ex["smax"], ex["name"]
        pu, pv, cuv, cvu = oracle.grid_pairs(inst.dims, inst.nbr, synth.offsets_for(2, 4))
        bf = oracle.brute_force(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct)
        assert bf["flow"] == ex["flow"]
        assert bf["smin"].tolist() == ex["smin"] and bf["smax"].tolist() == ex["smax"]
        a = oracle.ard_grid(inst, tile=(1, 2))
        assert a["flow"] == ex["flow"] and a["smin"].tolist() == ex["smin"]


@pytest.mark.parametrize("cfg", [0, 1])
def test_closed_form_no_nlinks(cfg):
    """All n-links zero: every vertex is independent, |f| = sum min(cs, ct),
    S_min = {cs > ct}, S_max = {cs >= ct}."""
    inst = synth.config(cfg)
    inst.nbr[:] = 0
    r = oracle.solve_grid(inst)
    cs = inst.cs.astype(np.int64)
    ct = inst.ct.astype(np.int64)
    assert r["flow"] == int(np.minimum(cs, ct).sum())
    assert (r["smin"] == (cs > ct)).all()
    assert (r["smax"] == (cs >= ct)).all()


def test_closed_form_strong_nlinks():
    """n-links stronger than every t-link together: the only candidate minimum
    cuts keep the grid in one piece, |f| = min(sum cs, sum ct)."""
    for seed, conn in [(5, 4), (6, 8)]:
        inst = synth.random_grid((20, 24), conn, seed)
        offs = synth.offsets_for(2, conn)
        big = int(inst.cs.sum() + inst.ct.sum() + 1)
        for k, off in enumerate(offs):
            valid = synth.grids._shift_valid(inst.dims, off).reshape(-1)
            inst.nbr[k] = np.where(valid, big, 0)
        r = oracle.solve_grid(inst)
        sc, st = int(inst.cs.sum()), int(inst.ct.sum())
        assert r["flow"] == min(sc, st)
        if sc < st:
            assert r["smin"].sum() == 0 and r["smax"].sum() == 0
        elif st < sc:
            assert r["smin"].all() and r["smax"].all()


@pytest.mark.parametrize("seed", range(20))
def test_chain_closed_form(seed):
    """A 1 x L chain fed at its left end and drained at its right end carries
    min(source, sink, every forward capacity)."""
    rng = np.random.default_rng(seed)
    L = int(rng.integers(2, 40))
    nbr = np.zeros((4, L), np.int32)
    fwd = rng.integers(1, 30, size=L - 1)
    nbr[0, :L - 1] = fwd
    nbr[1, 1:] = rng.integers(0, 30, size=L - 1)
    cs = np.zeros(L, np.int32)
    ct = np.zeros(L, np.int32)
    cs[0] = int(rng.integers(1, 50))
    ct[-1] = int(rng.integers(1, 50))
    inst = synth.GridInstance(dims=(1, L), conn=4, cs=cs, ct=ct, nbr=nbr)
    r = oracle.solve_grid(inst, method="pr")
    assert r["flow"] == min(int(cs[0]), int(ct[-1]), int(fwd.min()))
    d = oracle.solve_grid(inst, method="dinic")
    assert d["flow"] == r["flow"] and (d["smin"] == r["smin"]).all()


def test_workload0_solvers_agree_and_certify():
    inst = synth.config(0)
    r = oracle.solve_grid(inst, "pr")
    d = oracle.solve_grid(inst, "dinic")
    assert r["flow"] == d["flow"]
    assert (r["smin"] == d["smin"]).all() and (r["smax"] == d["smax"]).all()
    pu, pv, cuv, cvu = r["pairs"]
    oracle.certify(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct, r["r_uv"], r["r_vu"], r["rt"],
                   r["ex"], r["flow"], r["smin"], r["smax"])
    oracle.certify(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct, d["r_uv"], d["r_vu"], d["rt"],
                   d["ex"], d["flow"], d["smin"], d["smax"])


def test_certify_rejects_planted_mistakes():
    inst = synth.random_grid((8, 8), 4, 3)
    r = oracle.solve_grid(inst)
    pu, pv, cuv, cvu = r["pairs"]
    args = [inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct]
    good = [r["r_uv"], r["r_vu"], r["rt"], r["ex"], r["flow"], r["smin"], r["smax"]]
    oracle.certify(*args, *good)
    # a wrong flow value
    with pytest.raises(AssertionError):
        oracle.certify(*args, *good[:4], good[4] + 1, good[5], good[6])
    # a cut that is not minimal
    wrong = good[5].copy()
    wrong[np.argmax(wrong == 0)] = 1
    if oracle.cut_cost(wrong, pu, pv, cuv, cvu, inst.cs, inst.ct) != good[4]:
        with pytest.raises(AssertionError):
            oracle.certify(*args, *good[:5], wrong, None)
    # a residual pair that lost a unit
    bad = good[0].copy()
    i = int(np.argmax(bad > 0))
    bad[i] -= 1
    with pytest.raises(AssertionError):
        oracle.certify(*args, bad, *good[1:])


# ---------------------------------------------------------------------------
# The paper's method on the CPU (reference ARD)
# ---------------------------------------------------------------------------

CASES = [((12, 13), 4, (4, 5)), ((16, 16), 8, (8, 8)), ((9, 20), 4, (3, 7)),
         ((6, 7, 8), 6, (3, 4, 4)), ((10, 10), 8, (10, 10)), ((15, 9), 8, (2, 2))]


@pytest.mark.parametrize("seed", range(24))
def test_reference_ard_exact_and_invariants(seed):
    dims, conn, tile = CASES[seed % len(CASES)]
    inst = synth.random_grid(dims, conn, seed, tile=tile)
    r = oracle.solve_grid(inst)
    for parallel in (True, False):
        a = oracle.ard_grid(inst, parallel=parallel, checks=oracle.CHK_ALL)
        assert a["flow"] == r["flow"]
        assert (a["smin"] == r["smin"]).all() and (a["smax"] == r["smax"]).all()
        assert a["sweeps"] <= 2 * max(a["bsize"], 1) ** 2 + 1
        pu, pv, cuv, cvu = a["pairs"]
        oracle.certify(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct, a["r_uv"], a["r_vu"],
                       a["rt"], a["ex"], a["flow"], a["smin"], a["smax"])


@pytest.mark.parametrize("strength", [5, 40, 150, 400])
def test_reference_ard_paper_family(strength):
    """The synthetic family of Sec. 7.1 (excess in [-500, 500], constant strength)."""
    for seed in range(3):
        inst = synth.paper_e1_grid((30, 30), 8, seed, strength, tile=(15, 15))
        r = oracle.solve_grid(inst)
        a = oracle.ard_grid(inst, checks=oracle.CHK_ALL)
        assert a["flow"] == r["flow"] and (a["smin"] == r["smin"]).all()
        s = oracle.ard_grid(inst, parallel=False, checks=oracle.CHK_ALL)
        assert s["flow"] == r["flow"]


def test_reference_ard_single_region_is_one_sweep():
    inst = synth.random_grid((14, 11), 8, 11)
    a = oracle.ard_grid(inst, tile=(14, 11))
    r = oracle.solve_grid(inst)
    assert a["bsize"] == 0 and a["sweeps"] == 1 and a["flow"] == r["flow"]


def test_reference_ard_boundary_size_closed_form():
    """|B| for a tiling = vertices with a grid neighbour in another tile; for
    box tiles this is n minus the product of per-axis non-edge coordinates."""
    for dims, conn, tile in [((64, 64), 4, (32, 32)), ((50, 37), 8, (16, 8)),
                             ((9, 10, 11), 6, (4, 4, 4))]:
        inst = synth.random_grid(dims, conn, 0, tile=tile)
        a = oracle.ard_grid(inst, checks=0)
        inner = 1
        for d, t in zip(dims, tile):
            x = np.arange(d)
            edge = ((x % t == 0) & (x > 0)) | ((x % t == t - 1) & (x < d - 1))
            inner *= int((~edge).sum())
        assert a["bsize"] == int(np.prod(dims)) - inner
    assert oracle.ard_grid(synth.config(0), checks=0)["bsize"] == 252


# ---------------------------------------------------------------------------
# Partial discharges (Sec. 6.2): sweep s runs only the stages k <= s
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(24))
def test_reference_ard_partial_exact_and_invariants(seed):
    """Same flow and cuts as the textbook solvers; the labeling stays valid,
    monotone and below the exact region distance after every sweep."""
    dims, conn, tile = CASES[seed % len(CASES)]
    inst = synth.random_grid(dims, conn, 300 + seed, tile=tile)
    r = oracle.solve_grid(inst)
    for parallel in (True, False):
        a = oracle.ard_grid(inst, parallel=parallel, checks=oracle.CHK_ALL, partial=True)
        assert a["flow"] == r["flow"]
        assert (a["smin"] == r["smin"]).all() and (a["smax"] == r["smax"]).all()
        # the cap reaches d_inf after d_inf sweeps, from there on the sweeps are full
        B = max(a["bsize"], 1)
        assert a["sweeps"] <= B + 2 * B ** 2 + 1
        pu, pv, cuv, cvu = a["pairs"]
        oracle.certify(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct, a["r_uv"], a["r_vu"],
                       a["rt"], a["ex"], a["flow"], a["smin"], a["smax"])


def _region_flow_sum(inst, tile):
    """Sum over regions of the max flow of the region alone (its inner pairs and
    its t-links; pairs to other regions dropped), by the textbook solver."""
    pu, pv, cuv, cvu = oracle.grid_pairs(inst.dims, inst.nbr, oracle._offsets(inst))
    region = oracle.grid_regions(inst.dims, tile)
    total = 0
    for rk in np.unique(region):
        vs = np.flatnonzero(region == rk)
        idx = -np.ones(inst.n, np.int64)
        idx[vs] = np.arange(len(vs))
        keep = (region[pu] == rk) & (region[pv] == rk)
        total += oracle.solve_pairs(len(vs), idx[pu[keep]], idx[pv[keep]], cuv[keep], cvu[keep],
                                    inst.cs[vs], inst.ct[vs])["flow"]
    return total


def test_reference_ard_partial_first_sweep_is_regionwise_maxflow():
    """With partial discharges sweep 0 runs stage 0 only: paths to the sink.
    No flow crosses a region border, and the flow after the sweep is the sum of
    the regions' own max flows.  Without the cap some flow does cross."""
    crossed_full = 0
    for seed in range(8):
        dims, conn, tile = CASES[seed % len(CASES)]
        inst = synth.random_grid(dims, conn, 400 + seed, tile=tile)
        pu, pv, cuv, cvu = oracle.grid_pairs(inst.dims, inst.nbr, oracle._offsets(inst))
        region = oracle.grid_regions(inst.dims, tile)
        cross = region[pu] != region[pv]
        a = oracle.ard_grid(inst, partial=True, max_sweeps=1, stop_early=True)
        assert a["sweeps"] == 1
        assert (a["r_uv"][cross] == cuv[cross]).all() and (a["r_vu"][cross] == cvu[cross]).all()
        assert a["flow"] == _region_flow_sum(inst, tile)
        f = oracle.ard_grid(inst, partial=False, max_sweeps=1, stop_early=True)
        crossed_full += int((f["r_uv"][cross] != cuv[cross]).any())
    assert crossed_full > 0


@pytest.mark.parametrize("dims,conn", [((12, 10), 4), ((9, 7), 8), ((4, 5, 6), 6)])
def test_serpentine_closed_form(dims, conn):
    """A single residual path through every vertex: flow = c(last, t), the
    minimal source side is the path, the maximal source side is everything."""
    from tests.helpers import serpentine_instance
    inst, path = serpentine_instance(dims, conn, tile=dims)
    assert len(set(path.tolist())) == len(path) and 0 < len(path) < inst.n
    r = oracle.solve_grid(inst)
    assert r["flow"] == 30
    want = np.zeros(inst.n, np.uint8)
    want[path] = 1
    assert (r["smin"] == want).all()
    assert (r["smax"] == 1).all()
    for tile in ((3,) * len(dims), tuple(max(1, d // 2) for d in dims)):
        inst.tile = tile
        a = oracle.ard_grid(inst, checks=oracle.CHK_ALL)
        assert a["flow"] == 30 and (a["smin"] == want).all() and (a["smax"] == 1).all()


# ---------------------------------------------------------------------------
# Boundary relabel heuristic (Sec. 6.1)
# ---------------------------------------------------------------------------

def _region_distance(n, pu, pv, r_uv, r_vu, region, rt, dinf):
    """Exact d*B (Sec. 4.1) by 0-1 breadth-first search towards t: an arc
    between regions has length 1, one inside a region length 0."""
    from collections import deque
    rev = [[] for _ in range(n)]  # v -> (u, length) for residual arcs u -> v
    for a, b, x, y in zip(pu, pv, r_uv, r_vu):
        ln = int(region[a] != region[b])
        if x > 0:
            rev[b].append((a, ln))
        if y > 0:
            rev[a].append((b, ln))
    dist = np.full(n, dinf, np.int64)
    dq = deque()
    for v in np.flatnonzero(rt > 0):
        dist[v] = 0
        dq.append(v)
    while dq:
        v = dq.popleft()
        for u, ln in rev[v]:
            if dist[v] + ln < dist[u]:
                dist[u] = dist[v] + ln
                (dq.appendleft if ln == 0 else dq.append)(u)
    return dist


def _assert_valid(pu, pv, r_uv, r_vu, region, rt, d):
    """Validity of Sec. 4.1 on every residual arc, and d = 0 wherever r_t > 0."""
    ln = (region[pu] != region[pv]).astype(np.int64)
    d = d.astype(np.int64)
    assert (d[pu][r_uv > 0] <= (d[pv] + ln)[r_uv > 0]).all()
    assert (d[pv][r_vu > 0] <= (d[pu] + ln)[r_vu > 0]).all()
    assert (d[rt > 0] == 0).all()


@pytest.mark.parametrize("L,w", [(6, 8), (3, 5), (9, 4)])
def test_boundary_relabel_region_chain_closed_form(L, w):
    """After the first sweep the labels are 1 in every region but the last;
    the heuristic lifts region j to L - 1 - j, its exact region distance."""
    from tests.helpers import region_chain_instance
    inst = region_chain_instance(L, w)
    j = np.repeat(np.arange(L), w)
    plain = oracle.ard_grid(inst, max_sweeps=1, stop_early=True)
    assert (plain["labels"] == np.where(j < L - 1, 1, 0)).all()
    brl = oracle.ard_grid(inst, max_sweeps=1, stop_early=True, boundary_relabel=True)
    assert (brl["labels"] == L - 1 - j).all()
    # the stand-alone heuristics (C and Python) on the plain state agree
    pu, pv, _, _ = plain["pairs"]
    region = oracle.grid_regions(inst.dims, inst.tile)
    for f in (oracle.boundary_relabel, oracle.boundary_relabel_c):
        got = f(inst.n, pu, pv, plain["r_uv"], plain["r_vu"], region, plain["labels"], plain["bsize"])
        assert (got == L - 1 - j).all()
    full = oracle.ard_grid(inst, boundary_relabel=True)
    assert full["flow"] == L * 10 == oracle.solve_grid(inst)["flow"]


BRL_CASES = [((12, 13), 4, (4, 5)), ((16, 16), 8, (4, 8)), ((6, 7, 8), 6, (3, 4, 4)),
             ((20, 9), 8, (5, 3)), ((5, 9, 13), 6, (5, 4, 6)), ((30, 30), 4, (6, 6))]


@pytest.mark.parametrize("seed", range(18))
def test_boundary_relabel_valid_lower_bound_and_two_implementations(seed):
    """On the state after s plain sweeps: the C heuristic and the separate
    Python one give the same labels, which never decrease, form a valid
    labeling and never exceed the exact region distance d*B."""
    dims, conn, tile = BRL_CASES[seed % len(BRL_CASES)]
    maker = synth.blob_grid if seed % 2 else synth.random_grid
    inst = (maker(dims, conn, 1500 + seed, 3, 2.0, 6.0, tile=tile) if seed % 2
            else maker(dims, conn, 1500 + seed, tile=tile))
    region = oracle.grid_regions(inst.dims, tile)
    lifted = 0
    for s in (1, 2, 3):
        a = oracle.ard_grid(inst, max_sweeps=s, stop_early=True)
        pu, pv, _, _ = a["pairs"]
        d0 = a["labels"]
        dinf = a["bsize"] if a["bsize"] > 0 else 1
        py = oracle.boundary_relabel(inst.n, pu, pv, a["r_uv"], a["r_vu"], region, d0, dinf)
        c = oracle.boundary_relabel_c(inst.n, pu, pv, a["r_uv"], a["r_vu"], region, d0, dinf)
        assert (py == c).all()
        assert (c >= d0).all() and (c <= dinf).all()
        _assert_valid(pu, pv, a["r_uv"], a["r_vu"], region, a["rt"], c)
        dstar = _region_distance(inst.n, pu, pv, a["r_uv"], a["r_vu"], region, a["rt"], dinf)
        assert (c <= dstar).all()
        lifted += int((c > d0).sum())
        if a["complete"]:
            break
    print(f"{inst.name}: {lifted} labels lifted", flush=True)


def test_boundary_relabel_lifts_labels_somewhere():
    """The heuristic is not the identity on the random families above."""
    lifted = 0
    for seed in range(6):
        dims, conn, tile = BRL_CASES[seed]
        inst = synth.random_grid(dims, conn, 1600 + seed, tile=tile)
        region = oracle.grid_regions(inst.dims, tile)
        a = oracle.ard_grid(inst, max_sweeps=1, stop_early=True)
        pu, pv, _, _ = a["pairs"]
        c = oracle.boundary_relabel_c(inst.n, pu, pv, a["r_uv"], a["r_vu"], region, a["labels"],
                                      max(a["bsize"], 1))
        lifted += int((c > a["labels"]).sum())
    assert lifted > 0


@pytest.mark.parametrize("partial", [False, True])
@pytest.mark.parametrize("seed", range(12))
def test_reference_ard_boundary_relabel_exact_and_invariants(seed, partial):
    """P-ARD with the heuristic after every sweep: the flow is the textbook
    maximum, the per-sweep checks (validity, monotone labels, labels below the
    exact region distance) hold, and the sweep count stays within 2|B|^2+1."""
    dims, conn, tile = BRL_CASES[seed % len(BRL_CASES)]
    inst = synth.random_grid(dims, conn, 1700 + seed, tile=tile)
    ref = oracle.solve_grid(inst)
    a = oracle.ard_grid(inst, partial=partial, boundary_relabel=True, checks=oracle.CHK_ALL)
    assert a["flow"] == ref["flow"]
    assert (a["smin"] == ref["smin"]).all() and (a["smax"] == ref["smax"]).all()
    assert a["sweeps"] <= 2 * max(a["bsize"], 1) ** 2 + 1
    s = oracle.ard_grid(inst, parallel=False, partial=partial, boundary_relabel=True,
                        checks=oracle.CHK_ALL)
    assert s["flow"] == ref["flow"]


# ---------------------------------------------------------------------------
# Push-relabel region discharge (Sec. 3, Proc. PRD; Alg. 1 and 2)
# ---------------------------------------------------------------------------

PRD_CASES = [((12, 13), 4, (4, 5)), ((16, 16), 8, (4, 8)), ((6, 7, 8), 6, (3, 4, 4)),
             ((20, 9), 8, (5, 3)), ((5, 9, 13), 6, (5, 4, 6)), ((30, 30), 4, (6, 6))]


@pytest.mark.parametrize("parallel", [True, False])
@pytest.mark.parametrize("seed", range(12))
def test_reference_prd_exact_and_invariants(seed, parallel):
    """P-PRD / S-PRD: the textbook flow and both cuts, distance labels valid and
    monotone after every sweep, at most 2n^2 sweeps."""
    dims, conn, tile = PRD_CASES[seed % len(PRD_CASES)]
    inst = synth.random_grid(dims, conn, 1800 + seed, tile=tile)
    ref = oracle.solve_grid(inst)
    p = oracle.prd_grid(inst, parallel=parallel)
    assert p["flow"] == ref["flow"]
    assert (p["smin"] == ref["smin"]).all() and (p["smax"] == ref["smax"]).all()
    assert p["sweeps"] <= 2 * inst.n ** 2
    # without the gap it still ends, with the same result
    q = oracle.prd_grid(inst, parallel=parallel, gap=False)
    assert q["flow"] == ref["flow"]


def test_reference_prd_single_region_is_one_sweep():
    """With one region Proc. PRD is plain push-relabel: one sweep solves it."""
    inst = synth.random_grid((14, 15), 8, 1850, tile=(14, 15))
    p = oracle.prd_grid(inst)
    assert p["sweeps"] == 1 and p["flow"] == oracle.solve_grid(inst)["flow"]


def test_ard_sweeps_below_prd_sweeps():
    """The paper's comparison (Tables 1 and 2): on the same partition ARD needs
    fewer sweeps than PRD, here summed over a family of random grids."""
    ard = prd = 0
    for seed in range(6):
        dims, conn, tile = PRD_CASES[seed]
        inst = synth.random_grid(dims, conn, 1900 + seed, tile=tile)
        ard += oracle.ard_grid(inst)["sweeps"]
        prd += oracle.prd_grid(inst)["sweeps"]
    print(f"P-ARD {ard} sweeps, P-PRD {prd} sweeps", flush=True)
    assert ard < prd


# ---------------------------------------------------------------------------
# Region reduction (Alg. 5, Sec. 8)
# ---------------------------------------------------------------------------

RR_CASES = [((30, 30), 8, (10, 10)), ((8, 9, 10), 6, (4, 3, 5)), ((24, 26), 4, (8, 13)),
            ((64, 64), 4, (32, 32))]


def _region_networks(inst, tile):
    """Yield, per region, the region network of Sec. 8: R, its boundary B^R and
    every pair touching R, as (global ids, in-R mask, pair arrays, s- and t-links
    of R)."""
    pu, pv, cuv, cvu = oracle.grid_pairs(inst.dims, inst.nbr,
                                         synth.offsets_for(len(inst.dims), inst.conn))
    region = oracle.grid_regions(inst.dims, tile)
    for rk in np.unique(region):
        inR = region == rk
        touch = inR[pu] | inR[pv]
        verts = np.unique(np.concatenate([np.flatnonzero(inR), pu[touch], pv[touch]]))
        idx = -np.ones(inst.n, np.int64)
        idx[verts] = np.arange(len(verts))
        rin = inR[verts]
        cs = np.where(rin, inst.cs[verts], 0)
        ct = np.where(rin, inst.ct[verts], 0)
        yield verts, rin, idx[pu[touch]], idx[pv[touch]], cuv[touch], cvu[touch], cs, ct


def _two_auxiliary_problems(inst, tile, solve, big=1 << 20):
    """The classes of Sec. 8 from the two auxiliary problems the section starts
    from: every boundary vertex joined to t without bound (N_t), or supplied
    from s without bound (N_s), each solved on its own by ``solve`` (returning
    the extremal cuts).  Strong source = minimal source side of N_t; strong sink
    = outside the maximal source side of N_s; weak source = in the maximal but
    not the minimal source side of N_t (it reaches neither t nor B^R in a
    maximum flow of N_t); weak sink = the same for N_s (neither s nor B^R
    reaches it).  Alg. 5 finds one flow whose residual network gives these four
    sets (its steps 1+3 are a maximum flow of N_t, its steps 1+4 one of N_s)."""
    cls = np.zeros(inst.n, np.uint8)
    for verts, rin, la, lb, cuv, cvu, cs, ct in _region_networks(inst, tile):
        bnd = ~rin
        nt = solve(len(verts), la, lb, cuv, cvu, cs, np.where(bnd, big, ct))
        ns = solve(len(verts), la, lb, cuv, cvu, np.where(bnd, big, cs), ct)
        c = np.zeros(len(verts), np.uint8)
        c[nt["smin"] == 1] |= oracle.REDUCE_STRONG_SOURCE
        c[ns["smax"] == 0] |= oracle.REDUCE_STRONG_SINK
        c[(nt["smax"] == 1) & (nt["smin"] == 0)] |= oracle.REDUCE_WEAK_SOURCE
        c[(ns["smax"] == 1) & (ns["smin"] == 0)] |= oracle.REDUCE_WEAK_SINK
        cls[verts[rin]] = c[rin]
    return cls


def _semantics_hold(cls, smin, smax):
    """The definitions of Sec. 8 against the extremal optimal cuts of the whole
    network: a strong source node is in every optimal source side (so in the
    minimal one), a strong sink node in none (not in the maximal one), a weak
    source node in some (the maximal one), a weak sink node outside some (not in
    the minimal one)."""
    ss = (cls & oracle.REDUCE_STRONG_SOURCE) > 0
    st = (cls & oracle.REDUCE_STRONG_SINK) > 0
    ws = (cls & oracle.REDUCE_WEAK_SOURCE) > 0
    wk = (cls & oracle.REDUCE_WEAK_SINK) > 0
    return bool((~ss | smin).all() and (~st | ~smax).all() and (~ws | smax).all()
                and (~wk | ~smin).all() and not (ss & st).any()
                and not ((ss | st) & (ws | wk)).any())


RR_TINY = [((4, 4), 4, (2, 2)), ((4, 4), 8, (2, 2)), ((4, 4), 4, (4, 2)), ((2, 2, 4), 6, (2, 2, 2)),
           ((3, 5), 8, (3, 2))]


def _brute(n, pu, pv, cuv, cvu, cs, ct):
    return oracle.brute_force(n, pu, pv, cuv, cvu, cs, ct)


@pytest.mark.parametrize("seed", range(100))
def test_region_reduction_tiny_against_brute_force(seed):
    """Networks of at most 16 vertices: the four classes of Alg. 5 equal the
    auxiliary problems solved by enumerating every cut of each region network,
    and agree with every optimal cut of the whole network (enumerated too)."""
    dims, conn, tile = RR_TINY[seed % len(RR_TINY)]
    inst = synth.random_grid(dims, conn, 2300 + seed)
    cls = oracle.region_reduction(inst, tile)
    assert (cls == _two_auxiliary_problems(inst, tile, _brute)).all()
    pu, pv, cuv, cvu = oracle.grid_pairs(inst.dims, inst.nbr,
                                         synth.offsets_for(len(inst.dims), inst.conn))
    bf = oracle.brute_force(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct)
    assert _semantics_hold(cls, bf["smin"] == 1, bf["smax"] == 1)


RR_FUZZ = [((4, 4), 4, (2, 2)), ((6, 5), 8, (3, 2)), ((8, 8), 4, (4, 3)), ((5, 6, 4), 6, (2, 3, 2)),
           ((12, 10), 8, (5, 4))]


def test_region_reduction_fuzz_against_auxiliary_problems():
    """600 random tilings: Alg. 5 (Dinic augmentations) gives exactly the
    classes of the two auxiliary problems solved by push-relabel, and they obey
    the definitions against the whole network's extremal cuts."""
    for seed in range(600):
        dims, conn, tile = RR_FUZZ[seed % len(RR_FUZZ)]
        inst = synth.random_grid(dims, conn, 5000 + seed)
        cls = oracle.region_reduction(inst, tile)
        aux = _two_auxiliary_problems(inst, tile, oracle.solve_pairs)
        assert (cls == aux).all(), seed
        ref = oracle.solve_grid(inst)
        assert _semantics_hold(cls, ref["smin"] == 1, ref["smax"] == 1), seed


def test_region_reduction_preflow_augment_is_caught():
    """Planted mistake: Augment as a maximum preflow (excess parked inside R and
    then ignored) is not a flow; the pins above reject it."""
    caught = 0
    for seed in range(60):
        dims, conn, tile = RR_FUZZ[seed % len(RR_FUZZ)]
        inst = synth.random_grid(dims, conn, 5000 + seed)
        wrong = oracle.region_reduction(inst, tile, augment="pr")
        ref = oracle.solve_grid(inst)
        if (not (wrong == _two_auxiliary_problems(inst, tile, oracle.solve_pairs)).all()
                or not _semantics_hold(wrong, ref["smin"] == 1, ref["smax"] == 1)):
            caught += 1
    assert caught >= 30


@pytest.mark.parametrize("seed", range(8))
def test_region_reduction_classes_against_global_cuts(seed):
    """All four classes obey the definitions of Sec. 8 against the textbook
    extremal cuts and equal the two auxiliary problems, on blob grids and random
    grids in 2D and 3D.  B^S and B^T are disjoint (asserted inside)."""
    dims, conn, tile = RR_CASES[seed % len(RR_CASES)]
    inst = (synth.blob_grid(dims, conn, 2100 + seed, 4, 3.0, 9.0, zero_frac=0.1) if seed % 2
            else synth.random_grid(dims, conn, 2100 + seed))
    cls = oracle.region_reduction(inst, tile)
    ref = oracle.solve_grid(inst)
    assert _semantics_hold(cls, ref["smin"] == 1, ref["smax"] == 1)
    assert (cls == _two_auxiliary_problems(inst, tile, oracle.solve_pairs)).all()


def test_region_reduction_single_region_decides_everything():
    """One region has no boundary: Augment(s, t) is the whole maximum flow, so
    the strong source nodes are the minimal source side, the strong sink nodes
    the complement of the maximal one, and every other vertex reaches no
    boundary and is reached from none: weak source and weak sink at once."""
    inst = synth.random_grid((14, 15), 8, 2200)
    cls = oracle.region_reduction(inst, (14, 15))
    ref = oracle.solve_grid(inst)
    smin, smax = ref["smin"] == 1, ref["smax"] == 1
    both = oracle.REDUCE_WEAK_SOURCE | oracle.REDUCE_WEAK_SINK
    want = np.where(smin, oracle.REDUCE_STRONG_SOURCE,
                    np.where(~smax, oracle.REDUCE_STRONG_SINK, both)).astype(np.uint8)
    assert (cls == want).all()


# ---------------------------------------------------------------------------
# Region relabel (Alg. 3) on a given state
# ---------------------------------------------------------------------------

def _alg3_brute(n, pu, pv, r_uv, r_vu, rt, region, labels, dinf):
    """The definition of the region relabel, vertex by vertex: the smallest
    stage k such that u reaches T_k in its region network (forward search from u
    over residual arcs inside the region)."""
    from collections import deque
    out_arcs = [[] for _ in range(n)]
    for a, b, x, y in zip(pu, pv, r_uv, r_vu):
        if x > 0:
            out_arcs[a].append(b)
        if y > 0:
            out_arcs[b].append(a)
    res = np.full(n, dinf, np.int64)
    for u in range(n):
        seen = {u}
        q = deque([u])
        best = dinf
        while q:
            x = q.popleft()
            if rt[x] > 0:
                best = 0
                break
            for w in out_arcs[x]:
                if region[w] != region[x]:
                    if labels[w] < dinf:
                        best = min(best, int(labels[w]) + 1)
                elif w not in seen:
                    seen.add(w)
                    q.append(w)
        res[u] = min(best, dinf)
    return res


@pytest.mark.parametrize("seed", range(40))
def test_region_relabel_against_its_definition(seed):
    """oracle.region_relabel (Alg. 3 steps) equals the definition evaluated
    vertex by vertex, on states left by the reference ARD after one or two
    sweeps and on random residual states with random labels."""
    cases = [((9, 11), 4, (3, 4)), ((8, 8), 8, (4, 4)), ((4, 5, 6), 6, (2, 3, 3)), ((12, 7), 4, (5, 7))]
    dims, conn, tile = cases[seed % len(cases)]
    inst = synth.random_grid(dims, conn, 2600 + seed, tile=tile)
    pu, pv, cuv, cvu = oracle.grid_pairs(inst.dims, inst.nbr, synth.offsets_for(len(dims), conn))
    region = oracle.grid_regions(dims, tile)
    rng = np.random.default_rng(seed)
    dinf = 1 + int(rng.integers(3, 30))
    if seed % 2:
        a = oracle.ard_grid(inst, tile=tile, max_sweeps=1 + seed % 3, stop_early=True)
        r_uv, r_vu, rt, labels = a["r_uv"], a["r_vu"], a["rt"], np.minimum(a["labels"], dinf)
    else:
        r_uv = cuv * (rng.random(cuv.size) < 0.7)
        r_vu = cvu * (rng.random(cvu.size) < 0.7)
        rt = inst.ct * (rng.random(inst.n) < 0.15)
        labels = rng.integers(0, dinf + 1, inst.n)
    got = oracle.region_relabel(inst.n, pu, pv, r_uv, r_vu, rt, region, labels, dinf)
    want = _alg3_brute(inst.n, pu, pv, r_uv, r_vu, rt, region, labels, dinf)
    assert (got == want).all()


@pytest.mark.parametrize("seed", range(12))
def test_region_distance_helpers_agree(seed):
    """The tests' two computations of d*B (0-1 breadth-first search, and
    Dijkstra with near-zero weights for the arcs inside a region) agree on the
    states the reference ARD leaves."""
    from tests.helpers import region_distance
    cases = [((9, 11), 4, (3, 4)), ((8, 8), 8, (4, 4)), ((4, 5, 6), 6, (2, 3, 3))]
    dims, conn, tile = cases[seed % len(cases)]
    inst = synth.random_grid(dims, conn, 2700 + seed, tile=tile)
    pu, pv, _, _ = oracle.grid_pairs(inst.dims, inst.nbr, synth.offsets_for(len(dims), conn))
    region = oracle.grid_regions(dims, tile)
    a = oracle.ard_grid(inst, tile=tile, max_sweeps=1 + seed % 3, stop_early=True)
    dinf = 50
    d1 = _region_distance(inst.n, pu, pv, a["r_uv"], a["r_vu"], region, a["rt"], dinf)
    d2 = region_distance(inst.n, pu, pv, a["r_uv"], a["r_vu"], region, a["rt"], dinf)
    assert (d1 == d2).all()


def test_region_reduction_union_matches_alg5():
    """The all-regions-at-once form (two textbook max flows over the regions
    with their arcs to other regions turned into terminal links) gives the
    classes of Alg. 5's steps on every case of the fuzz family and on blob
    grids."""
    for seed in range(300):
        dims, conn, tile = RR_FUZZ[seed % len(RR_FUZZ)]
        inst = synth.random_grid(dims, conn, 5000 + seed)
        assert (oracle.region_reduction_union(inst, tile) == oracle.region_reduction(inst, tile)).all(), seed
    for seed, (dims, conn, tile) in enumerate(RR_CASES):
        inst = synth.blob_grid(dims, conn, 2150 + seed, 4, 3.0, 9.0, zero_frac=0.1)
        assert (oracle.region_reduction_union(inst, tile) == oracle.region_reduction(inst, tile)).all()
