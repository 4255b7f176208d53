"""Host-side validation of the general-network entry point (mf_create_graph):
every malformed input is rejected with its status before any device call, so
these run without a GPU; and the synthetic network generators' contracts."""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def mf():
    from paper_1109_1146_amd import mf as _mf
    _mf.load()
    return _mf


def _base():
    pu = np.array([0, 1, 2], np.int32)
    pv = np.array([1, 2, 3], np.int32)
    c = np.array([3, 4, 5], np.int32)
    cs = np.array([5, 0, 0, 0], np.int32)
    ct = np.array([0, 0, 0, 5], np.int32)
    return dict(n=4, pu=pu, pv=pv, cuv=c.copy(), cvu=c.copy(), cs=cs, ct=ct)


@pytest.mark.parametrize("case", ["self_loop", "vertex_high", "vertex_negative", "negative_cap",
                                  "negative_link", "negative_region", "region_size_zero"])
def test_invalid_networks_are_rejected(mf, case):
    a = _base()
    region, region_size = None, 2
    if case == "self_loop":
        a["pv"][1] = a["pu"][1]
    elif case == "vertex_high":
        a["pv"][2] = 4
    elif case == "vertex_negative":
        a["pu"][0] = -1
    elif case == "negative_cap":
        a["cvu"][0] = -2
    elif case == "negative_link":
        a["ct"][3] = -1
    elif case == "negative_region":
        region = np.array([0, 0, -1, 1], np.int32)
    elif case == "region_size_zero":
        region_size = 0
    with pytest.raises(mf.MFError) as e:
        mf.Graph(region=region, region_size=region_size, **a)
    assert e.value.status == mf.MF_E_INVAL


@pytest.mark.parametrize("case", ["pair_sum", "inflow"])
def test_overflowing_networks_are_rejected(mf, case):
    a = _base()
    big = np.int32(2 ** 31 - 1)
    if case == "pair_sum":
        a["cuv"][0], a["cvu"][0] = big, 1
    else:
        # c(s, 1) plus the capacities into vertex 1 exceed int32
        a["cs"][1] = big - 3
        a["cuv"][0] = 4
    with pytest.raises(mf.MFError) as e:
        mf.Graph(region_size=2, **a)
    assert e.value.status == mf.MF_E_OVERFLOW


def test_random_graph_contract():
    g = synth.random_graph(500, 6, 3)
    assert g.pu.dtype == np.int32 and (g.pu != g.pv).all()
    assert g.pu.min() >= 0 and max(g.pu.max(), g.pv.max()) < g.n
    assert (g.cuv >= 0).all() and (g.cvu >= 0).all() and (g.cs >= 0).all() and (g.ct >= 0).all()
    assert abs(g.npairs - 1500) < 50
    # a deterministic function of the seed
    h = synth.random_graph(500, 6, 3)
    assert all((x == y).all() for x, y in zip(g.arrays(), h.arrays()))


def test_grid26_graph_is_the_26_neighbourhood():
    dims = (4, 5, 6)
    g = synth.grid26_graph(dims, 1)
    D, H, W = dims
    # pairs of a box under the 26-neighbourhood: for each of the 13 half-offsets
    want = sum((D - abs(dz)) * (H - abs(dy)) * (W - abs(dx)) for dz, dy, dx in synth.graphs.OFFSETS_26)
    assert g.npairs == want
    z, r = np.divmod(g.pu, H * W)
    y, x = np.divmod(r, W)
    z2, r2 = np.divmod(g.pv, H * W)
    y2, x2 = np.divmod(r2, W)
    cheb = np.maximum(np.maximum(abs(z - z2), abs(y - y2)), abs(x - x2))
    assert (cheb == 1).all()
    assert g.cuv.max() <= 100 and (g.cuv == g.cvu).all()
    # the oracle solves it (push-relabel and Dinic agree)
    a = oracle.solve_pairs(g.n, *g.arrays())
    b = oracle.solve_pairs(g.n, *g.arrays(), method="dinic")
    assert a["flow"] == b["flow"] and (a["smin"] == b["smin"]).all() and (a["smax"] == b["smax"]).all()


def _write_dimacs(path, N, s, t, arcs, comment=True):
    with open(path, "w") as f:
        if comment:
            f.write("c a max-flow problem\n")
        f.write(f"p max {N} {len(arcs)}\n")
        f.write(f"n {s} s\nn {t} t\n")
        for u, v, c in arcs:
            f.write(f"a {u} {v} {c}\n")


def _random_dimacs(seed, N=40, m=160):
    rng = np.random.default_rng(seed)
    s, t = (int(x) for x in rng.choice(np.arange(1, N + 1), size=2, replace=False))
    arcs = []
    for _ in range(m):
        u, v = (int(x) for x in rng.integers(1, N + 1, size=2))
        arcs.append((u, v, int(rng.integers(0, 30))))
    # every special kind of arc at least once
    arcs += [(s, t, 7), (t, s, 5), (s, s, 3), (t, 1 if t != 1 else 2, 4)]
    return N, s, t, arcs


@pytest.mark.parametrize("seed", range(6))
def test_dimacs_reader_keeps_the_max_flow(mf, tmp_path, seed):
    """The reader's pair form (s- and t-links, s -> t arcs as a constant) has the
    maximum flow of the file's network, computed here on the file's own arcs by
    scipy's maximum_flow, and the vertex numbering is the file's ids without s
    and t in increasing order."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow
    N, s, t, arcs = _random_dimacs(seed)
    path = tmp_path / "g.max"
    _write_dimacs(path, N, s, t, arcs)
    d = mf.read_dimacs(path)
    assert d["n"] == N - 2
    assert list(d["vertex_id"]) == [i for i in range(1, N + 1) if i not in (s, t)]
    assert d["st_capacity"] == sum(c for u, v, c in arcs if u == s and v == t)
    # the file's network, parallel arcs summed, self-arcs dropped
    cap = {}
    for u, v, c in arcs:
        if u != v:
            cap[(u - 1, v - 1)] = cap.get((u - 1, v - 1), 0) + c
    rows, cols, vals = zip(*[(u, v, c) for (u, v), c in cap.items()])
    g = csr_matrix((np.array(vals, np.int32), (np.array(rows), np.array(cols))), shape=(N, N))
    want = maximum_flow(g, s - 1, t - 1).flow_value
    got = oracle.solve_pairs(d["n"], d["pu"], d["pv"], d["cuv"], d["cvu"], d["cs"], d["ct"])["flow"]
    assert got + d["st_capacity"] == want


@pytest.mark.parametrize("case", ["no_problem", "bad_arc", "id_range", "count", "no_sink", "huge_cap",
                                  "missing_file"])
def test_dimacs_reader_rejects_bad_files(mf, tmp_path, case):
    path = tmp_path / "bad.max"
    status = mf.MF_E_INVAL
    if case == "no_problem":
        path.write_text("n 1 s\nn 2 t\na 1 2 3\n")
    elif case == "bad_arc":
        path.write_text("p max 3 1\nn 1 s\nn 2 t\na 1 x 3\n")
    elif case == "id_range":
        path.write_text("p max 3 1\nn 1 s\nn 2 t\na 1 4 3\n")
    elif case == "count":
        path.write_text("p max 3 2\nn 1 s\nn 2 t\na 1 3 3\n")
    elif case == "no_sink":
        path.write_text("p max 3 1\nn 1 s\na 1 3 3\n")
    elif case == "huge_cap":
        path.write_text("p max 3 1\nn 1 s\nn 2 t\na 1 3 3000000000\n")
        status = mf.MF_E_OVERFLOW
    else:
        path = tmp_path / "absent.max"
    with pytest.raises(mf.MFError) as e:
        mf.read_dimacs(path)
    assert e.value.status == status
