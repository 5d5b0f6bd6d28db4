"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Unique results are compared bit for bit: BFS levels, min-id component labels,
the rooting of a given forest (rst_root_forest vs DFS rooting), list ranks,
and the whole parent array on tree inputs (where the RST is unique).  Where
several answers are valid (which spanning tree hooking returns, which BFS
parent wins a race) the output is checked by the oracle's verifier, and the
forest edges by |F| = n - c plus component equality.
"""
import numpy as np
import pytest

import oracle
from paper_2603_11645_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11645_amd as rst
    return rst.Context(0)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def upload(g):
    return dev(g.offsets_typed()), dev(g.cols)


def small_graphs():
    gs = [
        I.path(1), I.path(2), I.path(257), I.star(300, 0), I.star(300, 299),
        I.grid(13, 29, 0.0, seed=1), I.grid(31, 37, 0.3, seed=2), I.grid_permuted(64, seed=1),
        I.road_mesh(96, 0.15, 0.01, seed=2), I.rmat_lcc(11, 16, seed=3),
        I.long_chain(3000, 0.005, 64, seed=4, offset_bytes=8),
    ]
    for s in range(4):
        gs.append(I.random_graph(1000 + 97 * s, 800, seed=s, connected=False))
        gs.append(I.random_graph(1500 + 13 * s, 4000, seed=50 + s, connected=True))
        gs.append(I.random_tree(2000 + 31 * s, seed=s))
    # isolated vertices only, self-loops and duplicate arcs
    gs.append(I.csr_from_edges(700, np.zeros(0, np.int32), np.zeros(0, np.int32), name="empty"))
    eu = np.array([0, 0, 1, 1, 2, 3, 3, 5], np.int32)
    ev = np.array([0, 1, 1, 2, 2, 4, 4, 5], np.int32)
    g = I.csr_from_edges(6, eu, ev, name="loops")
    # re-add duplicates/self-loops the builder removed (the library must tolerate them)
    cols = np.concatenate([g.cols, np.array([1, 0, 5], np.int32)])
    deg = np.diff(g.offsets)
    src = np.concatenate([np.repeat(np.arange(6), deg), np.array([0, 1, 5])])
    order = np.argsort(src, kind="stable")
    off = np.zeros(7, np.int64)
    np.add.at(off, src + 1, 1)
    gs.append(I.Graph("dups", 6, np.cumsum(off), cols[order]))
    return gs


SMALL = small_graphs()


@pytest.mark.parametrize("gi", range(len(SMALL)))
def test_components_bit_exact(ctx, gi):
    g = SMALL[gi]
    off, cols = upload(g)
    label, k = ctx.components(off, cols)
    k_ref, lab_ref = oracle.components(g.n, g.offsets, g.cols)
    assert k == k_ref
    assert np.array_equal(label.cpu().numpy(), lab_ref)


@pytest.mark.parametrize("gi", range(len(SMALL)))
def test_spanning_forest_edges(ctx, gi):
    g = SMALL[gi]
    off, cols = upload(g)
    label, tu, tv, t = ctx.spanning_forest(off, cols)
    label, tu, tv = label.cpu().numpy(), tu.cpu().numpy(), tv.cpu().numpy()
    k_ref, lab_ref = oracle.components(g.n, g.offsets, g.cols)
    assert np.array_equal(label, lab_ref)
    used = tu >= 0
    assert t == g.n - k_ref == int(used.sum())
    # slots that stayed roots are exactly the component labels
    assert np.array_equal(np.nonzero(~used)[0], np.unique(lab_ref))
    fu, fv = tu[used], tv[used]
    for a, b in zip(fu[:5000], fv[:5000]):
        assert b in g.cols[g.offsets[a]:g.offsets[a + 1]]
    # n - c edges whose components equal G's components form a spanning forest
    f = I.csr_from_edges(g.n, fu, fv)
    assert f.m == t
    k_f, lab_f = oracle.components(g.n, f.offsets, f.cols)
    assert k_f == k_ref and np.array_equal(lab_f, lab_ref)


@pytest.mark.parametrize("gi", range(len(SMALL)))
def test_root_forest_bit_exact(ctx, gi):
    g = SMALL[gi]
    label, fu, fv = oracle.uf_forest(g.n, g.offsets, g.cols)
    rs = np.random.RandomState(gi)
    comps = np.unique(label)
    roots = [int(rs.choice(np.nonzero(label == c)[0])) for c in comps[: max(1, len(comps) // 2)]]
    exp = oracle.dfs_root(g.n, fu, fv, roots)
    par = ctx.root_forest(g.n, dev(fu), dev(fv), dev(np.array(roots, np.int32)))
    assert np.array_equal(par.cpu().numpy(), exp)


@pytest.mark.parametrize("gi", range(len(SMALL)))
def test_spanning_tree_gconn_verified(ctx, gi):
    g = SMALL[gi]
    off, cols = upload(g)
    for root in sorted({0, g.n // 2, g.n - 1}):
        par = ctx.spanning_tree(off, cols, root, "gconn").cpu().numpy()
        k, _ = oracle.components(g.n, g.offsets, g.cols)
        assert ctx.last_status == (0 if k == 1 else -4)
        code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par, [root])
        assert code == 0, (oracle.VERIFY_CODES[code], bad)
        if g.m == g.n - 1 and k == 1:      # a tree: the RST is unique
            _, p_bfs, _ = oracle.bfs(g.n, g.offsets, g.cols, root)
            assert np.array_equal(par, p_bfs)


@pytest.mark.parametrize("gi", range(len(SMALL)))
def test_bfs_levels_bit_exact(ctx, gi):
    g = SMALL[gi]
    off, cols = upload(g)
    root = g.n // 3
    level, parent, st = ctx.bfs(off, cols, root, stats=True)
    level, parent = level.cpu().numpy(), parent.cpu().numpy()
    lref, _, ecc = oracle.bfs(g.n, g.offsets, g.cols, root)
    assert np.array_equal(level, lref)
    assert st["bfs_levels"] == ecc
    reach = lref >= 0
    assert np.all(parent[~reach] == -1)
    assert parent[root] == root
    v = np.nonzero(reach)[0]
    v = v[v != root]
    assert np.all(lref[parent[v]] == lref[v] - 1)
    for x in v[:3000]:
        assert parent[x] in g.cols[g.offsets[x]:g.offsets[x + 1]]


@pytest.mark.parametrize("gi", range(len(SMALL)))
def test_spanning_tree_bfs_verified(ctx, gi):
    g = SMALL[gi]
    off, cols = upload(g)
    par = ctx.spanning_tree(off, cols, 0, "bfs").cpu().numpy()
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par, [0])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)


def test_list_rank_bit_exact(ctx):
    rs = np.random.RandomState(1)
    for A in (1, 2, 255, 256, 257, 4097, 100003):
        order = rs.permutation(A)
        cuts = np.sort(rs.choice(np.arange(1, A), size=min(A - 1, 37), replace=False)) \
            if A > 1 else np.array([], int)
        succ = np.full(A, -1, np.int32)
        for piece in np.split(order, cuts):
            succ[piece[:-1]] = piece[1:]
        exp, _ = oracle.list_rank(succ)
        got = ctx.list_rank(dev(succ)).cpu().numpy()
        assert np.array_equal(got, exp)


def _local_lists(A, block, seed):
    """Lists that mostly stay inside blocks of consecutive ids (tour-like locality)."""
    rs = np.random.RandomState(seed)
    order = np.concatenate([b0 + rs.permutation(min(block, A - b0)) for b0 in range(0, A, block)])
    # a few long-range hops: swap some pieces across blocks
    k = max(1, A // 5000)
    idx = rs.choice(A, size=2 * k, replace=False)
    order[idx[:k]], order[idx[k:]] = order[idx[k:]].copy(), order[idx[:k]].copy()
    return order


def test_list_rank_tiled_locality(ctx):
    """Lists with tile locality (few segment exits) and across many tiles."""
    rs = np.random.RandomState(3)
    for A, block, nlists in ((16384, 16384, 1), (16385, 3000, 3), (200000, 7000, 1),
                             (1 << 20, 20000, 17), (50001, 1, 1)):
        order = _local_lists(A, block, A) if block > 1 else np.arange(A)
        cuts = np.sort(rs.choice(np.arange(1, A), size=nlists - 1, replace=False))
        succ = np.full(A, -1, np.int32)
        for piece in np.split(order, cuts):
            succ[piece[:-1]] = piece[1:]
        exp, k = oracle.list_rank(succ)
        assert k == nlists
        got = ctx.list_rank(dev(succ)).cpu().numpy()
        assert np.array_equal(got, exp)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_spanning_tree_unaligned_cols(ctx, shift):
    """Neighbour ids at an address that is not 16-byte aligned (a view into a
    larger buffer): the tile pass reads them without vector loads; labels and
    the parent array must come out the same as from an aligned copy."""
    for g in (I.road_mesh(160, 0.15, 0.01, seed=9), I.grid(100, 300, 0.2, seed=4)):
        off = dev(g.offsets_typed())
        buf = torch.zeros(g.nnz + shift, dtype=torch.int32, device="cuda")
        buf[shift:] = dev(g.cols)
        cols = buf[shift:]
        assert cols.data_ptr() % 16 != 0
        k_ref, lab_ref = oracle.components(g.n, g.offsets, g.cols)
        label, k = ctx.components(off, cols)
        assert k == k_ref and np.array_equal(label.cpu().numpy(), lab_ref)
        par = ctx.spanning_tree(off, cols, 3, "gconn").cpu().numpy()
        code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par, [3])
        assert code == 0, (oracle.VERIFY_CODES[code], bad)


@pytest.mark.gpu
@pytest.mark.parametrize("shift", [1, 2, 3])
def test_spanning_tree_unaligned_offsets(ctx, shift):
    """Offsets (4- and 8-byte) at an address that is not 16-byte aligned: the
    tile pass reads them without vector loads; labels and the parent array
    must come out right."""
    for g in (I.road_mesh(160, 0.15, 0.01, seed=9), I.grid(100, 300, 0.2, seed=4)):
        cols = dev(g.cols)
        for dt in (torch.int32, torch.int64):
            o = torch.from_numpy(g.offsets.astype(np.int64)).to(dt)
            buf = torch.zeros(g.n + 1 + shift, dtype=dt, device="cuda")
            buf[shift:] = o.cuda()
            off = buf[shift:]
            # int64 with shift 2 lands on a 16-byte boundary again (vector path)
            assert (off.data_ptr() % 16 == 0) == (shift * off.element_size() % 16 == 0)
            k_ref, lab_ref = oracle.components(g.n, g.offsets, g.cols)
            label, k = ctx.components(off, cols)
            assert k == k_ref and np.array_equal(label.cpu().numpy(), lab_ref)
            par = ctx.spanning_tree(off, cols, 3, "gconn").cpu().numpy()
            code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par, [3])
            assert code == 0, (oracle.VERIFY_CODES[code], bad)


def _lists_with_heads(A, heads, rs):
    """Lists over 0..A-1 whose first elements are exactly `heads` (the other
    ids follow in random order, split among the lists)."""
    rest = rs.permutation(np.setdiff1d(np.arange(A), heads))
    cuts = np.sort(rs.choice(np.arange(1, len(rest)), size=len(heads) - 1, replace=False))
    succ = np.full(A, -1, np.int32)
    for h, piece in zip(heads, np.split(rest, cuts)):
        chain = np.concatenate([[h], piece])
        succ[chain[:-1]] = chain[1:]
    return succ


def test_list_rank_tile_rulers(ctx):
    """In-tile ranking at its limits (rulers every 4th arc): a list that runs
    through 12288 arcs off the stride before reaching a strided one (hundreds
    of opened rulers), and tiles with 2047 and 2048 segment heads off the
    stride (the last count that the ruler walk takes and the first that goes
    to all-arc jumping), also in a ragged multi-tile input."""
    rs = np.random.RandomState(5)
    T, S = 16384, 4
    ids = np.arange(T)
    order = np.concatenate([ids[ids % S != 0], ids[ids % S == 0]])
    succ = np.full(T, -1, np.int32)
    succ[order[:-1]] = order[1:]
    cases = [succ]
    off_stride = ids[ids % S != 0]
    for nh in (2047, 2048):
        heads = np.sort(rs.choice(off_stride, size=nh, replace=False))
        cases.append(_lists_with_heads(T, heads, rs))
    # three tiles and a ragged tail, each tile's lists kept inside it
    parts, base = [], 0
    for size, nh in ((T, 2047), (T, 1), (T, 2048), (4101, 9)):
        loc = np.arange(size)
        heads = np.sort(rs.choice(loc[loc % S != 0], size=nh, replace=False))
        sub = _lists_with_heads(size, heads, rs)
        parts.append(np.where(sub >= 0, sub + base, -1).astype(np.int32))
        base += size
    cases.append(np.concatenate(parts))
    for succ in cases:
        exp, _ = oracle.list_rank(succ)
        got = ctx.list_rank(dev(succ)).cpu().numpy()
        assert np.array_equal(got, exp)


def test_list_rank_contracted_heads(ctx):
    """The contracted list of exits ranked in one workgroup, with few and with
    many list heads: lists that cross tiles often (one long list and 40 lists
    over 3 tiles), and 6000 two-element lists inside one tile, whose 6000
    tails form a contracted list of 6000 one-word lists -- more heads than
    the ruler table takes, so that workgroup ranks all words by pointer
    jumping instead."""
    rs = np.random.RandomState(8)
    cases = []
    for A, nl in ((40000, 1), (45000, 40)):
        order = rs.permutation(A)
        cuts = np.sort(rs.choice(np.arange(1, A), size=nl - 1, replace=False))
        succ = np.full(A, -1, np.int32)
        for piece in np.split(order, cuts):
            succ[piece[:-1]] = piece[1:]
        cases.append(succ)
    order = rs.permutation(12000).reshape(-1, 2)
    succ = np.full(12000, -1, np.int32)
    succ[order[:, 0]] = order[:, 1]
    cases.append(succ)
    for succ in cases:
        exp, _ = oracle.list_rank(succ)
        got = ctx.list_rank(dev(succ)).cpu().numpy()
        assert np.array_equal(got, exp)


def _list_with_exits(M, tiles, seed, tile=16384):
    """One list over tiles * tile ids whose tour leaves its tile exactly M - 1
    times (runs alternate over the tiles), so that the tiled ranking has
    exactly M segment exits (the tail included)."""
    rs = np.random.RandomState(seed)
    runs_of = [[] for _ in range(tiles)]
    for t in range(tiles):
        n_t = len(range(t, M, tiles))              # runs r with r % tiles == t
        ids = t * tile + rs.permutation(tile)
        cuts = np.sort(rs.choice(np.arange(1, tile), size=n_t - 1, replace=False))
        runs_of[t] = np.split(ids, cuts)
    order = np.concatenate([runs_of[r % tiles][r // tiles] for r in range(M)])
    succ = np.full(tiles * tile, -1, np.int32)
    succ[order[:-1]] = order[1:]
    return succ


def test_list_rank_contracted_capacity(ctx):
    """Contracted lists of exactly as many words as one workgroup ranks
    (19,456: packed 32-bit words), one more (64-bit words and the multi-block
    rounds), and small ones: the ranks match the oracle in every case."""
    for M, seed in ((19456, 1), (19457, 2), (19455, 3), (3, 4)):
        succ = _list_with_exits(M, 3, seed)
        nxt = succ.astype(np.int64)
        tile_of = np.arange(len(succ)) // 16384
        exits = np.count_nonzero((nxt < 0) | (tile_of != np.where(nxt < 0, -1, nxt) // 16384))
        assert exits == M
        exp, k = oracle.list_rank(succ)
        assert k == 1
        got = ctx.list_rank(dev(succ)).cpu().numpy()
        assert np.array_equal(got, exp), M


def test_heavy_hub_paths(ctx):
    """A star whose centre exceeds the heavy-degree threshold many times over."""
    g = I.star(200001, 7)
    off, cols = upload(g)
    for method in ("gconn", "bfs"):
        par = ctx.spanning_tree(off, cols, 7, method).cpu().numpy()
        assert np.all(par == 7)
    par = ctx.spanning_tree(off, cols, 3, "gconn").cpu().numpy()
    assert par[3] == 3 and par[7] == 3 and np.all(np.delete(par, [3, 7]) == 7)


def test_invalid_arguments(ctx):
    import paper_2603_11645_amd as rst
    g = I.path(10)
    off, cols = upload(g)
    with pytest.raises(rst.RstError):
        ctx.spanning_tree(off, cols, 10)
    with pytest.raises(rst.RstError):
        ctx.spanning_tree(off, cols, -1)
    # two designated roots in one tree
    label, fu, fv = oracle.uf_forest(g.n, g.offsets, g.cols)
    with pytest.raises(rst.RstError):
        ctx.root_forest(g.n, dev(fu), dev(fv), dev(np.array([0, 5], np.int32)))
    # out-of-range neighbour id caught by validation
    bad = g.cols.copy(); bad[3] = 99
    ctx.set_option(rst.OPT_VALIDATE, 1)
    try:
        with pytest.raises(rst.RstError) as ei:
            ctx.spanning_tree(off, dev(bad), 0)
        assert ei.value.code == rst.RST_E_RANGE
    finally:
        ctx.set_option(rst.OPT_VALIDATE, 0)


def test_tunables_do_not_change_results(ctx):
    import paper_2603_11645_amd as rst
    g = I.rmat_lcc(12, 16, seed=5)
    off, cols = upload(g)
    lref, _, _ = oracle.bfs(g.n, g.offsets, g.cols, 0)
    for ept in (1, 2, 4, 8):
        for heavy in (32, 1024):
            ctx.set_option(rst.OPT_RANK_ELEMS_PER_THREAD, ept)
            ctx.set_option(rst.OPT_HEAVY_DEGREE, heavy)
            ctx.set_option(rst.OPT_BFS_LEVELS_PER_SYNC, 3)
            ctx.set_option(rst.OPT_BFS_GRID, 7)
            par = ctx.spanning_tree(off, cols, 0, "gconn").cpu().numpy()
            assert oracle.verify_rst(g.n, g.offsets, g.cols, par, [0])[0] == 0
            level, _ = ctx.bfs(off, cols, 0)
            assert np.array_equal(level.cpu().numpy(), lref)
    ctx.set_option(rst.OPT_RANK_ELEMS_PER_THREAD, 4)
    ctx.set_option(rst.OPT_HEAVY_DEGREE, 1024)
    ctx.set_option(rst.OPT_BFS_LEVELS_PER_SYNC, 32)
    ctx.set_option(rst.OPT_BFS_GRID, 0)
