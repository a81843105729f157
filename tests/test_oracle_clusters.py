"""Pins of the cluster-analysis oracle (Sec. 3).

Labelling: the scipy-based periodic labelling against an independent
breadth-first search, and against scipy's own non-periodic labelling where
no cluster touches the edges.  Attachment: hand-built cases with a known
nearest void (and a tie), plus identities that hold for any input.
"""
import numpy as np
import pytest

from oracle import clusters
from paper_0802_2488_amd import synth


def partition(lab):
    """Labels -> frozenset of frozensets of pixel indices (label values ignored)."""
    flat = lab.ravel()
    groups = {}
    for i, v in enumerate(flat):
        if v >= 0:
            groups.setdefault(int(v), []).append(i)
    return frozenset(frozenset(g) for g in groups.values())


@pytest.mark.parametrize("L,f,seed", [(8, 0.3, 0), (8, 0.6, 1), (16, 0.45, 2), (24, 0.55, 3), (5, 0.5, 4)])
def test_periodic_labels_equal_breadth_first_search(L, f, seed):
    phase = synth.bernoulli_mask(L, f, seed).astype(bool)
    a = clusters.label_periodic(phase)
    b = clusters.label_bfs(phase)
    assert np.array_equal(a, b)


def test_no_wrap_bonds_matches_scipy_non_periodic():
    from scipy import ndimage
    L = 20
    phase = synth.bernoulli_mask(L, 0.5, 7).astype(bool)
    phase[0, :] = phase[-1, :] = phase[:, 0] = phase[:, -1] = False
    lab, n = ndimage.label(phase)
    ref = np.where(lab > 0, lab, -1)
    assert partition(clusters.label_periodic(phase)) == partition(ref)


def test_wrap_around_bonds_join_clusters():
    L = 8
    phase = np.zeros((L, L), bool)
    phase[3, :2] = True
    phase[3, -2:] = True          # touches the first two pixels through the x1 edge
    phase[0, 5] = phase[L - 1, 5] = True   # and through the x2 edge
    lab = clusters.label_periodic(phase)
    assert len(np.unique(lab[lab >= 0])) == 2
    assert lab[3, 0] == lab[3, L - 1] == 3 * L
    assert lab[0, 5] == lab[L - 1, 5] == 5


def test_plastic_cluster_joins_its_nearest_void():
    L = 12
    void = np.zeros((L, L), bool)
    plastic = np.zeros((L, L), bool)
    void[1, 1] = True                 # index 13
    void[1, 11] = True                # index 23
    plastic[6, 0] = plastic[6, 11] = True       # one plastic cluster across the x1 edge
    plastic[1, 2] = True              # touches void 13
    lab, st = clusters.analyze(void, plastic)
    assert st["n_void_clusters"] == 2
    assert st["n_clusters_raw"] == 3
    assert st["n_plastic_only_clusters"] == 1
    assert st["n_isolated_void_clusters"] == 1     # the void at index 23
    # squared distances: (6, 11) to void 23 is 25; (6, 0) to void 13 is 26
    assert lab[6, 0] == lab[6, 11] == lab[1, 11] == 23
    assert st["n_clusters"] == 2 and st["largest"] == 3


def test_attachment_tie_goes_to_the_smaller_void_index():
    L = 9
    void = np.zeros((L, L), bool)
    plastic = np.zeros((L, L), bool)
    void[4, 1] = void[4, 7] = True    # equidistant from (4, 4)
    plastic[4, 4] = True
    lab, st = clusters.analyze(void, plastic)
    assert lab[4, 4] == 4 * L + 1


def _analyze_by_definition(void, plastic):
    """Slow reference of clusters.analyze for small grids: breadth-first
    labels, one scan per cluster, the brute-force nearest void."""
    L = void.shape[0]
    npx = L * L
    raw = clusters.label_bfs(void | plastic).ravel()
    vflat, pflat = void.ravel(), plastic.ravel()
    roots = sorted(set(int(x) for x in raw if x >= 0))
    void_idx = np.flatnonzero(vflat)
    parent = {r: r for r in roots}

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    only = [r for r in roots if not vflat[raw == r].any()]
    if len(void_idx):
        for r in only:
            _, v = clusters.nearest_void(L, np.flatnonzero(raw == r), void_idx)
            a, b = find(r), find(int(raw[v]))
            if a != b:
                parent[max(a, b)] = min(a, b)
    comp = np.array([find(int(x)) if x >= 0 else -1 for x in raw])
    final = np.full(npx, -1, dtype=np.int64)
    for c in set(comp[comp >= 0].tolist()):
        final[comp == c] = np.flatnonzero(comp == c).min()
    isolated = sum(1 for r in roots if vflat[raw == r].any() and not pflat[raw == r].any())
    return final.reshape(L, L), len(only), isolated


@pytest.mark.parametrize("L,fv,fp,seed", [(8, 0.1, 0.4, 0), (16, 0.05, 0.3, 1), (16, 0.02, 0.5, 2),
                                          (32, 0.03, 0.45, 3), (32, 0.005, 0.3, 4), (24, 0.2, 0.2, 5)])
def test_analyze_equals_its_definition(L, fv, fp, seed):
    """The grouped, vectorised analysis against the plain per-cluster one."""
    void = synth.bernoulli_mask(L, fv, seed).astype(bool)
    plastic = synth.bernoulli_mask(L, fp, 500 + seed).astype(bool) & ~void
    lab, st = clusters.analyze(void, plastic)
    ref, n_only, isolated = _analyze_by_definition(void, plastic)
    assert np.array_equal(lab, ref)
    assert st["n_plastic_only_clusters"] == n_only and st["n_isolated_void_clusters"] == isolated


@pytest.mark.parametrize("seed", range(8))
def test_local_nearest_void_equals_brute_force(seed):
    """Windowed search against the full distance scan, with ties: sparse and
    dense voids, clusters across the periodic edge, lattice-symmetric voids."""
    tie = np.zeros((16, 16), dtype=bool)
    tie[5, 2] = tie[5, 8] = True   # both 3 pixels from (5, 5): the smaller index wins
    assert clusters.nearest_void_local(16, np.array([5 * 16 + 5]), tie.ravel()) == (9, 5 * 16 + 2)
    rng = np.random.default_rng(seed)
    L = int(rng.choice([8, 16, 32, 64]))
    void = rng.random((L, L)) < rng.choice([0.003, 0.02, 0.2])
    if seed % 3 == 0:   # symmetric pair of voids around a pixel: an exact tie
        void[:] = False
        c = int(rng.integers(L))
        void[c, (c + 3) % L] = void[c, (c - 3) % L] = True
    if not void.any():
        void[0, 0] = True
    free = np.flatnonzero(~void.ravel())
    for k in (1, 3, 12):
        start = int(rng.choice(free))
        y, x = divmod(start, L)
        pix = {start}
        for _ in range(k - 1):   # a random walk, wrapping around the edges
            y, x = (y + int(rng.integers(-1, 2))) % L, (x + int(rng.integers(-1, 2))) % L
            if not void[y, x]:
                pix.add(y * L + x)
        pix = np.array(sorted(pix))
        assert clusters.nearest_void_local(L, pix, void.ravel()) == \
            clusters.nearest_void(L, pix, np.flatnonzero(void.ravel()))


@pytest.mark.parametrize("seed", range(4))
def test_counting_identities_and_symmetries(seed):
    L = 32
    void = synth.bernoulli_mask(L, 0.08, seed).astype(bool)
    plastic = synth.bernoulli_mask(L, 0.25, 100 + seed).astype(bool) & ~void
    lab, st = clusters.analyze(void, plastic)
    # plastic-only clusters each merge into exactly one void-holding cluster
    assert st["n_clusters"] == st["n_clusters_raw"] - st["n_plastic_only_clusters"]
    assert st["n_void"] + st["n_plastic"] == int((lab >= 0).sum())
    # every final cluster holds a void
    for r in np.unique(lab[lab >= 0]):
        assert void[lab == r].any()
    # translation and transposition leave every tie-independent count unchanged
    keys = ("n_void", "n_plastic", "n_void_clusters", "n_clusters_raw", "n_isolated_void_clusters",
            "n_plastic_only_clusters", "n_clusters")
    for tv, tp in ((np.roll(void, (3, -5), (0, 1)), np.roll(plastic, (3, -5), (0, 1))), (void.T, plastic.T)):
        _, s2 = clusters.analyze(tv, tp)
        assert all(s2[k] == st[k] for k in keys)


def test_indicators_of_an_unloaded_grid():
    L = 32
    void = synth.bernoulli_mask(L, 0.1, 3).astype(bool)
    _, st = clusters.analyze(void, np.zeros_like(void))
    ind = clusters.indicators(st, L)
    assert ind["i"] == 1.0 and ind["n"] == 1.0
    f = void.mean()
    assert ind["f_p"] == pytest.approx(f / (1 - f))


def test_path_derivatives_exact_for_quadratics():
    rng = np.random.default_rng(3)
    x = np.cumsum(rng.uniform(0.05, 0.5, 12))
    a, b, c = 0.4, -2.0, 1.5
    dy, d2y = clusters.path_derivatives(x, a + b * x + c * x * x)
    np.testing.assert_allclose(dy, b + 2 * c * x, rtol=0, atol=1e-10)
    np.testing.assert_allclose(d2y, 2 * c, rtol=0, atol=1e-9)


def test_path_derivatives_uniform_grid_and_second_order():
    # on a uniform grid the inner slope is the central difference
    x = np.linspace(0.0, 1.0, 11)
    y = np.exp(x)
    dy, d2y = clusters.path_derivatives(x, y)
    h = x[1] - x[0]
    np.testing.assert_allclose(dy[1:-1], (y[2:] - y[:-2]) / (2 * h), rtol=1e-12)
    np.testing.assert_allclose(d2y[1:-1], (y[2:] - 2 * y[1:-1] + y[:-2]) / h**2, rtol=1e-9)
    # errors fall as h^2 inside (ratio ~4 when h halves)
    errs = []
    for m in (21, 41):
        x = np.linspace(0.0, 1.0, m)
        dy, _ = clusters.path_derivatives(x, np.sin(x))
        errs.append(np.abs(dy[1:-1] - np.cos(x[1:-1])).max())
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_path_indicators_of_linear_curves():
    eps0 = np.array([0.1, 0.25, 0.3, 0.5, 0.8])
    ind = clusters.path_indicators(eps0, 2.0 - 0.5 * eps0, 3.0 * eps0 + 1.0)
    np.testing.assert_allclose(ind["r"], -0.5, atol=1e-12)
    np.testing.assert_allclose(ind["minus_d2sigma0"], 0.0, atol=1e-9)


def _hand_built_grid():
    """L = 8 periodic grid, (x2, x1) = (row, column).  Voids: A = (1, 1),
    B = (4, 4) + (4, 5), C = (6, 1).  Plastic: (1, 2) next to A, a path
    (2, 1) (3, 1) (4, 1) (4, 2) (4, 3) joining A to B, and a plastic-only
    pair (2, 6) (3, 6) whose nearest void is (4, 5) (distance^2 = 2 from
    (3, 6); A is at 10 from (2, 6), C at 18)."""
    L = 8
    void = np.zeros((L, L), bool)
    plastic = np.zeros((L, L), bool)
    for y, x in ((1, 1), (4, 4), (4, 5), (6, 1)):
        void[y, x] = True
    for y, x in ((1, 2), (2, 1), (3, 1), (4, 1), (4, 2), (4, 3), (2, 6), (3, 6)):
        plastic[y, x] = True
    return L, void, plastic


def test_indicators_of_a_hand_built_grid():
    """Sec. 3 indicators counted by hand: 3 void clusters (A, B, C); the
    void-plastic phase holds A-path-B (9 pixels), C, and the plastic-only pair
    that joins B's cluster, so 2 clusters, the largest of 11 pixels; only C
    has no plastic neighbour.  A wrong normalisation (void pixels instead of
    void clusters), the largest cluster taken before attachment, or f_p without
    the 1 - f factor each fail one of these values."""
    L, void, plastic = _hand_built_grid()
    lab, st = clusters.analyze(void, plastic)
    assert (st["n_void"], st["n_plastic"], st["n_void_clusters"]) == (4, 8, 3)
    assert (st["n_clusters_raw"], st["n_isolated_void_clusters"], st["n_plastic_only_clusters"]) == (3, 1, 1)
    assert (st["n_clusters"], st["largest"]) == (2, 11)
    assert lab[2, 6] == lab[4, 5] == lab[1, 1] and lab[6, 1] != lab[1, 1]
    ind = clusters.indicators(st, L)
    assert ind["v_p"] == pytest.approx(12 / 64, abs=1e-15)
    assert ind["f_p"] == pytest.approx((12 / 64) / (1 - 4 / 64), abs=1e-15)
    assert ind["v_max"] == pytest.approx(11 / 64, abs=1e-15)
    assert ind["i"] == pytest.approx(1 / 3, abs=1e-15)
    assert ind["n"] == pytest.approx(2 / 3, abs=1e-15)
    # an imposed f (the nominal porosity) replaces the realised one in f_p only
    ind2 = clusters.indicators(st, L, f=0.1)
    assert ind2["f_p"] == pytest.approx((12 / 64) / 0.9, abs=1e-15)
    assert ind2["v_max"] == ind["v_max"]
