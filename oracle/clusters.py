"""Void and plastic clusters of a solved grid (Sec. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Phases: void (mask = 1), plastic (matrix pixels on the yield surface, the
plastic mask of a solve) and elastic.  Clusters are sets of pixels of one
phase connected through nearest neighbours (the Hoshen-Kopelman labelling
the paper uses); the "void-plastic" phase is the union of voids and plastic
pixels.  A plastic cluster that touches no void is then connected to its
nearest void, so every cluster holds at least one void.

Readings (the paper is silent on them):
  * the lattice is periodic (the computations are on a periodic cell), so
    neighbours wrap around the edges;
  * "nearest" is the periodic Euclidean distance between pixel centres,
    from any pixel of the cluster to any void pixel; ties go to the void
    pixel of smallest index x2 * L + x1;
  * a cluster's label is the smallest pixel index it holds (canonical, so
    labellings compare exactly);
  * the largest cluster "spans" an axis when it occupies every column
    (every row) of the lattice.

Indicators of Sec. 3: the void-plastic fraction v_p and f_p = v_p / (1 - f),
v_max (largest void-plastic cluster / L^2), i (void clusters with no plastic
neighbour / void clusters) and n (void-plastic clusters / void clusters of
the unloaded grid, i.e. the void phase alone).
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def _uf_find(parent, x):
    while parent[x] != x:
        parent[x] = parent[parent[x]]
        x = parent[x]
    return x


def label_periodic(phase: np.ndarray) -> np.ndarray:
    """Periodic 4-connected components; label = smallest pixel index, -1 outside."""
    phase = np.asarray(phase).astype(bool)
    L = phase.shape[0]
    lab, n = ndimage.label(phase, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    parent = list(range(n + 1))

    def union(a, b):
        a, b = _uf_find(parent, a), _uf_find(parent, b)
        if a != b:
            parent[max(a, b)] = min(a, b)

    for i in range(L):   # wrap-around bonds
        if lab[i, 0] and lab[i, L - 1]:
            union(lab[i, 0], lab[i, L - 1])
        if lab[0, i] and lab[L - 1, i]:
            union(lab[0, i], lab[L - 1, i])
    root = np.array([_uf_find(parent, k) for k in range(n + 1)])
    comp = root[lab]
    out = np.full(L * L, -1, dtype=np.int64)
    flat = comp.ravel()
    idx = np.arange(L * L)
    inside = flat > 0
    # canonical label: smallest pixel index of the component
    mins = np.full(n + 1, L * L, dtype=np.int64)
    np.minimum.at(mins, flat[inside], idx[inside])
    out[inside] = mins[flat[inside]]
    return out.reshape(L, L)


def label_bfs(phase: np.ndarray) -> np.ndarray:
    """The same labelling by breadth-first search (independent check, small L)."""
    phase = np.asarray(phase).astype(bool)
    L = phase.shape[0]
    out = np.full((L, L), -1, dtype=np.int64)
    for p in range(L * L):
        y, x = divmod(p, L)
        if not phase[y, x] or out[y, x] >= 0:
            continue
        out[y, x] = p          # p is the smallest index of its component (visited in order)
        stack = [(y, x)]
        while stack:
            cy, cx = stack.pop()
            for ny, nx in ((cy, (cx + 1) % L), (cy, (cx - 1) % L), ((cy + 1) % L, cx), ((cy - 1) % L, cx)):
                if phase[ny, nx] and out[ny, nx] < 0:
                    out[ny, nx] = p
                    stack.append((ny, nx))
    return out


def nearest_void(L, pixels, void_idx):
    """(d2, void index) of the nearest void pixel to any of `pixels` (flat
    indices), periodic Euclidean distance, ties to the smallest void index."""
    py, px = np.divmod(np.asarray(pixels), L)
    vy, vx = np.divmod(np.asarray(void_idx), L)
    dy = np.abs(py[:, None] - vy[None, :])
    dx = np.abs(px[:, None] - vx[None, :])
    dy = np.minimum(dy, L - dy)
    dx = np.minimum(dx, L - dx)
    d2 = (dx * dx + dy * dy).min(axis=0)          # per void pixel: distance to the cluster
    best = d2.min()
    v = np.asarray(void_idx)[d2 == best].min()
    return int(best), int(v)


def nearest_void_local(L, pixels, void_flat, r_max=64):
    """The result of nearest_void, from the voids near the cluster only.

    Offsets (oy, ox) with |oy|, |ox| <= r around every cluster pixel are
    searched, r = 1, 2, 4, ...; a void at periodic distance d <= r from some
    cluster pixel lies in that pixel's window, so once the smallest squared
    offset found is <= r^2 it is the distance to the cluster and every void
    at that distance is among the candidates (ties to the smallest index as
    in nearest_void).  For r < L / 2 every offset is its own minimal periodic
    image.  Beyond r_max (very sparse voids) it defers to nearest_void."""
    py, px = np.divmod(np.asarray(pixels, dtype=np.int64), L)
    r = 1
    while 2 * r < L and r <= r_max:
        off = np.arange(-r, r + 1)
        oy, ox = np.meshgrid(off, off, indexing="ij")
        oy, ox = oy.ravel(), ox.ravel()
        vid = ((py[:, None] + oy[None, :]) % L) * L + (px[:, None] + ox[None, :]) % L
        d2 = np.broadcast_to(oy * oy + ox * ox, vid.shape)
        hit = void_flat[vid]
        if hit.any():
            best = int(d2[hit].min())
            if best <= r * r:
                return best, int(vid[hit & (d2 == best)].min())
        r *= 2
    return nearest_void(L, pixels, np.flatnonzero(void_flat))


def analyze(void: np.ndarray, plastic: np.ndarray):
    """Cluster labels (after attachment) and the counts behind the indicators."""
    void = np.asarray(void).astype(bool)
    plastic = np.asarray(plastic).astype(bool) & ~void
    L = void.shape[0]
    npx = L * L
    vp = void | plastic
    void_lab = label_periodic(void)
    raw = label_periodic(vp)
    roots = np.unique(raw[raw >= 0])
    flat = raw.ravel()
    vflat, pflat = void.ravel(), plastic.ravel()
    # raw labels are pixel indices: flag the clusters holding a void / a plastic pixel
    has_void = np.zeros(npx, dtype=bool)
    has_void[flat[vflat]] = True
    has_plastic = np.zeros(npx, dtype=bool)
    has_plastic[flat[pflat]] = True
    # the pixels of every raw cluster, grouped
    order = np.argsort(flat, kind="stable")
    sorted_lab = flat[order]
    # attach plastic-only clusters to the cluster of their nearest void
    parent = {int(r): int(r) for r in roots}

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    plastic_only = [int(r) for r in roots if not has_void[r]]
    if vflat.any():
        for r in plastic_only:
            lo, hi = np.searchsorted(sorted_lab, [r, r + 1])
            _, v = nearest_void_local(L, order[lo:hi], vflat)
            a, b = find(r), find(int(flat[v]))
            if a != b:
                parent[max(a, b)] = min(a, b)
    rep = np.full(npx, -1, dtype=np.int64)
    for r in roots:
        rep[r] = find(int(r))
    inside = flat >= 0
    comp = np.where(inside, rep[np.where(inside, flat, 0)], -1)
    # canonical labels again: smallest pixel index of each merged component
    mins = np.full(npx, npx, dtype=np.int64)
    np.minimum.at(mins, comp[inside], np.flatnonzero(inside))
    final = np.full(npx, -1, dtype=np.int64)
    final[inside] = mins[comp[inside]]
    final = final.reshape(L, L)
    labs, sizes = np.unique(final[final >= 0], return_counts=True)
    if len(labs):
        big = sizes.max()
        largest_label = int(labs[sizes == big].min())
        cells = final == largest_label
        spans_x1 = bool(cells.any(axis=0).all())
        spans_x2 = bool(cells.any(axis=1).all())
    else:
        big, largest_label, spans_x1, spans_x2 = 0, -1, False, False
    n_void_clusters = len(np.unique(void_lab[void_lab >= 0]))
    stats = dict(
        n_void=int(void.sum()), n_plastic=int(plastic.sum()),
        n_void_clusters=n_void_clusters,
        n_clusters_raw=len(roots),
        n_isolated_void_clusters=int(np.count_nonzero(has_void[roots] & ~has_plastic[roots])),
        n_plastic_only_clusters=len(plastic_only),
        n_clusters=len(labs), largest=int(big), largest_label=largest_label,
        spans_x1=spans_x1, spans_x2=spans_x2,
    )
    return final, stats


def indicators(stats, L, f=None):
    """Sec. 3 indicators from the counts (f defaults to the void fraction)."""
    npx = L * L
    f = stats["n_void"] / npx if f is None else f
    vp = (stats["n_void"] + stats["n_plastic"]) / npx
    nvc = max(stats["n_void_clusters"], 1)
    return dict(v_p=vp, f_p=vp / (1.0 - f), v_max=stats["largest"] / npx,
                i=stats["n_isolated_void_clusters"] / nvc, n=stats["n_clusters"] / nvc)


def path_derivatives(x, y):
    """First and second derivatives along a loading path (Sec. 3: r = dn/d eps0
    and the curvature -d2 sigma0 / d eps0^2 of the mean stress curve).  Each
    point takes the quadratic through three consecutive samples (its own and
    its neighbours; the first or last three at the ends) and differentiates
    it: a local fit with numpy.polyfit, not a difference formula."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    assert n >= 3 and np.all(np.diff(x) > 0)
    dy = np.empty(n)
    d2y = np.empty(n)
    for k in range(n):
        c = min(max(k, 1), n - 2)
        xs, ys = x[c - 1:c + 2], y[c - 1:c + 2]
        x0 = xs[1]                                   # centre the fit for conditioning
        coef = np.polyfit(xs - x0, ys, 2)            # exact through the three points
        dy[k] = np.polyval(np.polyder(coef), x[k] - x0)
        d2y[k] = 2.0 * coef[0]
    return dy, d2y


def path_indicators(eps0, n, sigma0):
    """r = dn/d eps0 and -d2 sigma0 / d eps0^2 at each step of a loading path."""
    r, _ = path_derivatives(eps0, n)
    _, s2 = path_derivatives(eps0, sigma0)
    return dict(r=r, minus_d2sigma0=-s2)
