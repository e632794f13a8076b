"""Geometry of the tile-binned particle/grid transfer (host-side, no GPU).

The transfer (Methods, fluid-filament interaction; read as Peskin's 4-point
kernel) puts a node whose home cell is h = floor(x) on the cells h-1 .. h+2
of each periodic axis.  The tile kernels of the binned transfer keep, per
tile (side 16, 32 or 64 cells), only the nodes whose home cell passes a keep rule, place each
kept node's four cells at window offsets d .. d+3 with d = (h - 1 - o) mod n
(o: window origin, three cells before the needed range) inside an LDS window
of side need + 6, and read the records from the home-tile bins of a few tile
columns.  The rules are separable, so one axis at a time suffices.

For every axis length 1..199, every tile and every Gaussian radius 1..8 this
checks, for the filter (needed: the density region of the tile, its
central-difference ring and R cells of filter support each side) and for the
spread (needed: the tile's own cells):
  * every node touching a needed cell is kept, its bin column is read, and
    its contribution lands on a window cell that the kernel reads for that
    grid cell (the single image when need + 3 <= n, else an image that the
    read sums);
  * every kept node's four cells stay inside the window;
  * the spread's kept nodes are kept by the filter and lie in the filter's
    bins (the filter hands the spread its record list);
  * a tile reads at most four bin columns in at most two runs, so a tile's
    bin set has at most eight runs (for every tile side: the margins, at most
    R + 3 = 11 cells, are shorter than a tile).

Two-layer markers (a marker's home cell is its node's shifted by -1, 0 or 1
cell, as the marker offset is at most one cell): the spread keeps nodes one
cell further out on each side (origin four cells before the tile) and
stages their gradient over a window two cells wider; a marker goes into the
one-layer window by the one-layer rule applied to its own home; the
spread's bins are those of the widened node range, and the integrate and
MDF gathers stage the velocity one cell wider on each side.  Checked: every
marker touching a tile cell is spread, its node kept and in the bins, its
contribution lands where the tile's cell is read, every kept node's
gradient support and every spread marker stay inside their windows, the
kept nodes lie in the filter's keep set and bins (the filter writes the
spread lists), and the gather supports stay inside the staged field.
"""
import numpy as np
import pytest

TILES = [16, 32, 64]
MAX_COLS = {16: 4, 32: 4, 64: 4}      # the kernels' TileCfg<TILE>::kMaxCols


def covering_columns(lo, hi, n, TILE=32):
    """Tile columns holding cells lo..hi of a periodic axis, capped at the
    kernels' column limit (the check below asserts the cap never binds)."""
    cap = MAX_COLS[TILE] + 1
    t = []
    if hi - lo + 1 >= n:
        k = 0
        while k * TILE < n and len(t) < cap:
            t.append(k)
            k += 1
        return t
    c = lo
    while c <= hi and len(t) < cap:
        cc = c % n
        tt = cc // TILE
        if tt not in t:
            t.append(tt)
        c += min((tt + 1) * TILE, n) - cc
    return t


def runs(cols):
    """Runs of consecutive column indices in the order listed."""
    r = 0
    for i, c in enumerate(cols):
        if i == 0 or c != cols[i - 1] + 1:
            r += 1
    return r


def check_reader(n, first, need, cols, bound_shift=0, side_shift=0, TILE=32):
    """Keep rule, window placement and bins of one reader on one axis.

    first: first needed cell (unwrapped); need: needed cells.  Returns the
    keep mask over home cells 0..n-1.  The shifts plant mistakes."""
    o = (first - 3) % n
    side = need + 6 + side_shift
    single = need + 3 <= n
    bound = (need + 2 if single else n) + bound_shift
    h = np.arange(n)
    d = (h - 1 - o) % n
    kept = d <= bound
    assert np.all(d[kept] + 3 <= side - 1), (n, first, need)
    in_bins = np.isin(h // TILE, cols)
    for k in range(4):
        c = (h - 1 + k) % n                   # grid cell of the contribution
        p = d + k                             # window offset it lands on
        rel = (c - first) % n
        needed = rel < need if need < n else np.ones(n, bool)
        assert np.all(kept[needed]), (n, first, need, k)
        assert np.all(in_bins[needed]), (n, first, need, k, cols)
        if single:
            assert np.all(p[needed] == 3 + rel[needed]), (n, first, need, k)
        else:
            assert np.all((p[needed] - 3 - rel[needed]) % n == 0), (n, first, need, k)
    return kept


def check_marker_reader(n, x0, tw, cols, TILE=32, node_bound_shift=0, g_side_shift=0):
    """Two-layer spread of the tile [x0, x0 + tw) on one axis: returns the
    node keep mask over home cells 0..n-1.  The shifts plant mistakes."""
    h = np.arange(n)
    dn = (h - 1 - (x0 - 4)) % n                # node support origin in the gradient window
    nbound = (tw + 4 if tw + 5 <= n else n) + node_bound_shift
    nkept = dn <= nbound
    g_side = TILE + 8 + g_side_shift
    assert np.all(dn[nkept] + 3 <= g_side - 1), (n, x0, tw)
    in_bins = np.isin(h // TILE, cols)
    single = tw + 3 <= n
    mbound = tw + 2 if single else n
    for s in (-1, 0, 1):
        mh = h + s                             # marker home, unwrapped
        dm = (mh - 1 - (x0 - 3)) % n           # marker support origin in the force window
        spread = dm <= mbound
        assert np.all(dm[spread] + 3 <= TILE + 5), (n, x0, tw, s)
        for k in range(4):
            c = (mh - 1 + k) % n
            p = dm + k
            rel = (c - x0) % n
            needed = rel < tw if tw < n else np.ones(n, bool)
            assert np.all(spread[needed]), (n, x0, tw, s, k)
            assert np.all(nkept[needed]), (n, x0, tw, s, k)
            assert np.all(in_bins[needed]), (n, x0, tw, s, k, cols)
            if single:
                assert np.all(p[needed] == 3 + rel[needed]), (n, x0, tw, s, k)
            else:
                assert np.all((p[needed] - 3 - rel[needed]) % n == 0), (n, x0, tw, s, k)
        # gathers of the tile's own nodes: staged cells x0 - 2 .. x0 + TILE + 2
        own = (h >= x0) & (h < x0 + tw)
        lo = mh[own] - 1 - (x0 - 2)
        assert np.all(lo >= 0) and np.all(lo + 3 <= TILE + 4), (n, x0, tw, s)
    return nkept


@pytest.mark.parametrize("TILE", TILES)
def test_binned_transfer_windows_and_bins(TILE):
    cases = 0
    top = 200 if TILE <= 32 else 300
    for n in range(1, top):
        for x0 in range(0, n, TILE):
            tw = min(TILE, n - x0)
            sp_cols = covering_columns(x0 - 3, x0 + tw + 1, n, TILE)   # widened for the markers
            assert len(sp_cols) <= MAX_COLS[TILE] and runs(sp_cols) <= 2
            sp_kept = check_reader(n, x0, tw, sp_cols, TILE=TILE)
            mk_kept = check_marker_reader(n, x0, tw, sp_cols, TILE=TILE)
            for R in range(1, 9):
                reg = TILE + 2 + 2 * R
                xo = x0 - R - 1
                f_cols = covering_columns(xo - 2, xo + reg, n, TILE)
                assert len(f_cols) <= MAX_COLS[TILE] and runs(f_cols) <= 2
                f_kept = check_reader(n, xo, reg, f_cols, TILE=TILE)
                h = np.arange(n)
                assert np.all(f_kept[sp_kept]), (n, x0, R)
                assert np.all(np.isin(h[sp_kept] // TILE, f_cols)), (n, x0, R)
                assert np.all(f_kept[mk_kept]), (n, x0, R)
                assert np.all(np.isin(h[mk_kept] // TILE, f_cols)), (n, x0, R)
                cases += 1
    assert cases > 2000


@pytest.mark.parametrize("TILE", TILES)
def test_column_limit_is_reached(TILE):
    # the column and run limits are tight: some axis and tile need them all
    worst = 0
    for n in range(1, 300):
        for x0 in range(0, n, TILE):
            R = 8
            reg = TILE + 2 + 2 * R
            worst = max(worst, len(covering_columns(x0 - R - 3, x0 - R - 1 + reg, n, TILE)))
    assert worst == MAX_COLS[TILE]


@pytest.mark.parametrize("mistake", ["dropped column", "keep bound one short", "window one short"])
def test_planted_mistakes_are_caught(mistake):
    # the check is sharp: a filter tile with one bin column left out, a keep
    # bound one cell short or a window one cell short fails it
    TILE = 32
    n, x0, R = 160, 64, 4
    reg = TILE + 2 + 2 * R
    cols = covering_columns(x0 - R - 1 - 2, x0 - R - 1 + reg, n)
    assert len(cols) == 3
    check_reader(n, x0 - R - 1, reg, cols)
    kw = {}
    if mistake == "dropped column":
        cols = cols[:-1]
    elif mistake == "keep bound one short":
        kw = {"bound_shift": -1}
    else:
        kw = {"side_shift": -1}
    with pytest.raises(AssertionError):
        check_reader(n, x0 - R - 1, reg, cols, **kw)


@pytest.mark.parametrize("mistake", ["node keep one short", "gradient window one short", "one-layer bins"])
def test_planted_marker_mistakes_are_caught(mistake):
    # the marker check is sharp too: a node keep bound one cell short, a
    # gradient window one cell short, or the one-layer spread bins on an
    # axis whose last tile is narrower than the extra cell fail it
    TILE = 32
    if mistake == "one-layer bins":
        n, x0 = 98, 0                          # last tile 2 cells wide: home 95 lies in tile 2
        tw = min(TILE, n - x0)
        check_marker_reader(n, x0, tw, covering_columns(x0 - 3, x0 + tw + 1, n, TILE))
        with pytest.raises(AssertionError):
            check_marker_reader(n, x0, tw, covering_columns(x0 - 2, x0 + tw, n, TILE))
        return
    n, x0 = 160, 64
    tw = TILE
    cols = covering_columns(x0 - 3, x0 + tw + 1, n)
    check_marker_reader(n, x0, tw, cols)
    kw = {"node_bound_shift": -1} if mistake == "node keep one short" else {"g_side_shift": -1}
    with pytest.raises(AssertionError):
        check_marker_reader(n, x0, tw, cols, **kw)
