"""Host-side measures of the charge-drop analysis (paper_2301_11735_amd.drop)
on configurations whose answers are known by construction; no GPU."""
import numpy as np

from paper_2301_11735_amd import drop

L = 16


def _neel():
    y, x = np.indices((L, L))
    return ((x + y) % 2).astype(np.int8)  # codes 0 (up) / 1 (down) alternating


def test_square_drop_in_a_neel_background():
    c = _neel()
    c[3:9, 5:11] = 2  # a 6 x 6 block of +1 charges
    st = drop.drop_stats(c, L)
    assert st["n_charged"] == 36
    assert st["drop"] == 1.0 and st["clusters"] == 1
    assert st["perim"] == 4 * 6 / 36  # 24 charge-spin bonds around the block
    assert st["af"] == 1.0  # the spins outside keep the Neel pattern


def test_isolated_charges_on_one_sublattice():
    c = _neel()
    y, x = np.indices((L, L))
    c[((x + y) % 2 == 0) & (x % 4 == 0)] = 2  # never two charges side by side
    st = drop.drop_stats(c, L)
    assert st["clusters"] == st["n_charged"] == 32
    assert st["drop"] == 1 / 32
    assert st["perim"] == 4.0


def test_clusters_join_across_the_periodic_edges():
    c = np.zeros((L, L), dtype=np.int8)
    c[7, 0] = c[7, L - 1] = 2        # neighbours through the left/right edge
    c[0, 4] = c[L - 1, 4] = 3        # neighbours through the top/bottom edge
    c[10, 10] = 2
    sizes = drop.charge_clusters(c, L)
    assert sizes.tolist() == [2, 2, 1]


def test_no_charges():
    st = drop.drop_stats(_neel(), L)
    assert st["n_charged"] == 0 and st["drop"] == 0.0 and st["af"] == 1.0


def test_doped_neel_start():
    c = drop.doped_neel(L, 20, 6, seed=5).reshape(L, L)
    assert (c == 2).sum() == 20 and (c == 3).sum() == 6
    y, x = np.indices((L, L))
    spins = c < 2
    assert np.array_equal(c[spins], ((x + y) % 2)[spins])  # the rest keeps the Neel pattern
    assert np.array_equal(drop.doped_neel(L, 20, 6, seed=5), drop.doped_neel(L, 20, 6, seed=5).copy())
