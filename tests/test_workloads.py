"""The seeded workload generators follow their stated recipes (no GPU needed)."""
import numpy as np

import workloads


def test_c4_tiles_recipe():
    tiles = workloads.c4()
    assert len(tiles) == 2048 and [t.index for t in tiles] == list(range(2048))
    shapes = {t.G.shape for t in tiles}
    assert shapes <= {(m, n) for m in workloads.C4_SIZES for n in workloads.C4_SIZES}
    assert len(shapes) == 16
    for t in tiles[:64]:
        m, n = t.G.shape
        assert t.V.shape == (256, m)
        assert np.all(t.G >= workloads.G_MIN) and np.all(t.G <= workloads.G_MAX * (1 + 1e-12))
        # differential pairs: at most one device of a pair carries weight
        gp, gm = t.G[:, 0::2], t.G[:, 1::2]
        assert np.all((gp == workloads.G_MIN) | (gm == workloads.G_MIN))
        if t.index % 2 == 0:
            assert set(np.unique(t.V)) <= {0.0, 0.5}
        else:
            assert np.all((t.V >= 0.0) & (t.V <= 0.5)) and len(np.unique(t.V)) > 2


def test_c4_filter_keeps_the_draws():
    """Filtering by n_t returns the same tiles (same draws) as the full workload."""
    full = workloads.c4(tiles=64)
    small = workloads.c4(tiles=64, max_n=64)
    want = [t for t in full if t.G.shape[1] <= 64]
    assert [t.index for t in small] == [t.index for t in want]
    for a, b in zip(small, want):
        assert np.array_equal(a.G, b.G) and np.array_equal(a.V, b.V)
