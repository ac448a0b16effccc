"""The ragged multi-scene batch generator (inputs only)."""
import numpy as np

import scenegen


def test_layout_is_seeded_and_ragged():
    a, b = scenegen.config4_layout(), scenegen.config4_layout()
    assert a == b and len(a) == 16
    px = np.array([s["pixels"] for s in a])
    assert px.min() >= 9_000 and px.max() <= 2_500_000
    drawn = scenegen.ragged_scene_sizes()
    assert np.all(px <= drawn) and np.all(px >= drawn - 2 * np.sqrt(drawn))
    blocks = [s for s in a if s["block"] > 1]
    assert len(blocks) == 4 and all(s["block"] == 15 for s in blocks)
    assert max(s["pixels"] for s in blocks) <= min(s["pixels"] for s in a if s["block"] == 1)
    assert sorted({s["atmosphere"] for s in a}) == [0, 1, 2, 3]


def test_block_footprints_partition_the_fine_grid():
    idx = scenegen.block_footprints(3, 4, 5)
    assert idx.shape == (12, 25)
    assert np.array_equal(np.sort(idx.ravel()), np.arange(3 * 5 * 4 * 5))
    # coarse pixel (1, 2) holds fine rows 5..9, columns 10..14
    fine_cols = 4 * 5
    want = [(r * fine_cols + c) for r in range(5, 10) for c in range(10, 15)]
    assert sorted(idx[1 * 4 + 2].tolist()) == want


def test_fine_states_and_mask():
    spec = {"scene": 3, "rows": 6, "cols": 7, "pixels": 42, "atmosphere": 3, "block": 15}
    st, mask = scenegen.config4_states(spec)
    assert st.shape == (6 * 15 * 7 * 15, 5) and mask.shape == (st.shape[0],)
    assert np.all(st[~mask, 0] == 0) and np.all(st[mask, 0] > 0)
    st2, _ = scenegen.config4_states(spec)
    assert np.array_equal(st, st2)
