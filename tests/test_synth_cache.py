"""The cached arg-min labels of the 2048x2048 degree-6 map equal the generator's
own arg-min on sampled rows (the cache only saves the ~90 s of CPU work)."""
import numpy as np

import synth


def test_c5_cache_matches_generator_rows():
    gm = synth.config_c5()
    assert (gm.H, gm.W) == (2048, 2048) and gm.N == int(gm.keep.size)
    rows = [0, 1, 513, 1024, 1777, 2047]
    raw = synth.config_c5_rows(rows)
    lab = gm.labels.reshape(gm.H, gm.W)[rows]
    assert np.array_equal(gm.keep[lab], raw)
