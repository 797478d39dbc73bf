"""Seeded input generators: deterministic, right shapes, subset selection
consistent with the full batch (no GPU)."""
import numpy as np

from paper_2503_09580_amd import workloads as wl


def test_c1_c2_shapes_and_determinism():
    h, p = wl.c1()
    assert h.shape == (1, 16, 16, 16) and p.shape == (1, 5)
    h2, _ = wl.c1()
    assert np.array_equal(h, h2)
    h, p = wl.c2(batch=3)
    assert h.shape == (3, 32, 32, 32)
    # bi-Maxwellian minus M: zero mass to grid accuracy
    assert np.all(np.abs(h.sum(axis=(1, 2, 3)) * 0.5 ** 3) < 1e-10)


def test_c3_subset_matches_full_batch():
    hs, ps = wl.c3(batch=64, cells=[3, 17, 63])
    hf, pf = wl.c3(batch=64)
    assert np.array_equal(hs, hf[[3, 17, 63]])
    assert np.array_equal(ps, pf[[3, 17, 63]])
    assert np.all(np.abs(pf[:, 0] - 1.0) <= 0.2 + 1e-12)
    assert np.all(np.abs(pf[:, 4] - 1.0) <= 0.2 + 1e-12)


def test_c5_temperatures_in_range():
    h, p = wl.c5(batch=16, cells=[0, 1])
    assert h.shape == (2, 64, 64, 64)
    _, pf = wl.c5(batch=16, cells=[])
    assert np.all((pf[:, 4] >= 0.5) & (pf[:, 4] <= 2.0))
