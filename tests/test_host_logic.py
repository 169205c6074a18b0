"""Host-side logic of the library (no device work): histogram peaks
against the oracle's definition, and the peak finder's own pins."""
import os

import numpy as np
import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2609_05467_amd", "libhra.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhra.so not built")


def test_peaks_single_spike(orc):
    from paper_2609_05467_amd import hra
    h = np.zeros(8192, np.uint32)
    b = orc.histogram_bin([0.3, -0.2, 0.9])
    h[b] = 7
    p = hra.histogram_peaks(h, 4)
    assert p["bins"] == [b] and p["mass"] == [7]
    c = orc.bin_centre(b)
    assert np.allclose(p["dirs"][0], c, atol=1e-6)
    # the bin centre lies inside its own bin
    assert orc.histogram_bin(c) == b


def test_peaks_match_oracle_random(orc):
    from paper_2609_05467_amd import hra
    rng = np.random.default_rng(0)
    for _ in range(5):
        h = rng.poisson(3.0, 8192).astype(np.uint32)
        for _ in range(6):
            h[rng.integers(8192)] += rng.integers(50, 500)
        p = hra.histogram_peaks(h, 16)
        o = orc.histogram_peaks(h, 16)
        assert p["bins"] == o["bins"] and p["mass"] == o["mass"]
        assert p["axis_mass"] == o["axis_mass"]


def test_peaks_azimuth_wrap(orc):
    from paper_2609_05467_amd import hra
    h = np.zeros(8192, np.uint32)
    h[10 * 128 + 127] = 5   # neighbours across the azimuth seam
    h[10 * 128 + 0] = 9
    p = hra.histogram_peaks(h, 4)
    assert p["bins"] == [10 * 128 + 0]


def test_axis_masses_partition_caps(orc):
    from paper_2609_05467_amd import hra
    h = np.ones(8192, np.uint32)
    p = hra.histogram_peaks(h, 1)
    # equal-area bins: each 45-degree cap holds (1 - cos 45) / 2 of the sphere
    frac = np.array(p["axis_mass"]) / 8192
    assert np.allclose(frac, (1 - np.sqrt(0.5)) / 2, atol=0.01)
