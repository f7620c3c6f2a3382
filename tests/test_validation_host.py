"""Host-side logic of the validation runs: the spectral peak finder used
for Strouhal numbers, and the paper's Table 1 values it is compared with."""
import numpy as np

from paper_2606_16765_amd.validation import TABLE1, dominant_frequency


def test_dominant_frequency_recovers_a_sine():
    n = 15000
    t = np.arange(n)
    rng = np.random.default_rng(0)
    for f in (1 / 2370.0, 1 / 812.5, 0.013):
        s = 0.3 + np.sin(2 * np.pi * f * t + 0.4) + 0.2 * rng.standard_normal(n)
        c = 0.5 * np.cos(2 * np.pi * f * t)
        got = dominant_frequency([s, c])
        assert abs(got - f) / f < 0.01, (got, f)


def test_table1_has_the_papers_rows():
    assert sorted(TABLE1) == [100, 500, 1000, 2000]
    assert TABLE1[1000][128] == 0.479 and TABLE1[1000][1024] == 0.472
    assert TABLE1[100]["ref"] == 1.08 and TABLE1[2000][256] == 0.407


def test_dominant_frequency_band_excludes_a_stronger_mode():
    n = 20000
    t = np.arange(n)
    shed, acoustic = 1 / 2400.0, 1 / 100.0
    s = 0.3 * np.sin(2 * np.pi * shed * t) + 2.0 * np.sin(2 * np.pi * acoustic * t)
    assert abs(dominant_frequency([s]) - acoustic) / acoustic < 0.01
    got = dominant_frequency([s], band=(1 / 10000.0, 1 / 1000.0))
    assert abs(got - shed) / shed < 0.02
