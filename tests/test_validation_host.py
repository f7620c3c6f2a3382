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


def test_cylinder_band_separates_shedding_from_the_duct_acoustic_mode():
    """The full-size cylinder's numbers: D = 64, u_in = 0.05, a 33,000-step
    window; shedding at St 0.21 under a stronger transverse acoustic mode of
    the 512-cell duct (c_s / 2 ny, St 0.72).  The cylinder run's band,
    St 0.05 - 0.5, recovers the shedding."""
    D, u, n = 64.0, 0.05, 33000
    t = np.arange(n)
    f_shed = 0.21 * u / D
    f_ac = (1 / np.sqrt(3.0)) / (2 * 512)
    assert abs(f_ac * D / u - 0.722) < 1e-3
    s = 0.5 * np.sin(2 * np.pi * f_shed * t) + 1.5 * np.sin(2 * np.pi * f_ac * t + 1.0)
    assert abs(dominant_frequency([s]) * D / u - 0.722) < 0.01
    st = dominant_frequency([s], band=(0.05 * u / D, 0.5 * u / D)) * D / u
    assert abs(st - 0.21) < 0.01, st
