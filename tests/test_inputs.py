"""The seeded input generator follows its stated recipe."""
import numpy as np

from paper_2405_04690_amd import inputs


def test_draw_sources_recipe_and_determinism():
    p = inputs.draw_sources(0, 4000, (1e-4, 1e-2), (-19, -15))
    q = inputs.draw_sources(0, 4000, (1e-4, 1e-2), (-19, -15))
    assert np.array_equal(p, q)
    assert p.shape == (4000, 8)
    la = np.log10(p[:, 0])
    assert la.min() >= -23 and la.max() <= -21
    assert p[:, 1].min() >= 1e-4 and p[:, 1].max() <= 1e-2
    lf = np.log10(p[:, 2])
    assert lf.min() >= -19 and lf.max() <= -15
    assert np.all((p[:, 3] >= 0) & (p[:, 3] <= 2 * np.pi))
    assert np.all((p[:, 4] >= 0) & (p[:, 4] <= np.pi))
    assert np.all((p[:, 5] >= 0) & (p[:, 5] <= np.pi))
    assert np.all((p[:, 6] >= 0) & (p[:, 6] <= 2 * np.pi))
    assert np.all(np.abs(p[:, 7]) <= np.pi / 2)
    # log-uniform f0: half the draws below the geometric mean
    assert abs(np.mean(p[:, 1] < 1e-3) - 0.5) < 0.05
    z = inputs.draw_sources(1, 10)
    assert np.all(z[:, 2] == 0)


def test_swap_batch_shapes():
    sb = inputs.paper_swap_batch(n_walkers=4, n_temps=3, n_src=5)
    assert sb.params_old.shape == (60, 8) and sb.params_new.shape == (60, 8)
    assert sb.res_idx.dtype == np.int32 and sb.res_idx.max() == 3
    full = inputs.paper_swap_batch(n_walkers=32, n_temps=24, n_src=130, mix="full")
    births = np.mean(full.params_old[:, 0] == 0)
    deaths = np.mean(full.params_new[:, 0] == 0)
    assert abs(births - 0.1) < 0.01 and abs(deaths - 0.1) < 0.01


def test_complex_normals_moments():
    g = inputs.complex_normals(3, (200000,))
    assert abs(np.mean(np.abs(g) ** 2) - 2.0) < 0.02
