"""The seeded input generators: deterministic, band-limited, unit RMS, and
the recipes the workloads state (tube split, tiling)."""
import numpy as np

from synth_inputs import (WORKLOADS, grid_shape, smooth_ic, smooth_noise, tiled_smooth_ic,
                          tube_ic, workload_ic)


def test_smooth_noise_is_seeded_band_limited_and_unit_rms():
    for extent in [(32, 24), (16, 12, 10)]:
        a = smooth_noise(extent, 7)
        assert a.shape == grid_shape(extent)
        assert np.array_equal(a, smooth_noise(extent, 7))
        assert not np.allclose(a, smooth_noise(extent, 8))
        assert abs(np.sqrt(np.mean(a * a)) - 1) < 1e-12 and abs(a.mean()) < 1e-12
        spec = np.fft.fftn(a)
        k2 = sum(np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n) ** 2 for n in a.shape], indexing="ij"))
        assert np.max(np.abs(spec[k2 > 64.0])) < 1e-9 * np.max(np.abs(spec))


def test_smooth_ic_amplitudes():
    rho, U, th = smooth_ic((24, 20, 16))
    assert abs(np.sqrt(np.mean((rho - 1) ** 2)) - 0.01) < 1e-12
    assert abs(np.sqrt(np.mean(U ** 2)) - 0.02) < 1e-12
    assert abs(np.sqrt(np.mean((th - 1) ** 2)) - 0.01) < 1e-12


def test_tube_recipe_matches_the_experiment():
    w = WORKLOADS["d3q95_11x11x800_tube"]
    rho, U, th = workload_ic(w)
    assert rho.shape == (800, 11, 11)
    assert np.all(rho[:400] == 4.0) and np.all(rho[400:] == 1.0)   # rho = p = 4 | 1, theta = 1
    assert np.all(th == 1.0) and np.all(U == 0.0)
    rho2, _, _ = tube_ic((3, 10), 5, (2.0, 1.0), (1.0, 1.0))
    assert np.all(rho2[:5] == 2.0) and np.all(rho2[5:] == 1.0)


def test_tiling_repeats_the_tile():
    rho, U, th = tiled_smooth_ic((16, 8, 8), (8, 4, 4))
    r1, U1, t1 = smooth_ic((8, 4, 4))
    assert np.array_equal(rho[4:, 4:, 8:], r1) and np.array_equal(U[:, :4, 4:, :8], U1)
