"""CPU checks of the spectral judge: single-mode spectra, Parseval, box
filter, and the error measure."""
import numpy as np

from paper_2602_14667_amd import spectral


def test_single_mode_lands_in_its_shell():
    n = 32
    x = np.arange(n)
    u = np.zeros((2, n, n)); b = np.zeros((2, n, n))
    u[0] = 0.1 * np.cos(2 * np.pi * 3 * x / n)[None, :]       # |kappa| = 3
    b[1] = 0.2 * np.sin(2 * np.pi * (4 * x[:, None] + 3 * x[None, :]) / n)  # 5
    e = spectral.shell_spectrum(u, b)
    assert abs(e[3] - 0.5 * 0.1 ** 2 / 2) < 1e-15
    assert abs(e[5] - 0.5 * 0.2 ** 2 / 2) < 1e-15
    assert abs(e.sum() - (e[3] + e[5])) < 1e-15


def test_parseval_matches_energies():
    rng = np.random.default_rng(0)
    n = 16
    u = rng.standard_normal((2, n, n)); b = rng.standard_normal((2, n, n))
    e = spectral.shell_spectrum(u, b)
    k = np.fft.fftfreq(n, 1 / n)
    kk = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    inside = kk < n / 2 + 0.5  # shells up to n/2 are kept
    tot = 0.0
    for f in (*u, *b):
        h = np.fft.fft2(f) / n ** 2
        tot += 0.5 * np.sum(np.abs(h[inside]) ** 2)
    assert abs(e.sum() - tot) < 1e-12


def test_box_filter_and_eps():
    a = np.arange(16.0).reshape(4, 4)
    f = spectral.box_filter(a, 2)
    assert np.allclose(f, [[2.5, 4.5], [10.5, 12.5]])
    e = np.array([0, 1.0, 2.0, 4.0])
    assert spectral.eps_spec(e, e, 3) == 0.0
    assert abs(spectral.eps_spec(1.1 * e, e, 3) - 0.1) < 1e-12


def test_kinetic_magnetic_split():
    """The two parts add up to E(k); a velocity-only field has no magnetic
    part and the single mode lands in its shell on the right side."""
    n = 32
    x = np.arange(n)
    u = np.zeros((2, n, n)); b = np.zeros((2, n, n))
    u[0] = 0.1 * np.cos(2 * np.pi * 3 * x / n)[None, :]
    b[1] = 0.2 * np.sin(2 * np.pi * (4 * x[:, None] + 3 * x[None, :]) / n)
    eu, eb = spectral.kinetic_magnetic_spectra(u, b)
    assert np.allclose(eu + eb, spectral.shell_spectrum(u, b), rtol=0, atol=1e-16)
    assert abs(eu[3] - 0.5 * 0.1 ** 2 / 2) < 1e-15 and eu[5] < 1e-30
    assert abs(eb[5] - 0.5 * 0.2 ** 2 / 2) < 1e-15 and eb[3] < 1e-30
