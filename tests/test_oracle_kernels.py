"""Pins of the oracle's time kernel K(t) = 2 pi Im g(-t) (Appendix A).

* the paper's own route: a numerical Fourier transform of
  delta g = g - g_1 - g_2 (g(xi) as printed in Appendix A) plus the printed
  analytic transforms of g_1 and g_2, which the oracle never evaluates;
* the printed asymptotes: 1/t^2 + sigma/t as t -> 0 (the g_1 term) and
  (sqrt(pi)/2) sigma^{3/2} t^{-1/2} as t -> inf (the g_2 term);
* sigma = 0 reduces to 1/t^2 (no contour deformation);
* the z-invariant kernel equals the general Laplace weight times the
  frequency factor kappa_w/2 (Appendix A.2), and equals half of 2 pi times the
  printed Appendix A.2 expression (the factor is fixed physically by the
  plate pins in test_oracle_force.py).
"""
import warnings

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.kernels import kernel_general, kernel_table, kernel_zinv2d


def g_paper(xi, s):
    return -1j * xi * (1 + 1j * s / xi) * (1 + 1j * s / (2 * xi)) / np.sqrt(1 + 1j * s / xi)


def im_g_minus_t_paper_route(t, s):
    """Im g(-t) = Im dg(-t) + (1/2pi)(1/t^2 + s/t) + s^{3/2}/(4 sqrt(pi) t^{1/2})."""
    def dg(x):
        return g_paper(x, s) - (x / 1j + s) - np.sqrt(1j) / 2 * s ** 1.5 / np.sqrt(x)
    A = 50.0 / t
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        i1 = quad(lambda x: dg(x).imag * np.cos(x * t) + dg(x).real * np.sin(x * t), 0, A,
                  limit=2000, epsabs=1e-14, epsrel=1e-13)[0]
        i2 = quad(lambda x: dg(x).imag, A, np.inf, weight="cos", wvar=t, limlst=200)[0]
        i3 = quad(lambda x: dg(x).real, A, np.inf, weight="sin", wvar=t, limlst=200)[0]
    return (i1 + i2 + i3) / (2 * np.pi) + (1 / t ** 2 + s / t) / (2 * np.pi) \
        + s ** 1.5 / (4 * np.sqrt(np.pi) * np.sqrt(t))


@pytest.mark.parametrize("sigma", [1.0, 10.0])
@pytest.mark.parametrize("t", [0.05, 0.3, 1.0, 3.0, 10.0])
def test_general_kernel_matches_paper_route(sigma, t):
    ref = 2 * np.pi * im_g_minus_t_paper_route(t, sigma)
    assert kernel_general(t, sigma) == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("sigma", [0.5, 1.0, 10.0])
def test_general_kernel_asymptotes(sigma):
    t0 = 1e-5 / sigma
    assert kernel_general(t0, sigma) / (1 / t0 ** 2 + sigma / t0) == pytest.approx(1.0, abs=1e-4)
    t1 = 1e5 / sigma
    tail = np.sqrt(np.pi) / 2 * sigma ** 1.5 / np.sqrt(t1)
    assert kernel_general(t1, sigma) / tail == pytest.approx(1.0, abs=1e-4)


def test_sigma_zero_limits():
    t = np.array([0.01, 0.1, 1.0, 7.0])
    np.testing.assert_allclose(kernel_general(t, 0.0), 1 / t ** 2, rtol=1e-15)
    np.testing.assert_allclose(kernel_general(t, 1e-9), 1 / t ** 2, rtol=1e-7)
    np.testing.assert_allclose(kernel_zinv2d(t, 0.0), 1 / t ** 3, rtol=1e-15)


@pytest.mark.parametrize("sigma", [1.0, 3.0])
@pytest.mark.parametrize("t", [0.1, 1.0, 4.0])
def test_zinv_kernel_is_general_weight_times_half_omega(sigma, t):
    """K_2D(t) = int w(k) (kappa_w / 2) e^{-k t} dk, w(k) = (k + s/2) sqrt(1 + s/k),
    kappa_w = sqrt(k (k + s)): the imaginary frequency of the contour point."""
    def integrand(k):
        return (k + sigma / 2) * np.sqrt(1 + sigma / k) * np.sqrt(k * (k + sigma)) / 2 * np.exp(-k * t)
    ref = quad(integrand, 0, np.inf, limit=500, epsrel=1e-13)[0]
    assert kernel_zinv2d(t, sigma) == pytest.approx(ref, rel=1e-10)


def test_zinv_kernel_vs_printed_expression():
    t = np.linspace(0.05, 20, 50)
    s = 1.7
    printed = (1 / (2 * np.pi)) * (2 / t ** 3 + 3 * s / (2 * t ** 2) + s ** 2 / (2 * t))
    np.testing.assert_allclose(kernel_zinv2d(t, s), 0.5 * 2 * np.pi * printed, rtol=1e-14)


def test_kernel_table_sampling():
    dt = 0.0125
    tab = kernel_table("general", 1.0, dt, 7)
    np.testing.assert_allclose(tab, kernel_general(dt * np.arange(1, 8), 1.0), rtol=0)
    assert np.all(np.isfinite(kernel_table("general", 1.0, 0.01, 100000)))
    assert np.all(np.diff(kernel_table("zinv2d", 1.0, 0.01, 1000)) < 0)
