"""Pins of the Hermite-Gauss basis (Sections 4 and 5) against textbook forms."""
import math

import numpy as np
import pytest

import oracle.wdd as O

EXPLICIT = [
    lambda t: np.ones_like(t),
    lambda t: 2 * t,
    lambda t: 4 * t ** 2 - 2,
    lambda t: 8 * t ** 3 - 12 * t,
    lambda t: 16 * t ** 4 - 48 * t ** 2 + 12,
]


def test_recurrence_matches_explicit_hermite_polynomials():
    t = np.linspace(-6, 6, 301)
    psi = O.hermite_functions(5, t)
    for n, hn in enumerate(EXPLICIT):
        ref = hn(t) * np.exp(-t * t / 2) / math.sqrt(2 ** n * math.factorial(n) * math.sqrt(math.pi))
        assert np.max(np.abs(psi[n] - ref)) < 1e-13


def test_continuous_orthonormality_by_gauss_hermite_quadrature():
    x, w = np.polynomial.hermite.hermgauss(40)      # exact for polynomial * exp(-x^2) up to degree 79
    psi = O.hermite_functions(16, x)
    gram = (psi * (w * np.exp(x * x))[None, :]) @ psi.T
    assert np.max(np.abs(gram - np.eye(16))) < 1e-12


def test_hermite_functions_are_eigenfunctions_of_the_centred_dft():
    """With sigma^2 = N / (2 pi) the sampled functions map to (-i)^n psi_n under the centred
    unitary forward DFT (equation eigenfunction-of-FT; the sign i^n there belongs to the
    opposite transform convention)."""
    n = 256
    sigma = math.sqrt(n / (2 * math.pi))
    psi = O.sampled_hermite(n, 8, sigma)
    for order in range(8):
        col = psi[:, order]
        ft = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(col))) / math.sqrt(n)
        assert np.max(np.abs(ft - (-1j) ** order * col)) < 1e-9


def test_parity_of_sampled_functions():
    psi = O.sampled_hermite(64, 8, 3.0)
    # grid index i <-> t = (i - 32) / sigma; mirror i -> 64 - i keeps t -> -t
    for order in range(8):
        col = psi[:, order]
        assert np.allclose(col[1:][::-1], (-1) ** order * col[1:], atol=1e-14)


def test_shell_order():
    assert O.basis_order(4).tolist() == [[0, 0], [0, 1], [1, 0], [1, 1]]
    assert sorted(map(tuple, O.basis_order(64).tolist())) == [(a, b) for a in range(8) for b in range(8)]
    k128 = O.basis_order(128)
    assert sorted(map(tuple, k128[:121].tolist())) == [(a, b) for a in range(11) for b in range(11)]
    assert k128[121:].tolist() == [[0, 11], [11, 0], [1, 11], [11, 1], [2, 11], [11, 2], [3, 11]]
    assert O.basis_size_1d(128) == 12 and O.basis_size_1d(256) == 16


def test_projection_is_the_papers_reduction_relabelled():
    """Phi^T vec(A) lists the entries of H(A) = psi_x^T A^T psi_y (Section 5)."""
    rng = np.random.default_rng(3)
    n, k, sigma = 16, 16, 2.0
    psi = O.sampled_hermite(n, 4, sigma)
    a = rng.normal(size=(n, n))
    red = psi.T @ a.T @ psi
    h = O.project(a[None], O.hg_basis(n, n, k, sigma))[0]
    for j, (ny, nx) in enumerate(O.basis_order(k)):
        assert abs(h[j] - red[nx, ny]) < 1e-12


def test_grid_orthonormality_is_close():
    phi = O.hg_basis(64, 64, 256, O.default_sigma(16.0, 256))
    gram = phi.T @ phi
    assert np.allclose(np.diag(gram), 1.0, atol=1e-12)
    assert np.max(np.abs(gram - np.eye(256))) < 1e-6


@pytest.mark.parametrize("radius,k", [(8.0, 64), (16.0, 256), (48.0, 128), (32.0, 64), (5.0, 7)])
def test_default_sigma_puts_the_highest_turning_point_on_the_rim(radius, k):
    """Reading R2: sigma is chosen so that the classical turning point of the highest 1D
    order n = L - 1 lies on the aperture rim.  The turning point is found from the Hermite
    differential equation psi'' = (t^2 - (2n + 1)) psi, i.e. where the second difference
    of the sampled function changes from oscillating (psi''/psi < 0) to decaying, not from
    the closed form in default_sigma."""
    sigma = O.default_sigma(radius, k)
    n = O.basis_size_1d(k) - 1
    x = np.linspace(0.5 * radius, 1.5 * radius, 200001)      # detector pixels from the centre
    h = x[1] - x[0]
    psi = O.hermite_functions(n + 1, x / sigma)[n]
    curv = (psi[2:] - 2 * psi[1:-1] + psi[:-2]) / (h * h) / psi[1:-1]   # psi''/psi in 1/px^2
    xm = x[1:-1]
    ok = np.abs(psi[1:-1]) > 1e-300
    # outermost sign change of psi''/psi from negative to positive
    s = np.sign(curv[ok])
    idx = np.nonzero((s[:-1] < 0) & (s[1:] > 0))[0]
    turn = xm[ok][idx[-1]]
    assert abs(turn - radius) <= 2 * h + 1e-9 * radius
