"""Pins of the assembled Kronecker-sum Laplacians (paper Section 2).

* constants are in the kernel (Neumann / periodic / pole-free ends), and
  lifted constants are stationary for the cylinder's Dirichlet end;
* the low spectrum converges at second order to the textbook eigenvalues
  of the continuous operators: Neumann Bessel zeros on the disk and the
  cylinder, -l(l+1) on the sphere, zeros of j_l' in the ball.  A wrong
  Kronecker order, a missing 1/rho^2 or 1/sin^2 scaling or a wrong 1D
  stencil moves these eigenvalues by O(1).
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import jnp_zeros, spherical_jn

from oracle import assemble


@pytest.mark.parametrize("geometry,n", [("disk", (7, 9)), ("sphere", (9, 7)),
                                        ("ball", (5, 6, 7)), ("cylinder", (5, 6, 7))])
def test_constants_in_kernel(geometry, n):
    M = assemble.laplacian(geometry, n, (1.0, 1.7))
    one = np.ones(M.shape[0])
    r = M @ one + assemble.dirichlet_lift(geometry, n, (1.0, 1.7))
    assert np.abs(r).max() <= 1e-12 * abs(M).max()


def _low_spectrum(geometry, n, k, extent=(1.0, 1.0)):
    M = assemble.laplacian(geometry, n, extent).toarray()
    ev = np.linalg.eigvals(M)
    assert np.abs(ev.imag).max() < 1e-8 * np.abs(M).max()
    return np.sort(-ev.real)[:k]


def _disk_exact(k):
    vals = [0.0]
    for m in range(0, 6):
        z = jnp_zeros(m, 4) if m > 0 else np.concatenate([jnp_zeros(0, 4)])
        for x in z:
            vals += [x * x] * (1 if m == 0 else 2)
    return np.sort(vals)[:k]


def _sphere_exact(k):
    vals = []
    for l in range(0, 8):
        vals += [l * (l + 1.0)] * (2 * l + 1)
    return np.sort(vals)[:k]


def _sph_jn_prime_zeros(l, count):
    f = lambda x: spherical_jn(l, x, derivative=True)  # noqa: E731
    xs = np.linspace(0.05, 30, 6000)
    fx = f(xs)
    roots = [brentq(f, a, b) for a, b, fa, fb in zip(xs[:-1], xs[1:], fx[:-1], fx[1:])
             if fa * fb < 0]
    return roots[:count]


def _ball_exact(k):
    vals = [0.0]
    for l in range(0, 5):
        for x in _sph_jn_prime_zeros(l, 3):
            vals += [x * x] * (2 * l + 1)
    return np.sort(vals)[:k]


def _cyl_exact(k, zs):
    radial = [0.0]
    for m in range(0, 5):
        for x in jnp_zeros(m, 3):
            radial += [x * x] * (1 if m == 0 else 2)
    vals = [r + (math.pi * (q - 0.5) / zs) ** 2 for r in radial for q in range(1, 4)]
    return np.sort(vals)[:k]


@pytest.mark.parametrize("geometry,grids,exact,k", [
    ("disk", [(10, 20), (20, 40)], _disk_exact, 6),
    ("sphere", [(16, 12), (32, 24)], _sphere_exact, 9),
    ("ball", [(6, 8, 8), (12, 16, 16)], _ball_exact, 4),
    ("cylinder", [(6, 10, 4), (12, 20, 8)], lambda k: _cyl_exact(k, 1.0), 4),
])
def test_spectrum_second_order(geometry, grids, exact, k):
    ex = exact(k)
    errs = []
    for n in grids:
        lo = _low_spectrum(geometry, n, k)
        errs.append(np.abs(lo - ex)[1:].max() if ex[0] == 0 else np.abs(lo - ex).max())
        if ex[0] == 0.0:
            assert abs(lo[0]) < 1e-8
    assert errs[1] < 0.05 * max(ex)
    assert errs[0] / errs[1] > 3.0, errs  # halving h: error ratio ~4


def test_sphere_radius_scaling():
    n = (16, 12)
    a = _low_spectrum("sphere", n, 4)
    b = _low_spectrum("sphere", n, 4, (2.0, 1.0))
    np.testing.assert_allclose(b, a / 4.0, atol=1e-10)


def test_layout_roundtrip():
    x = np.arange(2 * 3 * 4, dtype=float).reshape(4, 3, 2)  # [k][j][i]
    W = assemble.from_layout(x)
    assert W.shape == (2, 3, 4) and W[1, 2, 3] == x[3, 2, 1]
    # paper vectorisation: w_{i + (j-1) n1 + (k-1) n1 n2} <-> C-order storage
    np.testing.assert_array_equal(assemble.vec(W), x.ravel())
    np.testing.assert_array_equal(assemble.to_layout(W), x)
