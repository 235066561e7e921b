"""CPU checks of the C interface: exported symbols and the host-side FP64
set-up (grids, 1D operators, eigen-decompositions, phi_1 factors) against
the oracle.  No GPU work is launched here."""
import os
import re

import numpy as np
import pytest

import paper_2604_11558_amd as tg
from oracle import operators as op
from oracle.phi import phi1_matrix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "tgexp.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    names = set(re.findall(r"\b(tg_[a-z0-9_]+)\s*\(", header))
    assert len(names) >= 15
    L = tg.lib()
    for name in sorted(names):
        assert hasattr(L, name), name
    assert L.tg_version() == 1


def _oracle_ops(geometry, n, extent):
    return op.operators_1d(geometry, n, extent)


CASES = [("disk", (7, 12), (1.3, 1.0)), ("sphere", (10, 9), (1.0, 1.0)),
         ("ball", (8, 6, 11), (0.8, 1.0)), ("cylinder", (9, 10, 7), (1.2, 2.5)),
         ("ball", (64, 64, 128), (1.0, 1.0)),
         ("disk_lambda", (9, 12), (1.0, -1.95)), ("disk_lambda", (11, 8), (1.3, 0.5)),
         ("disk_lambda", (160, 160), (1.0, -1.95))]


@pytest.mark.parametrize("geometry,n,extent", CASES)
def test_grid_and_operators_match_oracle(geometry, n, extent):
    g = tg.Grid(geometry, n, extent)
    ref = _oracle_ops(geometry, n, extent)
    for m in range(1, len(n) + 1):
        np.testing.assert_allclose(g.coords(m), ref["grid"][m - 1], rtol=1e-15, atol=1e-15)
        A = ref["A"][m - 1]
        np.testing.assert_allclose(g.dense_operator(m), A, rtol=1e-14, atol=1e-14 * np.abs(A).max())


@pytest.mark.parametrize("geometry,n,extent", CASES)
def test_eigendecomposition(geometry, n, extent):
    g = tg.Grid(geometry, n, extent)
    for m in range(1, len(n) + 1):
        A = g.dense_operator(m)
        lam, V, Vi = g.eig(m)
        scale = np.abs(A).max()
        np.testing.assert_allclose(A @ V, V * lam[None, :], atol=2e-13 * scale * np.sqrt(n[m - 1]))
        np.testing.assert_allclose(V @ Vi, np.eye(n[m - 1]), atol=1e-12)
        np.testing.assert_allclose(np.sort(lam), np.sort(np.linalg.eigvals(A).real),
                                   atol=1e-11 * scale)


@pytest.mark.parametrize("geometry,n,extent", CASES[:4] + CASES[5:7])
@pytest.mark.parametrize("c", [1e-5, 3e-3, 0.2])
def test_phi1_factor_matches_oracle(geometry, n, extent, c):
    g = tg.Grid(geometry, n, extent)
    ref = _oracle_ops(geometry, n, extent)
    for m in range(1, len(n) + 1):
        P = g.phi1(m, c)
        R = phi1_matrix(ref["A"][m - 1], c)
        np.testing.assert_allclose(P, R, atol=2e-14 * n[m - 1], rtol=0)


def test_sigma_large_n():
    g = tg.Grid("sphere", (8, 2049))
    np.testing.assert_allclose(g.coords(2), op.phi_grid(2049), rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("geometry,n", [("disk", (2, 8)), ("ball", (4, 4, 1)), ("nope", (4, 4))])
def test_invalid_grid(geometry, n):
    with pytest.raises((tg.TGError, KeyError, ValueError)) as ei:
        tg.Grid(geometry, n)
    if isinstance(ei.value, tg.TGError):
        assert ei.value.code == -1


def test_invalid_extent():
    with pytest.raises(tg.TGError):
        tg.Grid("disk", (4, 4), (0.0, 1.0))
    # the anomalous disk: extent = (rho_*, lambda) with lambda < 1
    for ext in ((1.0, 1.0), (1.0, 2.0), (0.0, -1.0), (1.0, float("nan"))):
        with pytest.raises(tg.TGError):
            tg.Grid("disk_lambda", (4, 4), ext)


# the library's factors (own QL eigensolver on the symmetrised operator, or
# the closed-form Fourier basis for theta) against an independent route:
# Pade scaling-and-squaring exponential of the augmented matrix
# [[c A, I], [0, 0]], whose top-right block is phi_1(c A).  A_rho, A_phi,
# A_z and A_lambda are non-normal; by Proposition 1 their eigenvector
# matrices have condition number up to about sqrt(2 n), which bounds the
# eigen route's error (relative to the result's norm, in units of eps);
# scaling and squaring loses up to about ||c A|| eps (its squarings
# amplify the Pade approximant's rounding).  Two correct routes differ by
# less than 16 eps (sqrt(2 n) + ||c A||_inf) relative to max |phi_1|;
# measured up to 4e3 eps sqrt(2 n) (2.9e-11, z at n = 512, c = 0.4, where
# ||c A|| = 4.2e5).
PADE_CASES = [("rho2", "disk", lambda n: (n, 8), 1, (1.0, 1.0)),
              ("theta", "disk", lambda n: (4, n), 2, (1.0, 1.0)),
              ("rho3", "ball", lambda n: (n, 4, 4), 1, (1.0, 1.0)),
              ("phi", "sphere", lambda n: (4, n), 2, (1.0, 1.0)),
              ("z", "cylinder", lambda n: (4, 4, n), 3, (1.0, 1.0)),
              ("lambda", "disk_lambda", lambda n: (n, 4), 1, (1.0, -1.95))]


@pytest.mark.parametrize("name,geometry,shape,mode,extent", PADE_CASES)
@pytest.mark.parametrize("n", [64, 128, 256, 512])
def test_phi1_factor_against_pade_expm(name, geometry, shape, mode, extent, n):
    from oracle.phi import phi1_dense_expm
    g = tg.Grid(geometry, shape(n), extent)
    A = g.dense_operator(mode)
    for c in (5e-3, 0.4):  # tau d of the workloads: 5e-3 (ball u) ... 0.4 (sphere v at d = 40)
        P = g.phi1(mode, c)
        R = phi1_dense_expm(c * A)
        cA = c * np.abs(A).sum(axis=1).max()
        tol = 16 * 2.0 ** -52 * (np.sqrt(2.0 * n) + cA) * np.abs(R).max()
        err = np.abs(P - R).max()
        assert err < tol, (name, n, c, err, tol)
