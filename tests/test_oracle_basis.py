"""Pins of the oracle's 1-D basis and of its RK coefficients.

Nodes/weights are checked against numpy's Gauss-Legendre routine and the
Legendre-polynomial definition of the Lobatto nodes; D and the boundary
interpolants against exactness on monomials; the Lobatto operators against
the summation-by-parts identity; the LSERK4(5) coefficients against the
order conditions of a fourth-order Runge-Kutta method.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

NS = list(range(1, 10))


@pytest.mark.parametrize("N", NS)
def test_lg_nodes_match_numpy_gauss(orc, N):
    b = orc.basis(N, 0)
    x, w = npleg.leggauss(N + 1)
    assert np.allclose(b["x"], x, atol=1e-15, rtol=0)
    assert np.allclose(b["w"], w, atol=2e-15, rtol=0)


@pytest.mark.parametrize("N", NS)
def test_lgl_nodes_are_roots_of_dPN(orc, N):
    b = orc.basis(N, 1)
    c = np.zeros(N + 1)
    c[N] = 1.0
    roots = np.sort(npleg.legroots(npleg.legder(c))) if N > 1 else np.array([])
    assert b["x"][0] == -1.0 and b["x"][-1] == 1.0
    assert np.allclose(b["x"][1:-1], roots, atol=1e-14, rtol=0)


@pytest.mark.parametrize("nodes", [0, 1])
@pytest.mark.parametrize("N", NS)
def test_quadrature_exactness(orc, N, nodes):
    b = orc.basis(N, nodes)
    deg = 2 * N + 1 if nodes == 0 else 2 * N - 1
    for k in range(deg + 1):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.dot(b["w"], b["x"] ** k) - exact) < 1e-14
    # the next degree is not integrated exactly (even monomial)
    k = deg + 1
    exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
    assert abs(np.dot(b["w"], b["x"] ** k) - exact) > 1e-8


@pytest.mark.parametrize("nodes", [0, 1])
@pytest.mark.parametrize("N", NS)
def test_derivative_matrix_exact_on_polynomials(orc, N, nodes):
    b = orc.basis(N, nodes)
    x, D = b["x"], b["D"]
    assert np.abs(D @ np.ones(N + 1)).max() < 1e-13
    for k in range(1, N + 1):
        assert np.abs(D @ x ** k - k * x ** (k - 1)).max() < 1e-12 * max(1, N * N)
    for k in range(N + 1):
        assert abs(b["Lp"] @ x ** k - 1.0) < 1e-13
        assert abs(b["Lm"] @ x ** k - (-1.0) ** k) < 1e-13


@pytest.mark.parametrize("N", NS)
def test_lgl_summation_by_parts(orc, N):
    b = orc.basis(N, 1)
    W = np.diag(b["w"])
    Q = W @ b["D"]
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.abs(Q + Q.T - B).max() < 1e-13
    # split operator: zero diagonal, and boundary values are unit vectors
    assert np.abs(np.diag(b["DS"])).max() < 1e-13
    assert np.array_equal(b["Lm"], np.eye(N + 1)[0]) and np.array_equal(b["Lp"], np.eye(N + 1)[N])


def test_basis_rejects_bad_requests(orc):
    with pytest.raises(ValueError):
        orc.basis(0, 1)
    with pytest.raises(ValueError):
        orc.basis(3, 2)


def _butcher_from_2n(A, B):
    """Butcher tableau of a 2N-storage scheme dU <- A_s dU + dt R; U <- U + B_s dU."""
    s = len(A)
    a = np.zeros((s + 1, s))
    for i in range(1, s + 1):          # stage i+1 input (row i) uses K_1..K_i
        for j in range(i):
            acc = 0.0
            for r in range(j, i):
                prod = 1.0
                for m in range(j + 1, r + 1):
                    prod *= A[m]
                acc += B[r] * prod
            a[i, j] = acc
    return a[:s], a[s]


def test_lserk14_order_conditions(orc):
    """LSERK4-14 (Niegemann, Diehl & Busch): the same eight conditions.  The
    published coefficients carry 16 significant digits, so the conditions
    hold to about 5e-14 (sums of 14 terms of size up to 7); c to round-off."""
    A, B, C = orc.rk_coeffs(1)
    assert len(A) == 14
    a, b = _butcher_from_2n(A, B)
    c = a.sum(1)
    assert np.abs(c - C).max() < 1e-14
    conds = [
        (b.sum(), 1.0),
        (b @ c, 1 / 2),
        (b @ c ** 2, 1 / 3),
        (b @ (a @ c), 1 / 6),
        (b @ c ** 3, 1 / 4),
        (b @ (c * (a @ c)), 1 / 8),
        (b @ (a @ c ** 2), 1 / 12),
        (b @ (a @ (a @ c)), 1 / 24),
    ]
    for got, want in conds:
        assert abs(got - want) < 1e-13, (got, want)
    assert A[0] == 0.0
    A5, B5, C5 = orc.rk_coeffs(0)
    assert np.array_equal(np.concatenate([A5, B5, C5]), np.concatenate(orc.lserk_coeffs()))


def test_lserk_order_conditions(orc):
    A, B, C = orc.lserk_coeffs()
    a, b = _butcher_from_2n(A, B)
    c = a.sum(1)
    assert np.abs(c - C).max() < 1e-14
    conds = [
        (b.sum(), 1.0),
        (b @ c, 1 / 2),
        (b @ c ** 2, 1 / 3),
        (b @ (a @ c), 1 / 6),
        (b @ c ** 3, 1 / 4),
        (b @ (c * (a @ c)), 1 / 8),
        (b @ (a @ c ** 2), 1 / 12),
        (b @ (a @ (a @ c)), 1 / 24),
    ]
    for got, want in conds:
        assert abs(got - want) < 1e-14
    assert A[0] == 0.0
