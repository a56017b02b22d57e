"""Oracle FE building blocks pinned to closed forms and textbook values."""
import numpy as np
import pytest

from oracle import fe


def test_gll_closed_forms():
    assert np.allclose(fe.gll_points(1), [0, 1], atol=0)
    assert np.allclose(fe.gll_points(2), [0, 0.5, 1], atol=0)
    s5 = np.sqrt(5.0) / 10.0
    assert np.allclose(fe.gll_points(3), [0, 0.5 - s5, 0.5 + s5, 1], atol=1e-15)
    s21 = np.sqrt(21.0) / 14.0
    assert np.allclose(fe.gll_points(4), [0, 0.5 - s21, 0.5, 0.5 + s21, 1], atol=1e-15)
    # degree 6: interior points are the roots of P_6', symmetric about 1/2
    x = fe.gll_points(6)
    assert x[3] == 0.5 and np.allclose(x + x[::-1], 1.0, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_gauss_exactness(n):
    x, w = fe.gauss(n)
    for p in range(2 * n):
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 1e-14
    # not exact one degree higher (n-point Gauss has degree 2n-1)
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-10


def test_q1_stiffness_textbook():
    # trilinear hexahedron on the unit cube: 1/3 on the diagonal, 0 between
    # nodes on a common edge, -1/12 across face and body diagonals
    A = fe.reference_stiffness(1)
    for i in range(8):
        for j in range(8):
            d = sum(((i >> s) & 1) != ((j >> s) & 1) for s in range(3))
            want = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[d]
            assert abs(A[i, j] - want) < 1e-15


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_stiffness_properties(k):
    A = fe.reference_stiffness(k)
    n = k + 1
    assert np.allclose(A, A.T, atol=1e-13)
    # constants are in the kernel, linear functions give |grad|^2 * vol
    xi = fe.gll_points(k)
    pts = np.array([(xi[a], xi[b], xi[c]) for c in range(n) for b in range(n) for a in range(n)])
    assert np.abs(A @ np.ones(n ** 3)).max() < 1e-12
    g = np.array([0.7, -1.1, 0.4])
    u = pts @ g
    assert abs(u @ A @ u - g @ g) < 1e-12
    # a quadratic: u = x^2 has int |grad u|^2 = int 4x^2 = 4/3 (needs k >= 2)
    if k >= 2:
        u = pts[:, 0] ** 2
        assert abs(u @ A @ u - 4.0 / 3.0) < 1e-12
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-12 and np.sum(ev < 1e-10) == 1


def test_load_vector_integrates_polynomials():
    k = 3
    b = fe.reference_load(k, lambda p: p[:, 0] * p[:, 1] ** 2)
    # sum_i b_i = int f (partition of unity)
    assert abs(b.sum() - 0.5 * (1.0 / 3.0)) < 1e-15


# Lagrange polynomials on the Gauss-Lobatto nodes {0, 1} and {0, 1/2, 1},
# written out by hand as coefficient lists in ascending powers of t
_LAGRANGE = {1: [[1, -1], [0, 1]],                    # 1 - t, t
             2: [[1, -3, 2], [0, 4, -4], [0, -1, 2]]}  # 2(t-1/2)(t-1), -4t(t-1), 2t(t-1/2)


def _moment(p, coeffs):
    """int_0^1 t^p l(t) dt in exact rational arithmetic."""
    from fractions import Fraction
    return sum(Fraction(c, p + i + 1) for i, c in enumerate(coeffs))


@pytest.mark.parametrize("k,powers", [(1, (1, 2, 0)), (1, (0, 1, 2)), (2, (1, 2, 3)), (2, (3, 0, 2))])
def test_load_vector_entries_closed_form(k, powers):
    """Entry (a, b, c) of the load of f = x^px y^py z^pz is the product of the
    1D moments int t^p l_a, int t^p l_b, int t^p l_c (Gauss with k+1 points is
    exact for these degrees).  The powers differ per axis, so a swapped axis
    or a node order other than x fastest fails."""
    px, py, pz = powers
    b = fe.reference_load(k, lambda p: p[:, 0] ** px * p[:, 1] ** py * p[:, 2] ** pz)
    L = _LAGRANGE[k]
    n = k + 1
    for c in range(n):
        for bb in range(n):
            for a in range(n):
                want = _moment(px, L[a]) * _moment(py, L[bb]) * _moment(pz, L[c])
                assert abs(b[a + n * bb + n * n * c] - float(want)) < 1e-16, (a, bb, c)


def test_basis_partition_of_unity_and_gradients():
    rng = np.random.default_rng(0)
    xi = rng.uniform(0, 1, size=(20, 3))
    for k in (1, 2, 4, 6):
        assert np.allclose(fe.basis_at(k, xi).sum(axis=1), 1.0, atol=1e-12)
        g = fe.basis_gradient_at(k, xi)
        assert np.abs(g.sum(axis=1)).max() < 1e-10
