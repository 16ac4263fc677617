"""Pins of the oracle's design filter and projection (Sec. 2.1, oracle/design.py).

* filter_matrix: hand-computed cone weights on a 3 x 3 grid (centre element,
  r = 1.5 h: self r, edge neighbours r - h, corners r - sqrt(2) h); rows sum to
  one; identity for r below one element; translation invariance of interior
  rows; mirror symmetry of the whole operator; the boundary row and a row
  of rectangular elements by hand.
* projection / projection_deriv: P(0) = 0, P(1) = 1, P(eta) closed form,
  the small-beta limit P(x) -> x, central differences of P.
* filter_projection_backward: central differences of J(chi) = c . P(H chi).
"""
import numpy as np
import pytest

import oracle as O


def test_three_by_three_centre_row_by_hand():
    h = 1.0 / 3
    r = 1.5 * h
    H = O.filter_matrix(3, 3, r).toarray()
    w_self, w_edge, w_corner = r, r - h, r - np.sqrt(2) * h
    W = w_self + 4 * w_edge + 4 * w_corner
    expect = np.array([w_corner, w_edge, w_corner, w_edge, w_self, w_edge, w_corner, w_edge,
                       w_corner]) / W
    assert np.allclose(H[4], expect, rtol=1e-14, atol=0)


def test_corner_row_by_hand():
    """Element (0, 0) with r = 1.5 h keeps itself, (1, 0), (0, 1), (1, 1)."""
    h = 1.0 / 3
    r = 1.5 * h
    H = O.filter_matrix(3, 3, r).toarray()
    w = {0: r, 1: r - h, 3: r - h, 4: r - np.sqrt(2) * h}
    W = sum(w.values())
    expect = np.zeros(9)
    for k, v in w.items():
        expect[k] = v / W
    assert np.allclose(H[0], expect, rtol=1e-14, atol=0)


def test_rectangular_elements_row_by_hand():
    """nx = 4, ny = 2 (hx = 0.25, hy = 0.5), r = 0.55, element (1, 0): self 0.55,
    (0, 0) and (2, 0) at 0.25, (3, 0) and (1, 1) at 0.5; (0, 1) and (2, 1) at
    sqrt(0.3125) > r drop out."""
    H = O.filter_matrix(4, 2, 0.55).toarray()
    w = {1: 0.55, 0: 0.30, 2: 0.30, 3: 0.05, 5: 0.05}
    W = sum(w.values())
    expect = np.zeros(8)
    for k, v in w.items():
        expect[k] = v / W
    assert np.allclose(H[1], expect, rtol=1e-13, atol=0)


@pytest.mark.parametrize("nx,ny,r", [(7, 5, 0.3), (12, 12, 0.1), (9, 20, 0.17), (1, 1, 0.4)])
def test_rows_sum_to_one_and_constants_kept(nx, ny, r):
    H = O.filter_matrix(nx, ny, r)
    assert np.allclose(np.asarray(H.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-14)
    assert (H.toarray() >= 0).all()


def test_identity_below_one_element():
    H = O.filter_matrix(6, 4, 0.9 / 6)
    assert np.array_equal(H.toarray(), np.eye(24))


def test_interior_rows_translation_invariant_and_mirror_symmetric():
    nx = ny = 15
    r = 0.2   # three elements
    H = O.filter_matrix(nx, ny, r).toarray()
    def stencil(i, j):
        row = H[j * nx + i].reshape(ny, nx)
        return row[j - 3:j + 4, i - 3:i + 4]
    ref = stencil(7, 7)
    for i, j in [(3, 3), (10, 5), (5, 11), (11, 11)]:
        assert np.allclose(stencil(i, j), ref, rtol=1e-14, atol=0)
    # mirror x -> 1 - x maps H onto itself
    perm = np.array([j * nx + (nx - 1 - i) for j in range(ny) for i in range(nx)])
    assert np.allclose(H[np.ix_(perm, perm)], H, rtol=1e-14, atol=0)


@pytest.mark.parametrize("beta,eta", [(32.0, 0.5), (8.0, 0.3), (1.0, 0.9)])
def test_projection_closed_forms(beta, eta):
    den = np.tanh(beta * (1 - eta)) + np.tanh(beta * eta)
    assert O.projection(np.array([0.0]), beta, eta)[0] == pytest.approx(0.0, abs=1e-15)
    assert O.projection(np.array([1.0]), beta, eta)[0] == pytest.approx(1.0, rel=1e-15)
    assert O.projection(np.array([eta]), beta, eta)[0] == pytest.approx(
        np.tanh(beta * eta) / den, rel=1e-14)
    x = np.linspace(-0.2, 1.2, 57)
    assert (np.diff(O.projection(x, beta, eta)) >= 0).all()   # tanh saturates in FP64
    xm = eta + np.linspace(-0.5, 0.5, 21) / beta
    assert (np.diff(O.projection(xm, beta, eta)) > 0).all()
    h = 1e-6
    fd = (O.projection(x + h, beta, eta) - O.projection(x - h, beta, eta)) / (2 * h)
    assert np.allclose(O.projection_deriv(x, beta, eta), fd, rtol=1e-7, atol=1e-9)


def test_projection_small_beta_is_identity():
    x = np.linspace(0.0, 1.0, 11)
    assert np.allclose(O.projection(x, 1e-6, 0.4), x, rtol=0, atol=1e-11)
    assert np.array_equal(O.projection(x, 0.0, 0.4), x)
    assert np.array_equal(O.projection_deriv(x, 0.0, 0.4), np.ones_like(x))


@pytest.mark.parametrize("nx,ny,r,beta,eta", [(9, 7, 0.25, 8.0, 0.5), (10, 10, 0.15, 32.0, 0.45),
                                             (6, 11, 0.3, 0.0, 0.5)])
def test_backward_finite_differences(nx, ny, r, beta, eta):
    rng = np.random.default_rng(nx * ny)
    chi = rng.uniform(0.2, 0.8, nx * ny)
    c = rng.standard_normal(nx * ny)

    def J(x):
        return float(c @ O.filter_projection(x, nx, ny, r, beta, eta)[1])

    fil, _ = O.filter_projection(chi, nx, ny, r, beta, eta)
    g = O.filter_projection_backward(fil, c, nx, ny, r, beta, eta)
    for _ in range(4):
        d = rng.standard_normal(nx * ny)
        d /= np.linalg.norm(d)
        fd = (J(chi + 1e-6 * d) - J(chi - 1e-6 * d)) / 2e-6
        assert abs(fd - g @ d) <= 1e-6 * abs(g @ d) + 1e-9
