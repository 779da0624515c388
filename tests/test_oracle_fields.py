"""Pins of the prolongation oracle (oracle.fields)."""
import numpy as np

from oracle import fields, tt


def test_prolonged_fourier_mode_closed_form():
    """cos(2 pi k x) on M points: the even fine points are the coarse values;
    the odd ones, midway between x_j and x_(j+1), are the average
    (cos(2 pi k x_j) + cos(2 pi k x_(j+1))) / 2 = cos(pi k / M) cos(2 pi k
    (x_j + 1/(2M)))."""
    M, k = 32, 3
    x = np.arange(M) / M
    f = np.cos(2 * np.pi * k * x)
    g = fields.prolong_dense(f)
    xf = np.arange(2 * M) / (2 * M)
    want = np.cos(2 * np.pi * k * xf)
    want[1::2] *= np.cos(np.pi * k / M)
    assert np.allclose(g, want, atol=1e-15)


def test_prolongation_keeps_constants_and_is_second_order():
    c = fields.prolong_dense(np.full((8, 8, 8), 2.5))
    assert np.all(c == 2.5)
    errs = []
    for M in (16, 32, 64):
        x = np.arange(M) / M
        xf = np.arange(2 * M) / (2 * M)
        f = lambda t: np.exp(np.sin(2 * np.pi * t))  # noqa: E731
        errs.append(np.max(np.abs(fields.prolong_dense(f(x)) - f(xf))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.7 < r1 < 4.3 and 3.8 < r2 < 4.2, errs


def test_prolongation_of_separable_fields_is_separable():
    """Interpolation is linear and acts axis by axis: the prolongation of
    u(x1) v(x2) w(x3) is the product of the prolonged vectors, and its
    TT-SVD has rank 1 at the bonds between the dimensions."""
    rng = np.random.default_rng(3)
    u, v, w = (rng.standard_normal(8) for _ in range(3))
    F = np.einsum("i,j,k->ijk", u, v, w)
    G = fields.prolong_dense(F)
    want = np.einsum("i,j,k->ijk", fields.prolong_dense(u), fields.prolong_dense(v), fields.prolong_dense(w))
    assert np.allclose(G, want, atol=1e-14)
    cores, Gd = fields.prolong_tt(F, chi=16)
    assert np.allclose(tt.tt_full(cores).reshape(Gd.shape), Gd, atol=1e-13)
    exact = tt.tt_svd(Gd.reshape((2,) * 12), rel_tol=1e-12)
    r = tt.ranks(exact)
    assert r[4] == 1 and r[8] == 1, r
