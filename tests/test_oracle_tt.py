"""Pins of the tensor-train oracle (oracle.tt): brute force on small chains,
rounding error bounds, and eq. MPSdofs against the paper's stated reductions."""
import json
import os

import numpy as np
import pytest

from oracle import dense, tt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_tt(ranks, seed, decay=None):
    rng = np.random.default_rng(seed)
    cores = []
    for n in range(len(ranks) - 1):
        G = rng.standard_normal((ranks[n], 2, ranks[n + 1]))
        if decay is not None:
            G *= decay ** np.arange(ranks[n + 1])[None, None, :]
        cores.append(G)
    return cores


def test_tt_svd_round_trip():
    T = np.random.default_rng(0).standard_normal((2,) * 10)
    cores = tt.tt_svd(T, rel_tol=0.0)
    assert np.allclose(tt.tt_full(cores), T, atol=1e-12)


@pytest.mark.parametrize("ordering", ["serial", "interleaved"])
def test_mpo_product_brute_force(ordering):
    """Kronecker MPO of per-dimension 1-D operators equals the dense Kronecker
    product (bits permuted to the chain order), checked entry by entry."""
    bits, nd = 3, 3
    M = 1 << bits
    order = ([(d, b) for d in range(nd) for b in range(bits)] if ordering == "serial"
             else [(d, b) for b in range(bits) for d in range(nd)])
    A = [dense.d1_ghost(M), dense.d2_periodic(M) @ np.diag(np.arange(M) + 1.0), dense.d2_ghost(M)]
    mpo = tt.mpo_product([tt.operator_qtt(a) for a in A], order, nd)
    K = np.kron(np.kron(A[0], A[1]), A[2])  # serial bit order
    perm = tt.site_perm(order, bits)
    N = nd * bits
    Kp = K.reshape((2,) * (2 * N)).transpose(perm + [N + p for p in perm]).reshape(1 << N, 1 << N)
    assert np.allclose(tt.mpo_full(mpo), Kp, atol=1e-10 * np.abs(K).max())
    # MPO x MPS equals the dense matrix-vector product
    x = _random_tt([1] + [3] * (N - 1) + [1], 1)
    y = tt.mpo_apply(mpo, x)
    assert np.allclose(tt.tt_full(y).reshape(-1), Kp @ tt.tt_full(x).reshape(-1),
                       atol=1e-10 * np.abs(Kp).max() * 10)


def test_operator_ranks():
    """Bond dimensions of the 1-D CFD2 operators in quantics form: the cyclic
    shift has rank 2, so D1p/D2p have rank <= 3; the ghost-point versions add
    two corner projectors (rank <= 5)."""
    M = 128
    for A, rmax in ((dense.d1_periodic(M), 3), (dense.d2_periodic(M), 3),
                    (dense.d1_ghost(M), 5), (dense.d2_ghost(M), 5)):
        W = tt.operator_qtt(A)
        assert max(G.shape[-1] for G in W) <= rmax
        assert np.allclose(tt.mpo_full(W), A, atol=1e-9 * np.abs(A).max())


def test_sum_and_diag():
    x = _random_tt([1, 2, 3, 2, 1], 2)
    y = _random_tt([1, 3, 4, 2, 1], 3)
    s = tt.mps_sum([(0.5, x), (-2.0, y)])
    assert np.allclose(tt.tt_full(s), 0.5 * tt.tt_full(x) - 2.0 * tt.tt_full(y))
    D = tt.mpo_full(tt.mpo_diag(x))
    assert np.allclose(np.diag(D), tt.tt_full(x).reshape(-1))
    assert np.allclose(D - np.diag(np.diag(D)), 0.0)


def test_rounding_error_bounds():
    """Textbook rounding: ||T - R(T)||^2 = sum of discarded sigma^2 (up to
    rounding); simultaneous truncation: ||T - R(T)|| <= sum_n eps_n."""
    x = _random_tt([1, 2, 4, 8, 16, 16, 8, 4, 2, 1], 4, decay=0.55)
    T = tt.tt_full(x)
    for chi in (2, 4, 6):
        r, disc = tt.round_ttsvd(x, chi)
        err2 = np.sum((tt.tt_full(r) - T) ** 2)
        assert err2 <= sum(disc) * (1 + 1e-8) + 1e-28
        assert err2 >= max(disc) * (1 - 1e-8)  # at least the optimal error at the worst bond
        g, info = tt.round_det(x, chi)
        errg = np.sqrt(np.sum((tt.tt_full(g) - T) ** 2))
        assert errg <= sum(np.sqrt(d) for d in info["discarded"]) * (1 + 1e-8) + 1e-14
        assert max(tt.ranks(g)) <= chi


def test_round_det_untruncated_exact():
    x = _random_tt([1, 2, 4, 8, 4, 4, 2, 1], 5)
    y = tt.mps_sum([(1.0, x), (0.25, x)])
    g, _ = tt.round_det(y, 64)
    assert np.allclose(tt.tt_full(g), 1.25 * tt.tt_full(x), atol=1e-12)
    assert all(r <= c for r, c in zip(tt.ranks(g), tt.chain_caps(7, 64)))


def _gaussian_sketch(N, ell, seed):
    ranks = [min(ell, 2**n, 2 ** (N - n)) for n in range(N + 1)]
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((ranks[n], 2, ranks[n + 1])) for n in range(N)], ranks


def test_round_sketch_exact_when_ell_covers_rank():
    """With sketch ranks at the chain maxima the range finder is exact and
    rounding W x with chi = 2^(N/2) returns W x itself."""
    N = 8
    x = _random_tt([1, 2, 4, 8, 8, 8, 4, 2, 1], 6)
    W = tt.mpo_product([tt.operator_qtt(dense.d1_ghost(16)), tt.operator_qtt(dense.d2_ghost(16))],
                       [(0, b) for b in range(4)] + [(1, b) for b in range(4)], 2)
    Z, ell = _gaussian_sketch(N, 16, 7)
    out, _ = tt.round_sketch([(0.7, W, x), (-1.5, None, x)], Z, ell, 16)
    ref = 0.7 * tt.tt_full(tt.mpo_apply(W, x)) - 1.5 * tt.tt_full(x)
    assert np.allclose(tt.tt_full(out), ref, atol=1e-11 * np.abs(ref).max())


def test_round_sketch_quasi_optimal():
    """Randomized range finding + truncation stays within a small factor of the
    textbook SVD rounding error (Gaussian sketch, oversampling 8)."""
    x = _random_tt([1, 2, 4, 8, 16, 32, 16, 8, 4, 2, 1], 8, decay=0.7)
    chi = 6
    ref, _ = tt.round_ttsvd(x, chi)
    T = tt.tt_full(x)
    e_opt = np.linalg.norm(tt.tt_full(ref) - T)
    Z, ell = _gaussian_sketch(10, chi + 8, 9)
    out, info = tt.round_sketch([(1.0, None, x)], Z, ell, chi)
    e = np.linalg.norm(tt.tt_full(out) - T)
    assert e <= 3.0 * e_opt
    assert max(tt.ranks(out)) <= chi


@pytest.mark.parametrize("c", [0, 1, 4, 7])
def test_round_sketch_two_sided_exact_when_ell_covers_rank(c):
    """Two-sided range finding with the centre at any site: exact when both
    sketches have the chain's maximal ranks; the range-finder output is
    left-orthogonal left of the centre and right-orthogonal right of it."""
    N = 8
    x = _random_tt([1, 2, 4, 8, 8, 8, 4, 2, 1], 6)
    W = tt.mpo_product([tt.operator_qtt(dense.d1_ghost(16)), tt.operator_qtt(dense.d2_ghost(16))],
                       [(0, b) for b in range(4)] + [(1, b) for b in range(4)], 2)
    Zr, _ = _gaussian_sketch(N, 16, 7)
    Zl, _ = _gaussian_sketch(N, 16, 8)
    terms = [(0.7, W, x), (-1.5, None, x)]
    ref = 0.7 * tt.tt_full(tt.mpo_apply(W, x)) - 1.5 * tt.tt_full(x)
    mid, cc = tt.rand_orth_two_sided(terms, Zr, Zl, c)
    assert cc == c
    for n in range(c):
        A = mid[n].reshape(-1, mid[n].shape[2])
        assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-12)
    for n in range(c + 1, N):
        A = mid[n].reshape(mid[n].shape[0], -1)
        assert np.allclose(A @ A.T, np.eye(A.shape[0]), atol=1e-12)
    assert np.allclose(tt.tt_full(mid), ref, atol=1e-11 * np.abs(ref).max())
    out, _ = tt.round_sketch_two_sided(terms, Zr, Zl, 16, c=c)
    assert np.allclose(tt.tt_full(out), ref, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("c", [1, 5, 9])
def test_round_sketch_two_sided_truncation_bound(c):
    """With the ranges captured exactly, the simultaneous truncation of the
    mixed canonical form errs by at most the discarded Gram eigenvalues,
    summed over the bonds (a wrong choice of Gram matrix on either side of
    the centre breaks this), and it is within a small factor of TT-SVD."""
    x = _random_tt([1, 2, 4, 8, 16, 32, 16, 8, 4, 2, 1], 8, decay=0.7)
    N = 10
    Zr, _ = _gaussian_sketch(N, 32, 21)
    Zl, _ = _gaussian_sketch(N, 32, 22)
    T = tt.tt_full(x)
    for chi in (3, 6, 12):
        out, info = tt.round_sketch_two_sided([(1.0, None, x)], Zr, Zl, chi, c=c)
        e2 = np.linalg.norm(tt.tt_full(out) - T) ** 2
        assert e2 <= sum(info["discarded"]) * (1 + 1e-9) + 1e-24
        ref, _ = tt.round_ttsvd(x, chi)
        assert np.sqrt(e2) <= 3.0 * np.linalg.norm(tt.tt_full(ref) - T) + 1e-14
        assert max(tt.ranks(out)) <= chi


def test_nvpp_paper_claims():
    """eq. MPSdofs against the reductions the paper states for the 128^5 grid
    (N = 35): O(10^6) fewer parameters at chi = 32 (Abstract, Discussion),
    NVPP of order 1/10^5 of the grid at chi = 128 (Results), and NVPP = M^d
    exactly at the maximal chi = 2^floor(N/2) (Materials and Methods)."""
    with open(os.path.join(GOLDEN, "nvpp_claims.json")) as fh:
        claims = json.load(fh)
    for c in claims["claims"]:
        N, chi = c["N"], c["chi"]
        v = tt.nvpp(N, chi)
        if c["kind"] == "exact_grid":
            assert v == 2**N
        else:
            ratio = 2**N / v
            lo, hi = c["order_of_magnitude_range"]
            assert lo <= ratio <= hi, (N, chi, ratio)
    # the number of stored core entries minus the gauge freedom, by brute force
    N, chi = 12, 8
    caps = tt.chain_caps(N, chi)
    stored = sum(2 * caps[n] * caps[n + 1] for n in range(N))
    gauge = sum(caps[n] ** 2 for n in range(1, N))
    assert tt.nvpp(N, chi) == stored - gauge


def _graded_chain(sig, seed):
    """8-site MPS whose middle bond (bond 4, the only one above 8) has the
    singular values sig: T = U diag(sig) V^T with orthonormal U, V (16 x 16)."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((16, 16)))
    V, _ = np.linalg.qr(rng.standard_normal((16, 16)))
    T = (U * sig) @ V.T
    return tt.tt_svd(T.reshape((2,) * 8), rel_tol=0.0), U, V


def test_svd_truncation_resolves_below_sqrt_eps():
    """Singular values far below sqrt(eps) sigma_1 (1e-10 .. 1e-22) are cut
    exactly where they should be: the rounded chain equals U_k diag(s_k) V_k^T
    of the one truncated bond to rounding error (a Gram-matrix eigensolver
    cannot separate directions whose squared singular values are below
    eps sigma_1^2, and would err by up to ~1e-8 here).  The deterministic,
    the one-sided and the two-sided sketched roundings all agree with it."""
    sig = 10.0 ** (-1.5 * np.arange(16))
    x, U, V = _graded_chain(sig, 31)
    k = 8
    exact = ((U[:, :k] * sig[:k]) @ V[:, :k].T).reshape(-1)
    N = 8
    Zr, ell = _gaussian_sketch(N, 16, 32)
    Zl, _ = _gaussian_sketch(N, 16, 33)
    outs = {
        "ttsvd": tt.round_ttsvd(x, k)[0],
        "det": tt.round_det(x, k)[0],
        "sketch": tt.round_sketch([(1.0, None, x)], Zr, ell, k)[0],
        "two_sided": tt.round_sketch_two_sided([(1.0, None, x)], Zr, Zl, k)[0],
    }
    for name, r in outs.items():
        err = np.abs(tt.tt_full(r).reshape(-1) - exact).max()
        assert err < 1e-15, (name, err)
    g, info = tt.round_det(x, k)
    # singular values to absolute accuracy ~ eps sigma_1 (sigma_1 = 1)
    assert abs(np.sqrt(info["discarded"][4]) - np.sqrt(np.sum(sig[k:] ** 2))) < 1e-14
    assert np.allclose(info["sigmas"][4], sig, rtol=0, atol=1e-14)


@pytest.mark.parametrize("c", [2, 4, 6])
def test_mixed_truncation_matches_ttsvd_at_one_bond(c):
    """When only one bond is over its cap, simultaneous and sequential
    truncation coincide: the two-sided rounding with any centre reproduces
    the textbook rounding and the exact truncated SVD."""
    sig = 0.6 ** np.arange(16)
    x, U, V = _graded_chain(sig, 34)
    N = 8
    Zr, _ = _gaussian_sketch(N, 16, 35)
    Zl, _ = _gaussian_sketch(N, 16, 36)
    for k in (8,):  # chi = 8: every other bond of the 8-site chain is within its cap
        ref = tt.tt_full(tt.round_ttsvd(x, k)[0])
        out, info = tt.round_sketch_two_sided([(2.0, None, x)], Zr, Zl, k, c=c)
        assert np.abs(tt.tt_full(out) - 2.0 * ref).max() < 1e-13
        assert np.isclose(info["discarded"][4], 4.0 * np.sum(sig[k:] ** 2), rtol=1e-10)
