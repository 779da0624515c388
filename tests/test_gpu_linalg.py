"""FP64 factorisation kernels against LAPACK (needs an MI355X)."""
import numpy as np
import pytest

q = pytest.importorskip("paper_2407_09169_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("m,n", [(2, 1), (4, 4), (8, 5), (32, 16), (64, 64), (128, 64), (96, 90),
                                 (192, 96), (200, 100), (256, 128), (257, 129), (288, 144), (290, 140),
                                 (320, 160), (512, 256), (576, 288), (333, 257), (576, 32), (500, 30)])
def test_qr(ctx, m, n):
    rng = np.random.default_rng(m * 1000 + n)
    A = rng.standard_normal((3, m, n))
    A[1, :, n // 2:] = 0.0  # rank deficient
    A[2] *= np.logspace(0, -12, n)[None, :]  # graded columns
    Q, R = q.linalg_qr(ctx, A)
    for b in range(3):
        assert np.max(np.abs(Q[b].T @ Q[b] - np.eye(n))) < 50 * n * 2.2e-16, b
        assert np.max(np.abs(Q[b] @ R[b] - A[b])) <= 50 * n * 2.2e-16 * np.abs(A[b]).max(), b
        assert np.max(np.abs(np.tril(R[b], -1))) == 0.0


@pytest.mark.parametrize("m,n", [(288, 144), (256, 144), (256, 128), (192, 96), (144, 144), (160, 80), (128, 128),
                                 (100, 37), (64, 64), (48, 24), (32, 32), (576, 32)])
def test_qr_q_only_split(ctx, m, n):
    """One matrix, Q only (the sweeps' call): the factorising workgroup leaves
    the reflectors and Q is formed with one column per wavefront, reflectors
    taken in pairs (odd n leaves a single one per chunk; n = 37 leaves idle
    wavefronts in the last workgroup; m = 576 takes chunks of 8).  Same Q as
    the factorisation that forms Q itself (with R), to rounding, for random,
    exactly rank-deficient and graded matrices."""
    rng = np.random.default_rng(m * 13 + n)
    for kind in ("random", "rank deficient", "graded"):
        A = rng.standard_normal((1, m, n))
        if kind == "rank deficient":
            A[0, :, n // 2:] = 0.0
        if kind == "graded":
            A[0] *= np.logspace(0, -12, n)[None, :]
        Qs, _ = q.linalg_qr(ctx, A, with_r=False)
        Qf, R = q.linalg_qr(ctx, A)
        assert np.max(np.abs(Qs[0].T @ Qs[0] - np.eye(n))) < 50 * n * 2.2e-16, kind
        assert np.max(np.abs(Qs[0] @ R[0] - A[0])) <= 50 * n * 2.2e-16 * np.abs(A[0]).max(), kind
        assert np.max(np.abs(Qs[0] - Qf[0])) < 1e-12, kind


@pytest.mark.parametrize("m,n", [(576, 288), (576, 100), (500, 250), (400, 33), (333, 257)])
def test_qr_single_blocked(ctx, m, n):
    """One matrix beyond the register kernels: blocked Householder (register
    panels, compact WY updates).  Random, exactly rank-deficient and graded
    matrices; Q orthonormal, Q R = A, R upper triangular."""
    rng = np.random.default_rng(m * 7 + n)
    for kind in ("random", "rank deficient", "graded"):
        A = rng.standard_normal((1, m, n))
        if kind == "rank deficient":
            A[0, :, n // 2:] = 0.0
        if kind == "graded":
            A[0] *= np.logspace(0, -12, n)[None, :]
        Q, R = q.linalg_qr(ctx, A)
        Qb, Rb, Ab = Q[0], R[0], A[0]
        assert np.max(np.abs(Qb.T @ Qb - np.eye(n))) < 50 * n * 2.2e-16, kind
        assert np.max(np.abs(Qb @ Rb - Ab)) <= 50 * n * 2.2e-16 * np.abs(Ab).max(), kind
        assert np.max(np.abs(np.tril(Rb, -1))) == 0.0, kind
        Q2, _ = q.linalg_qr(ctx, A, with_r=False)
        assert np.array_equal(Q2, Q), kind


@pytest.mark.parametrize("n,keep", [(1, 1), (2, 1), (2, 2), (3, 2), (5, 3), (16, 16), (33, 20), (64, 48), (100, 100),
                                    (128, 120), (144, 128), (288, 256)])
def test_eigh(ctx, n, keep):
    rng = np.random.default_rng(n * 7 + keep)
    X = rng.standard_normal((3, n, n + 4)) * np.logspace(0, -6, n + 4)[None, None, :]
    G = X @ np.transpose(X, (0, 2, 1))
    G[1] = X[1][:, : max(1, n // 3)] @ X[1][:, : max(1, n // 3)].T  # rank deficient
    P, lam = q.linalg_eigh(ctx, G, keep)
    for b in range(3):
        ref = np.linalg.eigvalsh(G[b])[::-1]
        l1 = ref[0]
        assert np.max(np.abs(lam[b] - ref)) < 100 * n * 2.2e-16 * l1, b
        assert np.max(np.abs(P[b].T @ P[b] - np.eye(keep))) < 100 * n * 2.2e-16, b
        resid = G[b] @ P[b] - P[b] * lam[b][:keep][None, :]
        assert np.max(np.abs(resid)) < 100 * n * 2.2e-16 * l1, b


@pytest.mark.parametrize("m,n", [(8, 5), (64, 64), (288, 144), (576, 32)])
def test_qr_degenerate(ctx, m, n):
    """Exactly degenerate inputs: the zero matrix (every reflector is the
    identity: Q = [I; 0], R = 0) and a single nonzero column (R = Q^T A has
    one nonzero column); Q stays orthonormal and Q R = A, with and without R."""
    A = np.zeros((2, m, n))
    A[1, :, n // 2] = np.random.default_rng(m + n).standard_normal(m)
    Q, R = q.linalg_qr(ctx, A)
    Qs, _ = q.linalg_qr(ctx, A, with_r=False)
    assert np.array_equal(Q[0], np.eye(m, n)) and np.array_equal(R[0], np.zeros((n, n)))
    for b in range(2):
        assert np.max(np.abs(Q[b].T @ Q[b] - np.eye(n))) < 50 * n * 2.2e-16, b
        assert np.max(np.abs(Q[b] @ R[b] - A[b])) <= 50 * n * 2.2e-16 * max(1.0, np.abs(A[b]).max()), b
        assert np.max(np.abs(np.tril(R[b], -1))) == 0.0, b
        assert np.max(np.abs(Qs[b] - Q[b])) < 1e-12, b
    assert np.count_nonzero(np.abs(R[1]).max(axis=0) > 0) == 1


@pytest.mark.parametrize("n,keep", [(16, 8), (33, 20), (144, 128)])
def test_eigh_degenerate(ctx, n, keep):
    """Exactly repeated eigenvalues, with the cut inside a multiplet (only the
    eigenspace is unique there: the kept vectors must be orthonormal
    eigenvectors, the eigenvalues exact), the matrix 2 I, and the zero
    matrix (eigenvalues 0, orthonormal vectors)."""
    rng = np.random.default_rng(n * 31 + keep)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([4.0, 2.0, 1.0, 0.5], (n + 3) // 4)[:n].copy()
    lam[keep:keep + 2] = lam[keep - 1]  # the multiplet of lam[keep-1] reaches past the cut
    G = np.stack([(U * lam) @ U.T, 2.0 * np.eye(n), np.zeros((n, n))])
    refs = [lam, np.full(n, 2.0), np.zeros(n)]
    P, got = q.linalg_eigh(ctx, G, keep)
    for b in range(3):
        l1 = max(1.0, refs[b][0])
        assert np.max(np.abs(got[b] - refs[b])) < 100 * n * 2.2e-16 * l1, b
        assert np.max(np.abs(P[b].T @ P[b] - np.eye(keep))) < 100 * n * 2.2e-16, b
        resid = G[b] @ P[b] - P[b] * got[b][:keep][None, :]
        assert np.max(np.abs(resid)) < 100 * n * 2.2e-16 * l1, b
