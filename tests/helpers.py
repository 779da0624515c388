"""Shared test helpers (tests only)."""
import numpy as np

from oracle import tt


def random_tt(ranks, seed, decay=None):
    rng = np.random.default_rng(seed)
    cores = []
    for n in range(len(ranks) - 1):
        G = rng.standard_normal((ranks[n], 2, ranks[n + 1]))
        if decay is not None:
            G *= decay ** np.arange(ranks[n + 1])[None, None, :]
        cores.append(G)
    return cores


def full(cores):
    """Full tensor (2,)*N of an MPS given as cores (zero padding is harmless)."""
    return tt.tt_full([np.asarray(c) for c in cores])


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def gaussian_sketch(N, ell, seed):
    ranks = [min(ell, 2 ** n, 2 ** (N - n)) for n in range(N + 1)]
    rng = np.random.default_rng(seed)
    cores = [rng.standard_normal((ranks[n], 2, ranks[n + 1])) / np.sqrt(ranks[n]) for n in range(N)]
    return cores, ranks


# Tolerances of FP64 parity for results that went through truncating
# roundings (fixed numbers; tests/test_tolerances.py checks on the CPU that
# each case held to them satisfies the reading they rest on).
#
# The HIP path cuts every bond from the eigen-decomposition of an FP64 Gram
# matrix, whose entries carry absolute noise of about eps sigma_1^2, so
# singular directions below sqrt(eps) sigma_1 (1.5e-8 sigma_1) are not
# resolved; the oracle cuts from SVDs, resolved to about eps sigma_1.
#
# TRUNC_TOL_F64 -- time steps.  Their rounding inputs have weight below that
# floor, where the two may keep different mixtures.  The oracle's own
# schedule with the truncation emulated from LAPACK eigenvectors of Gram
# matrices stays within a third of this bound of the SVD oracle on every
# step case (largest: 2.5e-8 after three steps of the 16^5 grid with the
# x-fields), so 1e-7 leaves a margin of three.
TRUNC_TOL_F64 = 1e-7
# CUT_TOL_F64 -- roundings of random chains whose cuts sit on clear spectral
# gaps far above the floor: only the first-order (Davis-Kahan) movement of
# the kept subspaces remains, below a tenth of 3 sqrt(eps) on every case.
CUT_TOL_F64 = 3.0 * np.sqrt(2.0 ** -52)


def cut_sensitivity(infos, eps=2.2e-16):
    """First-order (Davis-Kahan) relative movement of the simultaneous
    truncations in `infos` (oracle rounding infos with per-bond singular
    values) under a relative perturbation eps of the Gram entries: at a cut
    between sigma_k and sigma_(k+1) the kept subspace turns by about
    m eps sigma_1^2 / (sigma_k^2 - sigma_(k+1)^2), moving the tensor by that
    angle times sigma_k; summed over bonds and roundings, with no cap (a cut
    at a degenerate pair gives infinity)."""
    total = 0.0
    for info in infos:
        for n, s in enumerate(info["sigmas"]):
            if s is None:
                continue
            k = info["ranks"][n]
            if k >= s.size:
                continue
            lam = s ** 2
            gap = lam[k - 1] - lam[k]
            if gap <= 0:
                return np.inf
            total += s.size * eps * lam[0] / gap * s[k - 1] / s[0]
    return total


def trunc_gram_mixed(cores, c, chi):
    """Emulation of the HIP path's truncation (tests only): the simultaneous
    truncation of a mixed canonical TT with every bond cut from the
    eigen-decomposition of its FP64 Gram matrix instead of an SVD."""
    N = len(cores)
    caps = tt.chain_caps(N, chi)
    G = [None] * (N + 1)
    if c >= 1:
        G[c] = np.einsum("ktz,Ktz->kK", cores[c], cores[c], optimize=True)
        for n in range(c - 1, 0, -1):
            G[n] = np.einsum("asb,bc,dsc->ad", cores[n], G[n + 1], cores[n], optimize=True)
    if c + 1 <= N - 1:
        G[c + 1] = np.einsum("ktz,ktZ->zZ", cores[c], cores[c], optimize=True)
        for n in range(c + 1, N - 1):
            G[n + 1] = np.einsum("ysz,yY,YsZ->zZ", cores[n], G[n], cores[n], optimize=True)
    P = [None] * (N + 1)
    for n in range(1, N):
        lam, U = np.linalg.eigh(G[n])
        P[n] = U[:, ::-1][:, :max(1, min(lam.size, caps[n]))]
    out = []
    for n in range(N):
        A = cores[n]
        if n > 0:
            A = np.tensordot(P[n].T, A, axes=(1, 0))
        if n < N - 1:
            A = np.tensordot(A, P[n + 1], axes=(2, 0))
        out.append(A)
    return out


def mps_diff_norm(a, b):
    """|| a - b ||_2 of two MPSs on the same sites (bond dimensions may
    differ), without densifying: the difference is written exactly as a block
    sum, left-orthogonalised by QR, and its norm read off the last core (no
    inner products are subtracted, so no cancellation)."""
    N = len(a)
    cores = []
    for n, (A, B) in enumerate(zip(a, b)):
        A = np.asarray(A, dtype=np.float64)
        B = np.asarray(B, dtype=np.float64)
        if n == 0:
            C = np.concatenate([A, B], axis=2)
        elif n == N - 1:
            C = np.concatenate([A, -B], axis=0)
        else:
            C = np.zeros((A.shape[0] + B.shape[0], 2, A.shape[2] + B.shape[2]))
            C[:A.shape[0], :, :A.shape[2]] = A
            C[A.shape[0]:, :, A.shape[2]:] = B
        cores.append(C)
    return float(np.linalg.norm(tt.left_orthogonalize(cores)[-1]))


def mps_norm(a):
    return float(np.linalg.norm(tt.left_orthogonalize([np.asarray(G, dtype=np.float64) for G in a])[-1]))


def mps_rel(a, b):
    """||a - b|| / ||b|| of two MPSs (see mps_diff_norm)."""
    return mps_diff_norm(a, b) / mps_norm(b)
