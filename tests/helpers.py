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


def truncation_sensitivity(infos, eps=2.2e-16):
    """First-order size of the change of a simultaneous SVD truncation under
    rounding noise, relative to the norm: at bond n the kept subspace of the
    Gram matrix moves by an angle ~ m eps lambda_1 / (lambda_k - lambda_{k+1})
    (Davis-Kahan), at most 1 (a cut among eigenvalues at the noise level can
    turn the kept vectors by any angle); the tensor moves by that angle times
    sigma_k.  Summed over bonds and roundings.  Bonds with nothing discarded
    contribute nothing."""
    total = 0.0
    for info in infos:
        lams, ranks = info["lams"], info["ranks"]
        for n, lam in enumerate(lams):
            if lam is None:
                continue
            k = ranks[n]
            if k >= lam.size:
                continue
            l1 = max(lam[0], 1e-300)
            gap = max(lam[k - 1] - lam[k], 1e-300 * l1)
            sk = np.sqrt(max(lam[k - 1], 0.0))
            total += min(1.0, lam.size * eps * l1 / gap) * sk / np.sqrt(l1)
    return total
