"""Quantics tensor-train (MPS / MPO) arithmetic in FP64 -- oracle (test infrastructure).

Conventions
-----------
* An MPS is a list of N cores A_n of shape (r_{n-1}, 2, r_n), r_0 = r_N = 1
  (one binary digit per core: the quantics encoding of the "Matrix product
  state encoding" section, each dimension split lengthscale by lengthscale,
  most significant bit first).
* An MPO is a list of cores W_n of shape (D_{n-1}, 2 (out), 2 (in), D_n).
* A site order is a list of (dimension, bit) pairs; "serial" ordering puts
  every bit of phi1 first, then phi2, x1, x2, x3.

Rounding (bond truncation by singular value decompositions, "Matrix product
state algorithm" section), all FP64 and plain LAPACK:

* ``round_ttsvd``: the textbook sweep -- QR left-orthogonalisation, then a
  right-to-left sweep of truncated SVDs (Oseledets 2011).  This is the
  rounding the paper describes.
* ``trunc_svd``: on a left-orthogonal TT every bond is truncated to its
  leading left singular vectors, taken by SVD of the bond's right factor.
  All bonds are truncated from the same untruncated tensor
  (simultaneously), so ||T - T~||^2 <= sum_n eps_n^2 where eps_n^2 is the
  discarded singular weight at bond n.  ``trunc_svd_mixed`` does the same
  for a mixed canonical TT (orthogonal from both ends towards a centre).
  No Gram matrix is formed, so singular values down to about eps sigma_1
  are resolved.
* ``rand_orth`` / ``rand_orth_two_sided``: randomized range finding for a
  sum of MPO-applied MPSs (Al Daas et al., "Randomized algorithms for
  rounding in the tensor-train format", SISC 2023,
  randomize-then-orthogonalize): partial sketches with Gaussian TTs, then QR
  sweeps on the sketched unfoldings.  The Gaussian sketches are inputs.

``round_det = trunc_svd o left_orthogonalize o right_orthogonalize`` is the
deterministic rounding of an explicit MPS; ``round_sketch = trunc_svd o
rand_orth`` and ``round_sketch_two_sided = trunc_svd_mixed o
rand_orth_two_sided`` round sum_j c_j W_j x_j without forming the bond-(r D)
product.

Pins: tests/test_oracle_tt.py (dense round trip, Kronecker brute force for
MPOs, rounding error bounds, eq. MPSdofs).
"""
from __future__ import annotations

import numpy as np


def _ein(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


# ----------------------------------------------------------------------------
# site orders and dense conversion
# ----------------------------------------------------------------------------


def site_perm(order, bits):
    """Axis permutation from the serial (C-order) bit layout to ``order``."""
    return [d * bits + b for (d, b) in order]


def dense_to_sites(T, order, bits):
    N = len(order)
    return T.reshape((2,) * N).transpose(site_perm(order, bits))


def sites_to_dense(S, order, bits, ndims):
    perm = site_perm(order, bits)
    inv = np.argsort(perm)
    return S.transpose(inv).reshape((1 << bits,) * ndims)


def tt_full(cores):
    """Contract an MPS to its full tensor of shape (2,)*N."""
    T = cores[0]
    for G in cores[1:]:
        T = np.tensordot(T, G, axes=(-1, 0))
    return T.reshape(T.shape[1:-1])


def mpo_full(cores):
    """Contract an MPO to a (2^N x 2^N) matrix, rows = out bits MSB first."""
    N = len(cores)
    T = cores[0]
    for W in cores[1:]:
        T = np.tensordot(T, W, axes=(-1, 0))
    T = T.reshape(T.shape[1:-1])  # (t1, s1, t2, s2, ...)
    perm = [2 * n for n in range(N)] + [2 * n + 1 for n in range(N)]
    return T.transpose(perm).reshape(1 << N, 1 << N)


def tt_svd(T, rel_tol=1e-14, chi=None):
    """TT-SVD of a full tensor T with shape (q,)*N (q = 2 for an MPS)."""
    shape = T.shape
    N = len(shape)
    cores = []
    r = 1
    C = T.reshape(1, -1)
    for n in range(N - 1):
        C = C.reshape(r * shape[n], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        k = max(1, int(np.sum(s > rel_tol * s[0]))) if s[0] > 0 else 1
        if chi is not None:
            k = min(k, chi)
        cores.append(U[:, :k].reshape(r, shape[n], k))
        C = s[:k, None] * Vt[:k]
        r = k
    cores.append(C.reshape(r, shape[-1], 1))
    return cores


def vector_qtt(v, rel_tol=1e-15):
    """QTT of a 1-D vector of length 2^b (TT-SVD)."""
    v = np.asarray(v, dtype=np.float64)
    b = int(np.log2(v.size))
    assert 1 << b == v.size
    return tt_svd(v.reshape((2,) * b), rel_tol)


def operator_qtt(A, rel_tol=1e-14):
    """1-D MPO of a dense (2^b x 2^b) matrix by TT-SVD of its (t_k, s_k) pairs."""
    M = A.shape[0]
    b = int(np.log2(M))
    T = A.reshape((2,) * (2 * b))
    perm = []
    for k in range(b):
        perm += [k, b + k]
    T = T.transpose(perm).reshape((4,) * b)
    cores = tt_svd(T, rel_tol)
    return [G.reshape(G.shape[0], 2, 2, G.shape[-1]) for G in cores]


def identity_mpo(n_sites):
    I = np.eye(2).reshape(1, 2, 2, 1)
    return [I.copy() for _ in range(n_sites)]


# ----------------------------------------------------------------------------
# products over dimensions, sums, MPO algebra
# ----------------------------------------------------------------------------


def _kron_over_dims(per_dim, order, ndims, mpo):
    """Combine per-dimension (Q)TTs into one chain in the given site order.

    per_dim[d] is a list of `bits` cores for dimension d (None = all-ones
    vector for an MPS, identity for an MPO).  At each site the core of its
    dimension is tensored with identities on the bonds of all other
    dimensions; the combined bond index is raveled with dimension 0 slowest.
    """
    bits = len(order) // ndims
    if mpo:
        default = [np.eye(2).reshape(1, 2, 2, 1)] * bits
    else:
        default = [np.ones((1, 2, 1))] * bits
    pd = [per_dim[d] if per_dim[d] is not None else default for d in range(ndims)]
    pos = [0] * ndims
    bond = lambda d, p: pd[d][p].shape[0] if p < bits else 1  # noqa: E731
    out = []
    for (d, b) in order:
        assert pos[d] == b
        G = pd[d][b]
        pre = int(np.prod([bond(e, pos[e]) for e in range(d)]))
        post = int(np.prod([bond(e, pos[e]) for e in range(d + 1, ndims)]))
        Ip, Iq = np.eye(pre), np.eye(post)
        if mpo:
            K = _ein("pP,atsb,qQ->paqtsPbQ", Ip, G, Iq)
            K = K.reshape(pre * G.shape[0] * post, 2, 2, pre * G.shape[-1] * post)
        else:
            K = _ein("pP,asb,qQ->paqsPbQ", Ip, G, Iq)
            K = K.reshape(pre * G.shape[0] * post, 2, pre * G.shape[-1] * post)
        out.append(K)
        pos[d] += 1
    return out


def mps_product(per_dim, order, ndims):
    return _kron_over_dims(per_dim, order, ndims, mpo=False)


def mpo_product(per_dim, order, ndims):
    return _kron_over_dims(per_dim, order, ndims, mpo=True)


def mps_sum(terms):
    """sum_j c_j x_j as a block-diagonal MPS (exact, bonds add up)."""
    N = len(terms[0][1])
    if N == 1:
        return [sum(c * x[0] for c, x in terms)]
    out = []
    for n in range(N):
        blocks = [x[n] for _, x in terms]
        if n == 0:
            out.append(np.concatenate([c * x[0] for c, x in terms], axis=2))
        elif n == N - 1:
            out.append(np.concatenate(blocks, axis=0))
        else:
            rl = sum(G.shape[0] for G in blocks)
            rr = sum(G.shape[2] for G in blocks)
            G = np.zeros((rl, 2, rr))
            i = j = 0
            for B in blocks:
                G[i:i + B.shape[0], :, j:j + B.shape[2]] = B
                i += B.shape[0]
                j += B.shape[2]
            out.append(G)
    return out


def mpo_compose(A, B):
    """MPO of the matrix product A @ B."""
    out = []
    for Wa, Wb in zip(A, B):
        W = _ein("atub,cusd->actsbd", Wa, Wb)
        out.append(W.reshape(Wa.shape[0] * Wb.shape[0], 2, 2, Wa.shape[3] * Wb.shape[3]))
    return out


def mpo_diag(x):
    """MPO of diag(x) for an MPS x: W[a,t,s,b] = x[a,s,b] delta_ts."""
    out = []
    for G in x:
        W = np.zeros((G.shape[0], 2, 2, G.shape[2]))
        W[:, 0, 0, :] = G[:, 0, :]
        W[:, 1, 1, :] = G[:, 1, :]
        out.append(W)
    return out


def mpo_apply(W, x):
    """Exact MPO x MPS product (bond r*D)."""
    out = []
    for Wn, G in zip(W, x):
        Y = _ein("atsb,csd->catdb", Wn, G)
        out.append(Y.reshape(G.shape[0] * Wn.shape[0], 2, G.shape[2] * Wn.shape[3]))
    return out


def inner(a, b):
    E = np.ones((1, 1))
    for A, B in zip(a, b):
        E = _ein("ab,asc,bsd->cd", E, A, B)
    return float(E[0, 0])


def ranks(cores):
    return [1] + [G.shape[-1] for G in cores]


# ----------------------------------------------------------------------------
# rounding
# ----------------------------------------------------------------------------


def chain_caps(N, chi):
    return [min(chi, 1 << n, 1 << (N - n)) for n in range(N + 1)]


def left_orthogonalize(cores):
    """QR sweep left to right; returns a left-orthogonal copy (last core carries the norm)."""
    out = [G.copy() for G in cores]
    N = len(out)
    for n in range(N - 1):
        rl, _, rr = out[n].shape
        Q, R = np.linalg.qr(out[n].reshape(rl * 2, rr))
        k = Q.shape[1]
        out[n] = Q.reshape(rl, 2, k)
        out[n + 1] = np.tensordot(R, out[n + 1], axes=(1, 0))
    return out


def round_ttsvd(cores, chi, rel_tol=1e-14):
    """Textbook TT rounding: QR sweep, then right-to-left truncated SVDs.

    Returns (cores, discarded) with discarded[n] the sum of the squared
    singular values dropped at bond n (n = 1..N-1).
    """
    X = left_orthogonalize(cores)
    N = len(X)
    caps = chain_caps(N, chi)
    disc = [0.0] * (N + 1)
    for n in range(N - 1, 0, -1):
        rl, _, rr = X[n].shape
        U, s, Vt = np.linalg.svd(X[n].reshape(rl, 2 * rr), full_matrices=False)
        k = max(1, int(np.sum(s > rel_tol * s[0]))) if s[0] > 0 else 1
        k = min(k, caps[n])
        disc[n] = float(np.sum(s[k:] ** 2))
        X[n] = Vt[:k].reshape(k, 2, rr)
        X[n - 1] = np.tensordot(X[n - 1], U[:, :k] * s[:k], axes=(2, 0))
    return X, disc


def _cut(s, cap, rel_tol):
    """Number of singular values kept at a bond: at most cap, with rel_tol > 0
    also only those above rel_tol * sigma_1 (at least one)."""
    k = s.size
    if rel_tol > 0 and s.size and s[0] > 0:
        k = int(np.sum(s > rel_tol * s[0]))
    return max(1, min(k, cap))


def _project(cores, P):
    """Cores P_n^T A_n P_(n+1) (P_0 = P_N = None: no projection)."""
    N = len(cores)
    out = []
    for n in range(N):
        A = cores[n]
        if n > 0:
            A = np.tensordot(P[n].T, A, axes=(1, 0))
        if n < N - 1:
            A = np.tensordot(A, P[n + 1], axes=(2, 0))
        out.append(A)
    return out


def _right_factors(cores, last, first):
    """Left singular vectors and singular values of the right factor at bonds
    last, last-1, ..., first, for a chain whose cores right of `last` are
    right-orthogonal: at bond `last` the factor is core `last` itself
    (rows = its left bond); going left, the factor at bond n is core n
    contracted with U_(n+1) S_(n+1), the factor of bond n+1 up to its
    orthogonal right part.  SVDs of these factors, never of their Gram
    matrices, so singular values far below sqrt(eps) sigma_1 are resolved."""
    U, S = {}, {}
    C = None
    for n in range(last, first - 1, -1):
        A = cores[n]
        B = A if C is None else np.tensordot(A, C, axes=(2, 0))
        u, s, _ = np.linalg.svd(B.reshape(B.shape[0], -1), full_matrices=False)
        U[n], S[n] = u, s
        C = u * s
    return U, S


def _left_factors(cores, first, last):
    """Mirror image of _right_factors: right singular vectors and singular
    values of the left factor at bonds first+1, ..., last+1 for a chain whose
    cores left of `first` are left-orthogonal (bond n + 1 is right of core n)."""
    V, S = {}, {}
    C = None
    for n in range(first, last + 1):
        A = cores[n]
        B = A if C is None else np.tensordot(C, A, axes=(1, 0))
        _, s, vt = np.linalg.svd(B.reshape(-1, B.shape[2]), full_matrices=False)
        V[n + 1], S[n + 1] = vt.T, s
        C = s[:, None] * vt
    return V, S


def _trunc_from_factors(cores, chi, rel_tol, vecs, svals):
    N = len(cores)
    caps = chain_caps(N, chi)
    P = [None] * (N + 1)
    ranks_out = [1] * (N + 1)
    disc = [0.0] * (N + 1)
    sig = [None] * (N + 1)
    for n in range(1, N):
        s = svals[n]
        k = _cut(s, caps[n], rel_tol)
        P[n] = vecs[n][:, :k]
        ranks_out[n] = k
        disc[n] = float(np.sum(s[k:] ** 2))
        sig[n] = s
    s1 = svals[1]
    return _project(cores, P), {"ranks": ranks_out, "discarded": disc,
                                "norm2": float(np.sum(s1 ** 2)), "sigmas": sig}


def trunc_svd(X, chi, rel_tol=0.0):
    """Simultaneous SVD truncation of every bond of a left-orthogonal TT.

    At bond n the unfolding is Left_n Right_n with Left_n orthonormal, so its
    singular values and left singular vectors are those of the right factor
    Right_n, taken by SVD (``_right_factors``).  Keep the k_n = min(cap_n, .)
    leading left singular vectors P_n (with rel_tol > 0, also only those
    above rel_tol * sigma_1) and form the cores P_(n-1)^T X_n P_n.  All bonds
    are cut from the same untruncated tensor, so ||T - T~||^2 <= sum_n of the
    discarded sigma^2, and when cap_n covers the bond nothing is dropped.
    Returns (cores, info) with info = {"ranks", "discarded" (sum of dropped
    sigma^2 per bond), "norm2", "sigmas" (singular values per bond,
    descending)}.
    """
    N = len(X)
    if N == 1:
        return [X[0].copy()], {"ranks": [1, 1], "discarded": [0.0, 0.0],
                               "norm2": float(np.sum(X[0] ** 2)), "sigmas": [None, None]}
    U, S = _right_factors(X, N - 1, 1)
    return _trunc_from_factors(X, chi, rel_tol, U, S)


def right_orthogonalize(cores):
    """LQ sweep right to left; returns a right-orthogonal copy (first core carries the norm)."""
    rev = [np.ascontiguousarray(G.transpose(2, 1, 0)) for G in cores[::-1]]
    out = left_orthogonalize(rev)
    return [np.ascontiguousarray(G.transpose(2, 1, 0)) for G in out[::-1]]


def round_det(cores, chi, rel_tol=0.0):
    """Deterministic rounding of an explicit MPS.

    An LQ sweep (right to left) and a QR sweep (left to right) bring every
    bond down to at most min(2^n, 2^(N-n), input bond) with a left-orthogonal
    TT; the simultaneous SVD truncation then cuts each bond to chi.
    """
    return trunc_svd(left_orthogonalize(right_orthogonalize(cores)), chi, rel_tol)


def _as_term(t):
    c, W, x = t
    if W is None:
        W = identity_mpo(len(x))
    return c, W, x


def rand_orth(terms, Z, ell):
    """Randomized range finding for Y = sum_j c_j W_j x_j.

    terms: [(c_j, W_j or None, x_j)].  Z: Gaussian TT cores (ell_{n-1}, 2, ell_n),
    ell: sketch ranks ell_0..ell_N.  Returns a left-orthogonal TT X with ranks
    ell (its last core carries the norm) that spans the sketched ranges:

    right sketches  Wsk_n = Right_n(Y) Right_n(Z)^T,
    left sweep      S_n = [Q_{n-1}^T ... Y]_n Wsk_{n+1},  Q_n = qr(S_n).
    """
    terms = [_as_term(t) for t in terms]
    N = len(Z)
    J = len(terms)
    # right partial sketches: R[j][n] has shape (r_{n}, D_{n}, ell_{n}) for the bond
    # left of site n (0-based), R[j][N] = ones((1,1,1))
    R = []
    for (c, W, x) in terms:
        Rj = [None] * (N + 1)
        Rj[N] = np.ones((1, 1, 1))
        for n in range(N - 1, 0, -1):
            T1 = _ein("bBy,zty->bBtz", Rj[n + 1], Z[n])
            T2 = _ein("AtsB,bBtz->bAsz", W[n], T1)
            Rj[n] = _ein("asb,bAsz->aAz", x[n], T2)
        R.append(Rj)
    X = []
    Mj = [np.ones((1, 1, 1)) for _ in range(J)]  # (ell_{n-1}, r_{n-1}, D_{n-1})
    for n in range(N - 1):
        Cs = []
        S = 0.0
        for j, (c, W, x) in enumerate(terms):
            U1 = _ein("kaA,asb->kAsb", Mj[j], x[n])
            C = _ein("kAsb,AtsB->ktbB", U1, W[n])
            Cs.append(C)
            S = S + c * _ein("ktbB,bBz->ktz", C, R[j][n + 1])
        lp = S.shape[0]
        S = S.reshape(lp * 2, -1)
        Q, _ = np.linalg.qr(S)
        ln = Q.shape[1]
        X.append(Q.reshape(lp, 2, ln))
        Q3 = Q.reshape(lp, 2, ln)
        Mj = [_ein("ktz,ktbB->zbB", Q3, C) for C in Cs]
    last = 0.0
    for j, (c, W, x) in enumerate(terms):
        U1 = _ein("kaA,asb->kAsb", Mj[j], x[N - 1])
        C = _ein("kAsb,AtsB->ktbB", U1, W[N - 1])
        last = last + c * C.reshape(C.shape[0], 2, 1)
    X.append(last)
    return X


def round_sketch(terms, Z, ell, chi, rel_tol=0.0):
    return trunc_svd(rand_orth(terms, Z, ell), chi, rel_tol)


def rand_orth_two_sided(terms, Zr, Zl, c=None):
    """Two-sided randomized range finding for Y = sum_j c_j W_j x_j.

    The chain is orthogonalised from both ends towards a centre site c
    (default N // 2): bonds 1..c get left-orthogonal cores X_0..X_(c-1) from
    the right sketches Right_n(Y) Right_n(Zr)^T (the one-sided sweep of
    rand_orth stopped at c); bonds c+1..N-1 get right-orthogonal cores
    V_(c+1)..V_(N-1) from the left sketches Left_n(Zl)^T Left_n(Y), sweeping
    from the right end.  The centre core is X_(<c)^T Y V_(>c)^T.  Returns
    (cores, c): a mixed canonical TT with ranks ell (those of the sketches).
    """
    terms = [_as_term(t) for t in terms]
    N = len(Zr)
    if c is None:
        c = N // 2
    # right partial sketches R[j][n] (r_n, D_n, ell_n), bond left of site n
    R = []
    for (_, W, x) in terms:
        Rj = [None] * (N + 1)
        Rj[N] = np.ones((1, 1, 1))
        for n in range(N - 1, 0, -1):
            T1 = _ein("bBy,zty->bBtz", Rj[n + 1], Zr[n])
            T2 = _ein("AtsB,bBtz->bAsz", W[n], T1)
            Rj[n] = _ein("asb,bAsz->aAz", x[n], T2)
        R.append(Rj)
    # left partial sketches L[j][n] (ell_n, r_n, D_n), bond left of site n
    Lk = []
    for (_, W, x) in terms:
        Lj = [None] * (N + 1)
        Lj[0] = np.ones((1, 1, 1))
        for n in range(N - 1):
            T1 = _ein("yaA,ytz->aAtz", Lj[n], Zl[n])
            T2 = _ein("AtsB,aAtz->aBsz", W[n], T1)
            Lj[n + 1] = _ein("asb,aBsz->zbB", x[n], T2)
        Lk.append(Lj)
    # left sweep over sites 0..c-1
    X = []
    Mj = [np.ones((1, 1, 1)) for _ in terms]  # (ell_n, r_n, D_n)
    for n in range(c):
        Cs = []
        S = 0.0
        for j, (cj, W, x) in enumerate(terms):
            C = _ein("kAsb,AtsB->ktbB", _ein("kaA,asb->kAsb", Mj[j], x[n]), W[n])
            Cs.append(C)
            S = S + cj * _ein("ktbB,bBz->ktz", C, R[j][n + 1])
        lp = S.shape[0]
        Q, _ = np.linalg.qr(S.reshape(lp * 2, -1))
        Q3 = Q.reshape(lp, 2, Q.shape[1])
        X.append(Q3)
        Mj = [_ein("ktz,ktbB->zbB", Q3, C) for C in Cs]
    # right sweep over sites N-1..c+1
    V = [None] * N
    Mr = [np.ones((1, 1, 1)) for _ in terms]  # (r_n, D_n, ell_n) right of bond n
    for n in range(N - 1, c, -1):
        Cs = []
        S = 0.0
        for j, (cj, W, x) in enumerate(terms):
            C = _ein("AtsB,asBz->aAtz", W[n], _ein("asb,bBz->asBz", x[n], Mr[j]))
            Cs.append(C)
            S = S + cj * _ein("yaA,aAtz->ytz", Lk[j][n], C)
        ln = S.shape[0]
        rr = S.shape[2]
        Q, _ = np.linalg.qr(S.reshape(ln, 2 * rr).T)  # S = (Q R)^T: rows of Q^T orthonormal
        V3 = Q.T.reshape(Q.shape[1], 2, rr)
        V[n] = V3
        Mr = [_ein("aAtz,ytz->aAy", C, V3) for C in Cs]
    # centre core
    G = 0.0
    for j, (cj, W, x) in enumerate(terms):
        C = _ein("kAsb,AtsB->ktbB", _ein("kaA,asb->kAsb", Mj[j], x[c]), W[c])
        G = G + cj * _ein("ktbB,bBz->ktz", C, Mr[j])
    return X + [G] + V[c + 1:], c


def trunc_svd_mixed(cores, c, chi, rel_tol=0.0):
    """Simultaneous SVD truncation of a mixed canonical TT (cores 0..c-1 left
    orthogonal, c+1..N-1 right orthogonal).  At a bond n <= c the left part
    is orthonormal, so the singular structure is that of the right factor:
    the centre core, then going left through X_(c-1)..X_n (``_right_factors``
    from the centre); at a bond n > c the right part is orthonormal and the
    left factor decides: the centre core, then going right through
    V_(c+1).. (``_left_factors``).  With P_n the leading singular vectors,
    the cores become P_n^T A_n P_(n+1).  Returns (cores, info) as trunc_svd."""
    N = len(cores)
    if N == 1:
        return [cores[0].copy()], {"ranks": [1, 1], "discarded": [0.0, 0.0],
                                   "norm2": float(np.sum(cores[0] ** 2)), "sigmas": [None, None]}
    vecs, svals = {}, {}
    if c >= 1:
        U, S = _right_factors(cores, c, 1)
        vecs.update(U)
        svals.update(S)
    if c + 1 <= N - 1:
        V, S = _left_factors(cores, c, N - 2)
        vecs.update(V)
        svals.update(S)
    return _trunc_from_factors(cores, chi, rel_tol, vecs, svals)


def round_sketch_two_sided(terms, Zr, Zl, chi, rel_tol=0.0, c=None):
    cores, c = rand_orth_two_sided(terms, Zr, Zl, c)
    return trunc_svd_mixed(cores, c, chi, rel_tol)


# ----------------------------------------------------------------------------
# eq. MPSdofs
# ----------------------------------------------------------------------------


def nvpp(N, chi):
    """Number of variables parameterising the PDF, eq. MPSdofs."""
    p = lambda n: min(2**n, 2 ** (N - n), chi)  # noqa: E731
    return 2 * sum(p(n - 1) * p(n) for n in range(1, N + 1)) - sum(p(n) ** 2 for n in range(1, N))
