"""Prolongation of x-fields (tt_prolong) against the oracle's dense periodic
linear interpolation (needs an MI355X)."""
import numpy as np
import pytest

import workloads
from oracle import fields, tt
from tests.helpers import rel

q = pytest.importorskip("paper_2407_09169_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


def _dense(cores, bits, ndims):
    return tt.tt_full([np.asarray(G) for G in cores]).reshape((1 << bits,) * ndims)


def _field(M, seed, decay):
    """A periodic field with a decaying Fourier spectrum on an M^3 grid."""
    rng = np.random.default_rng(seed)
    F = np.zeros((M, M, M))
    x = np.arange(M) / M
    for k in range(1, 6):
        a = rng.standard_normal(3) * decay ** k
        th = rng.uniform(0, 2 * np.pi, 3)
        F += a[0] * np.einsum("i,j,k->ijk", np.cos(2 * np.pi * k * x + th[0]), np.sin(2 * np.pi * x + th[1]),
                              np.ones(M))
        F += a[1] * np.einsum("i,j,k->ijk", np.ones(M), np.cos(2 * np.pi * k * x + th[1]),
                              np.cos(2 * np.pi * (k - 1) * x + th[2]))
        F += a[2] * np.cos(2 * np.pi * k * (x[:, None, None] + x[None, :, None] + x[None, None, :]) + th[2])
    return F


@pytest.mark.parametrize("bits", [3, 4])
def test_prolong_untruncated_matches_oracle(ctx, bits):
    M = 1 << bits
    F = _field(M, 11 + bits, 0.6)
    x = q.TT.from_cores(ctx, tt.tt_svd(F.reshape((2,) * (3 * bits)), rel_tol=1e-14))
    y, disc = q.prolong(ctx, x, 3, bits, 1024)
    want = fields.prolong_dense(F)
    assert rel(_dense(y.cores(), bits + 1, 3), want) < 1e-12
    assert disc < 1e-20 * np.sum(want ** 2)


def test_prolong_truncated_is_quasi_optimal(ctx):
    """Cut to chi = 6 after every dimension: within a factor 2 of the
    oracle's TT-SVD of the fine field at the same chi, and the discarded
    weight bounds the error."""
    bits = 4
    F = _field(1 << bits, 17, 0.8)
    x = q.TT.from_cores(ctx, tt.tt_svd(F.reshape((2,) * (3 * bits)), rel_tol=1e-14))
    y, disc = q.prolong(ctx, x, 3, bits, 6)
    cores, G = fields.prolong_tt(F, 6)
    e_gpu = np.linalg.norm(_dense(y.cores(), bits + 1, 3) - G)
    e_opt = np.linalg.norm(tt.tt_full(cores).reshape(G.shape) - G)
    assert e_opt > 1e-6 * np.linalg.norm(G)  # truncation is active
    assert e_gpu <= 2.0 * e_opt
    assert e_gpu <= (1 + 1e-6) * np.sqrt(disc) * np.sqrt(3) + 1e-12


def test_prolong_full_size_sampled(ctx):
    """The seeded separable x-field on the 256^3 grid prolonged twice to
    1024^3 (bond 16, nothing cut), checked on 400 sampled points against the
    interpolation of its separable terms (interpolation acts axis by axis, so
    each 1-D vector is interpolated on its own)."""
    w = workloads.get_workload("t_5d_M8_chi16", bits=8)
    terms = workloads.flow_field_terms(w)["G"]
    x = q.from_separable(ctx, 3, 8, q.TT_SERIAL, terms, 16)
    y1, d1 = q.prolong(ctx, x, 3, 8, 16)
    y2, d2 = q.prolong(ctx, y1, 3, 9, 16)
    cores = [np.asarray(G) for G in y2.cores()]
    assert len(cores) == 30
    M = 1024
    ones = np.ones(256)
    fine = [(c, [fields.prolong_dense(fields.prolong_dense(ones if v is None else v)) for v in vecs])
            for c, vecs in terms]
    rng = np.random.default_rng(5)
    pts = rng.integers(0, M, size=(400, 3))
    pts[:8] = [[0, 0, 0], [M - 1, M - 1, M - 1], [1, 2, 3], [M - 1, 0, 1], [511, 512, 513], [2, 1023, 7],
               [1023, 1, 1022], [3, 3, 3]]
    got, want = [], []
    for p in pts:
        bitsq = [int(b) for d in range(3) for b in format(int(p[d]), "010b")]
        v = np.ones((1,))
        for n, G in enumerate(cores):
            v = v @ G[:, bitsq[n], :]
        got.append(float(v[0]))
        want.append(sum(c * u[0][p[0]] * u[1][p[1]] * u[2][p[2]] for c, u in fine))
    got, want = np.array(got), np.array(want)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert d1 + d2 < 1e-20
