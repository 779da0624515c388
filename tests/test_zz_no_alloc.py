"""tt_inner_noalloc (the entry point that allocates no device memory) against
tt_inner on the same inputs, through the C ABI: two calls in a row, the
second with smaller chains, each agreeing to the FP64 bar (both run the same
kernels in the same order, so the results are expected bitwise equal; the
test allows 1e-14 relative)."""
import numpy as np
import pytest

from tests.helpers import random_tt

q = pytest.importorskip("paper_2407_09169_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


def _pair(ctx, N, cap, seed):
    caps = [min(2 ** n, 2 ** (N - n), cap) for n in range(N + 1)]
    a = random_tt(caps, seed)
    b = random_tt(caps, seed + 1)
    return q.TT.from_cores(ctx, a), q.TT.from_cores(ctx, b)


def test_inner_noalloc_matches_inner(ctx):
    import torch
    out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    for N, cap, seed in ((24, 160, 71), (12, 24, 73)):  # the second call is smaller
        a, b = _pair(ctx, N, cap, seed)
        ref = q.inner(ctx, a, b)
        q.inner_noalloc(ctx, a, b, out)
        ctx.synchronize()
        got = float(out.cpu()[0])
        print(f"N={N} cap={cap}: inner {ref:.17g} noalloc {got:.17g}", flush=True)
        assert np.isfinite(got)
        assert abs(got - ref) <= 1e-14 * abs(ref), (N, cap, got, ref)


def test_inner_noalloc_rejects_oversize(ctx):
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    a, b = _pair(ctx, 22, 1024, 75)  # environments of 1024 x 1024: beyond the buffer
    with pytest.raises(q.QttError, match="static scratch"):
        q.inner_noalloc(ctx, a, b, out)
    assert float(out.cpu()[0]) == 0.0
