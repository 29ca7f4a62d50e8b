"""The entry point that allocates nothing (vr_relabel_min_noalloc) against
vr_relabel_min, through the C ABI: the same canonical labels, bit for bit,
on two calls in a row (the second smaller, so it must not see what the
first left in the shared scratch), no workspace taken from the context, and
sizes beyond the fixed scratch refused."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def labels(rng, n, n_groups):
    """Canonical labels (smallest member of each group; -1 for none), group
    sizes spread around the min_size used below."""
    g = rng.integers(0, n_groups, n)
    g[rng.random(n) < 0.1] = -1
    low = np.full(n_groups, n, np.int64)
    ok = g >= 0
    np.minimum.at(low, g[ok], np.nonzero(ok)[0])
    return np.where(ok, low[np.maximum(g, 0)], -1).astype(np.int32)


def test_noalloc_matches_relabel_min():
    from paper_1902_01010_amd import vr
    ctx = vr.Context(0)
    rng = np.random.default_rng(77)
    for n, ng, min_size in ((3_000_000, 150_000, 20), (200_000, 40_000, 5)):
        lab = torch.from_numpy(labels(rng, n, ng)).cuda()
        ref = ctx.relabel_min(lab, min_size).cpu().numpy()
        before = ctx.workspace_bytes()
        out = torch.full((n,), -9, dtype=torch.int32, device="cuda")
        got = ctx.relabel_min_noalloc(lab, min_size, out=out).cpu().numpy()
        assert ctx.workspace_bytes() == before
        np.testing.assert_array_equal(got, ref)
        assert (ref >= 0).any() and (ref < 0).any()
    # a fresh context that never allocated: the call takes no workspace
    fresh = vr.Context(0)
    small = torch.from_numpy(labels(rng, 1000, 40)).cuda()
    got = fresh.relabel_min_noalloc(small, 10).cpu().numpy()
    assert fresh.workspace_bytes() == 0
    np.testing.assert_array_equal(got, ctx.relabel_min(small, 10).cpu().numpy())
    # beyond the fixed scratch, and a label >= n: errors, nothing hangs
    big = torch.zeros(vr.NOALLOC_MAX_LABELS + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(vr.VrError) as e:
        fresh.relabel_min_noalloc(big, 1)
    assert e.value.code == vr.VR_ERR_INVALID_ARG and "fixed scratch" in str(e.value)
    bad = small.clone()
    bad[3] = 5000
    with pytest.raises(vr.VrError):
        fresh.relabel_min_noalloc(bad, 1)
    # and it still works after the error
    np.testing.assert_array_equal(fresh.relabel_min_noalloc(small, 10).cpu().numpy(), got)
    fresh.close()
    ctx.close()
