"""The allocation-free scores entry point (MI355X only).

fsa_scores_noalloc takes fsa_scores' arguments and runs its kernels, but
stages everything in a fixed device array instead of allocating.  Checked
through the C ABI: the same scores as fsa_scores on two calls in a row (the
second smaller, so stale staged values from the first would show), no block
requested from a registered allocator (fsa_scores requests its blocks there),
its counter of bad variances cleared between calls, and sizes beyond the
fixed array refused on the host."""
import sys

import numpy as np
import pytest

from oracle import fsa_oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    from paper_2405_14492_amd import fsa
    fsa.lib()
    return fsa


def data(n, seed):
    rng = np.random.default_rng(seed)
    y = rng.normal(size=n)
    mu = y + 0.3 * rng.normal(size=n)
    var = rng.uniform(0.05, 2.0, size=n)
    return y, mu, var


def test_noalloc_scores_match_fsa_scores_on_two_calls(F):
    import torch
    alloc = F.TorchAllocator()
    F.fsa_set_allocator(alloc)
    try:
        for call, n in enumerate((200_000, 1_537)):
            say(f"case: fsa_scores_noalloc call {call} n={n}")
            y, mu, var = data(n, 40 + call)
            before = alloc.allocs
            got = F.fsa_scores_noalloc(y, mu, var)
            assert alloc.allocs == before, "the allocation-free entry point requested a device block"
            ref = F.fsa_scores(y, mu, var)
            assert alloc.allocs > before  # the allocating one goes through the registered allocator
            assert np.array_equal(np.array(got), np.array(ref)), (got, ref)
            np.testing.assert_allclose(got, O.scores(y, mu, var), rtol=1e-12)
        torch.cuda.synchronize()
    finally:
        F.fsa_set_allocator(None)
    F.fsa_pool_trim()
    assert alloc.releases == alloc.allocs and not alloc.live


def test_noalloc_counter_is_cleared_and_limits_are_checked(F):
    y, mu, var = data(5000, 7)
    bad = var.copy()
    bad[17] = -1.0
    say("case: fsa_scores_noalloc with one bad variance, then a good call")
    with pytest.raises(F.FsaError):
        F.fsa_scores_noalloc(y, mu, bad)
    got = F.fsa_scores_noalloc(y, mu, var)
    assert np.array_equal(np.array(got), np.array(F.fsa_scores(y, mu, var)))
    say("case: fsa_scores_noalloc past its fixed size is refused on the host")
    big = F.SCORES_NOALLOC_MAX_N + 1
    z = np.ones(big)
    with pytest.raises(F.FsaError, match="exceeds its fixed scratch"):
        F.fsa_scores_noalloc(z, z, z)
    # the largest size it accepts
    y2, mu2, var2 = data(F.SCORES_NOALLOC_MAX_N, 9)
    got = F.fsa_scores_noalloc(y2, mu2, var2)
    assert np.array_equal(np.array(got), np.array(F.fsa_scores(y2, mu2, var2)))
