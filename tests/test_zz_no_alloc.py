"""The allocation-free mature entry point (swgs_mature_noalloc) against the
allocating one (swgs_mature), through the C ABI: the same record bytes, the
same pool afterwards, on two calls in a row (the second on a smaller pool,
so the shared scratch holds the first call's contents), and the size limit
rejected before anything is launched."""
import sys

import numpy as np
import pytest
import torch

from paper_2409_07759_amd import synth as S

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def sw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_07759_amd import swgs
    return swgs


def test_mature_noalloc_equals_mature_on_two_calls(sw):
    ctx = sw.Context(0)
    for num_gs, swin, deg, st, seed in ((6000, 5, 3, 7, 31), (1500, 3, 1, 9, 32)):
        say("mature noalloc", num_gs, swin, deg, st)
        pool = S.steady_window_pool(num_gs, swin, deg, st, seed)
        a = sw.Pool.from_synth(pool, train=False)
        b = sw.Pool.from_synth(pool, train=False)
        rec_a, cnt_a = sw.mature(ctx, a, st + 1)
        buf = torch.full((sw.swgs_record_bytes(num_gs, deg),), 0xAB, dtype=torch.uint8, device="cuda")
        rec_b, cnt_b = sw.mature_noalloc(ctx, b, st + 1, buf)
        assert cnt_a == cnt_b == num_gs // swin
        assert rec_a.numel() == rec_b.numel()
        assert torch.equal(rec_a, rec_b)
        for name in ("params", "birth", "start", "expire"):
            assert np.array_equal(host(getattr(a, name)), host(getattr(b, name))), name
    ctx.close()


def test_mature_noalloc_rejects_pools_beyond_its_scratch(sw):
    ctx = sw.Context(0)
    n = int(sw.swgs_mature_noalloc_max_gs()) + 1
    say("mature noalloc limit", n)
    z = np.zeros(2 * n, np.int32)
    big = sw.Pool(np.zeros((14, 2 * n), np.float32), z, z, z + 1, n, 4, 0, "cuda", train=False)
    rec = torch.empty(sw.swgs_record_bytes(n, 0), dtype=torch.uint8, device="cuda")
    with pytest.raises(sw.SwgsError) as e:
        sw.mature_noalloc(ctx, big, 1, rec)
    assert e.value.status == sw.SWGS_ERR_CAPACITY
    assert host(big.start).max() == 0        # nothing was written
    ctx.close()
