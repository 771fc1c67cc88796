"""The allocation-free Gram entry point (bkts_gram_noalloc) against bkts_gram through the C ABI.

Each case makes two calls in a row, the second on a smaller block, so the second result must not
depend on partials left in the shared scratch array by the first.  Both results are also checked
against an FP64 product on the host, and free device memory must not change across the calls.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# (dtype, k, ld, first N, second N)
CASES = [
    ("f64", 16, 16, 300001, 4099),
    ("f32", 4, 4, 2000000, 1000),
    ("f64", 32, 40, 50000, 77),
    ("f32", 3, 3, 123457, 1),
    ("f64", 8, 8, 70001, 2),
]


def _block(torch, N, k, ld, dtype, seed):
    rng = np.random.default_rng(seed)
    full = rng.standard_normal((N, ld))
    t = torch.from_numpy(full).to(torch.float64 if dtype == "f64" else torch.float32).cuda()
    return t[:, :k]


def test_gram_noalloc_matches_gram():
    import torch
    from paper_2504_02117_amd import bkts
    assert torch.cuda.is_available()
    ctx = bkts.bkts_ctx_create(0, torch.cuda.current_stream())
    try:
        # warm the module and torch's caching allocator before watching free memory
        blocks = []
        for ci, (dtype, k, ld, n1, n2) in enumerate(CASES):
            for n, s in ((n1, 10 * ci), (n2, 10 * ci + 5)):
                blocks.append((dtype, k, n, _block(torch, n, k, ld, dtype, s), _block(torch, n, k, ld, dtype, s + 1)))
        outs = [(torch.zeros((b[1], b[1]), dtype=torch.float64, device="cuda"),
                 torch.full((b[1], b[1]), 7.0, dtype=torch.float64, device="cuda")) for b in blocks]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for (dtype, k, n, X, Y), (g_ref, g_na) in zip(blocks, outs):
            say(f"gram_noalloc {dtype} k={k} ld={X.stride(0)} N={n}")
            bkts.bkts_gram_noalloc(ctx, X, Y, g_na)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 == free0, (free0, free1)
        for (dtype, k, n, X, Y), (g_ref, g_na) in zip(blocks, outs):
            bkts.bkts_gram(ctx, X, Y, g_ref)
        torch.cuda.synchronize()
        for (dtype, k, n, X, Y), (g_ref, g_na) in zip(blocks, outs):
            ref = g_ref.cpu().numpy()
            got = g_na.cpu().numpy()
            host = X.double().cpu().numpy().T @ Y.double().cpu().numpy()
            scale = max(np.abs(host).max(), 1.0)
            assert np.abs(got - ref).max() <= 1e-12 * scale, (dtype, k, n)
            assert np.abs(got - host).max() <= 1e-11 * scale, (dtype, k, n)
    finally:
        torch.cuda.synchronize()
        bkts.bkts_ctx_destroy(ctx)


def test_gram_noalloc_rejections():
    import torch
    from paper_2504_02117_amd import bkts
    ctx = bkts.bkts_ctx_create(0, torch.cuda.current_stream())
    try:
        X = torch.zeros((10, 4), dtype=torch.float64, device="cuda")
        G = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
        with pytest.raises(bkts.BktsError) as e:  # ld < k
            bkts._check(bkts._lib.bkts_gram_noalloc(ctx, bkts.BKTS_F64, 10, 4, bkts._ptr(X), 3, bkts._ptr(X), 4,
                                                    bkts._ptr(G)))
        assert e.value.status == bkts.BKTS_EINVAL
        with pytest.raises(bkts.BktsError) as e:  # k beyond the maximum block width
            bkts._check(bkts._lib.bkts_gram_noalloc(ctx, bkts.BKTS_F64, 10, 33, bkts._ptr(X), 33, bkts._ptr(X), 33,
                                                    bkts._ptr(G)))
        assert e.value.status == bkts.BKTS_EINVAL
    finally:
        torch.cuda.synchronize()
        bkts.bkts_ctx_destroy(ctx)
