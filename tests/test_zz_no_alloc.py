"""sur_topk_noalloc (the top-k selection with the library's static scratch,
for callers that cannot allocate) against sur_topk through the C ABI: equal
index lists on two calls in a row, the second on a smaller input, with ties,
NaN and signed zeros in the scores (the refusal of sizes beyond the static
scratch is a CPU test: it returns before any device call)."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _scores(n, seed):
    rng = np.random.default_rng(seed)
    s = rng.normal(0, 1, n).astype(np.float32)
    s[rng.integers(0, n, n // 50)] = 0.5            # ties at common values
    s[rng.integers(0, n, 17)] = np.nan
    s[rng.integers(0, n, 9)] = -0.0
    s[rng.integers(0, n, 9)] = 0.0
    return s


def test_noalloc_topk_matches_the_workspace_entry_point():
    import torch
    from paper_2502_11129_amd import surrogate as SU
    lib = SU.load()
    sur = SU.Surrogate()
    for n, k, seed in ((3_000_017, 150_001, 1), (200_003, 10_007, 2), (1, 1, 3)):
        _say(f"[no-alloc topk] n={n} k={k}")
        sc = torch.from_numpy(_scores(n, seed)).cuda()
        ref = sur.topk(sc, k).cpu().numpy()
        out = torch.full((k,), -1, dtype=torch.int32, device="cuda")
        err = C.create_string_buffer(256)
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = lib.sur_topk_noalloc(n, C.c_void_p(sc.data_ptr()), k, C.c_void_p(out.data_ptr()), st, err, 256)
        assert rc == 0, err.value
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        # the binding's wrapper gives the same list
        np.testing.assert_array_equal(SU.topk_noalloc(sc, k).cpu().numpy(), ref)
