"""The allocation-free search entry point (``knn_db_search_noalloc``) against
``knn_db_search`` with a caller workspace: same kernels, the workspace taken from the
library's fixed device scratch instead (run on an MI355X; collected last)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2206_14286_amd import datagen, knn

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _noalloc(db, Q, K, L, rerank, bins):
    M = Q.shape[0]
    ov = torch.full((M, K), 3.0, device=DEV)
    oi = torch.full((M, K), -3, dtype=torch.int32, device=DEV)
    bv = torch.full((M, L), 3.0, device=DEV) if bins else None
    bi = torch.full((M, L), -3, dtype=torch.int32, device=DEV) if bins else None
    st = knn.lib().knn_db_search_noalloc(db.handle, knn._ptr(Q), knn._in_dtype(Q), M, K, L, 0.95, -1, rerank,
                                         knn._ptr(ov), knn._ptr(oi), knn._ptr(bv), knn._ptr(bi), knn._stream())
    assert st == 0, knn.lib().knn_last_error()
    return (ov, oi, bv, bi) if bins else (ov, oi)


@pytest.mark.parametrize("metric,compute,rerank,bins", [("l2", "bf16", 40, False), ("cosine", "fp8", 0, True),
                                                       ("mips", "fp32", 20, True)])
def test_noalloc_search_equals_workspace_search_twice(metric, compute, rerank, bins):
    """Two calls in a row, the second with fewer queries and rows' worth of bins than the
    first: each equals knn_db_search with a caller workspace bit for bit, so nothing the
    first call left in the shared scratch leaks into the second."""
    print(f"noalloc {metric} {compute} rerank={rerank} bins={bins}", flush=True)
    N, D, K = 30000, 96, 10
    X = torch.from_numpy(datagen.normal(N, D, 81)).to(DEV)
    db = knn.Database(X, metric, compute)
    for M, L in ((1000, 600), (37, 200)):
        Q = torch.from_numpy(datagen.normal(M, D, 82 + M)).to(DEV)
        want = db.search(Q, K, L, rerank=rerank, return_bins=bins)
        got = _noalloc(db, Q, K, L, rerank, bins)
        torch.cuda.synchronize()
        for g, w in zip(got, want):
            assert torch.equal(g, w)
    sys.stdout.flush()


def test_noalloc_rejects_searches_beyond_its_scratch():
    """A search whose workspace exceeds the fixed scratch is refused before anything is
    enqueued; the outputs stay untouched."""
    N, D, K = 20000, 64, 10
    db = knn.Database(torch.from_numpy(datagen.normal(N, D, 83)).to(DEV), "mips", "fp32")
    cap = int(knn.lib().knn_noalloc_scratch_bytes())
    M, L = 8192, 2000  # bins alone: 8192 x 2000 x 8 bytes = 131 MB
    assert db.workspace_size(M, K, L) > cap
    Q = torch.from_numpy(datagen.normal(M, D, 84)).to(DEV)
    ov = torch.full((M, K), 3.0, device=DEV)
    oi = torch.full((M, K), -3, dtype=torch.int32, device=DEV)
    st = knn.lib().knn_db_search_noalloc(db.handle, knn._ptr(Q), knn.F32, M, K, L, 0.95, -1, 0, knn._ptr(ov),
                                         knn._ptr(oi), None, None, knn._stream())
    assert st == 1 and b"scratch" in knn.lib().knn_last_error()
    torch.cuda.synchronize()
    assert torch.all(ov == 3.0) and torch.all(oi == -3)
