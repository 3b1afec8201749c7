"""kd_knn_noalloc (scratch in a fixed library array, no device allocation)
against kd_knn on the same inputs, through the C ABI.

Bar: indices byte-identical and squared distances bit-identical to kd_knn
(same kernels; only where the scratch lives differs).  Two calls in a row,
the second with fewer queries, so that state the first call leaves in the
shared array (counters, cursors, hand-off rows) must not leak into the
second; then the largest query count the array holds, and one more, which
must be refused before anything runs."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2210_12859_amd as kd  # noqa: E402
from paper_2210_12859_amd import datagen  # noqa: E402

# largest Q whose scratch fits KD_NOALLOC_SCRATCH_BYTES (dim 2, 3 / dim 4)
MAX_Q_D3 = 1_104_800
MAX_Q_D4 = 616_042


def _dev():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda:0")


def _both(tree, q, k, maxr=math.inf):
    print(f"[gpu] noalloc vs kd_knn Q={q.shape[0]} k={k} maxr={maxr}", flush=True)
    ni, nd = kd.kd_knn_noalloc(tree, q, k, maxr)
    torch.cuda.synchronize()
    ri, rd = kd.kd_knn(tree, q, k, maxr)
    torch.cuda.synchronize()
    return ni.cpu().numpy(), nd.cpu().numpy(), ri.cpu().numpy(), rd.cpu().numpy()


def _same(ni, nd, ri, rd, ctx):
    bad = np.nonzero((ni.reshape(ni.shape[0], -1) != ri.reshape(ri.shape[0], -1)).any(axis=1))[0]
    assert len(bad) == 0, f"{ctx}: indices differ at rows {bad[:5]}"
    assert np.array_equal(nd.view(np.uint32), rd.view(np.uint32)), f"{ctx}: d2 bits differ"


@pytest.fixture(scope="module")
def gmm_tree():
    P = datagen.gmm(262_144, 3, 0)
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    yield tree
    tree.close()


def test_two_calls_second_smaller(gmm_tree):
    Qa = torch.from_numpy(datagen.gmm(200_000, 3, 1)).to(_dev())
    Qb = torch.from_numpy(datagen.gmm(3_001, 3, 5)).to(_dev())
    for q, k, ctx in [(Qa, 8, "first call, 200000 queries"), (Qb, 8, "second call, 3001 queries"),
                      (Qb, 1, "third call, fcp")]:
        _same(*_both(gmm_tree, q, k), ctx)


def test_bounded_radius_and_k64(gmm_tree):
    q = torch.from_numpy(datagen.uniform(50_000, 3, 9)).to(_dev())
    _same(*_both(gmm_tree, q, 64), "k=64")
    _same(*_both(gmm_tree, q, 5, 0.01), "k=5 maxR=0.01")


def test_largest_query_count_and_one_more():
    P = datagen.uniform(1 << 20, 3, 0)
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(datagen.uniform(MAX_Q_D3 + 1, 3, 1)).to(_dev())
    _same(*_both(tree, q[:MAX_Q_D3], 8), f"Q={MAX_Q_D3}")
    with pytest.raises(kd.KdError) as ei:
        kd.kd_knn_noalloc(tree, q, 8)
    assert ei.value.status == kd.KD_EINVAL and "fixed scratch" in str(ei.value)
    tree.close()


def test_dim4_and_empty_tree():
    P = datagen.uniform(70_000, 4, 3)
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(datagen.uniform(MAX_Q_D4, 4, 4)).to(_dev())
    _same(*_both(tree, q, 8), f"dim 4, Q={MAX_Q_D4}")
    q1 = torch.from_numpy(datagen.uniform(MAX_Q_D4 + 1, 4, 4)).to(_dev())
    with pytest.raises(kd.KdError):
        kd.kd_knn_noalloc(tree, q1, 8)
    tree.close()
    empty = kd.kd_build(torch.zeros((0, 3), dtype=torch.float32, device=_dev()))
    qe = torch.from_numpy(datagen.uniform(100, 3, 2)).to(_dev())
    ni, nd = kd.kd_knn_noalloc(empty, qe, 4)
    torch.cuda.synchronize()
    assert (ni.cpu().numpy() == -1).all() and np.isinf(nd.cpu().numpy()).all()
    empty.close()


def test_call_allocates_no_device_memory(gmm_tree):
    q = torch.from_numpy(datagen.uniform(400_000, 3, 11)).to(_dev())
    oi = torch.empty((q.shape[0], 8), dtype=torch.int32, device=_dev())
    od = torch.empty((q.shape[0], 8), dtype=torch.float32, device=_dev())
    kd.kd_knn_noalloc(gmm_tree, q[:1000], 8, out_idx=oi[:1000], out_d2=od[:1000])  # module and lookup warm
    torch.cuda.synchronize()
    s = torch.cuda.Stream()  # a stream no call has used: kd_knn would allocate its scratch here
    with torch.cuda.stream(s):
        od.fill_(0.0)  # the runtime sets up the stream's queue on its first launch (no tensor allocated)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    with torch.cuda.stream(s):
        kd.kd_knn_noalloc(gmm_tree, q, 8, out_idx=oi, out_d2=od, stream=s)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, f"free device memory changed by {free0 - free1} bytes"
    ri, rd = kd.kd_knn(gmm_tree, q, 8)
    torch.cuda.synchronize()
    _same(oi.cpu().numpy(), od.cpu().numpy(), ri.cpu().numpy(), rd.cpu().numpy(), "side stream")
