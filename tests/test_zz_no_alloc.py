"""The allocation-free batched entry point against the ordinary batched one: two calls in
a row through the C ABI (the second with fewer and smaller graphs), each output equal to
vdmc_count_batch's element by element, and the size limits reported as errors."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def v():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_11655_amd as v
    v.load()
    v.init()
    return v


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("k", [3, 4])
def test_noalloc_equals_batch(v, k):
    import torch
    first = gg.er_batch(300, 20, 500, 2.0, 8.0, seed=41)
    second = gg.er_batch(37, 10, 120, 1.0, 5.0, seed=42)
    stream = torch.cuda.Stream()
    for graphs in (first, second):
        Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
        with torch.cuda.stream(stream):
            want = v.count_batch(Gs, k, stream=stream)
            outs = [torch.full((g.n, v.num_classes(k)), -1, dtype=torch.int64, device="cuda") for g in graphs]
            v.count_batch_noalloc(Gs, k, outs, stream=stream)
            stream.synchronize()
        for a, b in zip(outs, want):
            assert (_np(a) == _np(b)).all()
        sc = v.shape_counts(Gs[-1])
        T = sum(sc.values())
        assert int(_np(outs[-1]).sum()) == k * T


def test_noalloc_limits(v):
    import torch
    big = gg.er_directed(2000, 0.002, 3)          # more vertices than the whole-graph kernel takes
    G = v.Graph(big.n, big.src, big.dst)
    o = torch.empty((big.n, 199), dtype=torch.int64, device="cuda")
    with pytest.raises(v.VdmcError) as e:
        v.count_batch_noalloc([G], 4, [o])
    assert e.value.name == "UNSUPPORTED"
    small = gg.er_directed(30, 0.1, 4)
    Gs = v.Graph(small.n, small.src, small.dst)
    os_ = torch.empty((small.n, 199), dtype=torch.int64, device="cuda")
    with pytest.raises(v.VdmcError) as e:
        v.count_batch_noalloc([Gs] * 8193, 4, [os_] * 8193)
    assert e.value.name == "INVALID_ARG"
    assert v.count_batch_noalloc([], 4, []) == []
