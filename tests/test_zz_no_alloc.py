"""tn_sample_noalloc (staging in the library's static device array) against
tn_sample, through the C ABI: identical samples on two calls in a row, the
second with a smaller input; unsliced and sliced plans; the size limit; no
growth of device memory use across calls."""
import numpy as np
import pytest

from paper_2405_14060_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T(gpu):
    import paper_2405_14060_amd as T
    T.lib()
    return T


@pytest.mark.parametrize("sliced", [False, True])
def test_noalloc_sampling_matches_tn_sample(T, sliced):
    import torch
    net = W.grid_mrf(5, 6, 3)
    kw = dict(semirings=T.SUM_PRODUCT)
    if sliced:
        sc = T.Plan(T.Network(net), **kw).info()["sc"]
        kw["max_log2_size"] = sc - 2
    P = T.Plan(T.Network(net), **kw)
    assert (P.info()["n_sliced"] > 0) == sliced
    # two calls in a row, the second smaller (the static array keeps the
    # first call's rows beyond the second's)
    for n, seed in ((30000, 11), (7000, 12)):
        got = P.sample_noalloc(n, seed)
        want = P.sample(n, seed)
        assert got.shape == (n, net.n_vars)
        assert np.array_equal(got, want), (n, seed)
        assert got.min() >= 0 and got.max() < 2
    # device memory does not grow across allocation-free calls (a plain
    # tn_sample of this size grows the plan's staging by 9.6 MB)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for n, seed in ((80000, 13), (5000, 14)):
        P.sample_noalloc(n, seed)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_sampling_size_limit(T):
    net = W.grid_mrf(4, 4, 0)
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT)
    n_max = (1 << 22) // net.n_vars
    s = P.sample_noalloc(n_max, 5)
    assert np.array_equal(s, P.sample(n_max, 5))
    with pytest.raises(T.TNError) as e:
        P.sample_noalloc(n_max + 1, 5)
    assert e.value.status == 4  # TN_E_TOO_LARGE
    # zero samples: only the p(e) > 0 check
    assert P.sample_noalloc(0, 5).shape == (0, net.n_vars)
