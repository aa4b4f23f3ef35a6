"""heom_propagate_noalloc (work buffers in the library's static device array)
against heom_propagate through the C ABI: the same kernels in the same order,
so the results agree bit for bit; two calls in a row, the second on a smaller
state, and the size limit.  Tolerance: exact equality (identical arithmetic)."""

import numpy as np
import pytest

import workloads as w
from oracle import model as om

P = pytest.importorskip("paper_2601_20550_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_propagate_matches_propagate_twice(prec):
    params = w.cfg2()[0]
    params["depth"] = 3
    o = om.build(params)
    m = P.heom_model_build(params)
    for call, (n_traj, steps, every) in enumerate([(6, 7, 3), (2, 5, 0)]):
        x = w.random_hierarchy(n_traj, len(o.hier), o.d, seed=60 + call, scale_by_depth=0.3 ** o.hier.n.sum(1))
        a, b = P.State(m, n_traj, prec), P.State(m, n_traj, prec)
        a.upload(x)
        b.upload(x)
        ta = P.heom_propagate(m, a, steps, sample_every=every)
        tb = P.heom_propagate_noalloc(m, b, steps, sample_every=every)
        assert np.array_equal(a.download(), b.download()), call
        if every:
            assert np.array_equal(ta, tb), call
        else:
            assert tb is None


def test_noalloc_kron_model_and_transposed_generator():
    # the three-mode model in FP32 runs the (S; 4, 4) kernel through both calls
    params = w.cfg3(depth=1)[0]
    o = om.build(params)
    m = P.heom_model_build(params)
    x = w.random_hierarchy(3, len(o.hier), o.d, seed=8)
    for adjoint in (False, True):
        a, b = P.State(m, 3, "fp32"), P.State(m, 3, "fp32")
        a.upload(x)
        b.upload(x)
        P.heom_propagate(m, a, 4, adjoint=adjoint)
        P.heom_propagate_noalloc(m, b, 4, adjoint=adjoint)
        assert np.array_equal(a.download(), b.download())


def test_noalloc_rejects_states_beyond_the_static_buffer():
    params = w.cfg3(depth=2)[0]
    m = P.heom_model_build(params)
    big = P.State(m, 128, "fp32")  # 128 x 55 x 51.2 KB x 2 stage buffers > 64 MiB
    big.set_ground()
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_propagate_noalloc(m, big, 1)
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
    assert "64 MiB" in str(e.value) or "67108864" in str(e.value)
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_propagate_noalloc(m, big, -1)
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
