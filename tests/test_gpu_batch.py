"""GPU parity of the multi-instance path (heom_batch_*): instances of different
sizes (d = 6, 25, 80) propagated by one launch per size class and RK4 stage,
against the CPU FP64 oracle instance by instance, and against the
single-model entry points.

Tolerances as in the single-model tests: FP64 1e-12 of the peak for a few RK4
steps and 1e-10 for a response; FP32 1e-5 for steps and 1e-4 for a response.
"""

import numpy as np
import pytest

import workloads as w
from oracle import heom as oh
from oracle import model as om

P = pytest.importorskip("paper_2601_20550_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _relerr(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _instances():
    """The smallest instance of each size class of the uneven 64-instance
    batch, plus a second one in the d = 25 class (two instances share a launch)."""
    inst = [p for p, _ in w.cfg4_instances()]
    sizes = []
    for p in inst:
        o = om.build(p)
        sizes.append((o.d, len(o.hier)))
    pick = []
    for d in (6, 25, 80):
        idx = sorted((n, i) for i, (dd, n) in enumerate(sizes) if dd == d)
        pick.append(idx[0][1])
        if d == 25:
            pick.append(idx[1][1])
    return [inst[i] for i in pick]


@pytest.fixture(scope="module")
def instances():
    ps = _instances()
    return ps, [om.build(p) for p in ps]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_batch_propagate_parity(instances, prec, tol, adjoint):
    ps, os_ = instances
    models = [P.heom_model_build(p) for p in ps]
    ntraj = [2, 3, 1, 2]
    xs, states = [], []
    for i, (m, o) in enumerate(zip(models, os_)):
        x = w.random_hierarchy(ntraj[i], len(o.hier), o.d, seed=30 + i,
                               scale_by_depth=0.3 ** o.hier.n.sum(1))
        s = P.State(m, ntraj[i], prec)
        s.upload(x)
        xs.append(x)
        states.append(s)
    b = P.heom_batch_create(models)
    P.heom_batch_propagate(b, states, 3, adjoint)
    for i, (o, x, s) in enumerate(zip(os_, xs, states)):
        ref = np.stack([oh.propagate(o, x[t], 3, adjoint=adjoint) for t in range(ntraj[i])])
        assert _relerr(s.download(), ref) < tol, i


def test_batch_propagate_matches_single_model_path(instances):
    ps, os_ = instances
    models = [P.heom_model_build(p) for p in ps]
    a, c = [], []
    for i, (m, o) in enumerate(zip(models, os_)):
        x = w.random_hierarchy(2, len(o.hier), o.d, seed=50 + i)
        sa, sc = P.State(m, 2, "fp32"), P.State(m, 2, "fp32")
        sa.upload(x)
        sc.upload(x)
        a.append(sa)
        c.append(sc)
    b = P.heom_batch_create(models)
    P.heom_batch_propagate(b, a, 5)
    for m, s in zip(models, c):
        P.heom_model_set_kernel(m, "fp32", "mfma_dyn")
        P.heom_propagate(m, s, 5)
    for sa, sc in zip(a, c):
        assert _relerr(sa.download(), sc.download()) < 1e-6


def test_batch_response_parity(instances):
    ps, os_ = instances
    grid = {"n1": 4, "n3": 4, "steps_per_sample": 5, "t2_steps": [0, 6]}
    models = [P.heom_model_build(p) for p in ps]
    rhos, refs = [], []
    for m, o in zip(models, os_):
        r = oh.propagate(o, oh.ground_state_hierarchy(o), 30)
        s = P.State(m, 1, "fp64")
        s.upload(r[None])
        rhos.append(s)
        refs.append(oh.response_2d(o, r, grid))
    b = P.heom_batch_create(models)
    got = P.heom_batch_response_2d(b, rhos, grid, "fp64")
    got32 = P.heom_batch_response_2d(b, rhos, grid, "fp32")
    for i, (m, rho, ref) in enumerate(zip(models, rhos, refs)):
        assert got[i].shape == ref.shape
        assert _relerr(got[i], ref) < 1e-10, i
        assert _relerr(got32[i], ref) < 1e-4, i
        single = P.heom_response_2d(m, rho, grid, "fp64", "adjoint")
        assert _relerr(got[i], single) < 1e-12, i


def test_batch_errors(instances):
    ps, _ = instances
    p2 = dict(ps[0])
    p2["dt"] = 0.05
    m1, m2 = P.heom_model_build(ps[0]), P.heom_model_build(p2)
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_batch_create([m1, m2])
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
    m3 = P.heom_model_build(ps[1])
    b = P.heom_batch_create([m1, m3])
    s1, s3 = P.State(m1, 1, "fp64"), P.State(m3, 1, "fp32")
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_batch_propagate(b, [s1, s3], 1)
    assert e.value.code == P.heom2dvs.HEOM_ERR_STATE
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_batch_propagate(b, [s3, s1], 1)
    assert e.value.code == P.heom2dvs.HEOM_ERR_STATE


def test_batch_six_row_block_class_and_wide_mode_rejected():
    # FP32 instances with d = 96 (six 16-row blocks: two waves per row block and
    # the 16-byte operand reads of the multi-instance kernel) next to a d = 80
    # instance, against the oracle; a mode of 12 kept levels is refused
    base = w.cfg3()[0]
    ps = []
    for keep, depth in (((4, 4, 6), 1), ((4, 4, 6), 2), ((4, 4, 5), 1)):
        p = dict(base)
        p["modes"] = [dict(md) for md in base["modes"]]
        p["depth"] = depth
        for md, k in zip(p["modes"], keep):
            md["n_keep"] = k
        ps.append(p)
    os_ = [om.build(p) for p in ps]
    models = [P.heom_model_build(p) for p in ps]
    states, xs = [], []
    for i, (m, o) in enumerate(zip(models, os_)):
        x = w.random_hierarchy(3, len(o.hier), o.d, seed=70 + i, scale_by_depth=0.3 ** o.hier.n.sum(1))
        s = P.State(m, 3, "fp32")
        s.upload(x)
        states.append(s)
        xs.append(x)
    P.heom_batch_propagate(P.heom_batch_create(models), states, 2)
    for o, x, s in zip(os_, xs, states):
        ref = np.stack([oh.propagate(o, x[t], 2) for t in range(3)])
        assert _relerr(s.download(), ref) < 1e-5
    wide = w.cfg2()[0]
    wide["depth"] = 1
    wide["modes"][0]["n_keep"] = 12
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_batch_create([P.heom_model_build(wide)])
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
