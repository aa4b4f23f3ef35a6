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
    grid = {"n1": 3, "n3": 3, "steps_per_sample": 4, "t2_steps": [0, 5]}
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


def _class_instances(with_nb4=True):
    """One instance per size class the single launch covers: d = 6, 25 and 80
    from the uneven batch, and the three-mode model kept at (4, 4, 3) and
    (4, 4, 4) levels (d = 48 and 64) at depth 1."""
    ps = [p for p in _instances()]
    base = w.cfg3()[0]
    for keep in ((4, 4, 3), (4, 4, 4)) if with_nb4 else ((4, 4, 3),):
        p = dict(base)
        p["modes"] = [dict(md) for md in base["modes"]]
        p["depth"] = 1
        for md, k in zip(p["modes"], keep):
            md["n_keep"] = k
        ps.append(p)
    return ps


def _random_states(models, os_, prec, seed):
    xs, states = [], []
    for i, (m, o) in enumerate(zip(models, os_)):
        nt = 1 + i % 3
        x = w.random_hierarchy(nt, len(o.hier), o.d, seed=seed + i, scale_by_depth=0.3 ** o.hier.n.sum(1))
        s = P.State(m, nt, prec)
        s.upload(x)
        xs.append(x)
        states.append(s)
    return xs, states


@pytest.mark.parametrize("with_nb4", [True, False])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_single_launch_parity(with_nb4, prec, tol, adjoint):
    # one launch per RK4 stage over five (or four) size classes: workgroups
    # split among the classes, narrower classes leaving the extra waves idle;
    # against the oracle and against the per-class launches
    ps = _class_instances(with_nb4)
    os_ = [om.build(p) for p in ps]
    models = [P.heom_model_build(p) for p in ps]
    xs, single = _random_states(models, os_, prec, 90)
    _, per_class = _random_states(models, os_, prec, 90)
    b = P.heom_batch_create(models)
    P.heom_batch_set_launch(b, "single")
    assert P.heom_batch_get_launch(b) == "single"
    P.heom_batch_propagate(b, single, 3, adjoint)
    P.heom_batch_set_launch(b, "per_class")
    P.heom_batch_propagate(b, per_class, 3, adjoint)
    for i, (o, x, s, c) in enumerate(zip(os_, xs, single, per_class)):
        ref = np.stack([oh.propagate(o, x[t], 3, adjoint=adjoint) for t in range(x.shape[0])])
        got = s.download()
        assert _relerr(got, ref) < tol, (i, o.d)
        assert _relerr(got, c.download()) < (1e-12 if prec == "fp64" else 2e-6), (i, o.d)


def test_single_launch_response_matches_per_class(instances):
    ps, os_ = instances
    grid = {"n1": 3, "n3": 3, "steps_per_sample": 4, "t2_steps": [0, 5]}
    models = [P.heom_model_build(p) for p in ps]
    rhos = []
    for m, o in zip(models, os_):
        s = P.State(m, 1, "fp64")
        s.upload(oh.propagate(o, oh.ground_state_hierarchy(o), 20)[None])
        rhos.append(s)
    b = P.heom_batch_create(models)
    ref = P.heom_batch_response_2d(b, rhos, grid, "fp64")
    P.heom_batch_set_launch(b, "single")
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-4)):
        got = P.heom_batch_response_2d(b, rhos, grid, prec)
        for g, r in zip(got, ref):
            assert _relerr(g, r) < tol


@pytest.mark.parametrize("launch", ["per_class", "single"])
def test_batch_graph_replays_match_direct_launches(instances, launch):
    # graph_steps = 2: a 7-step call replays its captured graph three times
    # and finishes with one direct step; three calls in a row with eager
    # work (traces) and synchronisations between them, every result compared
    # with direct launches bit for bit; then a response whose t1 / t3 / t2
    # loops replay one captured graph between the dipole and pairing launches
    import torch
    ps, os_ = instances
    models = [P.heom_model_build(p) for p in ps]
    _, sg = _random_states(models, os_, "fp32", 120)
    _, sd = _random_states(models, os_, "fp32", 120)
    bg, bd = P.heom_batch_create(models), P.heom_batch_create(models)
    for b in (bg, bd):
        P.heom_batch_set_launch(b, launch)
    P.heom_batch_set_graph_steps(bg, 2)
    for _ in range(3):
        P.heom_batch_propagate(bg, sg, 7)
        P.heom_batch_propagate(bd, sd, 7)
        for m, a, c in zip(models, sg, sd):
            assert np.array_equal(P.heom_trace(m, a), P.heom_trace(m, c))
        torch.cuda.synchronize()
        for a, c in zip(sg, sd):
            assert np.array_equal(a.download(), c.download())
    grid = {"n1": 3, "n3": 3, "steps_per_sample": 2, "t2_steps": [0, 4]}
    rhos = []
    for m, o in zip(models, os_):
        s = P.State(m, 1, "fp64")
        s.upload(oh.propagate(o, oh.ground_state_hierarchy(o), 20)[None])
        rhos.append(s)
    rg = P.heom_batch_response_2d(bg, rhos, grid, "fp32")
    rd = P.heom_batch_response_2d(bd, rhos, grid, "fp32")
    for a, c in zip(rg, rd):
        assert np.array_equal(a, c)


def test_batch_autotune_picks_the_faster_form(instances):
    ps, os_ = instances
    models = [P.heom_model_build(p) for p in ps]
    b = P.heom_batch_create(models)
    assert P.heom_batch_get_launch(b) == "per_class"
    chosen, ms = P.heom_batch_autotune(b, "fp32", n_traj=2, reps=2)
    assert np.isfinite(ms["per_class"]) and np.isfinite(ms["single"])
    assert chosen == ("single" if ms["single"] < ms["per_class"] else "per_class")
    assert P.heom_batch_get_launch(b) == chosen
    for nb in (1, 2, 5):  # the classes of these instances: a tuned shape each
        wg, lds = P.heom_batch_get_class_shape(b, nb)
        assert wg >= 1 and lds in ((0, 1) if nb <= 4 else (-1,))
    xs, st = _random_states(models, os_, "fp32", 140)
    P.heom_batch_propagate(b, st, 2)
    for o, x, s in zip(os_, xs, st):
        ref = np.stack([oh.propagate(o, x[t], 2) for t in range(x.shape[0])])
        assert _relerr(s.download(), ref) < 1e-5
    # a d = 96 instance (six row blocks) keeps the per-class form only
    base = w.cfg3()[0]
    p = dict(base)
    p["modes"] = [dict(md) for md in base["modes"]]
    p["depth"] = 1
    for md, k in zip(p["modes"], (4, 4, 6)):
        md["n_keep"] = k
    bw = P.heom_batch_create([models[0], P.heom_model_build(p)])
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_batch_set_launch(bw, "single")
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
    chosen, ms = P.heom_batch_autotune(bw, "fp32", n_traj=1, reps=1)
    assert chosen == "per_class" and np.isnan(ms["single"])


@pytest.mark.parametrize("wg,lds", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_per_class_launch_shapes_parity(wg, lds):
    # the per-class launch with either neighbour-sum form (registers / LDS)
    # and with one workgroup per CU, for the FP32 classes that have both forms
    # (d = 6, 25, 48, 64) and the d = 80 class, against the oracle
    ps = _class_instances(True)
    os_ = [om.build(p) for p in ps]
    models = [P.heom_model_build(p) for p in ps]
    xs, st = _random_states(models, os_, "fp32", 160)
    b = P.heom_batch_create(models)
    for nb in (1, 2, 3, 4):
        P.heom_batch_set_class_shape(b, nb, wg, lds)
        assert P.heom_batch_get_class_shape(b, nb) == (wg, lds)
    P.heom_batch_set_class_shape(b, 5, wg, -1)
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_batch_set_class_shape(b, 5, 0, 1)
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
    P.heom_batch_propagate(b, st, 2)
    for i, (o, x, s) in enumerate(zip(os_, xs, st)):
        ref = np.stack([oh.propagate(o, x[t], 2) for t in range(x.shape[0])])
        assert _relerr(s.download(), ref) < 1e-5, (i, o.d)
