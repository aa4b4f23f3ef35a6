"""Captured RK4 step sequences (heom_model_set_graph_steps): replays give the
same states as direct launches, bit for bit (same kernels in the same order),
over several replays with direct work and host synchronisation in between,
and after the kernel choice changes."""

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


@pytest.mark.parametrize("which,depth", [("cfg1", None), ("cfg2", 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_graph_replays_match_direct_launches(which, depth, prec, adjoint):
    p = getattr(w, which)()[0]
    if depth is not None:
        p["depth"] = depth
    o = om.build(p)
    x = w.random_hierarchy(3, len(o.hier), o.d, seed=4, scale_by_depth=0.3 ** o.hier.n.sum(1))
    mg = P.heom_model_build(p)
    md = P.heom_model_build(p)
    P.heom_model_set_graph_steps(mg, 8)
    P.heom_model_set_graph_steps(md, 0)
    sg, sd = P.State(mg, 3, prec), P.State(md, 3, prec)
    sg.upload(x)
    sd.upload(x)
    for n, kernel in ((19, "mfma"), (8, "mfma"), (17, "generic"), (16, "mfma_dyn")):
        for m in (mg, md):
            P.heom_model_set_kernel(m, prec, kernel)
        P.heom_propagate(mg, sg, n, adjoint)
        P.heom_propagate(md, sd, n, adjoint)
        a, b = sg.download(), sd.download()
        assert np.array_equal(a, b), (n, kernel)
        # direct work between replays
        t = P.State(mg, 3, prec)
        P.heom_rhs(mg, sg, t, adjoint)
    # and the result is the propagation the oracle computes
    tol = 1e-11 if prec == "fp64" else 1e-4
    ref = np.stack([oh.propagate(o, x[i], 60, adjoint=adjoint) for i in range(3)])
    got = sg.download()
    assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref))
