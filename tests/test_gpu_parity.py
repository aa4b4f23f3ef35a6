"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances.  FP64 kernels: relative 1e-12 of the largest output element for a
single right-hand side or step (different summation order only), looser for
long propagations where rounding accumulates.  FP32 kernels: relative 2e-6
per right-hand side (80-term FP32 dot products, unit round-off 6e-8), and
the response tolerance is 1e-4 of the peak, the accuracy target of the
FP32 path.
"""

import numpy as np
import pytest

import workloads as w
from oracle import heom as oh
from oracle import model as om

P = pytest.importorskip("paper_2601_20550_amd")

pytestmark = pytest.mark.gpu


def _gpu_or_skip():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    _gpu_or_skip()


def _depth_scale(model):
    # deeper ADOs are smaller in physical states; keeps the test inputs in a
    # realistic dynamic range
    return 0.3 ** model.hier.n.sum(1)


def _params(which, depth=None, **kw):
    p = getattr(w, which)()[0]
    if depth is not None:
        p["depth"] = depth
    p.update(kw)
    return p


def _relerr(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


CASES = [("cfg1", None), ("cfg2", None), ("cfg2", 2), ("cfg3", 2), ("paper_scale", 2)]


KERNELS = ["generic", "mfma", "mfma_dyn", "kron", "mfma_gh"]


def _kron_applies(which, prec):
    # the (S; 4, 4) matrix-core kernel: FP32, three modes of (4|5, 4, 4) levels
    return prec == "fp32" and which in ("cfg3", "paper_scale")


def _applies(kernel, which, prec):
    if kernel == "kron":
        return _kron_applies(which, prec)
    if kernel == "mfma_gh":  # FP32, d = 65..80 (the three-mode 4 x 4 x 5 model)
        return prec == "fp32" and which == "cfg3"
    return True


@pytest.mark.parametrize("which,depth", CASES)
@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kernel", KERNELS)
def test_rhs_parity(which, depth, adjoint, prec, kernel):
    params = _params(which, depth)
    o = om.build(params)
    m = P.heom_model_build(params)
    if not _applies(kernel, which, prec):
        with pytest.raises(P.heom2dvs.HeomError) as e:
            P.heom_model_set_kernel(m, prec, kernel)
        assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
        return
    P.heom_model_set_kernel(m, prec, kernel)
    x = w.random_hierarchy(3, len(o.hier), o.d, seed=11, scale_by_depth=_depth_scale(o))
    xin = P.State(m, 3, prec)
    xout = P.State(m, 3, prec)
    xin.upload(x)
    P.heom_rhs(m, xin, xout, adjoint)
    got = xout.download()
    ref = oh.rhs(o, x, adjoint=adjoint)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert _relerr(got, ref) < tol


@pytest.mark.parametrize("which,B", [("cfg1", 16384), ("cfg2", 2048)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_padded_matrices_many_per_workgroup(which, B, prec, tol):
    # d = 6 and 25 are padded to 16 and 32 in the LDS planes, and every
    # persistent workgroup processes hundreds of matrices: padding entries left
    # non-zero by one matrix must not reach the next (regression: they grew
    # from matrix to matrix until 0 * inf poisoned the matrix-core products)
    params = _params(which)
    o = om.build(params)
    m = P.heom_model_build(params)
    P.heom_model_set_kernel(m, prec, "mfma")
    s = P.State(m, B, prec)
    s.set_ground()
    x = w.random_hierarchy(3, len(o.hier), o.d, seed=9, hermitian=True, scale_by_depth=_depth_scale(o))
    picks = [0, B // 2 + 1, B - 1]
    for i, b in enumerate(picks):
        s.upload_range(b, x[i:i + 1])
    P.heom_propagate(m, s, 3)  # raises HEOM_ERR_UNSTABLE on a non-finite hierarchy
    ref = oh.propagate(o, x, 3)
    for i, b in enumerate(picks):
        assert _relerr(s.download_range(b, 1)[0], ref[i]) < tol
    g = oh.propagate(o, oh.ground_state_hierarchy(o), 3)
    assert _relerr(s.download_range(1, 1)[0], g) < tol


def test_rhs_parity_full_depth_three_modes():
    params = _params("cfg3")
    o = om.build(params)
    m = P.heom_model_build(params)
    x = w.random_hierarchy(2, len(o.hier), o.d, seed=5, scale_by_depth=_depth_scale(o))
    ref = oh.rhs(o, x)
    for kernel in KERNELS:
        for prec, tol in (("fp64", 1e-12), ("fp32", 2e-6)):
            if kernel in ("kron", "mfma_gh") and prec == "fp64":
                continue
            P.heom_model_set_kernel(m, prec, kernel)
            a, b = P.State(m, 2, prec), P.State(m, 2, prec)
            a.upload(x)
            P.heom_rhs(m, a, b)
            assert _relerr(b.download(), ref) < tol, (kernel, prec)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("kernel", KERNELS)
def test_rk4_steps_parity(prec, tol, kernel):
    params = _params("cfg3", 2) if kernel in ("kron", "mfma_gh") else _params("cfg2", 3)
    if kernel in ("kron", "mfma_gh") and prec == "fp64":
        pytest.skip("FP32-only kernel")
    o = om.build(params)
    m = P.heom_model_build(params)
    P.heom_model_set_kernel(m, prec, kernel)
    x = w.random_hierarchy(2, len(o.hier), o.d, seed=3, hermitian=True, scale_by_depth=_depth_scale(o))
    s = P.State(m, 2, prec)
    s.upload(x)
    P.heom_propagate(m, s, 5)
    ref = oh.propagate(o, x, 5)
    assert _relerr(s.download(), ref) < tol
    # the transposed generator
    s.upload(x)
    P.heom_propagate(m, s, 5, adjoint=True)
    ref = oh.propagate(o, x, 5, adjoint=True)
    assert _relerr(s.download(), ref) < tol


@pytest.fixture(scope="module")
def full_size_refs():
    params = _params("cfg3")
    o = om.build(params)
    x = w.random_hierarchy(1, len(o.hier), o.d, seed=77, hermitian=True,
                           scale_by_depth=_depth_scale(o))
    g = np.zeros_like(x)
    g[0, 0, 0, 0] = 1.0
    return params, x, oh.rk4_step(o, x), oh.rk4_step(o, g)


@pytest.mark.parametrize("kernel", ["mfma", "mfma_dyn", "kron", "mfma_gh"])
def test_full_size_batched_step_sampled(full_size_refs, kernel):
    """Three-mode depth-6 model, 128 trajectories (the benchmark batch) with
    either matrix-core instantiation the benchmark's autotuner may choose:
    one FP32 RK4 step on the whole batch; trajectories 0 (ground state) and
    77 (random) are compared with the oracle."""
    params, x, ref77, ref0 = full_size_refs
    m = P.heom_model_build(params)
    P.heom_model_set_kernel(m, "fp32", kernel)
    B = 128
    s = P.State(m, B, "fp32")
    s.set_ground()
    s.upload_range(77, x)
    P.heom_propagate(m, s, 1)
    got77 = s.download_range(77, 1)
    got0 = s.download_range(0, 1)
    assert _relerr(got77, ref77) < 1e-5
    assert _relerr(got0, ref0) < 1e-5
    # an untouched trajectory stays exactly the ground-state step
    got5 = s.download_range(5, 1)
    assert np.array_equal(got5, got0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_propagate_sampled_traces_parity(prec, tol):
    # detection traces tr(mu rho_0) recorded during heom_propagate against the
    # oracle's propagation sample by sample (n_steps not a multiple of the
    # sampling interval: the trailing steps are propagated, not sampled)
    params = _params("cfg2", 2)
    o = om.build(params)
    m = P.heom_model_build(params)
    x = w.random_hierarchy(2, len(o.hier), o.d, seed=8, scale_by_depth=_depth_scale(o))
    s = P.State(m, 2, prec)
    s.upload(x)
    tr = P.heom_propagate(m, s, 23, sample_every=5)
    assert tr.shape == (5, 2)
    ref = np.zeros((5, 2), dtype=complex)
    for b in range(2):
        y = x[b]
        for k in range(5):
            ref[k, b] = np.trace(o.mu @ y[0])
            y = oh.propagate(o, y, 5 if k < 4 else 3)
    assert _relerr(tr, ref) < tol
    assert _relerr(s.download(), np.stack([oh.propagate(o, x[b], 23) for b in range(2)])) < tol



@pytest.mark.parametrize("which,depth", [("cfg1", None), ("cfg2", 2), ("cfg3", 1), ("paper_scale", 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dipole_and_trace_parity(which, depth, prec):
    # d = 6, 25, 80, 64: the LDS-staged commutator kernel (d = 80 in FP64
    # fills 155 KB of LDS); larger d use the plain kernel (edge-model tests)
    params = _params(which, depth)
    o = om.build(params)
    m = P.heom_model_build(params)
    x = w.random_hierarchy(2, len(o.hier), o.d, seed=9)
    tol = 1e-13 if prec == "fp64" else 1e-6
    for op, D in (("mu", o.mu), ("mu_plus", o.mu_plus), ("mu_minus", o.mu_minus)):
        for tr in (False, True):
            s = P.State(m, 2, prec)
            s.upload(x)
            P.heom_apply_dipole(m, s, op, transpose=tr)
            Dm = D.T if tr else D
            assert _relerr(s.download(), oh.commutator(Dm, x)) < tol
        s = P.State(m, 2, prec)
        s.upload(x)
        got = P.heom_trace(m, s, op)
        ref = oh.trace_n0(D, x)
        assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref)) * 10


def test_equilibrate_parity_fixed_steps():
    params = _params("cfg1")
    o = om.build(params)
    m = P.heom_model_build(params)
    rho, steps, res = P.heom_equilibrate(m, tol=0.0, check_every=200, min_steps=0, max_steps=1000)
    ref, rsteps, rres = oh.equilibrate(o, 0.0, 200, 0, 1000)
    assert steps == rsteps == 1000
    assert _relerr(rho.download()[0], ref) < 1e-11
    assert abs(res - rres) < 1e-9 * rres
    # residual-based stop: start point of the stationary solution is not needed;
    # a loose tolerance must stop at the same check on both sides
    rho2, steps2, res2 = P.heom_equilibrate(m, tol=3e-3, check_every=100, min_steps=0, max_steps=5000)
    _, rsteps2, rres2 = oh.equilibrate(o, 3e-3, 100, 0, 5000)
    assert steps2 == rsteps2 and res2 <= 3e-3


def test_equilibrate_converges_to_stationary_state():
    # small model where the slowest relaxation is fast: the propagated state
    # reaches the sparse-solve stationary solution of the oracle
    mode = dict(omega=1.0, g3=-0.2, g4=0.02, V1=1.0, V2=0.1, zeta=1.0, gamma=1.0,
                mu1=1.0, mu2=0.2, n_basis=12, n_keep=4, K=2)
    params = {"modes": [mode], "couplings": [], "beta": 3.0, "depth": 4,
              "decomp": "pade", "dt": 0.05}
    o = om.build(params)
    m = P.heom_model_build(params)
    rho, steps, res = P.heom_equilibrate(m, tol=1e-11, check_every=200, min_steps=0,
                                         max_steps=60000, require_convergence=True)
    st = oh.stationary_state(o)
    assert res <= 1e-11
    assert _relerr(rho.download()[0], st) < 1e-8


def test_linear_response_brownian_parity():
    params = w.harmonic_pin(depth=4, K=2, dt=0.02, n_keep=6)
    o = om.build(params)
    m = P.heom_model_build(params)
    rho = P.State(m, 1, "fp64")
    rho.set_ground()
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        got = P.heom_linear_response(m, rho, 12, 50, prec)
        ref = oh.linear_response(o, oh.ground_state_hierarchy(o), 12, 50)
        assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref)), prec


def _response_case(which, depth, n, sps, t2, dt=None):
    params = _params(which, depth)
    if dt is not None:
        params["dt"] = dt
    o = om.build(params)
    m = P.heom_model_build(params)
    rho_ref = oh.propagate(o, oh.ground_state_hierarchy(o), 50)
    rho = P.State(m, 1, "fp64")
    rho.upload(rho_ref[None])
    grid = {"n1": n, "n3": n, "steps_per_sample": sps, "t2_steps": t2}
    ref = oh.response_2d(o, rho_ref, grid)
    return m, rho, grid, ref


RESP = [("cfg1", None, 8, 25, [0, 40], None), ("cfg2", 2, 6, 5, [0, 12], None),
        ("cfg3", 1, 4, 4, [0, 6], None), ("paper_scale", 1, 3, 3, [0, 4], None)]


@pytest.mark.parametrize("which,depth,n,sps,t2,dt", RESP)
@pytest.mark.parametrize("method", ["direct", "adjoint"])
def test_response_2d_parity(which, depth, n, sps, t2, dt, method):
    m, rho, grid, ref = _response_case(which, depth, n, sps, t2, dt)
    got = P.heom_response_2d(m, rho, grid, "fp64", method)
    assert got.shape == ref.shape
    assert _relerr(got, ref) < 1e-10
    got32 = P.heom_response_2d(m, rho, grid, "fp32", method)
    assert _relerr(got32, ref) < 1e-4


def test_response_2d_generic_kernel():
    m, rho, grid, ref = _response_case("cfg2", 2, 6, 5, [0, 12], None)
    for prec in ("fp64", "fp32"):
        P.heom_model_set_kernel(m, prec, "generic")
    got = P.heom_response_2d(m, rho, grid, "fp64", "adjoint")
    assert _relerr(got, ref) < 1e-10
    got32 = P.heom_response_2d(m, rho, grid, "fp32", "direct")
    assert _relerr(got32, ref) < 1e-4


def test_autotune_picks_a_measured_kernel():
    # (5, 5) levels: no compile-time shape, so "mfma_dyn" would run the same
    # code as "mfma" and is not timed; the single mode of 6 levels has one
    # (both are timed); the three-mode (4, 4, 5) model adds the (S; 4, 4)
    # kernel in FP32
    for which, depth, prec, want in (("cfg2", 3, "fp32", {"generic", "mfma"}),
                                     ("cfg1", None, "fp64", {"generic", "mfma", "mfma_dyn"}),
                                     ("cfg3", 1, "fp32", {"generic", "mfma", "kron", "mfma_gh"})):
        m = P.heom_model_build(_params(which, depth))
        P.heom_model_set_kernel(m, prec, "generic")
        best, ms = P.heom_autotune(m, 4, prec, reps=2)
        assert set(ms) == want, which
        assert best == min(ms, key=ms.get)
        assert P.heom_model_get_kernel(m, prec) == best


def test_response_2d_batching_and_methods_agree():
    m, rho, grid, ref = _response_case("cfg2", 2, 6, 5, [0, 7, 12], None)
    a = P.heom_response_2d(m, rho, grid, "fp64", "direct", max_batch=4)
    b = P.heom_response_2d(m, rho, grid, "fp64", "adjoint", max_batch=5)
    c = P.heom_response_2d(m, rho, grid, "fp64", "adjoint", max_batch=1)
    assert _relerr(a, ref) < 1e-10
    assert _relerr(b, ref) < 1e-10
    assert _relerr(c, b) < 1e-13


def test_spectrum_parity():
    rng = np.random.default_rng(4)
    for n1, n3 in ((8, 8), (5, 7)):
        RI = rng.standard_normal((n1, n3)) + 1j * rng.standard_normal((n1, n3))
        RII = rng.standard_normal((n1, n3)) + 1j * rng.standard_normal((n1, n3))
        got = P.heom_spectrum_2d(RI, RII, 0.7)
        ref = oh.correlation_spectrum(RI, RII, 0.7)
        assert got.shape == ref.shape == (2 * n3, 2 * n1)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_unstable_step_is_reported():
    params = _params("cfg1", dt=2.0)
    m = P.heom_model_build(params)
    s = P.State(m, 1, "fp64")
    s.set_ground()
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_propagate(m, s, 400)
    assert e.value.code == P.heom2dvs.HEOM_ERR_UNSTABLE


def test_state_errors():
    m1 = P.heom_model_build(_params("cfg1"))
    m2 = P.heom_model_build(_params("cfg1"))
    a, b = P.State(m1, 2, "fp64"), P.State(m2, 2, "fp64")
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_rhs(m1, a, b)
    assert e.value.code == P.heom2dvs.HEOM_ERR_STATE
    with pytest.raises(P.heom2dvs.HeomError):
        P.heom_rhs(m1, a, a)
    with pytest.raises(P.heom2dvs.HeomError) as e:
        a.download_range(1, 2)
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM


def test_timing_counters():
    params = _params("cfg2", 2)
    m = P.heom_model_build(params)
    s = P.State(m, 3, "fp32")
    s.set_ground()
    P.heom_timing_enable(m, True)
    P.heom_propagate(m, s, 2)
    ms, n, upd = P.heom_timing_read(m)
    P.heom_timing_enable(m, False)
    assert n == 8 and upd == 8 * 3 * m.n_ado and ms > 0


def test_response_2d_three_modes_depth2_parity():
    # the full pipeline on the three-mode model at depth 2 (55 ADOs, d = 80)
    m, rho, grid, ref = _response_case("cfg3", 2, 3, 2, [0, 2])
    got = P.heom_response_2d(m, rho, grid, "fp64", "adjoint")
    assert _relerr(got, ref) < 1e-10
    got32 = P.heom_response_2d(m, rho, grid, "fp32", "direct")
    assert _relerr(got32, ref) < 1e-4


def test_full_size_fp32_spectrum_matches_fp64():
    # full three-mode model (5005 ADOs): the FP32 path against the FP64 path on
    # a 16 x 16 grid (the oracle cannot run this size); accuracy target of the
    # FP32 path: 1e-4 of the peak for R and for S_C
    params = _params("cfg3")
    m = P.heom_model_build(params)
    rho = P.State(m, 1, "fp64")
    rho.set_ground()
    P.heom_propagate(m, rho, 100)
    grid = {"n1": 16, "n3": 16, "steps_per_sample": 10, "t2_steps": [0]}
    r64 = P.heom_response_2d(m, rho, grid, "fp64", "adjoint")
    r32 = P.heom_response_2d(m, rho, grid, "fp32", "adjoint")
    assert _relerr(r32, r64) < 1e-4
    dt_s = 10 * params["dt"]
    s64 = P.heom_spectrum_2d(r64[0, 0], r64[0, 1], dt_s)
    s32 = P.heom_spectrum_2d(r32[0, 0], r32[0, 1], dt_s)
    assert _relerr(s32, s64) < 1e-4


@pytest.mark.parametrize("which,depth", [("cfg1", None), ("cfg2", 2)])
def test_krylov_equilibration_reaches_stationary_state(which, depth):
    # the oracle's sparse direct solve; for the two-mode model (17,500
    # unknowns, minutes of CPU) it is stored by tests/golden/make_stationary.py
    params = _params(which, depth)
    if which == "cfg1":
        params["dt"] = 0.05
        ref = oh.stationary_state(om.build(params))
    else:
        import os
        z = np.load(os.path.join(os.path.dirname(__file__), "golden", "cfg2_depth2_rho_eq.npz"))
        assert int(z["depth"]) == depth
        ref = z["rho"]
    m = P.heom_model_build(params)
    rho, applies, res = P.heom_equilibrate_krylov(m, tol=1e-11)
    assert res <= 1e-11 and applies > 0
    got = rho.download()[0]
    assert np.max(np.abs(got - ref)) < 1e-8 * np.max(np.abs(ref))


def test_krylov_equilibration_three_modes_is_stationary():
    # d = 80 at depth 1 (the oracle's sparse direct solve is too slow at this
    # size): the state must be stationary under the oracle's generator, have
    # unit trace and a Hermitian system part
    params = _params("cfg3", 1)
    o = om.build(params)
    m = P.heom_model_build(params)
    rho, applies, res = P.heom_equilibrate_krylov(m, tol=1e-11)
    got = rho.download()[0]
    assert res <= 1e-11
    assert np.max(np.abs(oh.rhs(o, got))) < 1e-10
    assert abs(np.trace(got[0]) - 1.0) < 1e-12
    assert np.max(np.abs(got[0] - got[0].conj().T)) < 1e-10


PATHWAYS = [("mu", "mu", "mu"),                  # full response, all 8 Liouville terms
            ("mu_plus", "mu_plus", "mu_minus"),  # double-quantum (k1 + k2 - k3)
            ("mu_minus", "mu_plus", "mu_plus")]  # rephasing, as in heom_response_2d


@pytest.mark.parametrize("method", ["direct", "adjoint"])
def test_response_pathways_parity(method):
    params = _params("cfg2", 2)
    o = om.build(params)
    m = P.heom_model_build(params)
    rho_ref = oh.propagate(o, oh.ground_state_hierarchy(o), 50)
    rho = P.State(m, 1, "fp64")
    rho.upload(rho_ref[None])
    grid = {"n1": 4, "n3": 5, "steps_per_sample": 4, "t2_steps": [0, 6]}
    names = {"mu": o.mu, "mu_plus": o.mu_plus, "mu_minus": o.mu_minus}
    ref = oh.response_2d(o, rho_ref, grid,
                         pathways=[tuple(names[x] for x in pw) for pw in PATHWAYS])
    got = P.heom_response_2d_pathways(m, rho, grid, PATHWAYS, "fp64", method)
    assert got.shape == ref.shape
    assert _relerr(got, ref) < 1e-10
    got32 = P.heom_response_2d_pathways(m, rho, grid, PATHWAYS, "fp32", method)
    assert _relerr(got32, ref) < 1e-4
    # the standard call is the rephasing / non-rephasing pair of this one
    std = P.heom_response_2d(m, rho, grid, "fp64", method)
    assert _relerr(got[:, 2], std[:, 0]) < 1e-13
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_response_2d_pathways(m, rho, grid, [(0, 1, 7)], "fp64", method)
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM


def _edge_params(kind):
    p = _params("cfg2")
    if kind == "depth0":            # a single ADO: the system alone, no bath couplings
        p["depth"] = 0
    elif kind == "drude_only":      # K = 0: only the Drude term of each bath
        p["depth"] = 2
        for md in p["modes"]:
            md["K"] = 0
    elif kind == "no_bath":         # zeta = 0: every bath coefficient vanishes
        p["depth"] = 2
        for md in p["modes"]:
            md["zeta"] = 0.0
    elif kind == "max_d":           # d = 8 x 16 = 128, the largest product dimension
        p["depth"] = 1
        p["modes"][0]["n_keep"] = 8
        p["modes"][1]["n_keep"] = 16
        p["modes"][1]["n_basis"] = 20
    elif kind == "max_mfma32":      # d = 7 x 4 x 4 = 112, the largest FP32 matrix-core size
        p = _params("cfg3", 1)
        for mode, k in zip(p["modes"], (7, 4, 4)):
            mode["n_keep"] = k
    elif kind == "wide_mode":       # a mode of 12 kept levels: beyond the 8 x 8 v_s slot
        p["depth"] = 2
        p["modes"][0]["n_keep"] = 12
        p["modes"][1]["n_keep"] = 5
    return p


@pytest.mark.parametrize("kind", ["depth0", "drude_only", "no_bath", "max_d", "max_mfma32", "wide_mode"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rhs_parity_edge_models(kind, prec):
    params = _edge_params(kind)
    o = om.build(params)
    m = P.heom_model_build(params)
    x = w.random_hierarchy(2, len(o.hier), o.d, seed=17, scale_by_depth=_depth_scale(o))
    kernels = ["generic", "mfma"]
    # the matrix-core kernels stage three DP x (DP+1) planes in 160 KB of LDS:
    # d <= 112 in FP32, d <= 80 in FP64
    # (a mode of more than 8 kept levels does not fit the kernels' v_s slot):
    # those models start on the VALU kernel and refuse the matrix-core ones
    if kind in ("max_d", "wide_mode") or (kind == "max_mfma32" and prec == "fp64"):
        kernels = ["generic"]
        assert P.heom_model_get_kernel(m, prec) == "generic"
        with pytest.raises(P.heom2dvs.HeomError) as e:
            P.heom_model_set_kernel(m, prec, "mfma")
        assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
    for kernel in kernels:
        P.heom_model_set_kernel(m, prec, kernel)
        for adjoint in (False, True):
            xin, xout = P.State(m, 2, prec), P.State(m, 2, prec)
            xin.upload(x)
            P.heom_rhs(m, xin, xout, adjoint)
            ref = oh.rhs(o, x, adjoint=adjoint)
            tol = 1e-12 if prec == "fp64" else 4e-6
            assert _relerr(xout.download(), ref) < tol, (kernel, adjoint)


def test_response_2d_without_bath_hierarchy():
    # depth 0: the response of the isolated system, against the oracle
    params = _edge_params("depth0")
    o = om.build(params)
    m = P.heom_model_build(params)
    rho_ref = oh.propagate(o, oh.ground_state_hierarchy(o), 10)
    rho = P.State(m, 1, "fp64")
    rho.upload(rho_ref[None])
    grid = {"n1": 4, "n3": 4, "steps_per_sample": 3, "t2_steps": [0, 5]}
    ref = oh.response_2d(o, rho_ref, grid)
    for method in ("direct", "adjoint"):
        assert _relerr(P.heom_response_2d(m, rho, grid, "fp64", method), ref) < 1e-10


def test_empty_and_zero_work_requests():
    m = P.heom_model_build(_params("cfg1"))
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.State(m, 0, "fp64")
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM
    s = P.State(m, 2, "fp32")
    s.set_ground()
    before = s.download()
    P.heom_propagate(m, s, 0)
    assert np.array_equal(s.download(), before)
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_propagate(m, s, -1)
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM


@pytest.mark.parametrize("method", ["direct", "adjoint"])
def test_progress_reports_do_not_change_results(method):
    m, rho, grid, ref = _response_case("cfg2", 2, 4, 5, [0, 12], None)
    plain = P.heom_response_2d(m, rho, grid, "fp64", method)
    calls = []
    P.heom_model_set_progress(m, lambda ph, done, tot: calls.append((ph, done, tot)), 7)
    got = P.heom_response_2d(m, rho, grid, "fp64", method, max_batch=3)
    P.heom_model_set_progress(m, None)
    np.testing.assert_array_equal(got, P.heom_response_2d(m, rho, grid, "fp64", method, max_batch=3))
    assert _relerr(got, plain) < 1e-13 and _relerr(got, ref) < 1e-10
    # 2 pathways x 2 batches (4 t1 samples, 3 per batch) x steps per batch
    per_batch = 12 + (2 * 3 * 5 if method == "direct" else 0)
    total = 2 * 2 * per_batch
    assert calls and all(t == total for _, _, t in calls)
    done = [d for _, d, _ in calls]
    assert done == sorted(done) and all(x % 7 == 0 for x in done) and total - done[-1] < 7


@pytest.mark.parametrize("which,depth,cut", [("cfg2", 4, 2.0), ("cfg3", 3, 2.0)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kernel", KERNELS)
def test_rhs_parity_rate_filtered_hierarchy(which, depth, cut, prec, kernel):
    # non-triangular index set: neighbours outside the kept set are absent
    params = _params(which, depth, rate_cut=cut)
    o = om.build(params)
    assert len(o.hier) < len(om.build(_params(which, depth)).hier)
    m = P.heom_model_build(params)
    assert m.n_ado == len(o.hier)
    if not _applies(kernel, which, prec):
        pytest.skip("kernel not applicable to this model and precision")
    P.heom_model_set_kernel(m, prec, kernel)
    x = w.random_hierarchy(2, len(o.hier), o.d, seed=21, scale_by_depth=_depth_scale(o))
    xin = P.State(m, 2, prec)
    xout = P.State(m, 2, prec)
    xin.upload(x)
    for adjoint in (False, True):
        P.heom_rhs(m, xin, xout, adjoint)
        assert _relerr(xout.download(), oh.rhs(o, x, adjoint=adjoint)) < (1e-12 if prec == "fp64" else 2e-6)


@pytest.mark.parametrize("method", ["direct", "adjoint"])
def test_response_2d_parity_rate_filtered(method):
    params = _params("cfg2", 3, rate_cut=1.5)
    o = om.build(params)
    m = P.heom_model_build(params)
    rho_ref = oh.propagate(o, oh.ground_state_hierarchy(o), 50)
    rho = P.State(m, 1, "fp64")
    rho.upload(rho_ref[None])
    grid = {"n1": 5, "n3": 5, "steps_per_sample": 5, "t2_steps": [0, 10]}
    ref = oh.response_2d(o, rho_ref, grid)
    assert _relerr(P.heom_response_2d(m, rho, grid, "fp64", method), ref) < 1e-10
    assert _relerr(P.heom_response_2d(m, rho, grid, "fp32", method), ref) < 1e-4


def test_progress_reports_in_stationary_solve():
    params = _params("cfg1")
    params["dt"] = 0.05
    m = P.heom_model_build(params)
    ref, ref_applies, ref_res = P.heom_equilibrate_krylov(m, tol=1e-11, steps_per_apply=200)
    calls = []
    P.heom_model_set_progress(m, lambda ph, done, tot: calls.append((ph, done, tot)), 300)
    got, applies, res = P.heom_equilibrate_krylov(m, tol=1e-11, steps_per_apply=200)
    P.heom_model_set_progress(m, None)
    np.testing.assert_array_equal(got.download(), ref.download())
    assert (applies, res) == (ref_applies, ref_res)
    assert calls and all(ph == "stationary solve" for ph, _, _ in calls)
    done = [d for _, d, _ in calls]
    assert done == sorted(done) and all(x % 200 == 0 for x in done)
    # one report per crossing of a multiple of 300 steps, at the next application boundary
    assert len(done) == len({x // 300 for x in done})


def test_krylov_stationary_state_rate_filtered():
    params = _params("cfg1", rate_cut=3.0)
    params["dt"] = 0.05
    params["decomp"] = "pade"
    o = om.build(params)
    assert len(o.hier) < len(om.build(dict(params, rate_cut=0.0)).hier)
    ref = oh.stationary_state(o)
    m = P.heom_model_build(params)
    rho, applies, res = P.heom_equilibrate_krylov(m, tol=1e-11)
    assert res <= 1e-11 and applies > 0
    assert np.max(np.abs(rho.download()[0] - ref)) < 1e-8 * np.max(np.abs(ref))


def test_batch_with_rate_filtered_instance():
    insts = [_params("cfg2", 3, rate_cut=1.5), _params("cfg2", 3), _params("cfg1", 3, rate_cut=2.5)]
    for p in insts:
        p["dt"] = 0.05
    models = [P.heom_model_build(p) for p in insts]
    oracles = [om.build(p) for p in insts]
    states, refs = [], []
    for i, (m, o) in enumerate(zip(models, oracles)):
        x = w.random_hierarchy(2, len(o.hier), o.d, seed=40 + i, hermitian=True, scale_by_depth=_depth_scale(o))
        s = P.State(m, 2, "fp32")
        s.upload(x)
        states.append(s)
        refs.append(oh.propagate(o, x, 4))
    P.heom_batch_propagate(P.heom_batch_create(models), states, 4)
    for s, ref in zip(states, refs):
        assert _relerr(s.download(), ref) < 1e-5


@pytest.mark.parametrize("keep", [(4, 5), (6, 6), (4, 4, 3), (4, 4, 6)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kernel", ["mfma", "mfma_dyn"])
def test_rhs_parity_padded_multiple_of_four(keep, prec, kernel):
    # d = 20, 36, 48, 96: a multiple of four (16-byte rows in global memory and
    # in the padded LDS planes) but, for 20 and 36, not of 16 (zero-padded
    # tiles); d = 96 is the six-row-block shape (two waves per row block with
    # the 16-byte operand reads in FP32), which FP64 runs on the VALU kernel
    if prec == "fp64" and len(keep) == 3 and np.prod(keep) > 80:
        pytest.skip("FP64 matrix-core planes hold d <= 80")
    params = _params("cfg3" if len(keep) == 3 else "cfg2", 2)
    for mode, k in zip(params["modes"], keep):
        mode["n_keep"] = k
    o = om.build(params)
    m = P.heom_model_build(params)
    P.heom_model_set_kernel(m, prec, kernel)
    B = 600  # several matrices per persistent workgroup
    x = w.random_hierarchy(2, len(o.hier), o.d, seed=31, scale_by_depth=_depth_scale(o))
    xin = P.State(m, B, prec)
    xout = P.State(m, B, prec)
    xin.set_ground()
    xin.upload_range(0, x[:1])
    xin.upload_range(B - 1, x[1:])
    P.heom_rhs(m, xin, xout)
    ref = oh.rhs(o, x)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert _relerr(xout.download_range(0, 1)[0], ref[0]) < tol
    assert _relerr(xout.download_range(B - 1, 1)[0], ref[1]) < tol


@pytest.mark.parametrize("which", ["cfg3", "paper_scale"])
def test_device_basis_roundtrip_and_default_kernel(which):
    # three-mode (S; 4, 4) models keep their matrices in the reordered device
    # basis: upload / download must give back the caller's arrays exactly
    params = _params(which, 1)
    o = om.build(params)
    m = P.heom_model_build(params)
    assert P.heom_model_get_kernel(m, "fp32") == "mfma"
    x = w.random_hierarchy(3, len(o.hier), o.d, seed=2)
    s = P.State(m, 3, "fp64")
    s.upload(x)
    assert np.array_equal(s.download(), x)
    s.upload_range(1, x[2:3])
    assert np.array_equal(s.download_range(1, 1)[0], x[2])
    ops = m.operators()
    assert np.array_equal(ops["H"], o.H) or _relerr(ops["H"], o.H) < 1e-13


@pytest.mark.parametrize("which,depth,B", [("cfg3", 1, 3000), ("paper_scale", 1, 2000)])
def test_kron_many_items_per_wave(which, depth, B):
    # thousands of trajectories: every wave of the persistent grid processes
    # many (matrix, plane) items; picked trajectories against the oracle and
    # untouched ones against the ground-state step
    params = _params(which, depth)
    o = om.build(params)
    m = P.heom_model_build(params)
    P.heom_model_set_kernel(m, "fp32", "kron")
    s = P.State(m, B, "fp32")
    s.set_ground()
    x = w.random_hierarchy(3, len(o.hier), o.d, seed=4, scale_by_depth=_depth_scale(o))
    picks = [0, B // 2 + 3, B - 1]
    for i, b in enumerate(picks):
        s.upload_range(b, x[i:i + 1])
    P.heom_propagate(m, s, 2)
    ref = oh.propagate(o, x, 2)
    for i, b in enumerate(picks):
        assert _relerr(s.download_range(b, 1)[0], ref[i]) < 1e-5
    g = oh.propagate(o, oh.ground_state_hierarchy(o), 2)
    assert _relerr(s.download_range(1, 1)[0], g) < 1e-5
