"""Python binding of libheom2dvs.so (ctypes; argument marshalling only).

Every computation runs in the HIP library.  The functions carry the names of
the C entry points declared in include/heom2dvs.h; PyTorch, when present,
supplies the HIP stream (torch.cuda.current_stream()) and optionally its
caching allocator for device memory.

Host arrays are numpy complex128 of shape (n_traj, n_ado, d, d).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libheom2dvs.so")

HEOM_OK = 0
HEOM_ERR_PARAM = -1
HEOM_ERR_OOM = -2
HEOM_ERR_UNSTABLE = -3
HEOM_ERR_NOCONV = -4
HEOM_ERR_HIP = -5
HEOM_ERR_STATE = -6

HEOM_FP64, HEOM_FP32 = 0, 1
HEOM_PADE, HEOM_MATSUBARA = 0, 1
HEOM_OP_MU, HEOM_OP_MU_PLUS, HEOM_OP_MU_MINUS = 0, 1, 2
HEOM_RESP_DIRECT, HEOM_RESP_ADJOINT = 0, 1
HEOM_KERNEL_AUTO, HEOM_KERNEL_GENERIC, HEOM_KERNEL_MFMA, HEOM_KERNEL_MFMA_DYN, HEOM_KERNEL_KRON = 0, 1, 2, 3, 4
HEOM_KERNEL_MFMA_GH = 5
KERNELS = {"auto": 0, "generic": 1, "mfma": 2, "mfma_dyn": 3, "kron": 4, "mfma_gh": 5}
KERNEL_NAMES = {v: k for k, v in KERNELS.items()}

_PREC = {"fp64": HEOM_FP64, "fp32": HEOM_FP32, HEOM_FP64: HEOM_FP64, HEOM_FP32: HEOM_FP32}
_OPS = {"mu": HEOM_OP_MU, "mu_plus": HEOM_OP_MU_PLUS, "mu_minus": HEOM_OP_MU_MINUS}
_METHOD = {"direct": HEOM_RESP_DIRECT, "adjoint": HEOM_RESP_ADJOINT,
           HEOM_RESP_DIRECT: HEOM_RESP_DIRECT, HEOM_RESP_ADJOINT: HEOM_RESP_ADJOINT}


class HeomError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class heom_mode(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("omega", "g3", "g4", "V1", "V2", "zeta", "gamma", "mu1", "mu2")] + \
               [("n_basis", C.c_int), ("n_keep", C.c_int), ("K", C.c_int),
                ("omega_b", C.c_double)]


class heom_coupling(C.Structure):
    _fields_ = [("s", C.c_int), ("t", C.c_int), ("g_st", C.c_double), ("g_s2t", C.c_double),
                ("g_st2", C.c_double), ("mu_st", C.c_double)]


class heom_params(C.Structure):
    _fields_ = [("n_modes", C.c_int), ("modes", C.POINTER(heom_mode)),
                ("n_couplings", C.c_int), ("couplings", C.POINTER(heom_coupling)),
                ("beta", C.c_double), ("depth", C.c_int), ("decomp", C.c_int),
                ("dt", C.c_double), ("rate_cut", C.c_double)]


class heom_info(C.Structure):
    _fields_ = [("d", C.c_int), ("n_ado", C.c_int), ("n_terms", C.c_int), ("n_modes", C.c_int),
                ("dims", C.c_int * 4), ("depth", C.c_int), ("dt", C.c_double)]


class heom_grid(C.Structure):
    _fields_ = [("n1", C.c_int), ("n3", C.c_int), ("steps_per_sample", C.c_int),
                ("n_t2", C.c_int), ("t2_steps", C.POINTER(C.c_int))]


class heom_op_grad(C.Structure):
    _fields_ = [("dH", C.c_void_p), ("dv", C.c_void_p), ("dmu", C.c_void_p), ("dc", C.c_void_p),
                ("dnu", C.c_void_p), ("stationary_steps", C.c_int),
                ("stationary_residual", C.c_double)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_PROGRESS_FN = C.CFUNCTYPE(None, C.c_char_p, C.c_longlong, C.c_longlong, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

# name -> (restype, argtypes)
_SIGS = {
    "heom_last_error": (C.c_char_p, []),
    "heom_set_allocator": (C.c_int, [_ALLOC_FN, _FREE_FN, C.c_void_p]),
    "heom_device_query": (C.c_int, [C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_char_p, C.c_int]),
    "heom_model_build": (C.c_int, [C.POINTER(heom_params), C.c_void_p, C.POINTER(C.c_void_p)]),
    "heom_model_build_host": (C.c_int, [C.POINTER(heom_params), C.POINTER(C.c_void_p)]),
    "heom_model_free": (None, [C.c_void_p]),
    "heom_model_info": (C.c_int, [C.c_void_p, C.POINTER(heom_info)]),
    "heom_model_operators": (C.c_int, [C.c_void_p] + [C.c_void_p] * 9),
    "heom_model_bath": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "heom_state_create": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    "heom_state_free": (None, [C.c_void_p]),
    "heom_state_shape": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "heom_state_upload": (C.c_int, [C.c_void_p, C.c_void_p]),
    "heom_state_download": (C.c_int, [C.c_void_p, C.c_void_p]),
    "heom_state_upload_range": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "heom_state_download_range": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "heom_state_set_ground": (C.c_int, [C.c_void_p]),
    "heom_state_copy": (C.c_int, [C.c_void_p, C.c_void_p]),
    "heom_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "heom_propagate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "heom_propagate_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "heom_apply_dipole": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int]),
    "heom_trace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "heom_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "heom_equilibrate": (C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_int),
                                   C.POINTER(C.c_double)]),
    "heom_equilibrate_krylov": (C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                          C.POINTER(C.c_void_p), C.POINTER(C.c_int),
                                          C.POINTER(C.c_double)]),
    "heom_stationary_refine": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_int,
                                         C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "heom_linear_response": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                       C.c_void_p]),
    "heom_response_2d": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(heom_grid), C.c_int,
                                   C.c_int, C.c_int, C.c_void_p]),
    "heom_response_2d_pathways": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(heom_grid), C.c_int,
                                            C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "heom_spectrum_1d": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_void_p]),
    "heom_spectrum_2d": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_double,
                                   C.c_void_p]),
    "heom_response_2d_vjp": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(heom_grid), C.c_void_p,
                                       C.c_int, C.c_double, C.c_int, C.POINTER(heom_op_grad)]),
    "heom_spectrum_2d_vjp": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_void_p]),
    "heom_params_vjp": (C.c_int, [C.POINTER(heom_params), C.c_void_p, C.c_int, C.c_double,
                                  C.POINTER(heom_op_grad), C.c_void_p]),
    "heom_response_2d_backward": (C.c_int, [C.POINTER(heom_params), C.c_void_p, C.c_void_p,
                                            C.POINTER(heom_grid), C.c_void_p, C.c_int, C.c_double,
                                            C.c_int, C.c_void_p, C.c_int, C.c_double, C.c_void_p]),
    "heom_batch_create": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
    "heom_batch_free": (None, [C.c_void_p]),
    "heom_batch_propagate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int]),
    "heom_batch_response_2d": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(heom_grid), C.c_int,
                                         C.c_void_p]),
    "heom_batch_set_launch": (C.c_int, [C.c_void_p, C.c_int]),
    "heom_batch_get_launch": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "heom_batch_set_graph_steps": (C.c_int, [C.c_void_p, C.c_int]),
    "heom_batch_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "heom_batch_get_class_shape": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "heom_batch_set_class_shape": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "heom_model_set_kernel": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "heom_model_set_graph_steps": (C.c_int, [C.c_void_p, C.c_int]),
    "heom_model_set_progress": (C.c_int, [C.c_void_p, _PROGRESS_FN, C.c_void_p, C.c_int]),
    "heom_model_get_kernel": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "heom_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int),
                                C.c_void_p]),
    "heom_timing_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "heom_timing_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong),
                                   C.POINTER(C.c_longlong)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libheom2dvs.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "__graft_entry__.build() (there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc != HEOM_OK:
        msg = _lib.heom_last_error()
        raise HeomError(rc, msg.decode() if msg else "")


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


def _params_struct(params):
    modes = params["modes"]
    arr = (heom_mode * len(modes))()
    for i, m in enumerate(modes):
        for k in ("omega", "g3", "g4", "V1", "V2", "zeta", "gamma", "mu1", "mu2"):
            setattr(arr[i], k, float(m.get(k, 0.0)))
        arr[i].n_basis = int(m["n_basis"])
        arr[i].n_keep = int(m["n_keep"])
        arr[i].K = int(m["K"])
        arr[i].omega_b = float(m.get("omega_b", 0.0))
    cps = params.get("couplings", [])
    carr = (heom_coupling * max(1, len(cps)))()
    for i, c in enumerate(cps):
        carr[i].s, carr[i].t = int(c["s"]), int(c["t"])
        for k in ("g_st", "g_s2t", "g_st2", "mu_st"):
            setattr(carr[i], k, float(c.get(k, 0.0)))
    p = heom_params()
    p.n_modes = len(modes)
    p.modes = arr
    p.n_couplings = len(cps)
    p.couplings = carr
    p.beta = float(params["beta"])
    p.depth = int(params["depth"])
    p.decomp = HEOM_MATSUBARA if params.get("decomp", "pade") == "matsubara" else HEOM_PADE
    p.dt = float(params["dt"])
    p.rate_cut = float(params.get("rate_cut", 0.0))
    return p, (arr, carr)


def _torch_stream_handle():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return C.c_void_p(0)


_alloc_keepalive = []


def heom_set_allocator_torch():
    """Route device allocations through torch's caching allocator."""
    import torch
    lib = load_library()
    dev = torch.cuda.current_device()

    def _alloc(nbytes, ctx):
        return torch.cuda.caching_allocator_alloc(int(nbytes), dev)

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
    _alloc_keepalive[:] = [fa, ff]
    _check(lib.heom_set_allocator(fa, ff, None))


def heom_device_query():
    lib = load_library()
    cu, lds = C.c_int(), C.c_int()
    name = C.create_string_buffer(256)
    _check(lib.heom_device_query(C.byref(cu), C.byref(lds), name, 256))
    return {"cu_count": cu.value, "lds_bytes": lds.value, "name": name.value.decode()}


class Model:
    """A built model (host operators + device tables)."""

    def __init__(self, params, stream=None, device=True):
        lib = load_library()
        self.params = params
        p, keep = _params_struct(params)
        h = C.c_void_p()
        if device:
            s = _torch_stream_handle() if stream is None else C.c_void_p(stream)
            _check(lib.heom_model_build(C.byref(p), s, C.byref(h)))
        else:
            _check(lib.heom_model_build_host(C.byref(p), C.byref(h)))
        self.handle = h
        info = heom_info()
        _check(lib.heom_model_info(h, C.byref(info)))
        self.d, self.n_ado, self.n_terms = info.d, info.n_ado, info.n_terms
        self.n_modes = info.n_modes
        self.dims = tuple(info.dims[:info.n_modes])
        self.depth, self.dt = info.depth, info.dt

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.heom_model_free(self.handle)
            self.handle = None

    def operators(self):
        d, M = self.d, self.n_terms
        H = np.zeros((d, d))
        mu = np.zeros((d, d))
        mup = np.zeros((d, d))
        mum = np.zeros((d, d))
        v = np.zeros(sum(x * x for x in self.dims))
        nu = np.zeros(M)
        c = np.zeros(2 * M)
        n = np.zeros((self.n_ado, M), dtype=np.int32)
        tm = np.zeros(M, dtype=np.int32)
        _check(_lib.heom_model_operators(self.handle, _ptr(H), _ptr(mu), _ptr(mup), _ptr(mum),
                                         _ptr(v), _ptr(nu), _ptr(c), _ptr(n), _ptr(tm)))
        vs, off = [], 0
        for ds in self.dims:
            vs.append(v[off:off + ds * ds].reshape(ds, ds))
            off += ds * ds
        return {"H": H, "mu": mu, "mu_plus": mup, "mu_minus": mum, "v": vs, "nu": nu,
                "c": c[0::2] + 1j * c[1::2], "ado_n": n, "term_mode": tm}

    def bath(self):
        """(nu, c, c_bra) complex arrays of the exponential bath terms."""
        return heom_model_bath(self)


class State:
    """A device hierarchy of n_traj trajectories."""

    def __init__(self, model: Model, n_traj=1, precision="fp64", handle=None):
        self.model = model
        if handle is None:
            h = C.c_void_p()
            _check(_lib.heom_state_create(model.handle, int(n_traj), _PREC[precision], C.byref(h)))
            handle = h
        self.handle = handle
        nt, pr = C.c_int(), C.c_int()
        _check(_lib.heom_state_shape(self.handle, C.byref(nt), C.byref(pr)))
        self.n_traj, self.precision = nt.value, pr.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.heom_state_free(self.handle)
            self.handle = None

    @property
    def shape(self):
        m = self.model
        return (self.n_traj, m.n_ado, m.d, m.d)

    def upload(self, x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(self.shape))
        _check(_lib.heom_state_upload(self.handle, _ptr(x)))

    def download(self):
        out = np.zeros(self.shape, dtype=np.complex128)
        _check(_lib.heom_state_download(self.handle, _ptr(out)))
        return out

    def upload_range(self, first, x):
        m = self.model
        x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(-1, m.n_ado, m.d, m.d))
        _check(_lib.heom_state_upload_range(self.handle, int(first), x.shape[0], _ptr(x)))

    def download_range(self, first, count):
        m = self.model
        out = np.zeros((count, m.n_ado, m.d, m.d), dtype=np.complex128)
        _check(_lib.heom_state_download_range(self.handle, int(first), int(count), _ptr(out)))
        return out

    def set_ground(self):
        _check(_lib.heom_state_set_ground(self.handle))

    def copy_from(self, other: "State"):
        _check(_lib.heom_state_copy(self.handle, other.handle))


# ----------------------------------------------------- C-named functions --

def heom_model_build(params, stream=None) -> Model:
    return Model(params, stream=stream, device=True)


def heom_model_build_host(params) -> Model:
    return Model(params, device=False)


def heom_state_create(model, n_traj=1, precision="fp64") -> State:
    return State(model, n_traj, precision)


def heom_rhs(model, x_in: State, x_out: State, adjoint=False):
    _check(_lib.heom_rhs(model.handle, x_in.handle, x_out.handle, int(bool(adjoint))))


def heom_propagate(model, state: State, n_steps: int, adjoint=False, sample_every=0):
    """n_steps RK4 steps in place; with sample_every > 0 returns the detection
    traces tr(mu rho_0) as a complex array [n_steps // sample_every + 1][n_traj]."""
    if sample_every and sample_every > 0:
        n_traj = state.n_traj
        out = np.zeros((int(n_steps) // int(sample_every) + 1) * n_traj * 2)
        _check(_lib.heom_propagate(model.handle, state.handle, int(n_steps), int(bool(adjoint)),
                                   int(sample_every), _ptr(out)))
        return (out[0::2] + 1j * out[1::2]).reshape(-1, n_traj)
    _check(_lib.heom_propagate(model.handle, state.handle, int(n_steps), int(bool(adjoint)), 0, None))
    return None


def heom_propagate_noalloc(model, state: State, n_steps: int, adjoint=False, sample_every=0):
    """heom_propagate without device allocations (work buffers in the library's
    static 64 MiB device array); same return value."""
    if sample_every and sample_every > 0:
        n_traj = state.n_traj
        out = np.zeros((int(n_steps) // int(sample_every) + 1) * n_traj * 2)
        _check(_lib.heom_propagate_noalloc(model.handle, state.handle, int(n_steps), int(bool(adjoint)),
                                           int(sample_every), _ptr(out)))
        return (out[0::2] + 1j * out[1::2]).reshape(-1, n_traj)
    _check(_lib.heom_propagate_noalloc(model.handle, state.handle, int(n_steps), int(bool(adjoint)), 0, None))
    return None


def heom_apply_dipole(model, state: State, op="mu", transpose=False):
    _check(_lib.heom_apply_dipole(model.handle, state.handle, _OPS.get(op, op), int(bool(transpose))))


def heom_trace(model, state: State, op="mu"):
    out = np.zeros(2 * state.n_traj)
    _check(_lib.heom_trace(model.handle, state.handle, _OPS.get(op, op), _ptr(out)))
    return out[0::2] + 1j * out[1::2]


def heom_residual(model, state: State):
    r = C.c_double()
    _check(_lib.heom_residual(model.handle, state.handle, C.byref(r)))
    return r.value


def heom_equilibrate(model, tol=1e-10, check_every=100, min_steps=0, max_steps=10000,
                     require_convergence=False):
    h = C.c_void_p()
    steps, res = C.c_int(), C.c_double()
    rc = _lib.heom_equilibrate(model.handle, float(tol), int(check_every), int(min_steps),
                               int(max_steps), int(bool(require_convergence)), C.byref(h),
                               C.byref(steps), C.byref(res))
    if rc == HEOM_ERR_NOCONV and h.value:
        _lib.heom_state_free(h)
    _check(rc)
    return State(model, handle=h), steps.value, res.value


def heom_equilibrate_krylov(model, tol=1e-10, pre_steps=100, steps_per_apply=500, restart=100,
                            max_applies=400):
    """Stationary state by GMRES on (I - Phi^m); returns (state, applications, residual)."""
    h = C.c_void_p()
    applies, res = C.c_int(), C.c_double()
    rc = _lib.heom_equilibrate_krylov(model.handle, float(tol), int(pre_steps), int(steps_per_apply),
                                      int(restart), int(max_applies), C.byref(h), C.byref(applies),
                                      C.byref(res))
    if rc == HEOM_ERR_NOCONV and h.value:
        _lib.heom_state_free(h)
    _check(rc)
    return State(model, handle=h), applies.value, res.value


def heom_stationary_refine(model, state, tol=1e-10, steps_per_apply=500, restart=100, max_applies=100,
                           require_convergence=False):
    """GMRES corrections of `state` in place; returns (applications, residual)."""
    applies, res = C.c_int(), C.c_double()
    rc = _lib.heom_stationary_refine(model.handle, state.handle, float(tol), int(steps_per_apply),
                                     int(restart), int(max_applies), C.byref(applies), C.byref(res))
    if rc != HEOM_ERR_NOCONV or require_convergence:
        _check(rc)
    return applies.value, res.value


def heom_linear_response(model, rho_eq: State, n: int, steps_per_sample: int, precision="fp64"):
    out = np.zeros(2 * n)
    _check(_lib.heom_linear_response(model.handle, rho_eq.handle, int(n), int(steps_per_sample),
                                     _PREC[precision], _ptr(out)))
    return out[0::2] + 1j * out[1::2]


def heom_response_2d(model, rho_eq: State, grid, precision="fp64", method="direct", max_batch=0):
    """R[t2][pathway (I, II)][t1][t3] as complex128."""
    t2 = (C.c_int * len(grid["t2_steps"]))(*[int(s) for s in grid["t2_steps"]])
    g = heom_grid(int(grid["n1"]), int(grid["n3"]), int(grid["steps_per_sample"]),
                  len(grid["t2_steps"]), t2)
    n_t2 = len(grid["t2_steps"])
    out = np.zeros(n_t2 * 2 * grid["n1"] * grid["n3"] * 2)
    _check(_lib.heom_response_2d(model.handle, rho_eq.handle, C.byref(g), _PREC[precision],
                                 _METHOD[method], int(max_batch), _ptr(out)))
    z = out[0::2] + 1j * out[1::2]
    return z.reshape(n_t2, 2, grid["n1"], grid["n3"])


def heom_response_2d_pathways(model, rho_eq: State, grid, pathways, precision="fp64", method="adjoint",
                              max_batch=0):
    """R[t2][pathway][t1][t3] (complex128) for dipole triples (D1, D2, D3), each
    "mu", "mu_plus" or "mu_minus" (or a heom_operator value)."""
    ops = []
    for pw in pathways:
        if len(pw) != 3:
            raise ValueError("a pathway is a triple (D1, D2, D3)")
        ops += [int(_OPS.get(x, x)) for x in pw]
    arr = (C.c_int * len(ops))(*ops)
    g, keep = _grid_struct(grid)
    n_t2 = len(grid["t2_steps"])
    out = np.zeros(n_t2 * len(pathways) * grid["n1"] * grid["n3"] * 2)
    _check(_lib.heom_response_2d_pathways(model.handle, rho_eq.handle, C.byref(g), _PREC[precision],
                                          _METHOD[method], int(max_batch), len(pathways), arr, _ptr(out)))
    z = out[0::2] + 1j * out[1::2]
    return z.reshape(n_t2, len(pathways), grid["n1"], grid["n3"])


def heom_spectrum_1d(R1, dt_s):
    """Linear line shape I(W) on the 2n frequency grid (complex128)."""
    load_library()
    R1 = np.asarray(R1, dtype=complex)
    n = len(R1)
    inp = np.zeros(2 * n)
    inp[0::2], inp[1::2] = R1.real, R1.imag
    out = np.zeros(4 * n)
    _check(_lib.heom_spectrum_1d(_ptr(inp), n, float(dt_s), _ptr(out)))
    return out[0::2] + 1j * out[1::2]


def heom_spectrum_2d(R_I, R_II, dt_s):
    R_I = np.ascontiguousarray(np.asarray(R_I, dtype=np.complex128))
    R_II = np.ascontiguousarray(np.asarray(R_II, dtype=np.complex128))
    n1, n3 = R_I.shape
    S = np.zeros((2 * n3, 2 * n1))
    _check(load_library().heom_spectrum_2d(_ptr(R_I), _ptr(R_II), n1, n3, float(dt_s), _ptr(S)))
    return S


def _grid_struct(grid):
    t2 = (C.c_int * len(grid["t2_steps"]))(*[int(x) for x in grid["t2_steps"]])
    g = heom_grid(int(grid["n1"]), int(grid["n3"]), int(grid["steps_per_sample"]),
                  len(grid["t2_steps"]), t2)
    return g, t2


def _grad_arrays(d, dims, M):
    return {"H": np.zeros((d, d)), "v": np.zeros(sum(x * x for x in dims)), "mu": np.zeros((d, d)),
            "c": np.zeros((M, 2)), "nu": np.zeros(M)}


def _grad_struct(a):
    g = heom_op_grad()
    g.dH, g.dv, g.dmu = a["H"].ctypes.data, a["v"].ctypes.data, a["mu"].ctypes.data
    g.dc, g.dnu = a["c"].ctypes.data, a["nu"].ctypes.data
    return g


def heom_response_2d_vjp(model, rho_eq, grid, W, stationary=True, tol=1e-10, max_steps=1000000):
    """Operator gradients of J = Re sum W R (W: complex [n_t2][2][n1][n3]).

    Returns a dict: H (d x d), v (list of d_s x d_s), mu (d x d), c (n_terms x 2:
    d/dRe c_j, d/dIm c_j), nu (n_terms), stationary_steps, stationary_residual."""
    g, keep = _grid_struct(grid)
    Wi = np.zeros(W.size * 2)
    Wi[0::2] = np.real(W).ravel()
    Wi[1::2] = np.imag(W).ravel()
    a = _grad_arrays(model.d, model.dims, model.n_terms)
    st = _grad_struct(a)
    _check(_lib.heom_response_2d_vjp(model.handle, rho_eq.handle, C.byref(g), _ptr(Wi),
                                     int(bool(stationary)), float(tol), int(max_steps), C.byref(st)))
    vs, off = [], 0
    for ds in model.dims:
        vs.append(a["v"][off:off + ds * ds].reshape(ds, ds).copy())
        off += ds * ds
    return {"H": a["H"], "v": vs, "mu": a["mu"], "c": a["c"], "nu": a["nu"],
            "stationary_steps": st.stationary_steps, "stationary_residual": st.stationary_residual}


def heom_spectrum_2d_vjp(G, n1, n3, dt_s):
    """W[P][j][k] (complex, P = I, II) with sum G S_C(R_I, R_II) = Re sum W R."""
    load_library()
    G = np.ascontiguousarray(G, dtype=np.float64)
    if G.shape != (2 * n3, 2 * n1):
        raise ValueError("G must have shape (2 n3, 2 n1)")
    out = np.zeros(2 * n1 * n3 * 2)
    _check(_lib.heom_spectrum_2d_vjp(_ptr(G), int(n1), int(n3), float(dt_s), _ptr(out)))
    return (out[0::2] + 1j * out[1::2]).reshape(2, n1, n3)


def heom_params_vjp(params, dirs, grad, step=1e-6):
    """out[i] = <grad, d(operators)/d(params) along dirs[i]> (host)."""
    load_library()
    p, keep = _params_struct(params)
    structs = [_params_struct(x) for x in dirs]
    arr = (heom_params * max(1, len(dirs)))(*[x[0] for x in structs])
    a = {"H": np.ascontiguousarray(grad["H"], dtype=np.float64),
         "v": np.ascontiguousarray(np.concatenate([np.ravel(x) for x in grad["v"]]), dtype=np.float64),
         "mu": np.ascontiguousarray(grad["mu"], dtype=np.float64),
         "c": np.ascontiguousarray(grad["c"], dtype=np.float64),
         "nu": np.ascontiguousarray(grad["nu"], dtype=np.float64)}
    st = _grad_struct(a)
    out = np.zeros(len(dirs))
    _check(_lib.heom_params_vjp(C.byref(p), C.cast(arr, C.c_void_p), len(dirs), float(step),
                                C.byref(st), _ptr(out)))
    return out


def heom_response_2d_backward(params, model, rho_eq, grid, dL_dR, dirs, stationary=True, tol=1e-11,
                              max_steps=1000000, step=1e-6):
    """dL/dtheta_i for a loss L(R) of heom_response_2d's output: dL_dR is the
    complex array dL/dRe R + i dL/dIm R ([n_t2][2][n1][n3]), dirs the parameter
    directions d params / d theta_i (dictionaries with the layout of params)."""
    p, keep = _params_struct(params)
    structs = [_params_struct(x) for x in dirs]
    arr = (heom_params * max(1, len(dirs)))(*[x[0] for x in structs])
    g, gkeep = _grid_struct(grid)
    G = np.asarray(dL_dR, dtype=np.complex128)
    Gi = np.zeros(G.size * 2)
    Gi[0::2] = np.real(G).ravel()
    Gi[1::2] = np.imag(G).ravel()
    out = np.zeros(len(dirs))
    _check(_lib.heom_response_2d_backward(C.byref(p), model.handle, rho_eq.handle, C.byref(g), _ptr(Gi),
                                          int(bool(stationary)), float(tol), int(max_steps),
                                          C.cast(arr, C.c_void_p), len(dirs), float(step), _ptr(out)))
    return out


def response_2d_autograd():
    """torch.autograd.Function computing R(theta) = heom_response_2d on the
    stationary state of the model built from params_at(theta), with the
    reverse-mode gradient (heom_response_2d_vjp, then heom_params_vjp along the
    parameter directions d params / d theta) as its backward.

    Usage: R = response_2d_autograd().apply(theta, params_at, directions, grid,
    eq_tol, eq_max_steps); theta is a float64 tensor, R a complex128 tensor
    [n_t2][2][n1][n3] on the CPU."""
    import torch

    class _Response2D(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, params_at, directions, grid, eq_tol=1e-12, eq_max_steps=1000000):
            params = params_at(theta.detach().cpu().numpy())
            model = heom_model_build(params)
            rho, _, _ = heom_equilibrate_krylov(model, tol=eq_tol, max_applies=max(1, eq_max_steps // 500))
            R = heom_response_2d(model, rho, grid, "fp64", "adjoint")
            ctx.model, ctx.rho, ctx.params, ctx.grid = model, rho, params, grid
            ctx.directions = directions
            return torch.from_numpy(R)

        @staticmethod
        def backward(ctx, grad_R):
            # torch passes dL/dRe R + i dL/dIm R, the cotangent convention of
            # heom_response_2d_backward
            gt = heom_response_2d_backward(ctx.params, ctx.model, ctx.rho, ctx.grid,
                                           grad_R.detach().cpu().numpy(), ctx.directions,
                                           stationary=True, tol=1e-11)
            return torch.from_numpy(gt), None, None, None, None, None

    return _Response2D


class Batch:
    """Several models propagated together (one launch per size class and RK4 stage)."""

    def __init__(self, models):
        self.models = list(models)
        arr = (C.c_void_p * len(self.models))(*[m.handle.value for m in self.models])
        h = C.c_void_p()
        _check(_lib.heom_batch_create(arr, len(self.models), C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.heom_batch_free(self.handle)
            self.handle = None


def heom_batch_create(models) -> Batch:
    return Batch(models)


def heom_batch_propagate(batch: Batch, states, n_steps: int, adjoint=False):
    if len(states) != len(batch.models):
        raise ValueError("one state per batch instance")
    arr = (C.c_void_p * len(states))(*[s.handle.value for s in states])
    _check(_lib.heom_batch_propagate(batch.handle, arr, int(n_steps), int(bool(adjoint))))


def heom_batch_response_2d(batch: Batch, rho_eqs, grid, precision="fp32"):
    """List of R[t2][pathway][t1][t3] (complex128), one per instance (adjoint method)."""
    if len(rho_eqs) != len(batch.models):
        raise ValueError("one rho_eq per batch instance")
    t2 = (C.c_int * len(grid["t2_steps"]))(*[int(s) for s in grid["t2_steps"]])
    g = heom_grid(int(grid["n1"]), int(grid["n3"]), int(grid["steps_per_sample"]),
                  len(grid["t2_steps"]), t2)
    n_t2 = len(grid["t2_steps"])
    outs = [np.zeros(n_t2 * 2 * grid["n1"] * grid["n3"] * 2) for _ in batch.models]
    rho = (C.c_void_p * len(rho_eqs))(*[r.handle.value for r in rho_eqs])
    optr = (C.c_void_p * len(outs))(*[o.ctypes.data for o in outs])
    _check(_lib.heom_batch_response_2d(batch.handle, rho, C.byref(g), _PREC[precision], optr))
    return [(o[0::2] + 1j * o[1::2]).reshape(n_t2, 2, grid["n1"], grid["n3"]) for o in outs]


BATCH_LAUNCH = {"auto": 0, "per_class": 1, "single": 2}


def heom_batch_set_launch(batch: Batch, launch: str):
    """Launch form of the batch's RK4 stages: "per_class", "single" or "auto"."""
    _check(_lib.heom_batch_set_launch(batch.handle, BATCH_LAUNCH[launch]))


def heom_batch_get_launch(batch: Batch) -> str:
    out = C.c_int()
    _check(_lib.heom_batch_get_launch(batch.handle, C.byref(out)))
    return {v: k for k, v in BATCH_LAUNCH.items()}[out.value]


def heom_batch_get_class_shape(batch: Batch, nb: int):
    """(workgroups per CU, neighbour-sum form) of size class nb's launch."""
    wg, xl = C.c_int(), C.c_int()
    _check(_lib.heom_batch_get_class_shape(batch.handle, int(nb), C.byref(wg), C.byref(xl)))
    return wg.value, xl.value


def heom_batch_set_class_shape(batch: Batch, nb: int, wg_per_cu=0, lds_sums=-1):
    _check(_lib.heom_batch_set_class_shape(batch.handle, int(nb), int(wg_per_cu), int(lds_sums)))


def heom_batch_set_graph_steps(batch: Batch, steps: int):
    _check(_lib.heom_batch_set_graph_steps(batch.handle, int(steps)))


def heom_batch_autotune(batch: Batch, precision="fp32", n_traj=1, reps=2):
    """Times both launch forms; returns (form auto now resolves to,
    {"per_class": ms per RK4 step, "single": ms per RK4 step or NaN})."""
    ms = np.zeros(2)
    _check(_lib.heom_batch_autotune(batch.handle, _PREC[precision], int(n_traj), int(reps), _ptr(ms)))
    return heom_batch_get_launch(batch), {"per_class": float(ms[0]), "single": float(ms[1])}


def heom_model_set_graph_steps(model, steps):
    _check(_lib.heom_model_set_graph_steps(model.handle, int(steps)))


def heom_model_bath(model):
    """Rates nu_j, coefficients c_j and bra-side coefficients of the bath terms."""
    M = model.n_terms
    out = [np.zeros(2 * M) for _ in range(3)]
    _check(_lib.heom_model_bath(model.handle, *[_ptr(a) for a in out]))
    return tuple(a[0::2] + 1j * a[1::2] for a in out)


def heom_model_set_progress(model, fn, every_steps=50):
    """Call fn(phase, done, total) every `every_steps` RK4 steps of the batched
    t2 / t3 propagations of later response calls on this model; fn=None turns
    it off."""
    if fn is None:
        model._progress_cb = None
        _check(_lib.heom_model_set_progress(model.handle, _PROGRESS_FN(), None, 0))
        return
    cb = _PROGRESS_FN(lambda phase, done, total, ctx: fn(phase.decode(), int(done), int(total)))
    model._progress_cb = cb  # keep the thunk alive while the library holds it
    _check(_lib.heom_model_set_progress(model.handle, cb, None, int(every_steps)))


def heom_model_set_kernel(model, precision, kernel):
    _check(_lib.heom_model_set_kernel(model.handle, _PREC[precision], KERNELS.get(kernel, kernel)))


def heom_model_get_kernel(model, precision):
    k = C.c_int()
    _check(_lib.heom_model_get_kernel(model.handle, _PREC[precision], C.byref(k)))
    return KERNEL_NAMES[k.value]


def heom_autotune(model, n_traj, precision="fp32", reps=2):
    """Times the kernel variants; returns (chosen name, {name: ms per RK4 step})."""
    k = C.c_int()
    ms = np.full(HEOM_KERNEL_MFMA_GH + 1, np.nan)
    _check(_lib.heom_autotune(model.handle, int(n_traj), _PREC[precision], int(reps), C.byref(k),
                              _ptr(ms)))
    return KERNEL_NAMES[k.value], {KERNEL_NAMES[i]: float(ms[i]) for i in range(1, HEOM_KERNEL_MFMA_GH + 1)
                                    if np.isfinite(ms[i])}


def heom_timing_enable(model, enable=True):
    _check(_lib.heom_timing_enable(model.handle, int(bool(enable))))


def heom_timing_read(model):
    ms, n, upd = C.c_double(), C.c_longlong(), C.c_longlong()
    _check(_lib.heom_timing_read(model.handle, C.byref(ms), C.byref(n), C.byref(upd)))
    return ms.value, n.value, upd.value
