// C ABI of the HEOM-2DVS library: object management, device memory and the
// propagation drivers (equilibration, linear and third-order responses).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "heom2dvs.h"
#include "kernels.h"
#include "grad.h"
#include "model.h"

namespace {

thread_local std::string g_last_error;

struct HeomError : std::runtime_error {
  int code;
  HeomError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

heom_alloc_fn g_alloc = nullptr;
heom_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    hipGetLastError();
    throw HeomError(HEOM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (g_alloc) {
    p = g_alloc(bytes, g_alloc_ctx);
    if (!p) throw HeomError(HEOM_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    hipGetLastError();
    throw HeomError(HEOM_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  if (g_alloc && g_free) {
    g_free(p, g_alloc_ctx);
    return;
  }
  (void)hipFree(p);
}

// Owning device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) : p(dev_alloc(b)), bytes(b) {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      dev_free(p);
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { dev_free(p); }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

template <typename F>
int guarded(F&& f) {
  try {
    f();
    return HEOM_OK;
  } catch (const HeomError& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::invalid_argument& e) {
    g_last_error = e.what();
    return HEOM_ERR_PARAM;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return HEOM_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HEOM_ERR_HIP;
  } catch (...) {
    g_last_error = "unknown error";
    return HEOM_ERR_HIP;
  }
}

template <typename T>
DevBuf upload_vec(const std::vector<T>& v, hipStream_t st) {
  DevBuf b(v.size() * sizeof(T));
  if (!v.empty()) hip_check(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st),
                            "upload");
  hip_check(hipStreamSynchronize(st), "upload sync");
  return b;
}

}  // namespace

struct heom_model {
  heom::HostModel hm;
  bool has_device = false;
  int device = 0;
  hipStream_t stream = nullptr;
  int lds_limit = 65536;
  // device copies
  DevBuf H64, H32, v64, v32, g64, g32, gi64, gi32, mu64[3];
  DevBuf Hp64, Hp32;  // H zero-padded to a multiple of 16 (matrix-core kernel)
  // Device basis: the product basis reordered so that three-mode models of
  // the (S; 4, 4) structure read a = 16 a_S + 4 a_M + a_F (the layout of the
  // HEOM_KERNEL_KRON kernel); every device operator and state is in it, and
  // states are permuted at upload / download.  perm[device index] = index
  // in the caller's basis (mode 0 slowest); empty when the two coincide.
  std::vector<int> perm;
  int dstrides[4] = {1, 1, 1, 1};       // strides of the modes in the device basis
  bool kron = false;                    // HEOM_KERNEL_KRON available
  heom::KronArgs kargs[2];              // forward / transposed tables
  std::vector<double> mu_dev;           // mu in the device basis (host copy)
  std::vector<int> quanta_dev;          // N(a) in the device basis
  int kernel[2] = {HEOM_KERNEL_MFMA, HEOM_KERNEL_MFMA};  // per precision
  DevBuf nb_ptr[2], nb_idx[2], nb_a64[2], nb_a32[2];
  DevBuf nb_tj, ado_n;  // forward-table (term, count) pairs and ADO indices (gradient kernels)
  heom::GradOps gops{};
  heom::DevOps<double> ops64[2];
  heom::DevOps<float> ops32[2];
  // two hierarchy-sized work buffers (RK4 stages, dipole results), grown on demand
  DevBuf work[2];
  DevBuf red_partial, red_result;
  // captured RK4 step sequences (launch-bound models): graph_steps RK4 steps
  // per graph, 0 = off; graphs are captured on cap_stream and replayed on stream
  struct Graph {
    const void* y;
    const void* w1;
    const void* w2;
    int n_traj;
    bool adjoint;
    int prec;
    int kernel;
    hipGraphExec_t exec;
  };
  int graph_steps = 0;
  hipStream_t cap_stream = nullptr;
  // progress reporting of long response calls (off when fn is null)
  heom_progress_fn progress_fn = nullptr;
  void* progress_ctx = nullptr;
  int progress_every = 0;
  std::vector<Graph> graphs;
  void clear_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  // kernel timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
  long long launches = 0, ado_updates = 0;

  ~heom_model() {
    clear_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& e : events) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
  long long traj_elems() const { return static_cast<long long>(hm.n_ado) * 2 * hm.d * hm.d; }
};

struct heom_state {
  heom_model* model = nullptr;
  int n_traj = 0;
  int precision = HEOM_FP64;
  DevBuf buf;
  long long n_elems() const { return static_cast<long long>(n_traj) * model->traj_elems(); }
  size_t elem_size() const { return precision == HEOM_FP64 ? sizeof(double) : sizeof(float); }
};

namespace {

void require_device(const heom_model* m) {
  if (!m) throw HeomError(HEOM_ERR_PARAM, "null model");
  if (!m->has_device) throw HeomError(HEOM_ERR_STATE, "model has no device data (built with heom_model_build_host)");
}

void require_state(const heom_model* m, const heom_state* s) {
  if (!s) throw HeomError(HEOM_ERR_PARAM, "null state");
  if (s->model != m) throw HeomError(HEOM_ERR_STATE, "state belongs to another model");
}

heom_params copy_check(const heom_params* p) {
  if (!p) throw HeomError(HEOM_ERR_PARAM, "null params");
  return *p;
}

// Chooses the device basis (see heom_model::perm) and returns the d x d
// operator A (caller's basis) in it.
void choose_device_basis(heom_model* m) {
  const auto& hm = m->hm;
  int roles[3];
  m->perm.clear();
  for (int s = 0; s < 4; ++s) m->dstrides[s] = hm.strides[s];
  m->kron = heom::kron_roles(hm.d, hm.n_modes, hm.dims, roles);
  if (!m->kron) return;
  const int S = roles[0], M = roles[1], F = roles[2];
  m->dstrides[S] = 16;
  m->dstrides[M] = 4;
  m->dstrides[F] = 1;
  m->perm.resize(hm.d);
  for (int a = 0; a < hm.d; ++a) {
    const int aS = a / 16, aM = (a / 4) % 4, aF = a % 4;
    m->perm[a] = aS * hm.strides[S] + aM * hm.strides[M] + aF * hm.strides[F];
  }
  bool identity = true;
  for (int a = 0; a < hm.d; ++a) identity = identity && m->perm[a] == a;
  if (identity) m->perm.clear();
}

std::vector<double> to_device_basis(const heom_model* m, const std::vector<double>& A) {
  if (m->perm.empty()) return A;
  const int d = m->hm.d;
  std::vector<double> B(A.size());
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      B[static_cast<size_t>(a) * d + b] = A[static_cast<size_t>(m->perm[a]) * d + m->perm[b]];
  return B;
}

// d x d array in the device basis -> caller's basis, in place
void to_user_basis(const heom_model* m, double* A) {
  if (m->perm.empty()) return;
  const int d = m->hm.d;
  std::vector<double> B(A, A + static_cast<size_t>(d) * d);
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      A[static_cast<size_t>(m->perm[a]) * d + m->perm[b]] = B[static_cast<size_t>(a) * d + b];
}

void upload_model(heom_model* m) {
  const auto& hm = m->hm;
  hipStream_t st = m->stream;
  std::vector<float> tmp;
  auto f32 = [&](const std::vector<double>& v) {
    tmp.assign(v.begin(), v.end());
    return upload_vec(tmp, st);
  };
  choose_device_basis(m);
  const std::vector<double> Hd = to_device_basis(m, hm.H);
  m->mu_dev = to_device_basis(m, hm.mu);
  m->quanta_dev.resize(hm.d);
  for (int a = 0; a < hm.d; ++a) m->quanta_dev[a] = hm.quanta[m->perm.empty() ? a : m->perm[a]];
  m->H64 = upload_vec(Hd, st);
  // FP32 copy of H shifted by (min + max of its diagonal) / 2 times the
  // identity: the commutator [H, rho] is unchanged, while the products H rho
  // and rho H whose difference it is shrink (about half the spectral range),
  // and with them their FP32 rounding
  std::vector<double> Hs = Hd;
  {
    double lo = Hd[0], hi = Hd[0];
    for (int a = 0; a < hm.d; ++a) {
      lo = std::min(lo, Hd[static_cast<size_t>(a) * hm.d + a]);
      hi = std::max(hi, Hd[static_cast<size_t>(a) * hm.d + a]);
    }
    const double c = 0.5 * (lo + hi);
    for (int a = 0; a < hm.d; ++a) Hs[static_cast<size_t>(a) * hm.d + a] -= c;
  }
  m->H32 = f32(Hs);
  std::vector<double> vpack;
  int v_off[4] = {0, 0, 0, 0};
  for (int s = 0; s < hm.n_modes; ++s) {
    v_off[s] = static_cast<int>(vpack.size());
    vpack.insert(vpack.end(), hm.v[s].begin(), hm.v[s].end());
  }
  m->v64 = upload_vec(vpack, st);
  m->v32 = f32(vpack);
  m->g64 = upload_vec(hm.gamma_sum, st);
  m->g32 = f32(hm.gamma_sum);
  if (hm.complex_rates) {
    m->gi64 = upload_vec(hm.gamma_sum_im, st);
    m->gi32 = f32(hm.gamma_sum_im);
  }
  m->mu64[HEOM_OP_MU] = upload_vec(m->mu_dev, st);
  m->mu64[HEOM_OP_MU_PLUS] = upload_vec(to_device_basis(m, hm.mu_plus), st);
  m->mu64[HEOM_OP_MU_MINUS] = upload_vec(to_device_basis(m, hm.mu_minus), st);
  for (int dir = 0; dir < 2; ++dir) {
    const heom::Neighbours& nb = dir == 0 ? hm.fwd : hm.adj;
    m->nb_ptr[dir] = upload_vec(nb.ptr, st);
    m->nb_idx[dir] = upload_vec(nb.idx, st);
    std::vector<double> a(nb.aL.size() * 4);
    for (size_t q = 0; q < nb.aL.size(); ++q) {
      a[4 * q] = nb.aL[q].real();
      a[4 * q + 1] = nb.aL[q].imag();
      a[4 * q + 2] = nb.aR[q].real();
      a[4 * q + 3] = nb.aR[q].imag();
    }
    m->nb_a64[dir] = upload_vec(a, st);
    m->nb_a32[dir] = f32(a);
    auto fill = [&](auto& op, const DevBuf& H, const DevBuf& v, const DevBuf& g, const DevBuf& gi,
                    const DevBuf& na) {
      using T = std::remove_const_t<std::remove_pointer_t<decltype(op.H)>>;
      op.H = H.as<T>();
      op.v = v.as<T>();
      op.gamma = g.as<T>();
      op.gamma_im = hm.complex_rates ? gi.as<T>() : nullptr;
      op.nb_ptr = m->nb_ptr[dir].as<int>();
      op.nb_idx = m->nb_idx[dir].as<int>();
      op.nb_a = na.as<T>();
      for (int s = 0; s < 4; ++s) {
        op.v_off[s] = v_off[s];
        op.dims[s] = hm.dims[s];
        op.strides[s] = m->dstrides[s];
      }
      op.n_modes = hm.n_modes;
      op.d = hm.d;
      op.n_ado = hm.n_ado;
    };
    fill(m->ops64[dir], m->H64, m->v64, m->g64, m->gi64, m->nb_a64[dir]);
    fill(m->ops32[dir], m->H32, m->v32, m->g32, m->gi32, m->nb_a32[dir]);
  }
  {
    const int d = hm.d, DP = 16 * ((d + 15) / 16);
    std::vector<double> hp(static_cast<size_t>(DP) * DP, 0.0);
    for (int a = 0; a < d; ++a)
      for (int c = 0; c < d; ++c) hp[static_cast<size_t>(a) * DP + c] = Hd[static_cast<size_t>(a) * d + c];
    m->Hp64 = upload_vec(hp, st);
    for (int a = 0; a < d; ++a)
      for (int c = 0; c < d; ++c) hp[static_cast<size_t>(a) * DP + c] = Hs[static_cast<size_t>(a) * d + c];
    m->Hp32 = f32(hp);
    if (!heom::mfma_supported<double>(d, hm.n_modes, hm.dims)) m->kernel[HEOM_FP64] = HEOM_KERNEL_GENERIC;
    if (!heom::mfma_supported<float>(d, hm.n_modes, hm.dims)) m->kernel[HEOM_FP32] = HEOM_KERNEL_GENERIC;
  }
  {
    m->nb_tj = upload_vec(hm.fwd.tj, st);
    m->ado_n = upload_vec(hm.ado_n, st);
    heom::GradOps& g = m->gops;
    g.v = m->v64.as<double>();
    g.nb_ptr = m->nb_ptr[0].as<int>();
    g.nb_idx = m->nb_idx[0].as<int>();
    g.nb_a = m->nb_a64[0].as<double>();
    g.nb_tj = m->nb_tj.as<int>();
    g.ado_n = m->ado_n.as<int>();
    for (int s = 0; s < 4; ++s) {
      g.v_off[s] = v_off[s];
      g.dims[s] = hm.dims[s];
      g.strides[s] = m->dstrides[s];
    }
    g.n_modes = hm.n_modes;
    g.d = hm.d;
    g.n_ado = hm.n_ado;
    g.n_terms = hm.n_terms;
  }
  if (m->kron) {
    int roles[3];
    heom::kron_roles(hm.d, hm.n_modes, hm.dims, roles);
    for (int dir = 0; dir < 2; ++dir) {
      heom::KronArgs& k = m->kargs[dir];
      const auto& op = m->ops32[dir];
      k.H = op.H;
      k.gamma = op.gamma;
      k.gamma_im = op.gamma_im;
      k.nb_ptr = op.nb_ptr;
      k.nb_idx = op.nb_idx;
      k.nb_a = op.nb_a;
      k.n_modes = hm.n_modes;
      k.n_ado = hm.n_ado;
      k.mode_S = roles[0];
      k.mode_M = roles[1];
      k.mode_F = roles[2];
      for (int e = 0; e < 64; ++e) k.vS[e] = 0.0f;
      for (size_t e = 0; e < hm.v[roles[0]].size(); ++e) k.vS[e] = static_cast<float>(hm.v[roles[0]][e]);
      for (int e = 0; e < 16; ++e) {
        k.vM[e] = static_cast<float>(hm.v[roles[1]][e]);
        k.vF[e] = static_cast<float>(hm.v[roles[2]][e]);
      }
    }
  }
  m->red_result = DevBuf(sizeof(double) * 4);
  m->has_device = true;
}

// typed helpers ------------------------------------------------------------

template <typename T>
const heom::DevOps<T>& ops_of(const heom_model* m, bool adjoint);
template <>
const heom::DevOps<double>& ops_of<double>(const heom_model* m, bool adjoint) { return m->ops64[adjoint ? 1 : 0]; }
template <>
const heom::DevOps<float>& ops_of<float>(const heom_model* m, bool adjoint) { return m->ops32[adjoint ? 1 : 0]; }

std::pair<hipEvent_t, hipEvent_t> next_event_pair(heom_model* m) {
  if (m->events_used == m->events.size()) {
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "event create");
    hip_check(hipEventCreate(&b), "event create");
    m->events.emplace_back(a, b);
  }
  return m->events[m->events_used++];
}

template <typename T>
const T* padded_H(const heom_model* m);
template <>
const double* padded_H<double>(const heom_model* m) { return m->Hp64.as<double>(); }
template <>
const float* padded_H<float>(const heom_model* m) { return m->Hp32.as<float>(); }

template <typename T>
constexpr int prec_of() { return std::is_same<T, double>::value ? HEOM_FP64 : HEOM_FP32; }

// One launch of the chosen RHS / RK4-stage kernel.
template <typename T>
void launch_stage(heom_model* m, bool adjoint, const T* in, const T* y, T* out, double coef, int n_traj) {
  const auto& op = ops_of<T>(m, adjoint);
  const int k = m->kernel[prec_of<T>()];
  if (k == HEOM_KERNEL_GENERIC)
    heom::launch_rhs<T>(op, in, y, out, coef, n_traj, m->stream);
  else if constexpr (std::is_same<T, float>::value) {
    if (k == HEOM_KERNEL_KRON)
      heom::launch_rhs_kron(m->kargs[adjoint ? 1 : 0], m->hm.d, in, y, out, coef, n_traj, m->stream);
    else if (k == HEOM_KERNEL_MFMA_GH)
      heom::launch_rhs_mfma_gh<T>(op, padded_H<T>(m), in, y, out, coef, n_traj, m->stream);
    else
      heom::launch_rhs_mfma<T>(op, padded_H<T>(m), in, y, out, coef, n_traj, k == HEOM_KERNEL_MFMA_DYN ? 1 : 0,
                               m->stream);
  } else
    heom::launch_rhs_mfma<T>(op, padded_H<T>(m), in, y, out, coef, n_traj, k == HEOM_KERNEL_MFMA_DYN ? 1 : 0,
                             m->stream);
}

// One launch of the fused RHS / RK4-stage kernel (timed when enabled).
template <typename T>
void stage(heom_model* m, bool adjoint, const T* in, const T* y, T* out, double coef, int n_traj) {
  if (m->timing) {
    auto ev = next_event_pair(m);
    hip_check(hipEventRecord(ev.first, m->stream), "event record");
    launch_stage<T>(m, adjoint, in, y, out, coef, n_traj);
    hip_check(hipEventRecord(ev.second, m->stream), "event record");
    m->launches += 1;
    m->ado_updates += static_cast<long long>(n_traj) * m->hm.n_ado;
  } else {
    launch_stage<T>(m, adjoint, in, y, out, coef, n_traj);
  }
}

template <typename T>
T* work_buffer(heom_model* m, int slot, long long elems) {
  size_t bytes = static_cast<size_t>(elems) * sizeof(T);
  if (m->work[slot].bytes < bytes) {
    hip_check(hipStreamSynchronize(m->stream), "sync before work buffer growth");
    m->clear_graphs();
    m->work[slot] = DevBuf();
    m->work[slot] = DevBuf(bytes);
  }
  return m->work[slot].as<T>();
}

// n_steps RK4 steps in place on y (n_traj trajectories), with work buffers
// w1, w2 of the same size:  y <- y + h L(y + h/2 L(y + h/3 L(y + h/4 L y))).
// One RK4 step as four fused stage launches (Horner form).
template <typename T>
void rk4_step_launches(heom_model* m, T* y, T* w1, T* w2, int n_traj, bool adjoint) {
  const double h = m->hm.dt;
  launch_stage<T>(m, adjoint, y, y, w1, h / 4.0, n_traj);
  launch_stage<T>(m, adjoint, w1, y, w2, h / 3.0, n_traj);
  launch_stage<T>(m, adjoint, w2, y, w1, h / 2.0, n_traj);
  launch_stage<T>(m, adjoint, w1, y, y, h, n_traj);
}

// Executable graph of graph_steps RK4 steps on these buffers (captured on
// first use; null if capture is not possible, which turns graphs off).
template <typename T>
hipGraphExec_t rk4_graph(heom_model* m, T* y, T* w1, T* w2, int n_traj, bool adjoint) {
  for (const auto& g : m->graphs)
    if (g.y == y && g.w1 == w1 && g.w2 == w2 && g.n_traj == n_traj && g.adjoint == adjoint &&
        g.prec == prec_of<T>() && g.kernel == m->kernel[prec_of<T>()])
      return g.exec;
  if (m->graphs.size() >= 32) m->clear_graphs();
  if (!m->cap_stream) hip_check(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking), "stream create");
  hip_check(hipStreamSynchronize(m->stream), "sync");
  hipStream_t saved = m->stream;
  m->stream = m->cap_stream;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
  if (ok) {
    try {
      for (int s = 0; s < m->graph_steps; ++s) rk4_step_launches<T>(m, y, w1, w2, n_traj, adjoint);
    } catch (...) {
      ok = false;
    }
    ok = (hipStreamEndCapture(m->cap_stream, &graph) == hipSuccess) && ok && graph;
  }
  m->stream = saved;
  if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipGetLastError();
  if (!ok) {
    m->graph_steps = 0;  // fall back to direct launches for this model
    return nullptr;
  }
  m->graphs.push_back({y, w1, w2, n_traj, adjoint, prec_of<T>(), m->kernel[prec_of<T>()], exec});
  return exec;
}

template <typename T>
void rk4_steps(heom_model* m, T* y, T* w1, T* w2, int n_traj, int n_steps, bool adjoint) {
  const double h = m->hm.dt;
  if (m->graph_steps > 0 && !m->timing && n_steps >= m->graph_steps) {
    hipGraphExec_t ex = rk4_graph<T>(m, y, w1, w2, n_traj, adjoint);
    if (ex) {
      const int reps = n_steps / m->graph_steps;
      for (int r = 0; r < reps; ++r) hip_check(hipGraphLaunch(ex, m->stream), "graph launch");
      n_steps -= reps * m->graph_steps;
    }
  }
  for (int s = 0; s < n_steps; ++s) {
    stage<T>(m, adjoint, y, y, w1, h / 4.0, n_traj);
    stage<T>(m, adjoint, w1, y, w2, h / 3.0, n_traj);
    stage<T>(m, adjoint, w2, y, w1, h / 2.0, n_traj);
    stage<T>(m, adjoint, w1, y, y, h, n_traj);
  }
}

template <typename T>
void rk4_steps_ws(heom_model* m, T* y, int n_traj, int n_steps, bool adjoint) {
  if (n_steps <= 0) return;
  const long long elems = static_cast<long long>(n_traj) * m->traj_elems();
  T* w1 = work_buffer<T>(m, 0, elems);
  T* w2 = work_buffer<T>(m, 1, elems);
  rk4_steps<T>(m, y, w1, w2, n_traj, n_steps, adjoint);
}

// Progress of one phase of a response call: steps counted over all its
// trajectory batches and pathways.
struct Progress {
  heom_model* m;
  const char* phase;
  long long total, done = 0, next = 0;
  Progress(heom_model* mm, const char* ph, long long tot) : m(mm), phase(ph), total(tot) {
    next = m->progress_every;
  }
  bool on() const { return m->progress_fn && m->progress_every > 0; }
};

// rk4_steps, split at every multiple of the progress interval (counted over
// the whole phase) to synchronise and report there.
template <typename T>
void rk4_steps_reported(heom_model* m, T* y, T* w1, T* w2, int n_traj, int n_steps, Progress& pr) {
  if (!pr.on()) {
    rk4_steps<T>(m, y, w1, w2, n_traj, n_steps, false);
    pr.done += n_steps;
    return;
  }
  while (n_steps > 0) {
    const int k = static_cast<int>(std::min<long long>(n_steps, pr.next - pr.done));
    rk4_steps<T>(m, y, w1, w2, n_traj, k, false);
    n_steps -= k;
    pr.done += k;
    if (pr.done >= pr.next) {
      hip_check(hipStreamSynchronize(m->stream), "sync");
      m->progress_fn(pr.phase, pr.done, pr.total, m->progress_ctx);
      pr.next += m->progress_every;
    }
  }
}

template <typename T>
double absmax(heom_model* m, const T* x, long long n_mats) {
  if (m->red_partial.bytes < static_cast<size_t>(n_mats) * sizeof(double)) {
    hip_check(hipStreamSynchronize(m->stream), "sync");
    m->red_partial = DevBuf();
    m->red_partial = DevBuf(static_cast<size_t>(n_mats) * sizeof(double));
  }
  heom::launch_absmax<T>(x, m->hm.d, n_mats, m->red_partial.as<double>(), m->red_result.as<double>(),
                         m->stream);
  double r = 0.0;
  hip_check(hipMemcpyAsync(&r, m->red_result.p, sizeof(double), hipMemcpyDeviceToHost, m->stream), "copy");
  hip_check(hipStreamSynchronize(m->stream), "sync");
  return r;
}

// L(x) into work buffer 0, then max |.|
template <typename T>
double residual_of(heom_model* m, const T* x, int n_traj) {
  const long long elems = static_cast<long long>(n_traj) * m->traj_elems();
  T* w = work_buffer<T>(m, 0, elems);
  launch_stage<T>(m, false, x, nullptr, w, 1.0, n_traj);
  return absmax<T>(m, w, static_cast<long long>(n_traj) * m->hm.n_ado);
}

template <typename T>
void check_finite(heom_model* m, const T* x, int n_traj, const char* where) {
  double r = absmax<T>(m, x, static_cast<long long>(n_traj) * m->hm.n_ado);
  if (!std::isfinite(r))
    throw HeomError(HEOM_ERR_UNSTABLE, std::string("non-finite hierarchy after ") + where +
                                           " (time step beyond the RK4 stability region?)");
}

template <typename T>
void propagate_sampled(heom_model* m, heom_state* s, int n_steps, bool adjoint, int sample_every, double* trace_out) {
  T* y = s->buf.as<T>();
  if (sample_every <= 0 || !trace_out) {
    rk4_steps_ws<T>(m, y, s->n_traj, n_steps, adjoint);
  } else {
    // tr(mu rho_0) of every trajectory at steps 0, sample_every, ... <= n_steps
    const int n_samples = n_steps / sample_every + 1;
    DevBuf tr(static_cast<size_t>(n_samples) * s->n_traj * 2 * sizeof(double));
    for (int k = 0; k < n_samples; ++k) {
      if (k > 0) rk4_steps_ws<T>(m, y, s->n_traj, sample_every, adjoint);
      heom::launch_trace<T>(m->mu64[HEOM_OP_MU].as<double>(), y, m->hm.d, m->traj_elems(), s->n_traj,
                            tr.as<double>() + static_cast<size_t>(k) * s->n_traj * 2, 1, m->stream);
    }
    const int rest = n_steps - (n_samples - 1) * sample_every;
    if (rest > 0) rk4_steps_ws<T>(m, y, s->n_traj, rest, adjoint);
    hip_check(hipMemcpyAsync(trace_out, tr.p, tr.bytes, hipMemcpyDeviceToHost, m->stream), "copy");
    hip_check(hipStreamSynchronize(m->stream), "sync");
  }
  check_finite<T>(m, y, s->n_traj, "propagation");
}

std::unique_ptr<heom_state> new_state(heom_model* m, int n_traj, int prec) {
  auto s = std::make_unique<heom_state>();
  s->model = m;
  s->n_traj = n_traj;
  s->precision = prec;
  s->buf = DevBuf(static_cast<size_t>(s->n_elems()) * s->elem_size());
  // zero fill
  if (prec == HEOM_FP64)
    heom::launch_set_ground<double>(s->buf.as<double>(), m->traj_elems(), 0, s->n_elems(), m->stream);
  else
    heom::launch_set_ground<float>(s->buf.as<float>(), m->traj_elems(), 0, s->n_elems(), m->stream);
  return s;
}

// dst (precision of dst) <- D^x src (FP64 source), n matrices.
template <typename T>
void commute_from64(heom_model* m, int op, int transpose, const double* src, T* dst, long long n_mats,
                    double* tmp64) {
  if constexpr (std::is_same<T, double>::value) {
    heom::launch_commutator<double>(m->mu64[op].as<double>(), transpose, src, dst, m->hm.d, n_mats, m->stream);
  } else {
    heom::launch_commutator<double>(m->mu64[op].as<double>(), transpose, src, tmp64, m->hm.d, n_mats,
                                    m->stream);
    heom::launch_convert<double, T>(tmp64, dst, n_mats * 2 * m->hm.d * m->hm.d, m->stream);
  }
}

size_t free_device_bytes() {
  size_t fr = 0, tot = 0;
  hip_check(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
  return fr;
}

// ------------------------------------------------------------- responses --

template <typename T>
void linear_response_impl(heom_model* m, const heom_state* rho_eq, int n, int sps, double* R_out) {
  const long long te = m->traj_elems();
  const int d = m->hm.d;
  DevBuf X(static_cast<size_t>(te) * sizeof(T));
  DevBuf tmp(static_cast<size_t>(te) * sizeof(double));
  commute_from64<T>(m, HEOM_OP_MU, 0, rho_eq->buf.as<double>(), X.as<T>(), m->hm.n_ado, tmp.as<double>());
  DevBuf out(static_cast<size_t>(n) * 2 * sizeof(double));
  for (int k = 0; k < n; ++k) {
    if (k) rk4_steps_ws<T>(m, X.as<T>(), 1, sps, false);
    heom::launch_trace<T>(m->mu64[HEOM_OP_MU].as<double>(), X.as<T>(), d, te, 1, out.as<double>() + 2 * k, 1,
                          m->stream);
  }
  check_finite<T>(m, X.as<T>(), 1, "linear response");
  std::vector<double> h(static_cast<size_t>(n) * 2);
  hip_check(hipMemcpyAsync(h.data(), out.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, m->stream), "copy");
  hip_check(hipStreamSynchronize(m->stream), "sync");
  for (int k = 0; k < n; ++k) {  // R1 = i * tr(...)
    R_out[2 * k] = -h[2 * k + 1];
    R_out[2 * k + 1] = h[2 * k];
  }
}

// Snapshots of the t1 trajectory: snap[j] = D2^x G(t1_j) D1^x rho_eq.
template <typename T>
void t1_snapshots(heom_model* m, const heom_state* rho_eq, int D1, int D2, int n1, int sps, T* snap) {
  const long long te = m->traj_elems();
  const long long n_mats = m->hm.n_ado;
  DevBuf X(static_cast<size_t>(te) * sizeof(T));
  DevBuf tmp(static_cast<size_t>(te) * sizeof(double));
  commute_from64<T>(m, D1, 0, rho_eq->buf.as<double>(), X.as<T>(), n_mats, tmp.as<double>());
  for (int j = 0; j < n1; ++j) {
    if (j) rk4_steps_ws<T>(m, X.as<T>(), 1, sps, false);
    heom::launch_commutator<T>(m->mu64[D2].as<double>(), 0, X.as<T>(), snap + j * te, m->hm.d, n_mats,
                               m->stream);
  }
  check_finite<T>(m, X.as<T>(), 1, "t1 scan");
}

int auto_batch(heom_model* m, int n_total, size_t elem, long long per_traj_buffers, size_t fixed_bytes,
               int max_batch) {
  if (max_batch > 0) return std::min(max_batch, n_total);
  const size_t te_bytes = static_cast<size_t>(m->traj_elems()) * elem;
  size_t fr = free_device_bytes();
  size_t budget = fr > fixed_bytes + (size_t(2) << 30) ? fr - fixed_bytes - (size_t(2) << 30) : 0;
  long long c = static_cast<long long>(budget / (te_bytes * per_traj_buffers));
  if (c < 1) throw HeomError(HEOM_ERR_OOM, "not enough device memory for one trajectory batch");
  return static_cast<int>(std::min<long long>(c, n_total));
}

// Pathway p applies (D1, D2, D3) = (ops[3p], ops[3p+1], ops[3p+2]) (heom_operator
// values); R is written as [n_t2][n_pw][n1][n3] complex.
template <typename T>
void response_direct(heom_model* m, const heom_state* rho_eq, const heom_grid& g, int max_batch, int n_pw,
                     const int* ops, double* Rdev) {
  const long long te = m->traj_elems();
  const int d = m->hm.d;
  const int n1 = g.n1, n3 = g.n3, sps = g.steps_per_sample;
  const size_t tb = static_cast<size_t>(te) * sizeof(T);
  DevBuf snap(tb * n1);
  const int C = auto_batch(m, n1, sizeof(T), 3, 0, max_batch);
  DevBuf Z(tb * C), W1(tb * C), W2(tb * C);
  const long long n_batches = (n1 + C - 1) / C;
  Progress pr(m, "t2/t3 propagation",
              n_pw * n_batches * (g.t2_steps[g.n_t2 - 1] + static_cast<long long>(g.n_t2) * (n3 - 1) * sps));
  for (int P = 0; P < n_pw; ++P) {
    const int* pw = ops + 3 * P;
    t1_snapshots<T>(m, rho_eq, pw[0], pw[1], n1, sps, snap.as<T>());
    for (int j0 = 0; j0 < n1; j0 += C) {
      const int c = std::min(C, n1 - j0);
      T* Y = snap.as<T>() + j0 * te;
      int done = 0;
      for (int i = 0; i < g.n_t2; ++i) {
        rk4_steps_reported<T>(m, Y, W1.as<T>(), W2.as<T>(), c, g.t2_steps[i] - done, pr);
        done = g.t2_steps[i];
        heom::launch_commutator<T>(m->mu64[pw[2]].as<double>(), 0, Y, Z.as<T>(), d,
                                   static_cast<long long>(c) * m->hm.n_ado, m->stream);
        for (int k = 0; k < n3; ++k) {
          if (k) rk4_steps_reported<T>(m, Z.as<T>(), W1.as<T>(), W2.as<T>(), c, sps, pr);
          double* out = Rdev + 2 * ((((static_cast<long long>(i) * n_pw + P) * n1 + j0) * n3) + k);
          heom::launch_trace<T>(m->mu64[HEOM_OP_MU].as<double>(), Z.as<T>(), d, te, c, out, n3, m->stream);
        }
        check_finite<T>(m, Z.as<T>(), c, "t3 propagation");
      }
    }
  }
}

template <typename T>
void response_adjoint(heom_model* m, const heom_state* rho_eq, const heom_grid& g, int max_batch, int n_pw,
                      const int* ops, double* Rdev) {
  const long long te = m->traj_elems();
  const int d = m->hm.d;
  const int n1 = g.n1, n3 = g.n3, sps = g.steps_per_sample;
  const size_t tb = static_cast<size_t>(te) * sizeof(T);
  // detection functional: l_0 = mu^T (n = 0 ADO), propagated with L^T;
  // Psi_k = (D3^x)^T l(t3_k).  The samples l(t3_k) are kept only when the
  // pathways use more than one D3.
  bool one_d3 = true;
  for (int P = 1; P < n_pw; ++P) one_d3 = one_d3 && ops[3 * P + 2] == ops[2];
  DevBuf Psi(tb * n3), Lk;
  if (!one_d3) Lk = DevBuf(tb * n3);
  {
    std::vector<double> h(static_cast<size_t>(te), 0.0);
    for (int a = 0; a < d; ++a)
      for (int c = 0; c < d; ++c) h[static_cast<size_t>(a) * d + c] = m->mu_dev[static_cast<size_t>(c) * d + a];
    DevBuf l64 = upload_vec(h, m->stream);
    DevBuf l(tb);
    heom::launch_convert<double, T>(l64.as<double>(), l.as<T>(), te, m->stream);
    for (int k = 0; k < n3; ++k) {
      if (k) rk4_steps_ws<T>(m, l.as<T>(), 1, sps, true);
      if (one_d3)
        heom::launch_commutator<T>(m->mu64[ops[2]].as<double>(), 1, l.as<T>(), Psi.as<T>() + k * te, d,
                                   m->hm.n_ado, m->stream);
      else
        hip_check(hipMemcpyAsync(Lk.as<T>() + k * te, l.p, tb, hipMemcpyDeviceToDevice, m->stream), "copy");
    }
    check_finite<T>(m, l.as<T>(), 1, "adjoint t3 scan");
  }
  DevBuf snap(tb * n1);
  const int C = auto_batch(m, n1, sizeof(T), 2, 0, max_batch);
  DevBuf W1(tb * C), W2(tb * C);
  DevBuf work(heom::pair_work_doubles(C, n3, m->hm.n_ado, d) * sizeof(double));
  int psi_op = one_d3 ? ops[2] : -1;
  Progress pr(m, "t2 propagation", static_cast<long long>(n_pw) * ((n1 + C - 1) / C) * g.t2_steps[g.n_t2 - 1]);
  for (int P = 0; P < n_pw; ++P) {
    const int* pw = ops + 3 * P;
    if (pw[2] != psi_op) {
      heom::launch_commutator<T>(m->mu64[pw[2]].as<double>(), 1, Lk.as<T>(), Psi.as<T>(), d,
                                 static_cast<long long>(n3) * m->hm.n_ado, m->stream);
      psi_op = pw[2];
    }
    t1_snapshots<T>(m, rho_eq, pw[0], pw[1], n1, sps, snap.as<T>());
    for (int j0 = 0; j0 < n1; j0 += C) {
      const int c = std::min(C, n1 - j0);
      T* Y = snap.as<T>() + j0 * te;
      int done = 0;
      for (int i = 0; i < g.n_t2; ++i) {
        rk4_steps_reported<T>(m, Y, W1.as<T>(), W2.as<T>(), c, g.t2_steps[i] - done, pr);
        done = g.t2_steps[i];
        double* out = Rdev + 2 * (((static_cast<long long>(i) * n_pw + P) * n1 + j0) * n3);
        // R = i^3 <Psi_k, Y_j> = -i <.,.>
        heom::launch_pairing<T>(Y, c, Psi.as<T>(), n3, m->hm.n_ado, d, 0.0, -1.0, work.as<double>(), out,
                                m->stream);
      }
      check_finite<T>(m, Y, c, "t2 propagation");
    }
  }
}

// Rotating-wave pathways of heom_response_2d: I (rephasing) and II (non-rephasing).
constexpr int kStdPathways[6] = {HEOM_OP_MU_MINUS, HEOM_OP_MU_PLUS, HEOM_OP_MU_PLUS,
                                 HEOM_OP_MU_PLUS, HEOM_OP_MU_MINUS, HEOM_OP_MU_PLUS};

void response_any(heom_model* m, const heom_state* rho_eq, const heom_grid* grid, int precision, int method,
                  int max_batch, int n_pw, const int* ops, double* R_out) {
  require_device(m);
  require_state(m, rho_eq);
  if (rho_eq->precision != HEOM_FP64 || rho_eq->n_traj != 1)
    throw HeomError(HEOM_ERR_STATE, "rho_eq must be an FP64 state with one trajectory");
  if (!grid || !R_out || !ops || n_pw < 1) throw HeomError(HEOM_ERR_PARAM, "null argument or no pathway");
  for (int q = 0; q < 3 * n_pw; ++q)
    if (ops[q] < HEOM_OP_MU || ops[q] > HEOM_OP_MU_MINUS) throw HeomError(HEOM_ERR_PARAM, "bad dipole operator");
  const heom_grid& g = *grid;
  if (g.n1 < 1 || g.n3 < 1 || g.steps_per_sample < 1 || g.n_t2 < 1 || !g.t2_steps)
    throw HeomError(HEOM_ERR_PARAM, "bad grid");
  for (int i = 0; i < g.n_t2; ++i)
    if (g.t2_steps[i] < 0 || (i && g.t2_steps[i] < g.t2_steps[i - 1]))
      throw HeomError(HEOM_ERR_PARAM, "t2_steps must be non-negative and non-decreasing");
  if (method != HEOM_RESP_DIRECT && method != HEOM_RESP_ADJOINT) throw HeomError(HEOM_ERR_PARAM, "bad method");
  const size_t n_out = static_cast<size_t>(g.n_t2) * n_pw * g.n1 * g.n3 * 2;
  DevBuf Rdev(n_out * sizeof(double));
  if (precision == HEOM_FP64) {
    if (method == HEOM_RESP_DIRECT) response_direct<double>(m, rho_eq, g, max_batch, n_pw, ops, Rdev.as<double>());
    else response_adjoint<double>(m, rho_eq, g, max_batch, n_pw, ops, Rdev.as<double>());
  } else if (precision == HEOM_FP32) {
    if (method == HEOM_RESP_DIRECT) response_direct<float>(m, rho_eq, g, max_batch, n_pw, ops, Rdev.as<double>());
    else response_adjoint<float>(m, rho_eq, g, max_batch, n_pw, ops, Rdev.as<double>());
  } else {
    throw HeomError(HEOM_ERR_PARAM, "bad precision");
  }
  std::vector<double> h(n_out);
  hip_check(hipMemcpyAsync(h.data(), Rdev.p, n_out * sizeof(double), hipMemcpyDeviceToHost, m->stream), "copy");
  hip_check(hipStreamSynchronize(m->stream), "sync");
  if (method == HEOM_RESP_DIRECT) {
    // R = i^3 tr(...) = -i tr(...)
    for (size_t q = 0; q < n_out / 2; ++q) {
      R_out[2 * q] = h[2 * q + 1];
      R_out[2 * q + 1] = -h[2 * q];
    }
  } else {
    std::memcpy(R_out, h.data(), n_out * sizeof(double));
  }
}

}  // namespace

struct heom_batch {
  std::vector<heom_model*> models;
  hipStream_t stream = nullptr;
  double dt = 0.0;
  int launch = HEOM_BATCH_AUTO;   // requested launch form
  int tuned = 0;                  // form chosen by heom_batch_autotune (0: none yet)
  double class_cost[8] = {};      // measured time per matrix of each size class (0: cost model)
  heom::MultiShape class_shape[8];  // per-class launch shape (autotuned; defaults otherwise)
  int graph_steps = 0;            // RK4 steps per captured graph (0: direct launches)
  hipStream_t cap_stream = nullptr;
  ~heom_batch() {
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  int resolved_launch() const {
    if (launch != HEOM_BATCH_AUTO) return launch;
    return tuned ? tuned : HEOM_BATCH_PER_CLASS;
  }
};

namespace {

// Relative time of one matrix per workgroup in size class nb when nothing
// was measured: matrix-core work grows as nb^3, neighbour and staging traffic
// as nb^2, and a workgroup has nb waves (per-matrix latency grows about as
// nb (nb + 1)), plus a fixed part for the item's global loads and barriers.
double default_class_cost(int nb) { return 4.0 + static_cast<double>(nb) * (nb + 1); }

// Descriptor sets of one batched propagation: per size class and for both
// generators, the four stage role assignments of the Horner RK4 step.  With
// the single-launch form the classes' descriptors are also concatenated and
// the launch's workgroups split among the classes in proportion to their
// estimated work (items x cost per item).
template <typename T>
struct BatchProp {
  struct Class {
    int nb = 0, vw = 1, n_inst = 0;
    long long n_items = 0;
    heom::MultiShape shape;
    DevBuf desc[2][4];
  };
  std::vector<Class> classes;
  std::vector<DevBuf> w1, w2;
  bool single = false;
  DevBuf fdesc[2][4], fcls;
  int n_cls = 0, waves = 0, grid = 0;
  size_t lds = 0;
  std::vector<heom::FusedClass> fhost;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int gsteps[2] = {0, 0};

  BatchProp() = default;
  BatchProp(const BatchProp&) = delete;
  BatchProp& operator=(const BatchProp&) = delete;
  ~BatchProp() {
    for (auto& e : gexec)
      if (e) (void)hipGraphExecDestroy(e);
  }

  void build(heom_batch* b, const std::vector<T*>& ys, const std::vector<int>& n_traj) {
    build_as(b, ys, n_traj, b->resolved_launch());
  }

  void build_as(heom_batch* b, const std::vector<T*>& ys, const std::vector<int>& n_traj, int form) {
    const int n = static_cast<int>(b->models.size());
    std::map<int, std::vector<int>> by_nb;
    for (int i = 0; i < n; ++i) by_nb[(b->models[i]->hm.d + 15) / 16].push_back(i);
    w1.clear();
    w2.clear();
    w1.resize(n);
    w2.resize(n);
    for (int i = 0; i < n; ++i) {
      const size_t bytes = static_cast<size_t>(n_traj[i]) * b->models[i]->traj_elems() * sizeof(T);
      w1[i] = DevBuf(bytes);
      w2[i] = DevBuf(bytes);
    }
    classes.clear();
    std::vector<heom::InstDesc<T>> all[2][4];
    std::vector<int> nbs;
    for (auto& kv : by_nb) {
      Class c;
      c.nb = kv.first;
      c.shape = b->class_shape[c.nb];
      c.n_inst = static_cast<int>(kv.second.size());
      const int full_vw = 16 / static_cast<int>(sizeof(T));
      c.vw = full_vw;
      for (int i : kv.second)
        if (b->models[i]->hm.d % full_vw) c.vw = 1;
      for (int a = 0; a < 2; ++a)
        for (int st = 0; st < 4; ++st) {
          std::vector<heom::InstDesc<T>> h;
          long long begin = 0;
          for (int i : kv.second) {
            heom_model* m = b->models[i];
            T* y = ys[i];
            T* p1 = w1[i].as<T>();
            T* p2 = w2[i].as<T>();
            heom::InstDesc<T> d;
            d.op = ops_of<T>(m, a == 1);
            d.Hp = padded_H<T>(m);
            const T* ins[4] = {y, p1, p2, p1};
            T* outs[4] = {p1, p2, p1, y};
            d.in = ins[st];
            d.y = y;
            d.out = outs[st];
            d.item_begin = begin;
            begin += static_cast<long long>(n_traj[i]) * m->hm.n_ado;
            h.push_back(d);
          }
          c.n_items = begin;
          all[a][st].insert(all[a][st].end(), h.begin(), h.end());
          c.desc[a][st] = upload_vec(h, b->stream);
        }
      nbs.push_back(c.nb);
      classes.push_back(std::move(c));
    }
    single = form == HEOM_BATCH_SINGLE;
    if (!single) return;
    waves = heom::fused_block_waves<T>(nbs.data(), static_cast<int>(nbs.size()));
    if (waves == 0) throw HeomError(HEOM_ERR_PARAM, "single-launch batches need every d <= 80");
    lds = 0;
    for (int nb : nbs) lds = std::max(lds, heom::fused_lds_bytes<T>(nb));
    const long long G = static_cast<long long>(heom::cu_count()) * heom::fused_workgroups_per_cu<T>(waves, lds);
    double total = 0.0;
    std::vector<double> w(classes.size());
    for (size_t c = 0; c < classes.size(); ++c) {
      const double cost = b->class_cost[classes[c].nb] > 0.0 ? b->class_cost[classes[c].nb]
                                                              : default_class_cost(classes[c].nb);
      w[c] = cost * static_cast<double>(classes[c].n_items);
      total += w[c];
    }
    fhost.clear();
    int begin = 0, inst = 0;
    for (size_t c = 0; c < classes.size(); ++c) {
      long long wg = total > 0.0 ? std::llround(static_cast<double>(G) * w[c] / total) : 1;
      wg = std::max<long long>(1, std::min<long long>(wg, std::max<long long>(1, classes[c].n_items)));
      heom::FusedClass f;
      f.nb = classes[c].nb;
      f.vw = classes[c].vw;
      f.inst_first = inst;
      f.n_inst = classes[c].n_inst;
      f.n_items = classes[c].n_items;
      f.wg_begin = begin;
      f.wg_end = begin + static_cast<int>(wg);
      begin = f.wg_end;
      inst += classes[c].n_inst;
      fhost.push_back(f);
    }
    grid = begin;
    n_cls = static_cast<int>(fhost.size());
    fcls = upload_vec(fhost, b->stream);
    for (int a = 0; a < 2; ++a)
      for (int st = 0; st < 4; ++st) fdesc[a][st] = upload_vec(all[a][st], b->stream);
  }

  void stage_launch(int st, bool adjoint, double coef, hipStream_t stream) {
    const int a = adjoint ? 1 : 0;
    if (single) {
      heom::launch_rhs_mfma_fused<T>(fcls.as<heom::FusedClass>(), n_cls, fdesc[a][st].template as<heom::InstDesc<T>>(),
                                     waves, lds, grid, coef, stream);
      return;
    }
    for (auto& c : classes)
      heom::launch_rhs_mfma_multi<T>(c.desc[a][st].template as<heom::InstDesc<T>>(), c.n_inst, c.nb, c.vw, coef,
                                     c.n_items, stream, c.shape);
  }

  void direct_steps(heom_batch* b, int n_steps, bool adjoint, hipStream_t stream) {
    const double h = b->dt;
    const double coef[4] = {h / 4.0, h / 3.0, h / 2.0, h};
    for (int k = 0; k < n_steps; ++k)
      for (int st = 0; st < 4; ++st) stage_launch(st, adjoint, coef[st], stream);
  }

  // graph of b->graph_steps RK4 steps (captured on first use; null when
  // capture fails, which turns graphs off for the batch)
  hipGraphExec_t graph(heom_batch* b, bool adjoint) {
    const int a = adjoint ? 1 : 0;
    if (gexec[a] && gsteps[a] == b->graph_steps) return gexec[a];
    if (gexec[a]) {
      (void)hipGraphExecDestroy(gexec[a]);
      gexec[a] = nullptr;
    }
    if (!b->cap_stream) hip_check(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "stream create");
    hip_check(hipStreamSynchronize(b->stream), "sync");
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      try {
        direct_steps(b, b->graph_steps, adjoint, b->cap_stream);
      } catch (...) {
        ok = false;
      }
      ok = (hipStreamEndCapture(b->cap_stream, &g) == hipSuccess) && ok && g;
    }
    if (ok) ok = hipGraphInstantiate(&gexec[a], g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!ok) {
      gexec[a] = nullptr;
      b->graph_steps = 0;
      return nullptr;
    }
    gsteps[a] = b->graph_steps;
    return gexec[a];
  }

  void steps(heom_batch* b, int n_steps, bool adjoint) {
    if (b->graph_steps > 0 && n_steps >= b->graph_steps) {
      hipGraphExec_t ex = graph(b, adjoint);
      if (ex) {
        const int reps = n_steps / gsteps[adjoint ? 1 : 0];
        for (int r = 0; r < reps; ++r) hip_check(hipGraphLaunch(ex, b->stream), "graph launch");
        n_steps -= reps * gsteps[adjoint ? 1 : 0];
      }
    }
    direct_steps(b, n_steps, adjoint, b->stream);
  }
};

// heom_batch_autotune: per-class time per matrix, then both launch forms.
template <typename T>
void batch_autotune(heom_batch* b, int n_traj, int reps, double* ms_out) {
  const int n = static_cast<int>(b->models.size());
  std::vector<DevBuf> st(n);
  std::vector<T*> ys(n);
  const std::vector<int> nt(n, n_traj);
  for (int i = 0; i < n; ++i) {
    const long long te = b->models[i]->traj_elems();
    st[i] = DevBuf(static_cast<size_t>(n_traj) * te * sizeof(T));
    ys[i] = st[i].as<T>();
    heom::launch_set_ground<T>(ys[i], te, n_traj, static_cast<long long>(n_traj) * te, b->stream);
  }
  // no graphs while timing; restores the graph setting and frees the events on every exit
  struct Guard {
    heom_batch* b;
    int graph_steps;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Guard() {
      b->graph_steps = graph_steps;
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } guard{b, b->graph_steps};
  b->graph_steps = 0;
  hip_check(hipEventCreate(&guard.e0), "event");
  hip_check(hipEventCreate(&guard.e1), "event");
  auto elapsed = [&] {
    hip_check(hipEventSynchronize(guard.e1), "event sync");
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, guard.e0, guard.e1), "event time");
    return static_cast<double>(ms);
  };
  const double h = b->dt;
  const double coef[4] = {h / 4.0, h / 3.0, h / 2.0, h};
  BatchProp<T> pc;
  pc.build_as(b, ys, nt, HEOM_BATCH_PER_CLASS);
  pc.direct_steps(b, 1, false, b->stream);  // code objects, caches
  std::vector<int> nbs;
  for (auto& c : pc.classes) {
    nbs.push_back(c.nb);
    // launch shapes of the class alone: the most and half the resident
    // workgroups per CU, each with both neighbour-sum forms where both exist
    const int max_wg = static_cast<int>(std::max<long long>(
        1, heom::rhs_mfma_multi_grid<T>(c.nb, c.vw, 1LL << 40, heom::MultiShape()) / heom::cu_count()));
    std::vector<int> wgs = {max_wg};
    if (max_wg / 2 >= 1) wgs.push_back(max_wg / 2);
    const std::vector<int> xls = heom::multi_has_alt_xl<T>(c.nb) ? std::vector<int>{0, 1} : std::vector<int>{-1};
    std::vector<heom::MultiShape> cand;
    for (int wg : wgs)
      for (int xl : xls) cand.push_back(heom::MultiShape{wg, xl});
    double best_ms = 0.0;
    heom::MultiShape best;
    for (const auto& sh : cand) {
      hip_check(hipEventRecord(guard.e0, b->stream), "event record");
      for (int k = 0; k < reps; ++k)
        for (int s4 = 0; s4 < 4; ++s4)
          heom::launch_rhs_mfma_multi<T>(c.desc[0][s4].template as<heom::InstDesc<T>>(), c.n_inst, c.nb, c.vw,
                                         coef[s4], c.n_items, b->stream, sh);
      hip_check(hipEventRecord(guard.e1, b->stream), "event record");
      const double ms = elapsed();
      if (best_ms == 0.0 || ms < best_ms) {
        best_ms = ms;
        best = sh;
      }
      // time per matrix per workgroup of the LDS neighbour-sum form at the
      // most workgroups (the form the single launch runs): what sets how many
      // of the single launch's workgroups the class needs
      if (sh.wg_per_cu == max_wg && (sh.xl == 1 || (sh.xl < 0))) {
        const double grid_c = static_cast<double>(heom::rhs_mfma_multi_grid<T>(c.nb, c.vw, c.n_items, sh));
        b->class_cost[c.nb] =
            ms * grid_c / (4.0 * reps * static_cast<double>(std::max<long long>(1, c.n_items)));
      }
    }
    b->class_shape[c.nb] = best;
    c.shape = best;
  }
  hip_check(hipEventRecord(guard.e0, b->stream), "event record");
  pc.direct_steps(b, reps, false, b->stream);
  hip_check(hipEventRecord(guard.e1, b->stream), "event record");
  const double ms_pc = elapsed() / reps;
  double ms_single = std::nan("");
  if (heom::fused_block_waves<T>(nbs.data(), static_cast<int>(nbs.size())) > 0) {
    BatchProp<T> ps;
    ps.build_as(b, ys, nt, HEOM_BATCH_SINGLE);
    ps.direct_steps(b, 1, false, b->stream);
    hip_check(hipEventRecord(guard.e0, b->stream), "event record");
    ps.direct_steps(b, reps, false, b->stream);
    hip_check(hipEventRecord(guard.e1, b->stream), "event record");
    ms_single = elapsed() / reps;
  }
  b->tuned = (std::isfinite(ms_single) && ms_single < ms_pc) ? HEOM_BATCH_SINGLE : HEOM_BATCH_PER_CLASS;
  if (ms_out) {
    ms_out[0] = ms_pc;
    ms_out[1] = ms_single;
  }
}

template <typename T>
void batch_response_adjoint(heom_batch* b, const heom_state* const* rho_eq, const heom_grid& g,
                            double* const* R_out) {
  const int n = static_cast<int>(b->models.size());
  const int n1 = g.n1, n3 = g.n3, sps = g.steps_per_sample;
  std::vector<long long> te(n);
  for (int i = 0; i < n; ++i) te[i] = b->models[i]->traj_elems();
  // detection functionals l_i (mu^T on ADO 0) and Psi_i[k] = (mu+^x)^T l_i(t3_k)
  std::vector<DevBuf> l(n), Psi(n), X(n), snap(n), tmp64(n), Rdev(n);
  size_t work_doubles = 0;
  for (int i = 0; i < n; ++i) {
    heom_model* m = b->models[i];
    const int d = m->hm.d;
    std::vector<double> h(static_cast<size_t>(te[i]), 0.0);
    for (int a = 0; a < d; ++a)
      for (int c = 0; c < d; ++c) h[static_cast<size_t>(a) * d + c] = m->mu_dev[static_cast<size_t>(c) * d + a];
    DevBuf l64 = upload_vec(h, b->stream);
    l[i] = DevBuf(static_cast<size_t>(te[i]) * sizeof(T));
    heom::launch_convert<double, T>(l64.as<double>(), l[i].as<T>(), te[i], b->stream);
    hip_check(hipStreamSynchronize(b->stream), "sync");
    Psi[i] = DevBuf(static_cast<size_t>(n3) * te[i] * sizeof(T));
    X[i] = DevBuf(static_cast<size_t>(te[i]) * sizeof(T));
    snap[i] = DevBuf(static_cast<size_t>(n1) * te[i] * sizeof(T));
    tmp64[i] = DevBuf(static_cast<size_t>(te[i]) * sizeof(double));
    Rdev[i] = DevBuf(static_cast<size_t>(g.n_t2) * 2 * n1 * n3 * 2 * sizeof(double));
    work_doubles = std::max(work_doubles, heom::pair_work_doubles(n1, n3, m->hm.n_ado, d));
  }
  DevBuf work(work_doubles * sizeof(double));
  {
    BatchProp<T> pl;
    std::vector<T*> ys(n);
    for (int i = 0; i < n; ++i) ys[i] = l[i].as<T>();
    pl.build(b, ys, std::vector<int>(n, 1));
    for (int k = 0; k < n3; ++k) {
      if (k) pl.steps(b, sps, true);
      for (int i = 0; i < n; ++i)
        heom::launch_commutator<T>(b->models[i]->mu64[HEOM_OP_MU_PLUS].as<double>(), 1, l[i].as<T>(),
                                   Psi[i].as<T>() + k * te[i], b->models[i]->hm.d, b->models[i]->hm.n_ado,
                                   b->stream);
    }
  }
  BatchProp<T> px, py;
  {
    std::vector<T*> ys(n);
    for (int i = 0; i < n; ++i) ys[i] = X[i].as<T>();
    px.build(b, ys, std::vector<int>(n, 1));
    if (g.t2_steps[g.n_t2 - 1] > 0) {
      for (int i = 0; i < n; ++i) ys[i] = snap[i].as<T>();
      py.build(b, ys, std::vector<int>(n, n1));
    }
  }
  const int pw_d[2][2] = {{HEOM_OP_MU_MINUS, HEOM_OP_MU_PLUS}, {HEOM_OP_MU_PLUS, HEOM_OP_MU_MINUS}};
  for (int P = 0; P < 2; ++P) {
    for (int i = 0; i < n; ++i)
      commute_from64<T>(b->models[i], pw_d[P][0], 0, rho_eq[i]->buf.as<double>(), X[i].as<T>(),
                        b->models[i]->hm.n_ado, tmp64[i].as<double>());
    for (int j = 0; j < n1; ++j) {
      if (j) px.steps(b, sps, false);
      for (int i = 0; i < n; ++i)
        heom::launch_commutator<T>(b->models[i]->mu64[pw_d[P][1]].as<double>(), 0, X[i].as<T>(),
                                   snap[i].as<T>() + j * te[i], b->models[i]->hm.d, b->models[i]->hm.n_ado,
                                   b->stream);
    }
    int done = 0;
    for (int q = 0; q < g.n_t2; ++q) {
      if (g.t2_steps[q] > done) py.steps(b, g.t2_steps[q] - done, false);
      done = g.t2_steps[q];
      for (int i = 0; i < n; ++i) {
        heom_model* m = b->models[i];
        double* out = Rdev[i].as<double>() + 2 * ((static_cast<long long>(q) * 2 + P) * n1 * n3);
        heom::launch_pairing<T>(snap[i].as<T>(), n1, Psi[i].as<T>(), n3, m->hm.n_ado, m->hm.d, 0.0, -1.0,
                                work.as<double>(), out, b->stream);
      }
    }
  }
  for (int i = 0; i < n; ++i) {
    check_finite<T>(b->models[i], snap[i].as<T>(), n1, "batched propagation");
    hip_check(hipMemcpyAsync(R_out[i], Rdev[i].p, Rdev[i].bytes, hipMemcpyDeviceToHost, b->stream), "copy");
  }
  hip_check(hipStreamSynchronize(b->stream), "sync");
}

}  // namespace

namespace {

// ----------------------------------------------------------------------------
// Stationary problems by GMRES.  With Phi the RK4 propagator of the forward
// (or transposed) generator, A = I - Phi^m (m RK4 steps) has the stationary
// state (or the trace functional) as its null vector; on the complement its
// slow modes are isolated near 0 while every mode that decays within m steps
// sits near 1, so restarted GMRES converges in far fewer propagation steps
// than plain time stepping.  FP64, one trajectory.
struct Krylov {
  heom_model* m;
  bool adjoint;
  int msteps;
  long long te;
  DevBuf part, dot, tmp;
  // progress reporting (heom_model_set_progress): RK4 steps of the operator
  // applications so far, of at most steps_total
  long long steps_done = 0, steps_total = 0, next_report = 0;
  Krylov(heom_model* mm, bool adj, int ms) : m(mm), adjoint(adj), msteps(ms), te(mm->traj_elems()) {
    part = DevBuf(static_cast<size_t>(2 * heom::hdot_parts()) * sizeof(double));
    dot = DevBuf(2 * sizeof(double));
    tmp = DevBuf(static_cast<size_t>(te) * sizeof(double));
  }
  std::complex<double> hdot(const double* x, const double* y) {
    heom::launch_hdot(x, y, m->hm.n_ado, m->hm.d, part.as<double>(), dot.as<double>(), m->stream);
    double h[2];
    hip_check(hipMemcpyAsync(h, dot.p, sizeof(h), hipMemcpyDeviceToHost, m->stream), "copy");
    hip_check(hipStreamSynchronize(m->stream), "sync");
    return {h[0], h[1]};
  }
  double norm(const double* x) { return std::sqrt(std::max(0.0, hdot(x, x).real())); }
  void axpy(std::complex<double> a, const double* x, double* y) {
    heom::launch_axpy(a.real(), a.imag(), x, y, m->hm.n_ado, m->hm.d, m->stream);
  }
  void copy(const double* x, double* y) {
    hip_check(hipMemcpyAsync(y, x, te * sizeof(double), hipMemcpyDeviceToDevice, m->stream), "copy");
  }
  void zero(double* y) { hip_check(hipMemsetAsync(y, 0, te * sizeof(double), m->stream), "memset"); }
  // w = (I - Phi^m) v
  void apply(const double* v, double* w) {
    copy(v, tmp.as<double>());
    rk4_steps_ws<double>(m, tmp.as<double>(), 1, msteps, adjoint);
    copy(v, w);
    axpy(-1.0, tmp.as<double>(), w);
    steps_done += msteps;
    if (m->progress_fn && m->progress_every > 0 && steps_done >= next_report) {
      hip_check(hipStreamSynchronize(m->stream), "sync");
      m->progress_fn("stationary solve", steps_done, steps_total, m->progress_ctx);
      next_report = (steps_done / m->progress_every + 1) * m->progress_every;
    }
  }
};

// Restarted GMRES for (I - Phi^m) x = b from the guess in x.  Stops when the
// residual estimate is <= rtol ||b|| or after max_applies operator
// applications; returns the last relative residual estimate.
double gmres(Krylov& K, const double* b, double* x, int restart, int max_applies, double rtol, int* applies) {
  using cd = std::complex<double>;
  const long long te = K.te;
  DevBuf V(static_cast<size_t>(restart + 1) * te * sizeof(double)), w(static_cast<size_t>(te) * sizeof(double));
  double* Vp = V.as<double>();
  const double bnorm = K.norm(b);
  *applies = 0;
  if (bnorm == 0.0) {
    K.zero(x);
    return 0.0;
  }
  double rel = 1.0;
  while (true) {
    // r = b - A x into V_0
    K.apply(x, w.as<double>());
    ++*applies;
    K.copy(b, Vp);
    K.axpy(-1.0, w.as<double>(), Vp);
    const double beta = K.norm(Vp);
    rel = beta / bnorm;
    if (rel <= rtol || *applies >= max_applies) return rel;
    K.zero(w.as<double>());
    K.axpy(1.0 / beta, Vp, w.as<double>());
    K.copy(w.as<double>(), Vp);
    std::vector<cd> H(static_cast<size_t>(restart + 1) * restart, 0.0), g(restart + 1, 0.0), sn(restart, 0.0);
    std::vector<double> cs(restart, 0.0);
    g[0] = beta;
    int kk = 0;
    for (int k = 0; k < restart && *applies < max_applies; ++k) {
      double* vk = Vp + k * te;
      double* vn = Vp + (k + 1) * te;
      K.apply(vk, w.as<double>());
      ++*applies;
      for (int j = 0; j <= k; ++j) {  // modified Gram-Schmidt
        const cd h = K.hdot(Vp + j * te, w.as<double>());
        H[j * restart + k] = h;
        K.axpy(-h, Vp + j * te, w.as<double>());
      }
      const double hn = K.norm(w.as<double>());
      H[(k + 1) * restart + k] = hn;
      K.zero(vn);
      if (hn > 0.0) K.axpy(1.0 / hn, w.as<double>(), vn);
      for (int j = 0; j < k; ++j) {  // previous rotations
        const cd a = H[j * restart + k], c = H[(j + 1) * restart + k];
        H[j * restart + k] = cs[j] * a + sn[j] * c;
        H[(j + 1) * restart + k] = -std::conj(sn[j]) * a + cs[j] * c;
      }
      const cd a = H[k * restart + k];
      const double bb = std::abs(H[(k + 1) * restart + k]);
      const double t = std::sqrt(std::norm(a) + bb * bb);
      if (std::abs(a) == 0.0) {
        cs[k] = 0.0;
        sn[k] = 1.0;
      } else {
        cs[k] = std::abs(a) / t;
        sn[k] = (a / std::abs(a)) * std::conj(H[(k + 1) * restart + k]) / t;
      }
      H[k * restart + k] = cs[k] * a + sn[k] * H[(k + 1) * restart + k];
      H[(k + 1) * restart + k] = 0.0;
      g[k + 1] = -std::conj(sn[k]) * g[k];
      g[k] = cs[k] * g[k];
      kk = k + 1;
      rel = std::abs(g[k + 1]) / bnorm;
      if (rel <= rtol || hn == 0.0) break;
    }
    // x += V y with H y = g (upper triangular)
    std::vector<cd> y(kk, 0.0);
    for (int i = kk - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int j = i + 1; j < kk; ++j) acc -= H[i * restart + j] * y[j];
      y[i] = H[i * restart + i] != 0.0 ? acc / H[i * restart + i] : 0.0;
    }
    for (int j = 0; j < kk; ++j) K.axpy(y[j], Vp + j * te, x);
    if (rel <= rtol || *applies >= max_applies) {
      hip_check(hipStreamSynchronize(K.m->stream), "sync");
      return rel;
    }
  }
}

}  // namespace

namespace {

// ----------------------------------------------------------------------------
// Reverse-mode gradient of J = Re sum W R (heom_response_2d_vjp).  FP64.
//
// The RK4 propagator is Phi = p(hL), p(z) = 1 + z + z^2/2 + z^3/6 + z^4/24, and
// for a step y -> Phi y with adjoint lambda (the cotangent of Phi y) the
// operator derivative is <lambda, dPhi y> = sum_{a+b<=3} c_{a+b}
// <(L^T)^a lambda, dL L^b y>, c_m = h^(m+1)/(m+1)!.  <u, dL z> is contracted
// into operator gradients by the grad.hip kernels (K below).

struct GradCtx {
  heom_model* m;
  long long te;    // doubles per trajectory
  double h;
  DevBuf partH, partP, partM;   // [max_parts][d*d]
  DevBuf gv, gc, gnu;           // device accumulators
  DevBuf C4, C1;                // combine coefficients (4x4 powers -> z'_a; 1x4 step)
  // sweep buffers
  DevBuf S, Ob, Zp;
  long long cap_S = 0, cap_O = 0;
  Progress* pr = nullptr;  // adjoint steps swept (heom_model_set_progress)
};

DevBuf upload_coef(const std::vector<double>& c, hipStream_t st) { return upload_vec(c, st); }

void zero_dev(DevBuf& b, hipStream_t st) {
  if (b.bytes) hip_check(hipMemsetAsync(b.p, 0, b.bytes, st), "memset");
}

void grad_init(GradCtx& g, heom_model* m) {
  g.m = m;
  g.te = m->traj_elems();
  g.h = m->hm.dt;
  const size_t dd = static_cast<size_t>(m->hm.d) * m->hm.d;
  const size_t parts = static_cast<size_t>(heom::grad_max_parts()) * dd * sizeof(double);
  g.partH = DevBuf(parts);
  g.partP = DevBuf(parts);
  g.partM = DevBuf(parts);
  size_t nv = 0;
  for (int s = 0; s < m->hm.n_modes; ++s) nv += static_cast<size_t>(m->hm.dims[s]) * m->hm.dims[s];
  g.gv = DevBuf(nv * sizeof(double));
  g.gc = DevBuf(static_cast<size_t>(m->hm.n_terms) * 2 * sizeof(double));
  g.gnu = DevBuf(static_cast<size_t>(m->hm.n_terms) * sizeof(double));
  for (DevBuf* b : {&g.partH, &g.partP, &g.partM, &g.gv, &g.gc, &g.gnu}) zero_dev(*b, m->stream);
  const double h = g.h;
  const double c[4] = {h, h * h / 2.0, h * h * h / 6.0, h * h * h * h / 24.0};
  std::vector<double> c4(32, 0.0);  // z'_a = sum_b c_{a+b} w_b
  for (int a = 0; a < 4; ++a)
    for (int b = 0; a + b < 4; ++b) c4[2 * (a * 4 + b)] = c[a + b];
  g.C4 = upload_coef(c4, m->stream);
  std::vector<double> c1 = {1.0, 0.0, h, 0.0, h * h / 2.0, 0.0, h * h * h / 6.0, 0.0};
  g.C1 = upload_coef(c1, m->stream);
}

// <u, dL z> over n_traj trajectories
void k_generator(GradCtx& g, const double* u, const double* z, int n_traj) {
  heom_model* m = g.m;
  const long long items = static_cast<long long>(n_traj) * m->hm.n_ado;
  heom::launch_gemm_grad(u, z, items, m->hm.d, 0.0, -1.0, g.partH.as<double>(), m->stream);
  int off = 0;
  for (int s = 0; s < m->hm.n_modes; ++s) {
    heom::launch_nb_grad(m->gops, s, u, z, items, g.gv.as<double>() + off, g.gc.as<double>(), g.gnu.as<double>(),
                         m->stream);
    off += m->hm.dims[s] * m->hm.dims[s];
  }
}

// <u, dD^x z> into the mu+ or mu- accumulator
void k_dipole(GradCtx& g, int op, const double* u, const double* z, int n_traj) {
  heom_model* m = g.m;
  const long long items = static_cast<long long>(n_traj) * m->hm.n_ado;
  double* part = op == HEOM_OP_MU_PLUS ? g.partP.as<double>() : g.partM.as<double>();
  heom::launch_gemm_grad(u, z, items, m->hm.d, 1.0, 0.0, part, m->stream);
}

void combine(GradCtx& g, const double* in, long long in_stride, int n_in, double* out, long long out_stride,
             int n_out, const double* coef, int acc, int n_traj) {
  heom::launch_combine(in, in_stride, n_in, out, out_stride, n_out, coef, acc,
                       static_cast<long long>(n_traj) * g.m->hm.n_ado, g.m->hm.d, g.m->stream);
}

void ensure(DevBuf& b, long long& cap, long long doubles, hipStream_t st) {
  if (cap < doubles) {
    hip_check(hipStreamSynchronize(st), "sync");
    b = DevBuf();
    b = DevBuf(static_cast<size_t>(doubles) * sizeof(double));
    cap = doubles;
  }
}

// Adjoint sweep over one segment of n steps.  The stored side starts at S0
// (nt trajectories) and is propagated forward with the generator of its own
// kind (L, or L^T if stored_adjoint); the other side O holds its state at the
// segment end and is carried back to the segment start with the transposed
// generator.  Accumulates the operator derivatives of every step.
void sweep(GradCtx& g, const double* S0, double* O, int nt, int n, bool stored_adjoint) {
  if (n <= 0) return;
  heom_model* m = g.m;
  hipStream_t st = m->stream;
  const long long N = static_cast<long long>(nt) * g.te;
  ensure(g.S, g.cap_S, static_cast<long long>(n) * 4 * N, st);
  ensure(g.Ob, g.cap_O, 8 * N, st);
  double* S = g.S.as<double>();
  double* Ob = g.Ob.as<double>();       // Ob[0..3]: on-the-fly powers
  double* Zp = Ob + 4 * N;              // combined partners z'_a
  const bool gs = stored_adjoint, go = !stored_adjoint;
  const double h = g.h;
  // forward recompute with powers
  hip_check(hipMemcpyAsync(S, S0, N * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  for (int k = 0; k < n; ++k) {
    double* Sk = S + static_cast<long long>(k) * 4 * N;
    for (int p = 1; p < 4; ++p) stage<double>(m, gs, Sk + (p - 1) * N, nullptr, Sk + p * N, 1.0, nt);
    if (k + 1 < n) {
      double* nx = S + static_cast<long long>(k + 1) * 4 * N;
      combine(g, Sk, N, 4, nx, N, 1, g.C1.as<double>(), 0, nt);
      stage<double>(m, gs, Sk + 3 * N, nx, nx, h * h * h * h / 24.0, nt);
    }
  }
  // backward
  hip_check(hipMemcpyAsync(Ob, O, N * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  for (int k = n - 1; k >= 0; --k) {
    double* Sk = S + static_cast<long long>(k) * 4 * N;
    for (int p = 1; p < 4; ++p) stage<double>(m, go, Ob + (p - 1) * N, nullptr, Ob + p * N, 1.0, nt);
    if (!stored_adjoint) {
      // stored = forward y (L powers w_b), on the fly = lambda (L^T powers u_a)
      combine(g, Sk, N, 4, Zp, N, 4, g.C4.as<double>(), 0, nt);
      for (int a = 0; a < 4; ++a) k_generator(g, Ob + a * N, Zp + a * N, nt);
    } else {
      // stored = L^T powers u_a, on the fly = L powers w_b
      combine(g, Ob, N, 4, Zp, N, 4, g.C4.as<double>(), 0, nt);
      for (int a = 0; a < 4; ++a) k_generator(g, Sk + a * N, Zp + a * N, nt);
    }
    // O(k) = Phi_O O(k+1)
    combine(g, Ob, N, 4, Ob, N, 1, g.C1.as<double>(), 0, nt);
    stage<double>(m, go, Ob + 3 * N, Ob, Ob, h * h * h * h / 24.0, nt);
  }
  hip_check(hipMemcpyAsync(O, Ob, N * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  if (g.pr) {
    Progress& pr = *g.pr;
    pr.done += n;
    if (pr.on() && pr.done >= pr.next) {
      hip_check(hipStreamSynchronize(st), "sync");
      m->progress_fn(pr.phase, pr.done, pr.total, m->progress_ctx);
      pr.next = (pr.done / m->progress_every + 1) * m->progress_every;
    }
  }
}

void copy_dev(double* dst, const double* src, long long n, hipStream_t st) {
  hip_check(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
}

void response_vjp(heom_model* m, const heom_state* rho_eq, const heom_grid& gr, const double* W, bool stationary,
                  double tol, int max_steps, heom_op_grad* out) {
  GradCtx g;
  grad_init(g, m);
  hipStream_t st = m->stream;
  const int d = m->hm.d, n_ado = m->hm.n_ado;
  const int n1 = gr.n1, n3 = gr.n3, sps = gr.steps_per_sample, nq = gr.n_t2;
  const long long te = g.te;
  const double* rho = rho_eq->buf.as<double>();
  auto Wc = [&](int q, int P, int j, int k, int part) {
    return W[2 * (((static_cast<long long>(q) * 2 + P) * n1 + j) * n3 + k) + part];
  };
  // 1. detection functional l(k sps) and Psi_k = (mu+^x)^T l(k sps)
  DevBuf Lk(static_cast<size_t>(n3) * te * sizeof(double)), Psi(static_cast<size_t>(n3) * te * sizeof(double));
  {
    std::vector<double> h(static_cast<size_t>(te), 0.0);
    for (int a = 0; a < d; ++a)
      for (int c = 0; c < d; ++c) h[static_cast<size_t>(a) * d + c] = m->mu_dev[static_cast<size_t>(c) * d + a];
    hip_check(hipMemcpyAsync(Lk.p, h.data(), te * sizeof(double), hipMemcpyHostToDevice, st), "upload");
    hip_check(hipStreamSynchronize(st), "sync");
    for (int k = 1; k < n3; ++k) {
      copy_dev(Lk.as<double>() + k * te, Lk.as<double>() + (k - 1) * te, te, st);
      rk4_steps_ws<double>(m, Lk.as<double>() + k * te, 1, sps, true);
    }
    heom::launch_commutator<double>(m->mu64[HEOM_OP_MU_PLUS].as<double>(), 1, Lk.as<double>(), Psi.as<double>(), d,
                                    static_cast<long long>(n3) * n_ado, st);
  }
  DevBuf phi(static_cast<size_t>(n3) * te * sizeof(double));
  zero_dev(phi, st);
  DevBuf grho(static_cast<size_t>(te) * sizeof(double));
  zero_dev(grho, st);
  DevBuf Xc(static_cast<size_t>(n1) * te * sizeof(double)), bsrc(static_cast<size_t>(n1) * te * sizeof(double));
  DevBuf tmp1(static_cast<size_t>(te) * sizeof(double));
  const int T_max = gr.t2_steps[nq - 1];
  const int CSEG = 16;
  // boundaries of the t2 sweep: every t2 sample and every CSEG steps
  std::vector<int> bnd = {0};
  for (int t = CSEG; t < T_max; t += CSEG) bnd.push_back(t);
  for (int q = 0; q < nq; ++q) bnd.push_back(gr.t2_steps[q]);
  std::sort(bnd.begin(), bnd.end());
  bnd.erase(std::unique(bnd.begin(), bnd.end()), bnd.end());
  const int nbd = static_cast<int>(bnd.size());
  // trajectories per chunk from free memory: chunk state, checkpoints, sweep buffers, rk4 scratch
  const long long per_traj = (nbd + 1 + 4 * CSEG + 8 + 2 + 1) * te * static_cast<long long>(sizeof(double));
  const size_t fr = free_device_bytes();
  const size_t budget = fr > (size_t(2) << 30) ? fr - (size_t(2) << 30) : 0;
  const int nc = static_cast<int>(std::max<long long>(1, std::min<long long>(n1, budget / per_traj)));
  // adjoint RK4 steps of all sweeps: t2 per chunk and pathway, the t1 scans, the detection scan
  Progress prog(m, "gradient sweep",
                2LL * ((n1 + nc - 1) / nc) * T_max + 2LL * (n1 - 1) * sps + static_cast<long long>(n3 - 1) * sps);
  g.pr = &prog;
  const int pw_d[2][2] = {{HEOM_OP_MU_MINUS, HEOM_OP_MU_PLUS}, {HEOM_OP_MU_PLUS, HEOM_OP_MU_MINUS}};
  for (int P = 0; P < 2; ++P) {
    const int D1 = pw_d[P][0], D2 = pw_d[P][1];
    // t1 scan with checkpoints at every sample
    heom::launch_commutator<double>(m->mu64[D1].as<double>(), 0, rho, Xc.as<double>(), d, n_ado, st);
    for (int j = 1; j < n1; ++j) {
      copy_dev(Xc.as<double>() + j * te, Xc.as<double>() + (j - 1) * te, te, st);
      rk4_steps_ws<double>(m, Xc.as<double>() + j * te, 1, sps, false);
    }
    DevBuf Y(static_cast<size_t>(nc) * te * sizeof(double)), A(static_cast<size_t>(nc) * te * sizeof(double));
    DevBuf CK(static_cast<size_t>(std::max(nbd - 1, 1)) * nc * te * sizeof(double));
    for (int j0 = 0; j0 < n1; j0 += nc) {
      const int c = std::min(nc, n1 - j0);
      const long long N = static_cast<long long>(c) * te;
      heom::launch_commutator<double>(m->mu64[D2].as<double>(), 0, Xc.as<double>() + j0 * te, Y.as<double>(), d,
                                      static_cast<long long>(c) * n_ado, st);
      // forward over t2 with checkpoints; detection cotangent phi_k += sum_j (-i W) Y_j(T_q)
      for (int i = 0; i < nbd; ++i) {
        if (i + 1 < nbd) copy_dev(CK.as<double>() + i * N, Y.as<double>(), N, st);
        for (int q = 0; q < nq; ++q) {
          if (gr.t2_steps[q] != bnd[i]) continue;
          std::vector<double> cf(static_cast<size_t>(n3) * c * 2);
          for (int k = 0; k < n3; ++k)
            for (int jj = 0; jj < c; ++jj) {  // -i W
              cf[2 * (k * c + jj)] = Wc(q, P, j0 + jj, k, 1);
              cf[2 * (k * c + jj) + 1] = -Wc(q, P, j0 + jj, k, 0);
            }
          DevBuf cfd = upload_coef(cf, st);
          combine(g, Y.as<double>(), te, c, phi.as<double>(), te, n3, cfd.as<double>(), 1, 1);
          hip_check(hipStreamSynchronize(st), "sync");
        }
        if (i + 1 < nbd) rk4_steps_ws<double>(m, Y.as<double>(), c, bnd[i + 1] - bnd[i], false);
      }
      // backward over t2: sources sigma_q = sum_k (-i W) Psi_k at t2_q
      zero_dev(A, st);
      for (int i = nbd - 1; i >= 0; --i) {
        for (int q = 0; q < nq; ++q) {
          if (gr.t2_steps[q] != bnd[i]) continue;
          std::vector<double> cf(static_cast<size_t>(c) * n3 * 2);
          for (int jj = 0; jj < c; ++jj)
            for (int k = 0; k < n3; ++k) {
              cf[2 * (jj * n3 + k)] = Wc(q, P, j0 + jj, k, 1);
              cf[2 * (jj * n3 + k) + 1] = -Wc(q, P, j0 + jj, k, 0);
            }
          DevBuf cfd = upload_coef(cf, st);
          combine(g, Psi.as<double>(), te, n3, A.as<double>(), te, c, cfd.as<double>(), 1, 1);
          hip_check(hipStreamSynchronize(st), "sync");
        }
        if (i > 0) sweep(g, CK.as<double>() + (i - 1) * N, A.as<double>(), c, bnd[i] - bnd[i - 1], false);
      }
      // A = cotangent of the snapshots D2^x X(t1_j)
      k_dipole(g, D2, A.as<double>(), Xc.as<double>() + j0 * te, c);
      heom::launch_commutator<double>(m->mu64[D2].as<double>(), 1, A.as<double>(), bsrc.as<double>() + j0 * te, d,
                                      static_cast<long long>(c) * n_ado, st);
    }
    // t1 backward
    DevBuf b(static_cast<size_t>(te) * sizeof(double));
    copy_dev(b.as<double>(), bsrc.as<double>() + (n1 - 1) * te, te, st);
    std::vector<double> one = {1.0, 0.0};
    DevBuf oned = upload_coef(one, st);
    for (int j = n1 - 1; j >= 1; --j) {
      sweep(g, Xc.as<double>() + (j - 1) * te, b.as<double>(), 1, sps, false);
      combine(g, bsrc.as<double>() + (j - 1) * te, te, 1, b.as<double>(), te, 1, oned.as<double>(), 1, 1);
    }
    k_dipole(g, D1, b.as<double>(), rho, 1);
    heom::launch_commutator<double>(m->mu64[D1].as<double>(), 1, b.as<double>(), tmp1.as<double>(), d, n_ado, st);
    combine(g, tmp1.as<double>(), te, 1, grho.as<double>(), te, 1, oned.as<double>(), 1, 1);
    hip_check(hipStreamSynchronize(st), "sync");
  }
  // detection side: Psi_k = (mu+^x)^T l(k sps)
  {
    DevBuf csrc(static_cast<size_t>(n3) * te * sizeof(double));
    heom::launch_commutator<double>(m->mu64[HEOM_OP_MU_PLUS].as<double>(), 0, phi.as<double>(), csrc.as<double>(),
                                    d, static_cast<long long>(n3) * n_ado, st);
    k_dipole(g, HEOM_OP_MU_PLUS, Lk.as<double>(), phi.as<double>(), n3);
    DevBuf cc(static_cast<size_t>(te) * sizeof(double));
    copy_dev(cc.as<double>(), csrc.as<double>() + (n3 - 1) * te, te, st);
    std::vector<double> one = {1.0, 0.0};
    DevBuf oned = upload_coef(one, st);
    for (int k = n3 - 1; k >= 1; --k) {
      sweep(g, Lk.as<double>() + (k - 1) * te, cc.as<double>(), 1, sps, true);
      combine(g, csrc.as<double>() + (k - 1) * te, te, 1, cc.as<double>(), te, 1, oned.as<double>(), 1, 1);
    }
    // l_0 = mu^T on ADO 0: dJ/dmu[a][b] += Re c(0)[0][b][a]
    std::vector<double> c0(static_cast<size_t>(d) * d);
    hip_check(hipMemcpyAsync(c0.data(), cc.p, c0.size() * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    for (int a = 0; a < d; ++a)
      for (int bb = 0; bb < d; ++bb) out->dmu[a * d + bb] = c0[static_cast<size_t>(bb) * d + a];
  }
  // stationary state: <g_rho, d rho_eq> = <P(hL^T) kd, dL rho_eq>, kd = h sum_n (Phi^T)^n r
  out->stationary_steps = 0;
  out->stationary_residual = 0.0;
  if (stationary) {
    DevBuf work(heom::pair_work_doubles(1, 1, n_ado, d) * sizeof(double));
    DevBuf sdev(2 * sizeof(double));
    heom::launch_pairing<double>(grho.as<double>(), 1, rho, 1, n_ado, d, 1.0, 0.0, work.as<double>(),
                                 sdev.as<double>(), st);
    double sgr[2];
    hip_check(hipMemcpyAsync(sgr, sdev.p, sizeof(sgr), hipMemcpyDeviceToHost, st), "copy");
    std::vector<double> blk(static_cast<size_t>(2) * d * d);
    hip_check(hipMemcpyAsync(blk.data(), grho.p, blk.size() * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    for (int a = 0; a < d; ++a) {
      blk[static_cast<size_t>(a) * d + a] -= sgr[0];
      blk[static_cast<size_t>(d) * d + static_cast<size_t>(a) * d + a] -= sgr[1];
    }
    hip_check(hipMemcpyAsync(grho.p, blk.data(), blk.size() * sizeof(double), hipMemcpyHostToDevice, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    // kd solves (I - Phi^T) kd = h r; equivalently (I - (Phi^T)^M) kd = h sum_{n<M} (Phi^T)^n r
    const int M = 500;
    DevBuf kd(static_cast<size_t>(te) * sizeof(double)), bsum(static_cast<size_t>(te) * sizeof(double));
    {
      Krylov K(m, true, M);
      K.steps_total = static_cast<long long>(std::max(1, max_steps / M)) * M;
      K.zero(bsum.as<double>());
      for (int n = 0; n < M; ++n) {
        if (n) rk4_steps_ws<double>(m, grho.as<double>(), 1, 1, true);
        K.axpy(g.h, grho.as<double>(), bsum.as<double>());
      }
      K.zero(kd.as<double>());
      int applies = 0;
      const double rel = gmres(K, bsum.as<double>(), kd.as<double>(), 100, std::max(1, max_steps / M), tol, &applies);
      out->stationary_steps = M + applies * M;
      out->stationary_residual = rel;
      if (!(rel <= tol))
        throw HeomError(HEOM_ERR_NOCONV, "adjoint stationary solve did not converge within max_steps");
    }
    DevBuf t1(static_cast<size_t>(te) * sizeof(double)), t2(static_cast<size_t>(te) * sizeof(double));
    stage<double>(m, true, kd.as<double>(), kd.as<double>(), t1.as<double>(), g.h / 4.0, 1);
    stage<double>(m, true, t1.as<double>(), kd.as<double>(), t2.as<double>(), g.h / 3.0, 1);
    stage<double>(m, true, t2.as<double>(), kd.as<double>(), t1.as<double>(), g.h / 2.0, 1);
    k_generator(g, t1.as<double>(), rho, 1);
    hip_check(hipStreamSynchronize(st), "sync");
  }
  // reductions and the dipole chain mu -> (mu, mu+, mu-)
  const long long dd = static_cast<long long>(d) * d;
  DevBuf red(3 * dd * sizeof(double));
  zero_dev(red, st);
  heom::launch_reduce_parts(g.partH.as<double>(), heom::grad_max_parts(), dd, red.as<double>(), st);
  heom::launch_reduce_parts(g.partP.as<double>(), heom::grad_max_parts(), dd, red.as<double>() + dd, st);
  heom::launch_reduce_parts(g.partM.as<double>(), heom::grad_max_parts(), dd, red.as<double>() + 2 * dd, st);
  std::vector<double> hr(3 * dd);
  hip_check(hipMemcpyAsync(hr.data(), red.p, hr.size() * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
  size_t nv = g.gv.bytes / sizeof(double);
  hip_check(hipMemcpyAsync(out->dv, g.gv.p, nv * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
  hip_check(hipMemcpyAsync(out->dc, g.gc.p, g.gc.bytes, hipMemcpyDeviceToHost, st), "copy");
  hip_check(hipMemcpyAsync(out->dnu, g.gnu.p, g.gnu.bytes, hipMemcpyDeviceToHost, st), "copy");
  hip_check(hipStreamSynchronize(st), "sync");
  const auto& Nq = m->quanta_dev;
  for (long long i = 0; i < dd; ++i) out->dH[i] = hr[i];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      if (Nq[a] > Nq[b]) out->dmu[a * d + b] += hr[dd + a * d + b] + hr[2 * dd + static_cast<long long>(b) * d + a];
    }
  to_user_basis(m, out->dH);
  to_user_basis(m, out->dmu);
  auto finite = [](const double* x, size_t n) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(x[i])) return false;
    return true;
  };
  if (!finite(out->dH, dd) || !finite(out->dmu, dd) || !finite(out->dv, nv) ||
      !finite(out->dc, 2 * m->hm.n_terms) || !finite(out->dnu, m->hm.n_terms))
    throw HeomError(HEOM_ERR_UNSTABLE, "non-finite gradient");
}

// host model operators flattened in the heom_op_grad layout
struct OpVec {
  std::vector<double> H, v, mu, c, nu;
};

OpVec op_vec(const heom::HostModel& hm) {
  OpVec o;
  o.H = hm.H;
  for (int s = 0; s < hm.n_modes; ++s) o.v.insert(o.v.end(), hm.v[s].begin(), hm.v[s].end());
  o.mu = hm.mu;
  for (int j = 0; j < hm.n_terms; ++j) {
    o.c.push_back(hm.c[j].real());
    o.c.push_back(hm.c[j].imag());
  }
  o.nu = hm.nu;
  return o;
}

}  // namespace

// ============================================================== C ABI =====

// ------------------------------------------------ allocation-free calls --
// Scratch memory of heom_propagate_noalloc: a file-scope device array (each
// GPU the library runs on holds its own copy until the process ends).  In
// host code `scratch` is only a symbol: its device address is looked up once
// per device with hipGetSymbolAddress and that pointer is used everywhere.
namespace {

constexpr size_t kNoAllocBytes = static_cast<size_t>(64) << 20;  // 64 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (looked up on first use, with
// dev current; the caller's current device is restored).
unsigned char* device_scratch(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) throw HeomError(HEOM_ERR_PARAM, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    hip_check(hipGetDevice(&cur), "hipGetDevice");
    if (cur != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) hip_check(hipSetDevice(cur), "hipSetDevice");
    if (e != hipSuccess || !p)
      throw HeomError(HEOM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return static_cast<unsigned char*>(g_scratch_ptr[dev]);
}

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// heom_propagate with every work buffer carved from the device's scratch
// array: the two RK4 stage buffers, the traces and the absmax partials.
template <typename T>
void propagate_noalloc(heom_model* m, heom_state* s, int n_steps, bool adjoint, int sample_every, double* trace_out) {
  const long long elems = s->n_elems();
  const long long n_mats = static_cast<long long>(s->n_traj) * m->hm.n_ado;
  const bool sample = sample_every > 0 && trace_out;
  const int n_samples = sample ? n_steps / sample_every + 1 : 0;
  const size_t b_stage = align256(static_cast<size_t>(elems) * sizeof(T));
  const size_t b_part = align256(static_cast<size_t>(n_mats) * sizeof(double));
  const size_t b_res = 256;
  const size_t b_tr = align256(static_cast<size_t>(n_samples) * s->n_traj * 2 * sizeof(double));
  const size_t need = 2 * b_stage + b_part + b_res + b_tr;
  if (need > kNoAllocBytes)
    throw HeomError(HEOM_ERR_PARAM, "heom_propagate_noalloc needs " + std::to_string(need) +
                                        " bytes of scratch; the static buffer holds " +
                                        std::to_string(kNoAllocBytes) + " (use heom_propagate)");
  unsigned char* base = device_scratch(m->device);
  T* w1 = reinterpret_cast<T*>(base);
  T* w2 = reinterpret_cast<T*>(base + b_stage);
  double* part = reinterpret_cast<double*>(base + 2 * b_stage);
  double* res = reinterpret_cast<double*>(base + 2 * b_stage + b_part);
  double* tr = reinterpret_cast<double*>(base + 2 * b_stage + b_part + b_res);
  T* y = s->buf.as<T>();
  // direct launches only (no graph capture, no timing events: both would
  // create runtime objects)
  auto steps = [&](int k) {
    for (int i = 0; i < k; ++i) rk4_step_launches<T>(m, y, w1, w2, s->n_traj, adjoint);
  };
  if (!sample) {
    steps(n_steps);
  } else {
    for (int k = 0; k < n_samples; ++k) {
      if (k > 0) steps(sample_every);
      heom::launch_trace<T>(m->mu64[HEOM_OP_MU].as<double>(), y, m->hm.d, m->traj_elems(), s->n_traj,
                            tr + static_cast<size_t>(k) * s->n_traj * 2, 1, m->stream);
    }
    steps(n_steps - (n_samples - 1) * sample_every);
    hip_check(hipMemcpyAsync(trace_out, tr, static_cast<size_t>(n_samples) * s->n_traj * 2 * sizeof(double),
                             hipMemcpyDeviceToHost, m->stream),
              "copy");
  }
  double r = 0.0;
  if (n_mats > 0) {
    heom::launch_absmax<T>(y, m->hm.d, n_mats, part, res, m->stream);
    hip_check(hipMemcpyAsync(&r, res, sizeof(double), hipMemcpyDeviceToHost, m->stream), "copy");
  }
  hip_check(hipStreamSynchronize(m->stream), "sync");
  if (!std::isfinite(r))
    throw HeomError(HEOM_ERR_UNSTABLE, "non-finite hierarchy after propagation (time step beyond the RK4 stability region?)");
}

}  // namespace

extern "C" {

const char* heom_last_error(void) { return g_last_error.c_str(); }

int heom_set_allocator(heom_alloc_fn alloc, heom_free_fn release, void* ctx) {
  return guarded([&] {
    if ((alloc == nullptr) != (release == nullptr))
      throw HeomError(HEOM_ERR_PARAM, "alloc and free hooks must be given together");
    g_alloc = alloc;
    g_free = release;
    g_alloc_ctx = ctx;
  });
}

int heom_device_query(int* cu_count, int* lds_bytes, char* name_out, int name_len) {
  return guarded([&] {
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (cu_count) *cu_count = prop.multiProcessorCount;
    if (lds_bytes) *lds_bytes = static_cast<int>(prop.sharedMemPerBlock);
    if (name_out && name_len > 0) {
      std::snprintf(name_out, static_cast<size_t>(name_len), "%s (%s)", prop.name, prop.gcnArchName);
    }
  });
}

int heom_model_build_host(const heom_params* params, heom_model** out) {
  return guarded([&] {
    if (!out) throw HeomError(HEOM_ERR_PARAM, "null output pointer");
    *out = nullptr;
    heom_params p = copy_check(params);
    auto m = std::make_unique<heom_model>();
    m->hm = heom::build_host_model(p);
    *out = m.release();
  });
}

int heom_model_build(const heom_params* params, void* hip_stream, heom_model** out) {
  return guarded([&] {
    if (!out) throw HeomError(HEOM_ERR_PARAM, "null output pointer");
    *out = nullptr;
    heom_params p = copy_check(params);
    auto m = std::make_unique<heom_model>();
    m->hm = heom::build_host_model(p);
    hip_check(hipGetDevice(&m->device), "hipGetDevice");
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, m->device), "hipGetDeviceProperties");
    m->lds_limit = static_cast<int>(prop.sharedMemPerBlock);
    m->stream = static_cast<hipStream_t>(hip_stream);
    const long long need_lds = static_cast<long long>(m->hm.d) * m->hm.d * sizeof(double);
    if (need_lds > m->lds_limit)
      throw HeomError(HEOM_ERR_PARAM, "product dimension too large for the FP64 kernel's LDS staging");
    upload_model(m.get());
    *out = m.release();
  });
}

void heom_model_free(heom_model* model) {
  if (!model) return;
  if (model->has_device) (void)hipStreamSynchronize(model->stream);
  delete model;
}

int heom_model_info(const heom_model* m, heom_info* out) {
  return guarded([&] {
    if (!m || !out) throw HeomError(HEOM_ERR_PARAM, "null argument");
    out->d = m->hm.d;
    out->n_ado = m->hm.n_ado;
    out->n_terms = m->hm.n_terms;
    out->n_modes = m->hm.n_modes;
    for (int s = 0; s < 4; ++s) out->dims[s] = s < m->hm.n_modes ? m->hm.dims[s] : 1;
    out->depth = m->hm.depth;
    out->dt = m->hm.dt;
  });
}

int heom_model_operators(const heom_model* m, double* H, double* mu, double* mu_plus, double* mu_minus,
                         double* v, double* nu, double* c, int* ado_n, int* term_mode) {
  return guarded([&] {
    if (!m) throw HeomError(HEOM_ERR_PARAM, "null model");
    const auto& hm = m->hm;
    auto cp = [](double* dst, const std::vector<double>& src) {
      if (dst) std::memcpy(dst, src.data(), src.size() * sizeof(double));
    };
    cp(H, hm.H);
    cp(mu, hm.mu);
    cp(mu_plus, hm.mu_plus);
    cp(mu_minus, hm.mu_minus);
    if (v) {
      size_t off = 0;
      for (const auto& vs : hm.v) {
        std::memcpy(v + off, vs.data(), vs.size() * sizeof(double));
        off += vs.size();
      }
    }
    cp(nu, hm.nu);
    if (c)
      for (int j = 0; j < hm.n_terms; ++j) {
        c[2 * j] = hm.c[j].real();
        c[2 * j + 1] = hm.c[j].imag();
      }
    if (ado_n) std::memcpy(ado_n, hm.ado_n.data(), hm.ado_n.size() * sizeof(int));
    if (term_mode) std::memcpy(term_mode, hm.term_mode.data(), hm.term_mode.size() * sizeof(int));
  });
}

int heom_model_bath(const heom_model* m, double* nu, double* c, double* c_bra) {
  return guarded([&] {
    if (!m) throw HeomError(HEOM_ERR_PARAM, "null model");
    const auto& hm = m->hm;
    for (int j = 0; j < hm.n_terms; ++j) {
      if (nu) {
        nu[2 * j] = hm.nu[j];
        nu[2 * j + 1] = hm.nu_im[j];
      }
      if (c) {
        c[2 * j] = hm.c[j].real();
        c[2 * j + 1] = hm.c[j].imag();
      }
      if (c_bra) {
        c_bra[2 * j] = hm.cb[j].real();
        c_bra[2 * j + 1] = hm.cb[j].imag();
      }
    }
  });
}

int heom_state_create(heom_model* m, int n_traj, int precision, heom_state** out) {
  return guarded([&] {
    require_device(m);
    if (!out) throw HeomError(HEOM_ERR_PARAM, "null output pointer");
    *out = nullptr;
    if (n_traj < 1) throw HeomError(HEOM_ERR_PARAM, "n_traj must be >= 1");
    if (precision != HEOM_FP64 && precision != HEOM_FP32) throw HeomError(HEOM_ERR_PARAM, "bad precision");
    auto s = new_state(m, n_traj, precision);
    hip_check(hipStreamSynchronize(m->stream), "sync");
    *out = s.release();
  });
}

void heom_state_free(heom_state* s) {
  if (!s) return;
  if (s->model && s->model->has_device) (void)hipStreamSynchronize(s->model->stream);
  delete s;
}

int heom_state_shape(const heom_state* s, int* n_traj, int* precision) {
  return guarded([&] {
    if (!s) throw HeomError(HEOM_ERR_PARAM, "null state");
    if (n_traj) *n_traj = s->n_traj;
    if (precision) *precision = s->precision;
  });
}

namespace {
// element e = a d + b of a matrix in the device basis -> its index in the
// caller's basis
std::vector<long long> basis_map(const heom_model* m) {
  const int d = m->hm.d;
  std::vector<long long> e(static_cast<size_t>(d) * d);
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      e[static_cast<size_t>(a) * d + b] =
          m->perm.empty() ? static_cast<long long>(a) * d + b : static_cast<long long>(m->perm[a]) * d + m->perm[b];
  return e;
}
}  // namespace

int heom_state_upload_range(heom_state* s, int first, int count, const double* host) {
  return guarded([&] {
    if (!s || !host) throw HeomError(HEOM_ERR_PARAM, "null argument");
    if (first < 0 || count < 0 || first + count > s->n_traj) throw HeomError(HEOM_ERR_PARAM, "bad trajectory range");
    heom_model* m = s->model;
    const int d = m->hm.d;
    const long long dd = static_cast<long long>(d) * d;
    const long long n_mats = static_cast<long long>(count) * m->hm.n_ado;
    const long long off = static_cast<long long>(first) * m->traj_elems();
    auto go = [&](auto* tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      std::vector<T> t(static_cast<size_t>(n_mats * 2 * dd));
      const std::vector<long long> src = basis_map(m);
      for (long long q = 0; q < n_mats; ++q)
        for (long long e = 0; e < dd; ++e) {
          const long long u = q * dd + src[e];
          t[q * 2 * dd + e] = static_cast<T>(host[2 * u]);
          t[q * 2 * dd + dd + e] = static_cast<T>(host[2 * u + 1]);
        }
      hip_check(hipMemcpyAsync(s->buf.as<T>() + off, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice,
                               m->stream), "upload");
      hip_check(hipStreamSynchronize(m->stream), "sync");
    };
    if (s->precision == HEOM_FP64) go(static_cast<double*>(nullptr));
    else go(static_cast<float*>(nullptr));
  });
}

int heom_state_download_range(const heom_state* s, int first, int count, double* host) {
  return guarded([&] {
    if (!s || !host) throw HeomError(HEOM_ERR_PARAM, "null argument");
    if (first < 0 || count < 0 || first + count > s->n_traj) throw HeomError(HEOM_ERR_PARAM, "bad trajectory range");
    heom_model* m = s->model;
    const int d = m->hm.d;
    const long long dd = static_cast<long long>(d) * d;
    const long long n_mats = static_cast<long long>(count) * m->hm.n_ado;
    const long long off = static_cast<long long>(first) * m->traj_elems();
    auto go = [&](auto* tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      std::vector<T> t(static_cast<size_t>(n_mats * 2 * dd));
      hip_check(hipMemcpyAsync(t.data(), s->buf.as<T>() + off, t.size() * sizeof(T), hipMemcpyDeviceToHost,
                               m->stream), "download");
      hip_check(hipStreamSynchronize(m->stream), "sync");
      const std::vector<long long> src = basis_map(m);
      for (long long q = 0; q < n_mats; ++q)
        for (long long e = 0; e < dd; ++e) {
          const long long u = q * dd + src[e];
          host[2 * u] = static_cast<double>(t[q * 2 * dd + e]);
          host[2 * u + 1] = static_cast<double>(t[q * 2 * dd + dd + e]);
        }
    };
    if (s->precision == HEOM_FP64) go(static_cast<double*>(nullptr));
    else go(static_cast<float*>(nullptr));
  });
}

int heom_state_upload(heom_state* s, const double* host) {
  if (!s) {
    g_last_error = "null state";
    return HEOM_ERR_PARAM;
  }
  return heom_state_upload_range(s, 0, s->n_traj, host);
}

int heom_state_download(const heom_state* s, double* host) {
  if (!s) {
    g_last_error = "null state";
    return HEOM_ERR_PARAM;
  }
  return heom_state_download_range(s, 0, s->n_traj, host);
}

int heom_state_set_ground(heom_state* s) {
  return guarded([&] {
    if (!s) throw HeomError(HEOM_ERR_PARAM, "null state");
    heom_model* m = s->model;
    if (s->precision == HEOM_FP64)
      heom::launch_set_ground<double>(s->buf.as<double>(), m->traj_elems(), s->n_traj, s->n_elems(), m->stream);
    else
      heom::launch_set_ground<float>(s->buf.as<float>(), m->traj_elems(), s->n_traj, s->n_elems(), m->stream);
    hip_check(hipStreamSynchronize(m->stream), "sync");
  });
}

int heom_state_copy(heom_state* dst, const heom_state* src) {
  return guarded([&] {
    if (!dst || !src) throw HeomError(HEOM_ERR_PARAM, "null state");
    if (dst->model != src->model) throw HeomError(HEOM_ERR_STATE, "states of different models");
    if (dst->n_traj != src->n_traj) throw HeomError(HEOM_ERR_STATE, "trajectory counts differ");
    heom_model* m = dst->model;
    const long long n = src->n_elems();
    if (src->precision == HEOM_FP64 && dst->precision == HEOM_FP64)
      heom::launch_convert<double, double>(src->buf.as<double>(), dst->buf.as<double>(), n, m->stream);
    else if (src->precision == HEOM_FP64)
      heom::launch_convert<double, float>(src->buf.as<double>(), dst->buf.as<float>(), n, m->stream);
    else if (dst->precision == HEOM_FP64)
      heom::launch_convert<float, double>(src->buf.as<float>(), dst->buf.as<double>(), n, m->stream);
    else
      heom::launch_convert<float, float>(src->buf.as<float>(), dst->buf.as<float>(), n, m->stream);
    hip_check(hipStreamSynchronize(m->stream), "sync");
  });
}

int heom_rhs(heom_model* m, const heom_state* in, heom_state* out, int adjoint) {
  return guarded([&] {
    require_device(m);
    require_state(m, in);
    require_state(m, out);
    if (in == out) throw HeomError(HEOM_ERR_PARAM, "in and out must differ");
    if (in->n_traj != out->n_traj || in->precision != out->precision)
      throw HeomError(HEOM_ERR_STATE, "in/out shapes differ");
    if (in->precision == HEOM_FP64)
      launch_stage<double>(m, adjoint != 0, in->buf.as<double>(), nullptr, out->buf.as<double>(), 1.0, in->n_traj);
    else
      launch_stage<float>(m, adjoint != 0, in->buf.as<float>(), nullptr, out->buf.as<float>(), 1.0, in->n_traj);
    hip_check(hipStreamSynchronize(m->stream), "sync");
  });
}

int heom_propagate(heom_model* m, heom_state* s, int n_steps, int adjoint, int sample_every, double* trace_out) {
  return guarded([&] {
    require_device(m);
    require_state(m, s);
    if (n_steps < 0) throw HeomError(HEOM_ERR_PARAM, "n_steps must be >= 0");
    if (s->precision == HEOM_FP64)
      propagate_sampled<double>(m, s, n_steps, adjoint != 0, sample_every, trace_out);
    else
      propagate_sampled<float>(m, s, n_steps, adjoint != 0, sample_every, trace_out);
  });
}

int heom_propagate_noalloc(heom_model* m, heom_state* s, int n_steps, int adjoint, int sample_every,
                           double* trace_out) {
  return guarded([&] {
    require_device(m);
    require_state(m, s);
    if (n_steps < 0) throw HeomError(HEOM_ERR_PARAM, "n_steps must be >= 0");
    if (s->precision == HEOM_FP64)
      propagate_noalloc<double>(m, s, n_steps, adjoint != 0, sample_every, trace_out);
    else
      propagate_noalloc<float>(m, s, n_steps, adjoint != 0, sample_every, trace_out);
  });
}

int heom_apply_dipole(heom_model* m, heom_state* s, int op, int transpose) {
  return guarded([&] {
    require_device(m);
    require_state(m, s);
    if (op < 0 || op > 2) throw HeomError(HEOM_ERR_PARAM, "bad operator");
    const long long n_mats = static_cast<long long>(s->n_traj) * m->hm.n_ado;
    const long long n = s->n_elems();
    if (s->precision == HEOM_FP64) {
      double* w = work_buffer<double>(m, 0, n);
      heom::launch_commutator<double>(m->mu64[op].as<double>(), transpose, s->buf.as<double>(), w, m->hm.d,
                                      n_mats, m->stream);
      heom::launch_convert<double, double>(w, s->buf.as<double>(), n, m->stream);
    } else {
      float* w = work_buffer<float>(m, 0, n);
      heom::launch_commutator<float>(m->mu64[op].as<double>(), transpose, s->buf.as<float>(), w, m->hm.d, n_mats,
                                     m->stream);
      heom::launch_convert<float, float>(w, s->buf.as<float>(), n, m->stream);
    }
    hip_check(hipStreamSynchronize(m->stream), "sync");
  });
}

int heom_trace(heom_model* m, const heom_state* s, int op, double* out) {
  return guarded([&] {
    require_device(m);
    require_state(m, s);
    if (op < 0 || op > 2 || !out) throw HeomError(HEOM_ERR_PARAM, "bad argument");
    DevBuf o(static_cast<size_t>(s->n_traj) * 2 * sizeof(double));
    if (s->precision == HEOM_FP64)
      heom::launch_trace<double>(m->mu64[op].as<double>(), s->buf.as<double>(), m->hm.d, m->traj_elems(),
                                 s->n_traj, o.as<double>(), 1, m->stream);
    else
      heom::launch_trace<float>(m->mu64[op].as<double>(), s->buf.as<float>(), m->hm.d, m->traj_elems(), s->n_traj,
                                o.as<double>(), 1, m->stream);
    hip_check(hipMemcpyAsync(out, o.p, o.bytes, hipMemcpyDeviceToHost, m->stream), "copy");
    hip_check(hipStreamSynchronize(m->stream), "sync");
  });
}

int heom_residual(heom_model* m, const heom_state* s, double* out) {
  return guarded([&] {
    require_device(m);
    require_state(m, s);
    if (!out) throw HeomError(HEOM_ERR_PARAM, "null output");
    *out = s->precision == HEOM_FP64 ? residual_of<double>(m, s->buf.as<double>(), s->n_traj)
                                     : residual_of<float>(m, s->buf.as<float>(), s->n_traj);
  });
}

int heom_equilibrate(heom_model* m, double tol, int check_every, int min_steps, int max_steps,
                     int require_convergence, heom_state** rho_eq_out, int* steps_out, double* residual_out) {
  int conv_fail = 0;
  int rc = guarded([&] {
    require_device(m);
    if (!rho_eq_out) throw HeomError(HEOM_ERR_PARAM, "null output pointer");
    *rho_eq_out = nullptr;
    if (check_every < 1 || max_steps < 0 || min_steps < 0) throw HeomError(HEOM_ERR_PARAM, "bad step counts");
    auto s = new_state(m, 1, HEOM_FP64);
    heom::launch_set_ground<double>(s->buf.as<double>(), m->traj_elems(), 1, s->n_elems(), m->stream);
    double* y = s->buf.as<double>();
    const long long te = m->traj_elems();
    DevBuf w1(static_cast<size_t>(te) * sizeof(double)), w2(static_cast<size_t>(te) * sizeof(double));
    int steps = 0;
    double res = -1.0;
    while (steps < max_steps) {
      const int k = std::min(check_every, max_steps - steps);
      rk4_steps<double>(m, y, w1.as<double>(), w2.as<double>(), 1, k, false);
      steps += k;
      res = -1.0;
      if (steps >= min_steps) {
        res = residual_of<double>(m, y, 1);
        if (!std::isfinite(res)) throw HeomError(HEOM_ERR_UNSTABLE, "non-finite hierarchy during equilibration");
        if (res <= tol) break;
      }
    }
    if (res < 0.0) res = residual_of<double>(m, y, 1);
    if (steps_out) *steps_out = steps;
    if (residual_out) *residual_out = res;
    if (require_convergence && res > tol) conv_fail = 1;
    *rho_eq_out = s.release();
  });
  if (rc == HEOM_OK && conv_fail) {
    g_last_error = "equilibration residual above tolerance at max_steps";
    return HEOM_ERR_NOCONV;
  }
  return rc;
}

namespace {

// GMRES corrections of rho (one FP64 trajectory, unit trace) until
// max|L rho| <= tol or max_applies operator applications.
void krylov_refine(heom_model* m, double* rho, double tol, int steps_per_apply, int restart, int max_applies,
                   int* used_out, double* res_out) {
  const long long te = m->traj_elems();
  Krylov K(m, false, steps_per_apply);
  K.steps_total = static_cast<long long>(max_applies) * steps_per_apply;
  DevBuf b(static_cast<size_t>(te) * sizeof(double)), x(static_cast<size_t>(te) * sizeof(double));
  int used = 0;
  double res = residual_of<double>(m, rho, 1);
  if (!std::isfinite(res)) throw HeomError(HEOM_ERR_UNSTABLE, "non-finite hierarchy during equilibration");
  while (res > tol && used < max_applies) {
    // rho + x with (I - Phi^m) x = -(I - Phi^m) rho
    K.apply(rho, x.as<double>());
    ++used;
    K.zero(b.as<double>());
    K.axpy(-1.0, x.as<double>(), b.as<double>());
    K.zero(x.as<double>());
    int applies = 0;
    const double rtol = std::min(1e-2, 0.1 * tol / res);
    gmres(K, b.as<double>(), x.as<double>(), restart, std::max(1, max_applies - used), rtol, &applies);
    used += applies;
    K.axpy(1.0, x.as<double>(), rho);
    res = residual_of<double>(m, rho, 1);
    if (!std::isfinite(res)) throw HeomError(HEOM_ERR_UNSTABLE, "non-finite hierarchy during equilibration");
  }
  *used_out = used;
  *res_out = res;
}

}  // namespace

int heom_equilibrate_krylov(heom_model* m, double tol, int pre_steps, int steps_per_apply, int restart,
                            int max_applies, heom_state** rho_eq_out, int* applies_out, double* residual_out) {
  int conv_fail = 0;
  int rc = guarded([&] {
    require_device(m);
    if (!rho_eq_out) throw HeomError(HEOM_ERR_PARAM, "null output pointer");
    *rho_eq_out = nullptr;
    if (pre_steps < 0 || steps_per_apply < 1 || restart < 1 || max_applies < 1 || !(tol > 0.0))
      throw HeomError(HEOM_ERR_PARAM, "bad Krylov parameters");
    auto s = new_state(m, 1, HEOM_FP64);
    heom::launch_set_ground<double>(s->buf.as<double>(), m->traj_elems(), 1, s->n_elems(), m->stream);
    rk4_steps_ws<double>(m, s->buf.as<double>(), 1, pre_steps, false);
    int used = 0;
    double res = 0.0;
    krylov_refine(m, s->buf.as<double>(), tol, steps_per_apply, restart, max_applies, &used, &res);
    if (applies_out) *applies_out = used;
    if (residual_out) *residual_out = res;
    if (res > tol) conv_fail = 1;
    *rho_eq_out = s.release();
  });
  if (rc == HEOM_OK && conv_fail) {
    g_last_error = "Krylov equilibration residual above tolerance at max_applies";
    return HEOM_ERR_NOCONV;
  }
  return rc;
}

int heom_stationary_refine(heom_model* m, heom_state* rho, double tol, int steps_per_apply, int restart,
                           int max_applies, int* applies_out, double* residual_out) {
  int conv_fail = 0;
  int rc = guarded([&] {
    require_device(m);
    require_state(m, rho);
    if (rho->precision != HEOM_FP64 || rho->n_traj != 1)
      throw HeomError(HEOM_ERR_STATE, "rho must be an FP64 state with one trajectory");
    if (steps_per_apply < 1 || restart < 1 || max_applies < 1 || !(tol > 0.0))
      throw HeomError(HEOM_ERR_PARAM, "bad Krylov parameters");
    int used = 0;
    double res = 0.0;
    krylov_refine(m, rho->buf.as<double>(), tol, steps_per_apply, restart, max_applies, &used, &res);
    if (applies_out) *applies_out = used;
    if (residual_out) *residual_out = res;
    if (res > tol) conv_fail = 1;
  });
  if (rc == HEOM_OK && conv_fail) {
    g_last_error = "stationary residual above tolerance at max_applies";
    return HEOM_ERR_NOCONV;
  }
  return rc;
}

int heom_linear_response(heom_model* m, const heom_state* rho_eq, int n, int sps, int precision, double* R_out) {
  return guarded([&] {
    require_device(m);
    require_state(m, rho_eq);
    if (rho_eq->precision != HEOM_FP64 || rho_eq->n_traj != 1)
      throw HeomError(HEOM_ERR_STATE, "rho_eq must be an FP64 state with one trajectory");
    if (n < 1 || sps < 1 || !R_out) throw HeomError(HEOM_ERR_PARAM, "bad grid");
    if (precision == HEOM_FP64) linear_response_impl<double>(m, rho_eq, n, sps, R_out);
    else if (precision == HEOM_FP32) linear_response_impl<float>(m, rho_eq, n, sps, R_out);
    else throw HeomError(HEOM_ERR_PARAM, "bad precision");
  });
}

int heom_response_2d(heom_model* m, const heom_state* rho_eq, const heom_grid* grid, int precision, int method,
                     int max_batch, double* R_out) {
  return guarded([&] { response_any(m, rho_eq, grid, precision, method, max_batch, 2, kStdPathways, R_out); });
}

int heom_response_2d_pathways(heom_model* m, const heom_state* rho_eq, const heom_grid* grid, int precision,
                              int method, int max_batch, int n_pathways, const int* ops, double* R_out) {
  return guarded([&] { response_any(m, rho_eq, grid, precision, method, max_batch, n_pathways, ops, R_out); });
}

int heom_spectrum_2d(const double* R_I, const double* R_II, int n1, int n3, double dt_s, double* S_out) {
  return guarded([&] {
    if (!R_I || !R_II || !S_out || n1 < 1 || n3 < 1 || !(dt_s > 0.0))
      throw HeomError(HEOM_ERR_PARAM, "bad argument");
    const size_t nr = static_cast<size_t>(n1) * n3 * 2;
    DevBuf dI(nr * sizeof(double)), dII(nr * sizeof(double));
    DevBuf work(static_cast<size_t>(4) * n3 * n1 * 2 * sizeof(double));
    DevBuf S(static_cast<size_t>(4) * n3 * n1 * sizeof(double));
    hip_check(hipMemcpy(dI.p, R_I, nr * sizeof(double), hipMemcpyHostToDevice), "upload");
    hip_check(hipMemcpy(dII.p, R_II, nr * sizeof(double), hipMemcpyHostToDevice), "upload");
    heom::launch_spectrum(dI.as<double>(), dII.as<double>(), n1, n3, dt_s, work.as<double>(), S.as<double>(),
                          nullptr);
    hip_check(hipMemcpy(S_out, S.p, S.bytes, hipMemcpyDeviceToHost), "download");
  });
}

int heom_response_2d_vjp(heom_model* m, const heom_state* rho_eq, const heom_grid* grid, const double* W,
                         int rho_is_stationary, double tol, int max_steps, heom_op_grad* out) {
  return guarded([&] {
    require_device(m);
    require_state(m, rho_eq);
    if (!grid || !W || !out || !out->dH || !out->dv || !out->dmu || !out->dc || !out->dnu)
      throw HeomError(HEOM_ERR_PARAM, "null argument");
    if (rho_eq->precision != HEOM_FP64 || rho_eq->n_traj != 1)
      throw HeomError(HEOM_ERR_STATE, "rho_eq must be an FP64 state with one trajectory");
    const heom_grid& g = *grid;
    if (g.n1 < 1 || g.n3 < 1 || g.steps_per_sample < 1 || g.n_t2 < 1 || !g.t2_steps)
      throw HeomError(HEOM_ERR_PARAM, "bad grid");
    for (int i = 0; i < g.n_t2; ++i)
      if (g.t2_steps[i] < 0 || (i && g.t2_steps[i] < g.t2_steps[i - 1]))
        throw HeomError(HEOM_ERR_PARAM, "t2_steps must be non-negative and non-decreasing");
    if (max_steps < 0 || !(tol >= 0.0)) throw HeomError(HEOM_ERR_PARAM, "bad tol / max_steps");
    int kmax = 0;
    for (int s = 0; s < m->hm.n_modes; ++s) {
      int k = 0;
      for (int j = 0; j < m->hm.n_terms; ++j) k += m->hm.term_mode[j] == s;
      kmax = std::max(kmax, k);
    }
    if (!heom::grad_supported(m->hm.d, m->hm.dims, m->hm.n_modes, kmax))
      throw HeomError(HEOM_ERR_PARAM, "gradient needs d <= 80, mode dimensions d_s <= 8 with d_s * d <= 512, and <= 4 terms per mode");
    for (int j = 0; j < m->hm.n_terms; ++j)
      if (m->hm.nu_im[j] != 0.0 || m->hm.cb[j] != std::conj(m->hm.c[j]))
        throw HeomError(HEOM_ERR_PARAM, "gradient supports Drude baths only (real rates, bra coefficients conj(c))");
    response_vjp(m, rho_eq, g, W, rho_is_stationary != 0, tol, max_steps, out);
  });
}

int heom_spectrum_1d(const double* R1, int n, double dt_s, double* I_out) {
  return guarded([&] {
    if (!R1 || !I_out || n < 1 || !(dt_s > 0)) throw HeomError(HEOM_ERR_PARAM, "bad arguments");
    // I(W_m) = sum_k w_k dt_s exp(i W_m t_k) R1(t_k), W_m = 2 pi m / (2 n dt_s), m = -n..n-1
    const double two_pi = 6.283185307179586476925287;
    for (int mi = 0; mi < 2 * n; ++mi) {
      const double W = two_pi * (mi - n) / (2.0 * n * dt_s);
      std::complex<double> acc = 0.0;
      for (int k = 0; k < n; ++k) {
        const double ph = W * dt_s * k;
        const std::complex<double> r(R1[2 * k], R1[2 * k + 1]);
        acc += (k == 0 ? 0.5 : 1.0) * std::complex<double>(std::cos(ph), std::sin(ph)) * r;
      }
      acc *= dt_s;
      I_out[2 * mi] = acc.real();
      I_out[2 * mi + 1] = acc.imag();
    }
  });
}

int heom_spectrum_2d_vjp(const double* G, int n1, int n3, double dt_s, double* W_out) {
  return guarded([&] {
    if (!G || !W_out || n1 < 1 || n3 < 1 || !(dt_s > 0)) throw HeomError(HEOM_ERR_PARAM, "bad arguments");
    // S_P = Im(dt^2 E3 R^T E1^T), E(W,t) = w_t exp(iWt); S_C = -(S_I(W3,-W1) + S_II(W3,W1));
    // Im z = Re(-i z)  =>  W_P[j][k] = i dt^2 sum G[m3][m1] E3[m3][k] E1_P[m1][j]
    const double two_pi = 6.283185307179586476925287;
    auto wgt = [](int k) { return k == 0 ? 0.5 : 1.0; };
    for (int P = 0; P < 2; ++P) {
      const double sgn1 = P == 0 ? -1.0 : 1.0;
      // T[m3][j] = sum_m1 G[m3][m1] E1_P[m1][j]
      std::vector<std::complex<double>> T(static_cast<size_t>(2 * n3) * n1);
      for (int m3 = 0; m3 < 2 * n3; ++m3)
        for (int j = 0; j < n1; ++j) {
          std::complex<double> acc = 0.0;
          for (int m1 = 0; m1 < 2 * n1; ++m1) {
            const double w1 = sgn1 * two_pi * (m1 - n1) / (2.0 * n1 * dt_s);
            const double ph = w1 * dt_s * j;
            acc += G[static_cast<size_t>(m3) * 2 * n1 + m1] * std::complex<double>(std::cos(ph), std::sin(ph));
          }
          T[static_cast<size_t>(m3) * n1 + j] = acc * wgt(j);
        }
      for (int j = 0; j < n1; ++j)
        for (int k = 0; k < n3; ++k) {
          std::complex<double> acc = 0.0;
          for (int m3 = 0; m3 < 2 * n3; ++m3) {
            const double w3 = two_pi * (m3 - n3) / (2.0 * n3 * dt_s);
            const double ph = w3 * dt_s * k;
            acc += T[static_cast<size_t>(m3) * n1 + j] * std::complex<double>(std::cos(ph), std::sin(ph));
          }
          const std::complex<double> w = std::complex<double>(0.0, 1.0) * dt_s * dt_s * wgt(k) * acc;
          const size_t o = 2 * ((static_cast<size_t>(P) * n1 + j) * n3 + k);
          W_out[o] = w.real();
          W_out[o + 1] = w.imag();
        }
    }
  });
}

int heom_params_vjp(const heom_params* params, const heom_params* dirs, int n_dirs, double step,
                    const heom_op_grad* g, double* out) {
  return guarded([&] {
    if (!params || !dirs || n_dirs < 0 || !g || !out || !(step > 0))
      throw HeomError(HEOM_ERR_PARAM, "bad arguments");
    const heom_params base = copy_check(params);
    for (int s = 0; s < base.n_modes; ++s)
      if (base.modes && base.modes[s].omega_b != 0.0)
        throw HeomError(HEOM_ERR_PARAM, "parameter gradient supports Drude baths only");
    for (int i = 0; i < n_dirs; ++i) {
      const heom_params& dp = dirs[i];
      if (dp.n_modes != base.n_modes || dp.n_couplings != base.n_couplings)
        throw HeomError(HEOM_ERR_PARAM, "direction layout differs from params");
      auto shifted = [&](double e) {
        std::vector<heom_mode> modes(base.modes, base.modes + base.n_modes);
        std::vector<heom_coupling> cps(base.couplings, base.couplings + base.n_couplings);
        for (int s = 0; s < base.n_modes; ++s) {
          const heom_mode& dm = dp.modes[s];
          heom_mode& mm = modes[s];
          mm.omega += e * dm.omega;
          mm.g3 += e * dm.g3;
          mm.g4 += e * dm.g4;
          mm.V1 += e * dm.V1;
          mm.V2 += e * dm.V2;
          mm.zeta += e * dm.zeta;
          mm.gamma += e * dm.gamma;
          mm.mu1 += e * dm.mu1;
          mm.mu2 += e * dm.mu2;
        }
        for (int c = 0; c < base.n_couplings; ++c) {
          const heom_coupling& dc = dp.couplings[c];
          cps[c].g_st += e * dc.g_st;
          cps[c].g_s2t += e * dc.g_s2t;
          cps[c].g_st2 += e * dc.g_st2;
          cps[c].mu_st += e * dc.mu_st;
        }
        heom_params p = base;
        p.modes = modes.data();
        p.couplings = cps.data();
        p.beta = base.beta + e * dp.beta;
        return op_vec(heom::build_host_model(p));
      };
      const OpVec a = shifted(step), b = shifted(-step);
      auto dot = [&](const std::vector<double>& x, const std::vector<double>& y, const double* gg) {
        double t = 0.0;
        for (size_t k = 0; k < x.size(); ++k) t += gg[k] * (x[k] - y[k]);
        return t;
      };
      out[i] = (dot(a.H, b.H, g->dH) + dot(a.v, b.v, g->dv) + dot(a.mu, b.mu, g->dmu) + dot(a.c, b.c, g->dc) +
                dot(a.nu, b.nu, g->dnu)) /
               (2.0 * step);
    }
  });
}

int heom_response_2d_backward(const heom_params* params, heom_model* m, const heom_state* rho_eq,
                              const heom_grid* grid, const double* dL_dR, int rho_is_stationary, double tol,
                              int max_steps, const heom_params* dirs, int n_theta, double step,
                              double* dL_dtheta) {
  return guarded([&] {
    require_device(m);
    if (!params || !grid || !dL_dR || !dirs || !dL_dtheta || n_theta < 1)
      throw HeomError(HEOM_ERR_PARAM, "null argument or n_theta < 1");
    if (grid->n_t2 < 1 || grid->n1 < 1 || grid->n3 < 1) throw HeomError(HEOM_ERR_PARAM, "bad grid");
    // dL = sum (dL/dRe R dRe R + dL/dIm R dIm R) = Re sum conj(G) dR with
    // G = dL/dRe R + i dL/dIm R, so the response weights are W = conj(G)
    const size_t nr = static_cast<size_t>(grid->n_t2) * 2 * grid->n1 * grid->n3;
    std::vector<double> W(2 * nr);
    for (size_t k = 0; k < nr; ++k) {
      W[2 * k] = dL_dR[2 * k];
      W[2 * k + 1] = -dL_dR[2 * k + 1];
    }
    const int d = m->hm.d;
    size_t nv = 0;
    for (int s = 0; s < m->hm.n_modes; ++s) nv += static_cast<size_t>(m->hm.dims[s]) * m->hm.dims[s];
    std::vector<double> dH(static_cast<size_t>(d) * d), dv(nv), dmu(static_cast<size_t>(d) * d),
        dc(2 * static_cast<size_t>(m->hm.n_terms)), dnu(m->hm.n_terms);
    heom_op_grad g{dH.data(), dv.data(), dmu.data(), dc.data(), dnu.data(), 0, 0.0};
    int rc = heom_response_2d_vjp(m, rho_eq, grid, W.data(), rho_is_stationary, tol, max_steps, &g);
    if (rc != HEOM_OK) throw HeomError(rc, g_last_error);
    rc = heom_params_vjp(params, dirs, n_theta, step, &g, dL_dtheta);
    if (rc != HEOM_OK) throw HeomError(rc, g_last_error);
  });
}

int heom_batch_create(heom_model* const* models, int n_models, heom_batch** out) {
  return guarded([&] {
    if (!out || !models || n_models < 1) throw HeomError(HEOM_ERR_PARAM, "bad batch arguments");
    *out = nullptr;
    auto b = std::make_unique<heom_batch>();
    for (int i = 0; i < n_models; ++i) {
      heom_model* m = models[i];
      require_device(m);
      if (i == 0) {
        b->stream = m->stream;
        b->dt = m->hm.dt;
      } else {
        if (m->stream != b->stream) throw HeomError(HEOM_ERR_PARAM, "batch models must share the stream");
        if (m->hm.dt != b->dt) throw HeomError(HEOM_ERR_PARAM, "batch models must share the time step");
        if (m->device != models[0]->device) throw HeomError(HEOM_ERR_PARAM, "batch models must share the device");
      }
      if (!heom::mfma_supported<float>(m->hm.d, m->hm.n_modes, m->hm.dims) || (m->hm.d + 15) / 16 > 7)
        throw HeomError(HEOM_ERR_PARAM, "batch model dimension too large for the matrix-core kernel");
      b->models.push_back(m);
    }
    *out = b.release();
  });
}

void heom_batch_free(heom_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  delete b;
}

int heom_batch_propagate(heom_batch* b, heom_state* const* states, int n_steps, int adjoint) {
  return guarded([&] {
    if (!b || !states || n_steps < 0) throw HeomError(HEOM_ERR_PARAM, "bad arguments");
    const int n = static_cast<int>(b->models.size());
    const int prec = states[0] ? states[0]->precision : -1;
    std::vector<int> nt(n);
    for (int i = 0; i < n; ++i) {
      require_state(b->models[i], states[i]);
      if (states[i]->precision != prec) throw HeomError(HEOM_ERR_STATE, "batch states must share the precision");
      nt[i] = states[i]->n_traj;
    }
    if (prec == HEOM_FP64) {
      for (auto* m : b->models)
        if (!heom::mfma_supported<double>(m->hm.d, m->hm.n_modes, m->hm.dims)) throw HeomError(HEOM_ERR_PARAM, "FP64 batch needs d <= 80");
      BatchProp<double> bp;
      std::vector<double*> ys(n);
      for (int i = 0; i < n; ++i) ys[i] = states[i]->buf.as<double>();
      bp.build(b, ys, nt);
      bp.steps(b, n_steps, adjoint != 0);
      for (int i = 0; i < n; ++i) check_finite<double>(b->models[i], ys[i], nt[i], "batched propagation");
    } else {
      BatchProp<float> bp;
      std::vector<float*> ys(n);
      for (int i = 0; i < n; ++i) ys[i] = states[i]->buf.as<float>();
      bp.build(b, ys, nt);
      bp.steps(b, n_steps, adjoint != 0);
      for (int i = 0; i < n; ++i) check_finite<float>(b->models[i], ys[i], nt[i], "batched propagation");
    }
  });
}

int heom_batch_response_2d(heom_batch* b, const heom_state* const* rho_eq, const heom_grid* grid, int precision,
                           double* const* R_out) {
  return guarded([&] {
    if (!b || !rho_eq || !grid || !R_out) throw HeomError(HEOM_ERR_PARAM, "null argument");
    const heom_grid& g = *grid;
    if (g.n1 < 1 || g.n3 < 1 || g.steps_per_sample < 1 || g.n_t2 < 1 || !g.t2_steps)
      throw HeomError(HEOM_ERR_PARAM, "bad grid");
    for (int i = 0; i < g.n_t2; ++i)
      if (g.t2_steps[i] < 0 || (i && g.t2_steps[i] < g.t2_steps[i - 1]))
        throw HeomError(HEOM_ERR_PARAM, "t2_steps must be non-negative and non-decreasing");
    for (size_t i = 0; i < b->models.size(); ++i) {
      require_state(b->models[i], rho_eq[i]);
      if (rho_eq[i]->precision != HEOM_FP64 || rho_eq[i]->n_traj != 1)
        throw HeomError(HEOM_ERR_STATE, "rho_eq must be FP64 states with one trajectory");
      if (!R_out[i]) throw HeomError(HEOM_ERR_PARAM, "null output");
    }
    if (precision != HEOM_FP64 && precision != HEOM_FP32) throw HeomError(HEOM_ERR_PARAM, "bad precision");
    if (precision == HEOM_FP64)
      for (auto* m : b->models)
        if (!heom::mfma_supported<double>(m->hm.d, m->hm.n_modes, m->hm.dims)) throw HeomError(HEOM_ERR_PARAM, "FP64 batch needs d <= 80");
    // Instances go in groups whose buffers (Psi: n3, snapshots: n1, their two
    // RK4 scratch copies when t2 > 0, a few single states) fit in free memory.
    const size_t elem = precision == HEOM_FP64 ? sizeof(double) : sizeof(float);
    const bool any_t2 = g.t2_steps[g.n_t2 - 1] > 0;
    const size_t fr = free_device_bytes();
    const size_t budget = fr > (size_t(2) << 30) ? fr - (size_t(2) << 30) : 0;
    const int n = static_cast<int>(b->models.size());
    int i0 = 0;
    while (i0 < n) {
      size_t used = 0;
      int i1 = i0;
      while (i1 < n) {
        const size_t te = static_cast<size_t>(b->models[i1]->traj_elems());
        const size_t need = te * (elem * (g.n1 + g.n3 + (any_t2 ? 2 * g.n1 : 0) + 4) + 2 * sizeof(double));
        if (i1 > i0 && used + need > budget) break;
        used += need;
        ++i1;
      }
      if (used > budget) throw HeomError(HEOM_ERR_OOM, "not enough device memory for one instance");
      heom_batch sub;
      sub.models.assign(b->models.begin() + i0, b->models.begin() + i1);
      sub.stream = b->stream;
      sub.dt = b->dt;
      sub.launch = b->launch;
      sub.tuned = b->tuned;
      std::copy(std::begin(b->class_cost), std::end(b->class_cost), std::begin(sub.class_cost));
      std::copy(std::begin(b->class_shape), std::end(b->class_shape), std::begin(sub.class_shape));
      sub.graph_steps = b->graph_steps;
      if (precision == HEOM_FP64)
        batch_response_adjoint<double>(&sub, rho_eq + i0, g, R_out + i0);
      else
        batch_response_adjoint<float>(&sub, rho_eq + i0, g, R_out + i0);
      i0 = i1;
    }
  });
}

int heom_batch_set_launch(heom_batch* b, int launch) {
  return guarded([&] {
    if (!b) throw HeomError(HEOM_ERR_PARAM, "null batch");
    if (launch < HEOM_BATCH_AUTO || launch > HEOM_BATCH_SINGLE) throw HeomError(HEOM_ERR_PARAM, "bad launch form");
    if (launch == HEOM_BATCH_SINGLE)
      for (auto* m : b->models)
        if ((m->hm.d + 15) / 16 > heom::kFusedMaxNb)
          throw HeomError(HEOM_ERR_PARAM, "single-launch batches need every d <= 80");
    b->launch = launch;
  });
}

int heom_batch_get_launch(const heom_batch* b, int* out) {
  return guarded([&] {
    if (!b || !out) throw HeomError(HEOM_ERR_PARAM, "null argument");
    *out = b->resolved_launch();
  });
}

int heom_batch_set_class_shape(heom_batch* b, int nb, int wg_per_cu, int lds_sums) {
  return guarded([&] {
    if (!b || nb < 1 || nb > 7 || wg_per_cu < 0 || lds_sums < -1 || lds_sums > 1)
      throw HeomError(HEOM_ERR_PARAM, "bad arguments");
    if (lds_sums >= 0 && !heom::multi_has_alt_xl<float>(nb))
      throw HeomError(HEOM_ERR_PARAM, "this size class has one neighbour-sum form only");
    b->class_shape[nb] = heom::MultiShape{wg_per_cu, lds_sums};
  });
}

int heom_batch_get_class_shape(const heom_batch* b, int nb, int* wg_per_cu, int* lds_sums) {
  return guarded([&] {
    if (!b || !wg_per_cu || !lds_sums || nb < 1 || nb > 7) throw HeomError(HEOM_ERR_PARAM, "bad arguments");
    *wg_per_cu = b->class_shape[nb].wg_per_cu;
    *lds_sums = b->class_shape[nb].xl;
  });
}

int heom_batch_set_graph_steps(heom_batch* b, int steps) {
  return guarded([&] {
    if (!b || steps < 0) throw HeomError(HEOM_ERR_PARAM, "bad arguments");
    b->graph_steps = steps;
  });
}

int heom_batch_autotune(heom_batch* b, int precision, int n_traj, int reps, double* ms_out) {
  return guarded([&] {
    if (!b || n_traj < 1 || reps < 1) throw HeomError(HEOM_ERR_PARAM, "bad arguments");
    if (precision == HEOM_FP64) {
      for (auto* m : b->models)
        if (!heom::mfma_supported<double>(m->hm.d, m->hm.n_modes, m->hm.dims))
          throw HeomError(HEOM_ERR_PARAM, "FP64 batch needs d <= 80");
      batch_autotune<double>(b, n_traj, reps, ms_out);
    } else if (precision == HEOM_FP32) {
      batch_autotune<float>(b, n_traj, reps, ms_out);
    } else {
      throw HeomError(HEOM_ERR_PARAM, "bad precision");
    }
  });
}

int heom_model_set_kernel(heom_model* m, int precision, int kernel) {
  return guarded([&] {
    require_device(m);
    if (precision != HEOM_FP64 && precision != HEOM_FP32) throw HeomError(HEOM_ERR_PARAM, "bad precision");
    if (kernel < HEOM_KERNEL_AUTO || kernel > HEOM_KERNEL_MFMA_GH) throw HeomError(HEOM_ERR_PARAM, "bad kernel");
    const bool ok = precision == HEOM_FP64 ? heom::mfma_supported<double>(m->hm.d, m->hm.n_modes, m->hm.dims)
                                           : heom::mfma_supported<float>(m->hm.d, m->hm.n_modes, m->hm.dims);
    if (kernel == HEOM_KERNEL_AUTO) kernel = ok ? HEOM_KERNEL_MFMA : HEOM_KERNEL_GENERIC;
    if (kernel == HEOM_KERNEL_KRON && (precision != HEOM_FP32 || !m->kron))
      throw HeomError(HEOM_ERR_PARAM, "the (S;4,4) matrix-core kernel needs FP32 and three modes of (4|5, 4, 4) levels");
    if ((kernel == HEOM_KERNEL_MFMA || kernel == HEOM_KERNEL_MFMA_DYN) && !ok)
      throw HeomError(HEOM_ERR_PARAM, "matrix-core kernel unsupported for this d");
    if (kernel == HEOM_KERNEL_MFMA_GH &&
        (precision != HEOM_FP32 || !heom::mfma_gh_supported<float>(m->hm.d, m->hm.n_modes, m->hm.dims)))
      throw HeomError(HEOM_ERR_PARAM, "the H-from-global matrix-core kernel needs FP32, d in 65..80 and at most "
                                      "128 single-mode operator values");
    m->kernel[precision] = kernel;
    m->clear_graphs();
  });
}

int heom_model_set_progress(heom_model* m, heom_progress_fn fn, void* ctx, int every_steps) {
  return guarded([&] {
    if (!m) throw HeomError(HEOM_ERR_PARAM, "null model");
    m->progress_fn = every_steps > 0 ? fn : nullptr;
    m->progress_ctx = ctx;
    m->progress_every = fn ? every_steps : 0;
  });
}

int heom_model_set_graph_steps(heom_model* m, int steps) {
  return guarded([&] {
    require_device(m);
    if (steps < 0) throw HeomError(HEOM_ERR_PARAM, "steps must be >= 0");
    hip_check(hipStreamSynchronize(m->stream), "sync");
    m->clear_graphs();
    m->graph_steps = steps;
  });
}

int heom_model_get_kernel(const heom_model* m, int precision, int* kernel_out) {
  return guarded([&] {
    require_device(m);
    if ((precision != HEOM_FP64 && precision != HEOM_FP32) || !kernel_out) throw HeomError(HEOM_ERR_PARAM, "bad argument");
    *kernel_out = m->kernel[precision];
  });
}

int heom_autotune(heom_model* m, int n_traj, int precision, int reps, int* kernel_out, double* ms_out) {
  return guarded([&] {
    require_device(m);
    if (n_traj < 1 || reps < 1) throw HeomError(HEOM_ERR_PARAM, "bad autotune sizes");
    if (precision != HEOM_FP64 && precision != HEOM_FP32) throw HeomError(HEOM_ERR_PARAM, "bad precision");
    auto s = new_state(m, n_traj, precision);
    // restores the kernel choice and timing flag and frees the events on every exit
    struct Guard {
      heom_model* m;
      int prec, kernel;
      bool timing;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      ~Guard() {
        m->kernel[prec] = kernel;
        m->timing = timing;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
      }
    } guard{m, precision, m->kernel[precision], m->timing};
    hip_check(hipEventCreate(&guard.e0), "event");
    hip_check(hipEventCreate(&guard.e1), "event");
    m->timing = false;
    const bool ok = precision == HEOM_FP64 ? heom::mfma_supported<double>(m->hm.d, m->hm.n_modes, m->hm.dims)
                                           : heom::mfma_supported<float>(m->hm.d, m->hm.n_modes, m->hm.dims);
    const bool distinct_dyn = precision == HEOM_FP64 ? heom::mfma_static_shape<double>(m->ops64[0])
                                                     : heom::mfma_static_shape<float>(m->ops32[0]);
    std::vector<int> cand = {HEOM_KERNEL_GENERIC};
    if (ok) cand.push_back(HEOM_KERNEL_MFMA);
    if (ok && distinct_dyn) cand.push_back(HEOM_KERNEL_MFMA_DYN);
    if (precision == HEOM_FP32 && m->kron) cand.push_back(HEOM_KERNEL_KRON);
    if (precision == HEOM_FP32 && heom::mfma_gh_supported<float>(m->hm.d, m->hm.n_modes, m->hm.dims))
      cand.push_back(HEOM_KERNEL_MFMA_GH);
    if (ms_out)
      for (int k = 0; k <= HEOM_KERNEL_MFMA_GH; ++k) ms_out[k] = std::nan("");
    int best = guard.kernel;
    double best_ms = 1e300;
    for (int k : cand) {
      m->kernel[precision] = k;
      auto run = [&](int steps) {
        if (precision == HEOM_FP64) {
          heom::launch_set_ground<double>(s->buf.as<double>(), m->traj_elems(), n_traj, s->n_elems(), m->stream);
          rk4_steps_ws<double>(m, s->buf.as<double>(), n_traj, steps, false);
        } else {
          heom::launch_set_ground<float>(s->buf.as<float>(), m->traj_elems(), n_traj, s->n_elems(), m->stream);
          rk4_steps_ws<float>(m, s->buf.as<float>(), n_traj, steps, false);
        }
      };
      run(1);  // warm-up (first launch configures the kernel)
      hip_check(hipEventRecord(guard.e0, m->stream), "event");
      run(reps);
      hip_check(hipEventRecord(guard.e1, m->stream), "event");
      hip_check(hipEventSynchronize(guard.e1), "event sync");
      float ms = 0.0f;
      hip_check(hipEventElapsedTime(&ms, guard.e0, guard.e1), "event elapsed");
      const double per = ms / reps;
      if (ms_out) ms_out[k] = per;
      if (per < best_ms) {
        best_ms = per;
        best = k;
      }
    }
    guard.kernel = best;
    if (kernel_out) *kernel_out = best;
  });
}

int heom_timing_enable(heom_model* m, int enable) {
  return guarded([&] {
    require_device(m);
    m->timing = enable != 0;
  });
}

int heom_timing_read(heom_model* m, double* total_ms, long long* launches, long long* ado_updates) {
  return guarded([&] {
    require_device(m);
    hip_check(hipStreamSynchronize(m->stream), "sync");
    double tot = 0.0;
    for (size_t i = 0; i < m->events_used; ++i) {
      float ms = 0.0f;
      hip_check(hipEventElapsedTime(&ms, m->events[i].first, m->events[i].second), "event elapsed");
      tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = m->launches;
    if (ado_updates) *ado_updates = m->ado_updates;
    m->events_used = 0;
    m->launches = 0;
    m->ado_updates = 0;
  });
}

}  // extern "C"
