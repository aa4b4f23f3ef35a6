/*
 * heom2dvs.h -- C ABI of the MI355X (gfx950) HEOM-2DVS library.
 *
 * The library time-steps the hierarchical equations of motion (HEOM) of the
 * multi-mode anharmonic Brownian (MAB) oscillator model and evaluates linear
 * and third-order (2D IR) response functions and the 2D correlation
 * spectrum, following Hoshino & Tanimura, arXiv:2601.20550:
 *   model            Sec. II.A, Eqs. (Total Hamiltonian)-(h_int), (NLdip),
 *                    (counter1)-(sys_interaction)
 *   bath terms       Sec. II.B, Eqs. (drude), (L1), (L2), (counterterm),
 *                    (Pade1), (Pade2)
 *   HEOM             Sec. II.B, Eq. (HEOM_DB)
 *   responses        Sec. II.C, Eqs. (R1), (RFTIRI), (echo), (virtual-echo)
 *   spectra          Sec. II.C, Eqs. (2D-rephasing), (2D-nonrephasing),
 *                    (correlation-spectrum)
 *   integrator       Sec. III (fourth-order Runge-Kutta, fixed step)
 *
 * Conventions
 *   Units: hbar = 1; energies in units of omega0 (harmonic frequency of the
 *   reference mode); time in 1/omega0; beta is beta*hbar*omega0; m_s = 1.
 *   Product basis: mode 0 is the slowest index; each mode keeps the n_keep
 *   lowest eigenstates of its single-mode Hamiltonian (Sec. II.A).
 *   Hierarchy: ADOs n = (n_j), one entry per exponential bath term j
 *   (terms of mode 0 first, k = 0..K within a mode), truncated to
 *   |n| <= depth, ordered by depth and then ascending lexicographically.
 *   Host arrays of complex numbers are interleaved (re, im) doubles.
 *   A host hierarchy array has layout [n_traj][n_ado][d][d] complex, row-major.
 *
 * Errors: every int-returning call returns HEOM_OK (0) or a negative code;
 * heom_last_error() returns a thread-local message for the last failure.
 * No C++ exception crosses the ABI.  Pointers named *_out are caller-owned
 * host memory unless stated otherwise.  Objects returned through ** are owned
 * by the caller and released with the matching *_free call.
 */
#ifndef HEOM2DVS_H
#define HEOM2DVS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HEOM_OK = 0,
  HEOM_ERR_PARAM = -1,     /* invalid argument or parameter set          */
  HEOM_ERR_OOM = -2,       /* device allocation failed                   */
  HEOM_ERR_UNSTABLE = -3,  /* non-finite values during propagation       */
  HEOM_ERR_NOCONV = -4,    /* equilibration above tolerance at max_steps */
  HEOM_ERR_HIP = -5,       /* HIP runtime error (message has details)    */
  HEOM_ERR_STATE = -6      /* object mismatch (model/state/precision)    */
};

typedef enum { HEOM_FP64 = 0, HEOM_FP32 = 1 } heom_precision;
typedef enum { HEOM_PADE = 0, HEOM_MATSUBARA = 1 } heom_decomp;
/* Operators that the dipole/trace calls can apply. */
typedef enum { HEOM_OP_MU = 0, HEOM_OP_MU_PLUS = 1, HEOM_OP_MU_MINUS = 2 } heom_operator;
/* How heom_response_2d obtains the t3 dependence.
 * HEOM_RESP_DIRECT : the paper's order -- every t1 snapshot is propagated
 *                    over t2 and t3 and the trace is sampled (Sec. II.C).
 * HEOM_RESP_ADJOINT: the t3 propagation is replaced by one propagation of
 *                    the detection functional tr(mu .) under the transposed
 *                    HEOM; R is then the bilinear pairing of the two sets of
 *                    hierarchies.  Identical in exact arithmetic, including
 *                    the RK4 discretisation. */
typedef enum { HEOM_RESP_DIRECT = 0, HEOM_RESP_ADJOINT = 1 } heom_resp_method;

/* One vibrational mode s (Sec. II.A, II.B):
 *   H_A = omega (p^2 + q^2)/2 + g3 q^3/3! + g4 q^4/4!   (Eq. Potentials; g4 optional)
 *   V_s(q) = V1 q + V2 q^2/2                             (Eq. h_int, LL + SL)
 *   Drude bath (zeta, gamma) with K low-temperature terms (Eqs. drude, Pade1/2)
 *   dipole mu1 q + mu2 q^2/2                             (Eq. NLdip, s = s')
 *   n_basis harmonic levels are diagonalised, n_keep eigenstates are kept.
 * omega_b > 0 replaces the Drude density by the Brownian (underdamped
 * oscillator) density J(w) = (zeta/pi) gamma^2 omega_b^2 w /
 * ((omega_b^2 - w^2)^2 + gamma^2 w^2), one of the other spectral densities the
 * HEOM admits (Sec. II.B); it has the Drude counter-term constant zeta gamma/2
 * and K + 2 exponential terms: a complex-conjugate pair of rates
 * gamma/2 +- i sqrt(omega_b^2 - gamma^2/4) (two real rates when overdamped)
 * followed by the K low-temperature terms.  omega_b = gamma/2 (critical
 * damping) is rejected with HEOM_ERR_PARAM. */
typedef struct {
  double omega, g3, g4, V1, V2, zeta, gamma, mu1, mu2;
  int n_basis, n_keep, K;
  double omega_b;                   /* 0 = Drude bath                        */
} heom_mode;

/* Mode-mode coupling (Eq. Potential ss') and cross dipole (Eq. NLdip), s < t:
 *   g_st q_s q_t + (g_s2t q_s^2 q_t + g_st2 q_s q_t^2)/6 ;  mu_st q_s q_t */
typedef struct {
  int s, t;
  double g_st, g_s2t, g_st2, mu_st;
} heom_coupling;

typedef struct {
  int n_modes;                      /* 1..4                                  */
  const heom_mode* modes;
  int n_couplings;
  const heom_coupling* couplings;
  double beta;                      /* beta * hbar * omega0                  */
  int depth;                        /* hierarchy depth L                     */
  int decomp;                       /* heom_decomp                           */
  double dt;                        /* RK4 step (1/omega0)                   */
  /* Optional non-triangular filter (0 = off): keep only the ADOs whose
   * total damping rate sum_j n_j Re(nu_j) is at most rate_cut (relative
   * tolerance 1e-9), in addition to |n| <= depth.  The paper's own filter is
   * not stated; this rate rule keeps the set closed under n -> n - e_j (all
   * Re nu_j > 0), as the truncation of Eq. HEOM_DB requires. */
  double rate_cut;
} heom_params;

typedef struct {
  int d;                            /* product-basis dimension               */
  int n_ado;                        /* number of ADOs                        */
  int n_terms;                      /* M = sum_s (K_s + 1)                   */
  int n_modes;
  int dims[4];                      /* kept levels per mode                  */
  int depth;
  double dt;
} heom_info;

/* t1/t3 sampling grid and t2 values of a third-order response.
 * t1_j = j * steps_per_sample * dt, t3_k = k * steps_per_sample * dt and
 * t2 = t2_steps[i] * dt; t2_steps must be non-decreasing. */
typedef struct {
  int n1, n3, steps_per_sample;
  int n_t2;
  const int* t2_steps;
} heom_grid;

typedef struct heom_model heom_model;
typedef struct heom_state heom_state;

/* ------------------------------------------------------------ general -- */
const char* heom_last_error(void);
/* Device allocator hook (e.g. a framework's caching allocator).  NULL
 * functions restore hipMalloc/hipFree.  Applies to later allocations. */
typedef void* (*heom_alloc_fn)(size_t bytes, void* ctx);
typedef void (*heom_free_fn)(void* ptr, void* ctx);
int heom_set_allocator(heom_alloc_fn alloc, heom_free_fn release, void* ctx);
/* Device properties used by the launch heuristics: CU count and LDS bytes per
 * workgroup of the current device. */
int heom_device_query(int* cu_count, int* lds_bytes, char* name_out, int name_len);

/* -------------------------------------------------------------- model -- */
/* Builds the operators of Sec. II.A in the product eigenbasis, the bath terms
 * of Sec. II.B and the hierarchy tables (host, FP64), then uploads them to the
 * current device.  `hip_stream` (a hipStream_t, may be NULL for the null
 * stream) is used by every later call on this model.
 * Errors: HEOM_ERR_PARAM for n_keep > n_basis, n_modes outside 1..4, product
 * dimension > 128, |gamma^2 - nu_k^2| < 1e-12 (Eq. Pade1 singular), depth < 0,
 * dt <= 0, couplings with s >= t or out of range. */
int heom_model_build(const heom_params* params, void* hip_stream, heom_model** out);
/* Host part only (no device memory): for inspecting the operators. */
int heom_model_build_host(const heom_params* params, heom_model** out);
void heom_model_free(heom_model* model);
int heom_model_info(const heom_model* model, heom_info* out);
/* Copies the host FP64 operators.  Any pointer may be NULL.
 *   H, mu, mu_plus, mu_minus: [d][d];  v: per mode [dims[s]][dims[s]] packed
 *   one after another;  nu: [n_terms];  c: [n_terms] complex;
 *   ado_n: [n_ado][n_terms] ints;  term_mode: [n_terms] ints. */
int heom_model_operators(const heom_model* model, double* H, double* mu, double* mu_plus,
                         double* mu_minus, double* v, double* nu, double* c, int* ado_n,
                         int* term_mode);
/* Exponential terms of the bath correlations, C(t) = sum_j c_j exp(-nu_j t)
 * per mode, with the bra-side coefficients c_bra_j of the coupling
 * Theta_j X = c_j V X - c_bra_j X V: the coefficient of exp(-nu_j t) in
 * C(t)*, i.e. conj(c_j) for a real rate and the partner's conj(c) for a
 * complex-conjugate pair of rates (Brownian baths).  Each output [n_terms]
 * complex (interleaved doubles), may be NULL.  heom_model_operators' nu
 * holds the real parts. */
int heom_model_bath(const heom_model* model, double* nu, double* c, double* c_bra);

/* -------------------------------------------------------------- state -- */
/* A device hierarchy of n_traj independent trajectories (n_traj x n_ado
 * complex d x d matrices) in the given precision, zero-initialised. */
int heom_state_create(heom_model* model, int n_traj, int precision, heom_state** out);
void heom_state_free(heom_state* state);
int heom_state_shape(const heom_state* state, int* n_traj, int* precision);
/* host [n_traj][n_ado][d][d] complex <-> device (converted to the state's precision) */
int heom_state_upload(heom_state* state, const double* host);
int heom_state_download(const heom_state* state, double* host_out);
/* Same for trajectories first .. first+count-1 only (host [count][n_ado][d][d]). */
int heom_state_upload_range(heom_state* state, int first, int count, const double* host);
int heom_state_download_range(const heom_state* state, int first, int count, double* host_out);
/* rho_{n=0} = |0><0| and every other ADO zero, for every trajectory
 * (factorised initial condition of Sec. II.C). */
int heom_state_set_ground(heom_state* state);
/* dst <- src, converting precision; trajectory counts must match. */
int heom_state_copy(heom_state* dst, const heom_state* src);

/* ---------------------------------------------------------- hot path -- */
/* out = L in (adjoint = 0) or L^T in (adjoint = 1) for every trajectory,
 * L being the HEOM generator of Eq. (HEOM_DB).  L^T is the transpose for the
 * bilinear pairing <A, X> = sum_n sum_ab A_n[a,b] X_n[a,b]. */
int heom_rhs(heom_model* model, const heom_state* in, heom_state* out, int adjoint);
/* n_steps fixed-step fourth-order Runge-Kutta steps of d rho/dt = L rho (or
 * L^T rho) in place (Sec. III: fixed-step Runge-Kutta integration of Eq.
 * HEOM_DB).  The step is evaluated as y + h L(y + h/2 L(y + h/3 L(y + h/4 L
 * y))), which equals the classic four-stage scheme for this linear,
 * time-independent generator.  The arithmetic is the state's precision (the
 * state carries it, so there is no separate precision argument).
 * sample_every > 0 with trace_out != NULL records the detection trace
 * tr(mu rho_{b, n=0}) (FP64 accumulation, Eq. R1's trace) of every trajectory
 * b at steps 0, sample_every, 2 sample_every, ... <= n_steps:
 * trace_out is caller-owned host memory of
 * (n_steps / sample_every + 1) x n_traj complex values (interleaved re, im),
 * sample-major.  sample_every <= 0 or trace_out == NULL records nothing.
 * HEOM_ERR_PARAM for n_steps < 0; HEOM_ERR_UNSTABLE if the state becomes
 * non-finite (checked at the end). */
int heom_propagate(heom_model* model, heom_state* state, int n_steps, int adjoint, int sample_every,
                   double* trace_out);
/* heom_propagate for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, but every work buffer (two RK4 stage buffers,
 * the sampled traces, the finiteness-check partials) lives in one static
 * device array of 64 MiB per GPU that the library holds until the process
 * ends; no hipMalloc / hipFree or other allocating call is made.  The model
 * and state must exist already (building them allocates).  Needs
 * 2 x state bytes + 8 x n_traj x n_ado + 16 x n_traj x n_samples bytes
 * (each part rounded up to 256) <= 64 MiB, else HEOM_ERR_PARAM with the
 * size in the message.  Graph replay and timing (heom_model_set_graph_steps,
 * heom_timing_enable) do not apply to this call.  Calls on one GPU share its
 * array: calls that overlap in time on one GPU (different threads or
 * streams) race and must be serialised by the caller.  Arguments, outputs
 * and errors otherwise as heom_propagate. */
int heom_propagate_noalloc(heom_model* model, heom_state* state, int n_steps, int adjoint, int sample_every,
                           double* trace_out);
/* X <- D^x X = D X - X D on every ADO (transpose = 0), or
 * X <- (D^T)^x X (transpose = 1), D chosen by `op` (heom_operator). FP64
 * arithmetic on either precision. */
int heom_apply_dipole(heom_model* model, heom_state* state, int op, int transpose);
/* out[b] = tr(D rho_{b, n=0}) for each trajectory b, FP64 accumulation;
 * out: [n_traj] complex. */
int heom_trace(heom_model* model, const heom_state* state, int op, double* out);
/* max over trajectories, ADOs and elements of |(L rho)| (FP64 value). */
int heom_residual(heom_model* model, const heom_state* state, double* out);

/* Equilibration (Sec. II.C, first two steps of the recipe): from
 * rho_{n=0} = |0><0| propagate in FP64; after every check_every steps (once
 * min_steps are done) evaluate the residual max|L rho|; stop at the first
 * check <= tol or at max_steps.  Returns a new FP64 state with one
 * trajectory.  HEOM_ERR_NOCONV is returned (with the state still written)
 * when max_steps is reached above tol and require_convergence != 0.
 * Times are counted in RK4 steps of the model's fixed dt: the time limit is
 * t_max = max_steps dt and the equilibration time t_eq = (*steps_out) dt (a
 * step count is exact, a time would have to be rounded to the step grid). */
int heom_equilibrate(heom_model* model, double tol, int check_every, int min_steps,
                     int max_steps, int require_convergence, heom_state** rho_eq_out,
                     int* steps_out, double* residual_out);

/* Linear response (Eq. R1): R1(t_k) = i tr{mu G(t_k) mu^x rho_eq},
 * t_k = k * steps_per_sample * dt, k = 0..n-1.  R_out: [n] complex. */
/* Stationary state by restarted GMRES (Sec. II.C defines rho_eq as the
 * long-time limit of the propagation from |0><0|; this reaches the same fixed
 * point, L rho_eq = 0 with tr rho_eq,0 = 1, in fewer steps): after pre_steps
 * RK4 steps from |0><0|, corrections x solve (I - Phi^m) x = -(I - Phi^m) rho
 * with m = steps_per_apply RK4 steps per operator application and GMRES
 * restarted every `restart` applications, until max|L rho| <= tol (the
 * residual of heom_equilibrate) or max_applies applications.  Outputs as in
 * heom_equilibrate (applies_out: operator applications); HEOM_ERR_NOCONV (the
 * state is still returned) if tol is not reached. */
int heom_equilibrate_krylov(heom_model* model, double tol, int pre_steps, int steps_per_apply, int restart,
                            int max_applies, heom_state** rho_eq_out, int* applies_out, double* residual_out);
/* The same GMRES corrections applied in place to an existing FP64
 * one-trajectory state with unit trace (e.g. to continue a previous call in
 * chunks).  HEOM_ERR_NOCONV (state updated) if tol is not reached. */
int heom_stationary_refine(heom_model* model, heom_state* rho, double tol, int steps_per_apply, int restart,
                           int max_applies, int* applies_out, double* residual_out);

int heom_linear_response(heom_model* model, const heom_state* rho_eq, int n,
                         int steps_per_sample, int precision, double* R_out);

/* Third-order responses of the rephasing (I: k3+k2-k1) and non-rephasing
 * (II: k3-k2+k1) pathways (Eqs. echo, virtual-echo) with the rotating-wave
 * split of the dipole: (D1,D2,D3) = (mu-, mu+, mu+) for I and (mu+, mu-, mu+)
 * for II, mu+ keeping the elements that raise the total number of kept quanta.
 * R = i^3 tr{mu G(t3) D3^x G(t2) D2^x G(t1) D1^x rho_eq}.
 * rho_eq: FP64 state with one trajectory.  precision selects the arithmetic of
 * the propagations (dipoles, traces and pairings are FP64).  max_batch bounds
 * the number of trajectories propagated together (0 = automatic from free
 * device memory).  R_out: [n_t2][2][n1][n3] complex. */
int heom_response_2d(heom_model* model, const heom_state* rho_eq, const heom_grid* grid,
                     int precision, int method, int max_batch, double* R_out);

/* Third-order responses of arbitrary dipole pathways (the full 8-term
 * response of Eq. RFTIRI with D1 = D2 = D3 = mu, double-quantum and other
 * phase-matched pathways): pathway p applies (D1, D2, D3) = (ops[3p],
 * ops[3p+1], ops[3p+2]), each a heom_operator, i.e.
 * R_p = i^3 tr{mu G(t3) D3^x G(t2) D2^x G(t1) D1^x rho_eq} on the grid, with
 * the same methods, precisions and batching as heom_response_2d (which is
 * this call with the pathways I = (mu-, mu+, mu+) and II = (mu+, mu-, mu+)).
 * R_out: host [n_t2][n_pathways][n1][n3] complex.  HEOM_ERR_PARAM for an
 * operator outside heom_operator or n_pathways < 1. */
int heom_response_2d_pathways(heom_model* model, const heom_state* rho_eq, const heom_grid* grid,
                              int precision, int method, int max_batch, int n_pathways, const int* ops,
                              double* R_out);

/* 2D correlation spectrum (Eq. correlation-spectrum) from the two pathway
 * responses, computed on the device in FP64: trapezoid weights (1/2 at t=0),
 * zero padding to 2n, Omega_m = 2 pi m/(2 n dt_s), m = -n..n-1,
 * S_P(W3,W1) = Im sum_jk w_j w_k dt_s^2 exp(i W3 t3_k + i W1 t1_j) R_P[j][k],
 * S_C(W3,W1) = -[S_I(W3,-W1) + S_II(W3,W1)] (sign fixed so the 0->1->0 peak
 * is positive).  R_I, R_II: [n1][n3] complex host arrays; S_out:
 * [2 n3][2 n1] doubles (rows W3, columns W1). */
int heom_spectrum_2d(const double* R_I, const double* R_II, int n1, int n3, double dt_s,
                     double* S_out);

/* Linear absorption line shape from R1 (heom_linear_response): the same
 * trapezoid-weighted DFT as heom_spectrum_2d in one dimension,
 * I(W_m) = sum_k w_k dt_s exp(i W_m t_k) R1(t_k), W_m = 2 pi m/(2 n dt_s),
 * m = -n..n-1 (Sec. II.C, linear response).  R1: [n] complex; I_out: [2n]
 * complex host arrays.  Host computation, FP64. */
int heom_spectrum_1d(const double* R1, int n, double dt_s, double* I_out);

/* ------------------------------------------------------- gradients ----- */
/* Gradients of a real objective J = Re sum W[q][P][j][k] R[q][P][j][k] of the
 * third-order responses (weights W from the caller, e.g. heom_spectrum_2d_vjp
 * of dJ/dS_C) with respect to the operators the HEOM generator and the
 * dipoles are built from (Sec. II.A operators, Sec. II.B bath terms).  Every
 * entry is treated as independent (no symmetry imposed).  Caller-owned host
 * arrays:
 *   dH  [d*d]                 dJ/dH_S'[a][b]
 *   dv  [sum_s dims[s]^2]     dJ/dv_s[a][b], mode after mode (V_s = v_s on mode s)
 *   dmu [d*d]                 dJ/dmu[a][b]; mu+ = mu where N(a) > N(b), mu- = (mu+)^T
 *   dc  [n_terms*2]           dJ/dRe c_j, dJ/dIm c_j
 *   dnu [n_terms]             dJ/dnu_j
 * stationary_steps / stationary_residual are outputs (see heom_response_2d_vjp). */
typedef struct {
  double* dH;
  double* dv;
  double* dmu;
  double* dc;
  double* dnu;
  int stationary_steps;
  double stationary_residual;
} heom_op_grad;

/* Reverse-mode gradient of J through the response computation of
 * heom_response_2d (adjoint detection method, FP64 propagation): the
 * detection functional, both pathways' t1 scans, t2 propagations and t3
 * detection, with the exact discrete adjoint of the RK4 propagator (each
 * step's derivative is the sum over a + b <= 3 of h^(a+b+1)/(a+b+1)!
 * <(L^T)^a lambda, dL L^b y>).  Forward states are recomputed from
 * checkpoints.  rho_is_stationary = 1: rho_eq is the stationary state
 * (L rho_eq = 0, tr rho_eq,0 = 1) and its dependence on the operators is
 * included through the adjoint stationary equation, solved by restarted
 * GMRES on (I - (Phi^T)^500) k = h sum_{n<500} (Phi^T)^n r (Phi: the RK4
 * propagator) until the relative residual is <= tol, using at most max_steps
 * RK4 steps (stationary_steps / stationary_residual report them;
 * HEOM_ERR_NOCONV if not reached); 0: rho_eq is held fixed.  W: host
 * [n_t2][2][n1][n3] complex.  Needs d <= 80, every mode dimension d_s <= 8
 * with d_s * d <= 512, K + 1 <= 4 terms per mode, and Drude baths (real
 * rates; HEOM_ERR_PARAM otherwise). */
int heom_response_2d_vjp(heom_model* model, const heom_state* rho_eq, const heom_grid* grid, const double* W,
                         int rho_is_stationary, double tol, int max_steps, heom_op_grad* out);

/* Backward pass of heom_response_2d (the gradient of a loss L(R) of the
 * responses with respect to model parameters; Sec. II.B: the generator of Eq.
 * HEOM_DB is linear in H_S', V_s, c_j and nu_j, so every derivative is a
 * pairing of forward and adjoint hierarchies): heom_response_2d_vjp with the
 * weights W = conj(dL_dR), then heom_params_vjp along the directions dirs.
 * params: the parameters `model` was built from; dL_dR: host
 * [n_t2][2][n1][n3] complex, dL/dRe R + i dL/dIm R; dirs: n_theta parameter
 * directions (d params / d theta_i, layout of params); step: central-
 * difference step of the host build derivative; rho_is_stationary, tol and
 * max_steps as in heom_response_2d_vjp.  dL_dtheta: caller-owned host
 * [n_theta].  Errors and limits as heom_response_2d_vjp and
 * heom_params_vjp. */
int heom_response_2d_backward(const heom_params* params, heom_model* model, const heom_state* rho_eq,
                              const heom_grid* grid, const double* dL_dR, int rho_is_stationary, double tol,
                              int max_steps, const heom_params* dirs, int n_theta, double step,
                              double* dL_dtheta);

/* Adjoint of heom_spectrum_2d: weights W[P][j][k] (P = I, II; host,
 * [2][n1][n3] complex) with sum G . S_C(R_I, R_II) = Re sum W[P] R_P for the
 * real cotangent G ([2 n3][2 n1], e.g. dJ/dS_C).  Host computation, FP64. */
int heom_spectrum_2d_vjp(const double* G, int n1, int n3, double dt_s, double* W_out);

/* Chain from operator gradients to parameters: out[i] = sum over all
 * operator entries of g x d(operators)/d(params) along dirs[i], the
 * derivative of the host model build taken by central differences with the
 * given step (dirs[i] has the layout of params and holds the derivative of
 * every number; integer fields are ignored).  Host computation.  Drude
 * baths only (omega_b = 0 in every mode; HEOM_ERR_PARAM otherwise). */
int heom_params_vjp(const heom_params* params, const heom_params* dirs, int n_dirs, double step,
                    const heom_op_grad* g, double* out);

/* ------------------------------------------- several model instances -- */
/* A batch of models (instances) of possibly different sizes, propagated
 * together: every RK4 stage is one persistent matrix-core launch per size
 * class ceil(d/16), covering the matrices of all instances of that class
 * (workgroups re-stage H and v_s when they move to another instance), or one
 * launch over all classes (heom_batch_set_launch below).  The
 * models are borrowed and must outlive the batch; they must share the device,
 * the stream and the time step, and each needs d <= 112 (FP32) or d <= 80
 * (FP64).  HEOM_ERR_PARAM otherwise. */
typedef struct heom_batch heom_batch;
int heom_batch_create(heom_model* const* models, int n_models, heom_batch** out);
void heom_batch_free(heom_batch* batch);
/* n_steps RK4 steps (forward or transposed generator) of states[i] (a state
 * of models[i]; all states in one precision), batched across instances. */
int heom_batch_propagate(heom_batch* batch, heom_state* const* states, int n_steps, int adjoint);
/* Third-order responses of every instance with the adjoint detection method
 * (see heom_response_2d), all propagations batched across instances.
 * rho_eq[i]: FP64 one-trajectory state of models[i]; R_out[i]: host
 * [n_t2][2][n1][n3] complex for instance i. */
int heom_batch_response_2d(heom_batch* batch, const heom_state* const* rho_eq, const heom_grid* grid,
                           int precision, double* const* R_out);
/* Launch form of a batch's RK4 stages:
 *   HEOM_BATCH_PER_CLASS: one persistent launch per size class and stage.
 *   HEOM_BATCH_SINGLE   : one persistent launch per stage over every class:
 *                         its workgroups are split among the classes in
 *                         proportion to matrices x time per matrix per
 *                         workgroup (measured by heom_batch_autotune, else
 *                         a model 4 + nb (nb + 1)); a workgroup runs the
 *                         item code of its class, with the LDS and width of
 *                         the widest class.  Needs every d <= 80
 *                         (HEOM_ERR_PARAM otherwise).
 *   HEOM_BATCH_AUTO     : the form heom_batch_autotune chose, per class
 *                         before any tuning (the default).
 * Both forms compute the same stages (results equal to rounding order). */
typedef enum {
  HEOM_BATCH_AUTO = 0,
  HEOM_BATCH_PER_CLASS = 1,
  HEOM_BATCH_SINGLE = 2
} heom_batch_launch;
int heom_batch_set_launch(heom_batch* batch, int launch);
/* The form HEOM_BATCH_AUTO resolves to now (or the one set). */
int heom_batch_get_launch(const heom_batch* batch, int* launch_out);
/* Replay every `steps` RK4 steps of a batched propagation as one captured HIP
 * graph (0: direct launches, the default).  A graph is captured per
 * propagation call on a private stream and replayed on the batch's stream;
 * if capture fails the batch falls back to direct launches. */
int heom_batch_set_graph_steps(heom_batch* batch, int steps);
/* Measure the launch forms on scratch states of n_traj trajectories per
 * instance (ground state, precision HEOM_FP32 or HEOM_FP64): each size class
 * alone in its launch shapes (heom_batch_get_class_shape; the fastest is
 * kept, and the LDS form's time per matrix per workgroup becomes the single
 * launch's work weight), then `reps` RK4 steps per class launches and, where
 * allowed, as single launches; HEOM_BATCH_AUTO then resolves to the faster.
 * ms_out (may be null): [per-class, single] milliseconds per RK4 step (NaN
 * when the single form is not allowed).  Allocates 3 x n_traj hierarchies per
 * instance for the duration of the call. */
int heom_batch_autotune(heom_batch* batch, int precision, int n_traj, int reps, double* ms_out);
/* Launch shape heom_batch_autotune chose for the per-class launch of size
 * class nb = ceil(d/16) (1..7): resident workgroups per CU (0: as many as LDS
 * and registers allow) and the neighbour-sum form (1: accumulated in LDS,
 * 0: in registers, -1: the class's only / default form).  The tuner times,
 * per class alone, the most and half the workgroups per CU with both forms
 * where both exist, and keeps the fastest. */
int heom_batch_get_class_shape(const heom_batch* batch, int nb, int* wg_per_cu, int* lds_sums);
/* Set that shape by hand (same meanings; lds_sums 0 or 1 only for the FP32
 * classes nb <= 4, which have both forms; FP64 batches always use the LDS
 * form).  HEOM_ERR_PARAM for values outside these ranges. */
int heom_batch_set_class_shape(heom_batch* batch, int nb, int wg_per_cu, int lds_sums);

/* ------------------------------------------------------ kernel choice -- */
/* Implementations of the fused RHS / RK4-stage kernel:
 *   HEOM_KERNEL_GENERIC : VALU kernel, one workgroup of 64/256 threads per
 *                         matrix, any d <= 128.
 *   HEOM_KERNEL_MFMA    : matrix-core kernel (v_mfma 16x16x4, persistent
 *                         workgroups of ceil(d/16) waves), d zero-padded to a
 *                         multiple of 16; compile-time mode shapes for
 *                         (4,4,5) levels in FP64 and (6) levels, runtime shape
 *                         otherwise.
 *   HEOM_KERNEL_MFMA_DYN: the matrix-core kernel with the runtime mode shape
 *                         even where a compile-time one exists.
 *   HEOM_KERNEL_KRON    : FP32 matrix-core kernel for three-mode models of
 *                         (4 or 5, 4, 4) levels (d = 64 or 80, e.g. the
 *                         water-like sym / asym stretch + bend model), one
 *                         wave per real plane of an output matrix; the mode
 *                         couplings contract in registers (Kronecker
 *                         structure of V_s, Eq. sys_interaction).  Such
 *                         models keep their device matrices in the basis
 *                         a = 16 a_S + 4 a_M + a_F (slow mode S of 4 or 5
 *                         levels); state upload / download convert from and
 *                         to the caller's basis (mode 0 slowest), so the
 *                         reordering is invisible at this interface.
 * (measured slower than HEOM_KERNEL_MFMA on MI355X at the three-mode depth-6
 * benchmark shape, so it is not the default; heom_autotune times it).
 *   HEOM_KERNEL_MFMA_GH : FP32 matrix-core kernel for d in 65..80 (five
 *                         16-row blocks) whose models keep at most 128
 *                         single-mode operator values: HEOM_KERNEL_MFMA's
 *                         algorithm with H read from its zero-padded global
 *                         copy (L1 / L2 resident) instead of an LDS plane,
 *                         so that three workgroups share a CU instead of two
 *                         (measured slower than HEOM_KERNEL_MFMA at the
 *                         three-mode depth-6 shape; heom_autotune times it).
 * Models start on HEOM_KERNEL_MFMA where it fits the LDS (FP32 d <= 112, FP64 d <= 80) and
 * every mode keeps at most 8 levels (the single-mode operators are staged in
 * 8 x 8 LDS slots), and on HEOM_KERNEL_GENERIC otherwise;
 * heom_model_set_kernel refuses a kernel outside these limits
 * (HEOM_ERR_PARAM), and heom_batch_create refuses models outside the
 * HEOM_KERNEL_MFMA limits.  heom_autotune measures the candidates. */
typedef enum {
  HEOM_KERNEL_AUTO = 0,
  HEOM_KERNEL_GENERIC = 1,
  HEOM_KERNEL_MFMA = 2,
  HEOM_KERNEL_MFMA_DYN = 3,
  HEOM_KERNEL_KRON = 4,
  HEOM_KERNEL_MFMA_GH = 5
} heom_kernel;
int heom_model_set_kernel(heom_model* model, int precision, int kernel);
int heom_model_get_kernel(const heom_model* model, int precision, int* kernel_out);
/* RK4 propagations of this model of at least `steps` steps replay a HIP graph
 * of `steps` captured RK4 steps (four stage launches each) instead of
 * launching every stage (Sec. III fixed-step integration, launch overhead
 * only).  0 turns graphs off.  Graphs are captured on a private stream per
 * (buffers, trajectories, generator, precision, kernel) and launched on the
 * model's stream.  Default 0.  Timing mode (heom_timing_enable) always
 * launches directly. */
int heom_model_set_graph_steps(heom_model* model, int steps);
/* Progress of long calls: while set, the batched t2 (and, for the direct
 * method, t3) propagations of heom_response_2d / heom_response_2d_pathways
 * ("t2 propagation", "t2/t3 propagation": steps counted over all trajectory
 * batches and pathways of the call) and the GMRES operator applications of
 * heom_equilibrate_krylov / heom_stationary_refine and of the stationary
 * term of heom_response_2d_vjp ("stationary solve": steps of all
 * applications, of at most max_applies x steps_per_apply), and the adjoint
 * sweeps of heom_response_2d_vjp ("gradient sweep": adjoint RK4 steps over
 * the t2 chunks and pathways, the t1 scans and the detection scan; reported
 * at the end of a checkpoint segment) synchronise the model's stream every
 * `every_steps` RK4 steps (at the next application or segment boundary) and
 * call fn(phase, steps_done, steps_total, ctx) on the calling thread.
 * fn = NULL or every_steps <= 0 turns it off (default).  The callback must
 * not call into this library. */
typedef void (*heom_progress_fn)(const char* phase, long long done, long long total, void* ctx);
int heom_model_set_progress(heom_model* model, heom_progress_fn fn, void* ctx, int every_steps);
/* Times every kernel variant that applies to the model (variants that would
 * run the same code are timed once) on a scratch batch of n_traj
 * trajectories in the given precision (one warm-up step, then reps RK4
 * steps each) and keeps the fastest for this model and precision.  ms_out
 * (may be NULL; HEOM_KERNEL_MFMA_GH + 1 entries) receives the measured time per
 * RK4 step indexed by heom_kernel, NaN for variants not timed.  The
 * previous choice is kept when an error occurs. */
int heom_autotune(heom_model* model, int n_traj, int precision, int reps, int* kernel_out,
                  double* ms_out);

/* ------------------------------------------------------- measurement -- */
/* While enabled, every launch of the fused RHS/RK4-stage kernel on this model
 * is bracketed by HIP events on the model's stream; heom_timing_read returns
 * the summed kernel time (ms), the number of launches and the number of
 * ADO-matrix updates they performed, then resets the counters. */
int heom_timing_enable(heom_model* model, int enable);
int heom_timing_read(heom_model* model, double* total_ms, long long* launches,
                     long long* ado_updates);

#ifdef __cplusplus
}
#endif
#endif /* HEOM2DVS_H */
