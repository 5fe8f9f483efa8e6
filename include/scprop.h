/*
 * scprop.h -- C ABI of libscprop: differentiable propagation of composite
 * superconducting-qubit systems on one MI355X (gfx950).
 *
 * What is computed (arXiv:2406.18155, SuperGrad):
 *   - single-mode Hamiltonians of transmons and fluxoniums, diagonalised and
 *     truncated to their lowest d levels (Sec. 3.1 fluxonium Hamiltonian;
 *     App. D step 1);
 *   - the composite Hamiltonian as a sum of local one- and two-body terms
 *     (Sec. 2.1, Hamiltonian decomposition; Sec. 3.1 multipath coupling) with
 *     microwave drives c(t) = E(t) cos(omega_d t + phase) on one operator of a
 *     mode (App. C, microwave control Hamiltonian);
 *   - the time-ordered propagator over a fixed step grid (Sec. 2.3), here by
 *     classical RK4 in the interaction picture of the frame
 *     H_f = sum_m diag(eps^f_m) (fixed at build), applied one mode's local
 *     operator at a time (App. B, contraction of local operators with the
 *     state tensor);
 *   - the gate fidelity F = |Tr(T^dag P U P)|^2 / d_c^2 (Sec. 4.1, composite
 *     state-transfer cost; App. D average fidelity);
 *   - the gradient of L = 1 - F w.r.t. pulse and device parameters by a
 *     discrete adjoint of the RK4 steps with checkpoints (Sec. 2.5, the
 *     per-step derivative sum and the chain rule for the costate).
 *
 * Units: energies and rates in rad/ns (GHz * 2 pi), times in ns, hbar = 1.
 *
 * State layout: a block of S columns, each a vector of D = prod_m d_m
 * complex amplitudes, column-major (column s starts at s*D).  Within a
 * column the index is sum_m a_m * stride_m with mode 0 slowest
 * (stride_m = prod_{m' > m} d_m').  Precision 0 stores complex64
 * (interleaved float re, im), precision 1 complex128.
 *
 * Conventions for every call:
 *   - the caller owns every buffer it passes (device pointers come from the
 *     caller's allocator, e.g. torch); ``scp_system`` owns its device tables
 *     and is freed by ``scp_destroy``;
 *   - ``stream`` is a hipStream_t passed as void* (NULL = default stream);
 *     device work is enqueued asynchronously on it; calls that return values
 *     through host pointers synchronise that stream first;
 *   - no C++ exception crosses the ABI; every call returns an scp_status and
 *     records a message readable with scp_last_error() on the same thread;
 *   - scp_propagate / scp_propagate_adjoint / scp_apply_generator /
 *     scp_fidelity allocate no device memory (the workspace is the caller's).
 */
#ifndef SCPROP_H
#define SCPROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SCP_OK = 0,
  SCP_EINVAL = -1,       /* invalid argument or unsupported shape */
  SCP_ENOMEM = -2,       /* device allocation failed (build only) */
  SCP_EDEGENERATE = -3,  /* a kept level is degenerate with another level */
  SCP_ENONFINITE = -4,   /* a result is NaN or Inf */
  SCP_EHIP = -5,         /* a HIP runtime call failed */
  SCP_EBUSY = -6         /* serving queue full / request refused */
} scp_status;

enum { SCP_MODE_TRANSMON = 0, SCP_MODE_FLUXONIUM = 1, SCP_MODE_RAW = 2 };
enum { SCP_OP_N = 0, SCP_OP_PHI = 1 };
enum {
  SCP_ENV_GAUSS = 0,        /* par[0] * exp(-(t-T/2)^2 / (2 sigma^2))           */
  SCP_ENV_GAUSS_BASIS = 1,  /* sum_j par[j] exp(-(t-t_j)^2/(2 sigma^2)),
                               t_j = (j+1/2) T / n_par                          */
  SCP_ENV_COS_RAMP = 2,     /* par[0]/2 * (1 - cos(2 pi t / T))  (App. C)       */
  SCP_ENV_CONST = 3,        /* par[0]                                            */
  SCP_ENV_PWC = 4           /* par[floor(step * n_par / n_steps)]: the piece of
                               the step being taken (all four stages)           */
};

#define SCP_MAX_TRUNC 8     /* largest per-mode truncation d                    */
#define SCP_MAX_MODES 16    /* largest number of modes                          */

/* One mode.  TRANSMON: charge basis of basis_dim = 2 ncut + 1 states,
 * H = 4 EC (n - ng)^2 - EJ cos(phi); operator n only.
 * FLUXONIUM: basis_dim harmonic-oscillator states of 4 EC n^2 + EL phi^2/2,
 * H = 4 EC n^2 + EL phi^2 / 2 - EJ cos(phi - phiext); operators n and phi.
 * RAW: trunc energies raw_eps and operators raw_ops given directly.
 * Frame energies (interaction picture) default to the dressed energies of
 * the mode as built; has_frame = 1 takes frame_eps instead (used to hold the
 * frame fixed while parameters move).
 *
 * Modes may have different truncations d_m.  The system then runs at d =
 * max d_m: a mode with fewer levels carries d - d_m inert levels (zero rows
 * and columns in n, phi and their derivatives; the open-system jump
 * operators only lower levels), so nothing ever enters them and the d_m
 * levels evolve exactly as in the product space of the modes' own
 * truncations.  Their energies continue the top level spacing.  Every index below (columns, rows, labels, matrix entries) is in
 * the uniform space: product state (a_0, ..., a_{n-1}) at sum_m a_m
 * d^(n-1-m). */
typedef struct {
  int32_t kind;        /* SCP_MODE_*                                           */
  int32_t basis_dim;   /* basis size before truncation (ignored for RAW)      */
  int32_t trunc;       /* d_m, 2..SCP_MAX_TRUNC; modes may differ (see below)  */
  int32_t has_frame;   /* 1: use frame_eps                                    */
  double EC, EJ, EL, ng, phiext;
  const double* raw_eps;  /* RAW: d energies (host)                            */
  const double* raw_ops;  /* RAW: [2][d][d][2] = op n then op phi, row-major,
                             (re, im) pairs (host); both Hermitian            */
  double frame_eps[SCP_MAX_TRUNC];
} scp_mode_desc;

/* + g * op_i(mode i) (x) op_j(mode j), i != j. */
typedef struct {
  int32_t i, j, op_i, op_j;
  double g;
} scp_coupling_desc;

/* c(t) = envelope(t; par) * cos(omega_d t + phase) multiplying op on mode.
 * has_omega = 0: omega_d = frame_eps[1] - frame_eps[0] of the mode. */
typedef struct {
  int32_t mode, op, env, n_par;
  int32_t has_omega;
  int32_t pad_;
  double omega_d, phase, sigma;
  const double* par;   /* n_par envelope parameters (host)                  */
} scp_drive_desc;

typedef struct {
  int32_t n_modes, n_couplings, n_drives, n_steps;
  double T;            /* pulse length; step h = T / n_steps                */
  const scp_mode_desc* modes;
  const scp_coupling_desc* couplings;
  const scp_drive_desc* drives;
} scp_system_desc;

typedef struct {
  int32_t n_cols;      /* S, number of propagated columns                   */
  int32_t precision;   /* 0: complex FP32 fused on-chip path;
                          1: complex FP64 plain path (one launch per term)  */
  int32_t ckpt_every;  /* checkpoint interval for the adjoint; 0 = ceil(sqrt(N)) */
  int32_t with_ckpt;   /* propagate: 1 = keep checkpoints in the workspace  */
  size_t workspace_bytes;  /* size of the workspace passed with these opts; a
                              call whose workspace_size exceeds it is refused
                              (SCP_EINVAL) before any launch               */
} scp_solve_opts;

typedef struct scp_system scp_system;

/* Build a system: single-mode builders, FP64 eigensolves on the GPU
 * (one workgroup per mode, cyclic Jacobi), dressed truncation with a fixed
 * eigenvector sign (largest-magnitude entry positive, ties to the lowest
 * basis index), frame energies, carriers, and the FP64-reduced phase and
 * drive tables of every RK4 stage time.  Synchronises ``stream``.
 * Errors: SCP_EINVAL (shape/field), SCP_EDEGENERATE (a kept level within
 * 1e-9 relative of another level), SCP_ENOMEM, SCP_EHIP. */
scp_status scp_build_system(const scp_system_desc* desc, void* stream, scp_system** out);

/* Sizes: D = d^n_modes, number of gradient parameters (order: drive
 * parameters in drive then par order; then (EJ, EC, EL) of every mode; then
 * coupling g in coupling order), dims (n_modes ints, nullable: the levels of
 * every mode in the index space, d for all). */
scp_status scp_system_info(const scp_system* sys, int64_t* D, int32_t* n_params,
                           int32_t* n_modes, int32_t* dims);

/* Dressed data of one mode as built (host FP64): eps[d] (ground
 * referenced), frame[d], ops[2][d][d][2] (n then phi; phi zero for
 * transmons), carrier omega of every drive (omega[n_drives], nullable). */
scp_status scp_system_mode(const scp_system* sys, int32_t mode, double* eps, double* frame,
                           double* ops);
scp_status scp_system_carriers(const scp_system* sys, double* omega);

/* Evaluation of the FP32 stage generator.  With D(t) = exp(i H_f t) the
 * interaction-picture generator is D(t) R(t) D(t)^dag, R the sum of the
 * un-rotated local terms (Sec. 2.1; App. B).  When every term of R is real --
 * each single-mode operator (with its parameter derivatives) real or i times
 * real, both factors of a coupling term of the same kind, drives on real
 * operators: transmon devices, and fluxonium devices with n(x)n and
 * phi(x)phi couplings and phi drives -- the FP32 path applies R with real
 * operators between diagonal rotations of the stage vectors (the "real
 * frame", *real_frame = 1); otherwise it applies the rotated complex
 * operators (*real_frame = 0).  Both evaluate the same map; they differ by
 * FP32 rounding.  scp_system_set_frame(sys, 0) makes a real-frame system use
 * the complex evaluation, 1 restores the real frame (SCP_EINVAL if the
 * system does not allow it).  Not while a call on the system is in flight;
 * synchronous. */
scp_status scp_system_frame(const scp_system* sys, int32_t* real_frame);
scp_status scp_system_set_frame(scp_system* sys, int32_t real_frame);

/* Engine of the FP32 solves (scp_propagate, scp_propagate_adjoint).
 * engine 1: the fused register-layout stepper (a column spread over the
 * threads of a workgroup, several modes per thread in registers; Sec. 2.1's
 * local terms at compile-time register positions).  engine 2: the gather
 * engine (one workgroup per column held in LDS, every thread evaluating the
 * generator on its own elements by gathering their neighbours along the
 * contracted digits), for devices with 64 <= D <= 4096 and at most 10 modes
 * whose stage tables fit in LDS; its adjoint needs in addition at most 16
 * drives on 10 distinct operators, 16 couplings and 16 operator slots, else
 * that solve runs on engine 1.  engine 0 (the default): engine 2 where it
 * runs and the columns would occupy fewer than 64 of engine 1's workgroups,
 * else engine 1.  Both engines compute the same RK4 steps and the same
 * discrete adjoint in FP32 with a compensated state; results differ by
 * rounding.  scp_system_set_engine: SCP_EINVAL for engine 2 on a device the
 * gather engine cannot run; a change forgets the recorded checkpoints.
 * scp_solve_engine writes (host) which engine a solve with opts (and the
 * adjoint if with_grad) runs on: 1 or 2 (0 for precision 1, the plain FP64
 * path).  Not while a call on the system is in flight. */
scp_status scp_system_set_engine(scp_system* sys, int32_t engine);
scp_status scp_solve_engine(const scp_system* sys, const scp_solve_opts* opts, int32_t with_grad,
                            int32_t* engine);

/* Kernel timing for measurement: with enable = 1 every later launch of the
 * fused forward (scp_propagate, and the forward inside scp_propagate_adjoint
 * when psi0 is given), of the segment recompute and of the reverse kernel
 * (scp_propagate_adjoint) on this system is bracketed by HIP events recorded
 * on its stream (the events are created per launch).  scp_system_kernel_times
 * waits for the recorded events and writes ms_out[3] (total milliseconds) and
 * counts[3] (launches) for the kinds forward, recompute, reverse since the
 * last read, then forgets them.  enable = 0 drops unread events.  Not with
 * scp_propagate_adjoint_noalloc (it refuses while timing is on). */
scp_status scp_system_set_timing(scp_system* sys, int32_t enable);
scp_status scp_system_kernel_times(scp_system* sys, double* ms_out, int32_t* counts);

/* Static spectrum (Sec. 3.2): the composite static Hamiltonian
 * H0 = sum_m diag(eps_m) + sum_e g_e A_i (x) B_j in the dressed single-mode
 * bases (drives excluded) is diagonalised in FP64 on the device by cyclic
 * Jacobi (D <= 2048; the matrix in LDS up to D = 96, in device memory above).
 * Every bare product state k (natural order, mode 0 slowest) is labelled
 * with the eigenvector of largest overlap |<k|v>|^2 (ties to the lowest
 * eigenvector index; labels are not forced to be distinct, so near a
 * degeneracy two bare states can share an eigenvector and zeta loses its
 * meaning).  scp_energy_tensor writes the labelled energies
 * E_out[k] (host, D doubles, rad/ns).  scp_static_zz writes the static
 * longitudinal coupling of modes (qi, qj) with every other mode in its
 * ground state, zeta = E(0) + E(1_i 1_j) - E(1_i) - E(1_j) (rad/ns), and
 * (grad_out, host, nullable, n_params doubles in the gradient order of
 * scp_system_info) d zeta / d theta from <v| dH0 |v> over the four levels
 * (Hellmann-Feynman; drive parameters get 0).  Both synchronise the stream
 * and allocate temporary device memory.  Errors: SCP_EINVAL (D > 2048, a
 * complex static Hamiltonian, a bad pair), SCP_ENONFINITE, SCP_EHIP. */
scp_status scp_energy_tensor(const scp_system* sys, double* E_out, void* stream);
scp_status scp_static_zz(const scp_system* sys, int32_t qi, int32_t qj, double* zeta_out,
                         double* grad_out, void* stream);

/* Workspace bytes a propagate (+ adjoint if with_grad) needs for opts. */
scp_status scp_workspace_size(const scp_system* sys, const scp_solve_opts* opts, int32_t with_grad,
                              size_t* bytes);

/* V(t) y for the stage time of (step, stage) (stage 0..3 at t_n + c h,
 * c = 0, 1/2, 1/2, 1): the interaction-picture generator applied to the
 * n_cols columns y (complex64, D x n_cols) into out.  FP32, the fused
 * stepper's applicator code with the rotated complex operators (its complex
 * evaluation; a real-frame system's stepper evaluates the same map with real
 * operators between frame rotations, see scp_system_frame). */
scp_status scp_apply_generator(const scp_system* sys, int32_t step, int32_t stage, const void* y,
                               void* out, int32_t n_cols, void* stream);

/* Propagate psi0 (D x S) over all n_steps RK4 steps into psiT.  With
 * opts->with_ckpt the states every ckpt_every steps are kept in the
 * workspace for scp_propagate_adjoint, and the system records which
 * workspace holds them for which (n_cols, ckpt_every, n_steps); a propagate
 * without checkpoints clears that record.  psi0 and psiT may alias.
 * Precision 0 runs on the engine scp_solve_engine names (the fused
 * register-layout stepper, or for few columns of a small device the gather
 * engine, one workgroup per column in LDS, with the same RK4 arithmetic:
 * compensated FP32 state, FP32 stage tables).  The workspace layout is the
 * engine's.  SCP_EINVAL if opts->workspace_bytes is below
 * scp_workspace_size(opts, with_grad = 0). */
scp_status scp_propagate(scp_system* sys, const scp_solve_opts* opts, void* workspace,
                         const void* psi0, void* psiT, void* stream);

/* Fidelity on the computational subspace: tau = sum_ij conj(T_ij)
 * U[comp_rows[i], comp_cols[j]] accumulated in FP64 on the device,
 * F = |tau|^2 / d_c^2.  U: D x S (precision 0 complex64, 1 complex128);
 * comp_rows (int64, d_c), comp_cols (int32, d_c), target (complex128,
 * d_c x d_c row-major) and tau_out (complex128, 1) are device pointers.
 * cotangent (nullable, same precision and shape as U) receives the
 * costate of L = 1 - F: -(tau/d_c^2) T_ij at (comp_rows[i], comp_cols[j]),
 * zero elsewhere.  F_out (host, nullable) synchronises the stream. */
scp_status scp_fidelity(const void* U, int64_t D, int32_t S, int32_t precision, int32_t d_c,
                        const int64_t* comp_rows, const int32_t* comp_cols, const void* target,
                        void* tau_out, void* cotangent, double* F_out, void* stream);

/* Composite state-transfer cost (Sec. 4.1, eq. for the composite state cost)
 * against full target states: tau = sum_j <phi_j | U[:, cols[j]]>,
 * accumulated in FP64 on the device by one workgroup in a fixed order
 * (deterministic), F = |tau|^2 / n_t^2, L = 1 - F.  U: D x S (precision 0
 * complex64, 1 complex128); cols (int32, n_t) and targets (complex128,
 * D x n_t column-major, phi_j = column j) and tau_out (complex128, 1) are
 * device pointers owned by the caller.  cotangent (nullable, same precision
 * and shape as U) receives the costate of L: -(tau/n_t^2) phi_j in column
 * cols[j], zero elsewhere (columns not named in cols included).  With
 * targets U_t|e_s> over a complete basis this is the gate fidelity of
 * scp_fidelity.  F_out (host, nullable) synchronises the stream.  A column
 * index outside [0, S) makes tau NaN (SCP_ENONFINITE when F_out is asked).
 * Errors: SCP_EINVAL, SCP_ENONFINITE, SCP_EHIP. */
scp_status scp_fidelity_states(const void* U, int64_t D, int32_t S, int32_t precision,
                               int32_t n_t, const int32_t* cols, const void* targets,
                               void* tau_out, void* cotangent, double* F_out, void* stream);

/* Fidelity with error-free single-qubit phase gates before and after the
 * gate (the compensation of App. D, restricted to Z rotations: virtual Z).
 * d_c = 2^n_qubits computational states, in binary order with qubit 0 most
 * significant (comp_rows / comp_cols as for scp_fidelity).  The block
 * M_ij = U[comp_rows[i], comp_cols[j]] is gathered on the device into
 * block_out (complex128, d_c x d_c row-major, device, caller-owned); on the
 * host the phases a (after the gate) and c (before it) that maximise |tau|,
 *   tau = sum_ij conj(T_ij) e^{i theta_i} M_ij e^{i chi_j},
 *   theta_i = sum_q a_q bit_q(i),  chi_j = sum_q c_q bit_q(j),
 * are found by coordinate ascent -- in turn a_0..a_{n-1}, then c_0..c_{n-1},
 * each phase is set to arg A - arg B where tau = A + e^{i p} B (B: the terms
 * whose bit of that qubit is set), until |tau| grows by at most 1e-14
 * relative or after 200 sweeps -- from each of a fixed set of starts, keeping
 * the largest |tau|: zero for one qubit; for more, 16 starts, start k with
 * a_q = 2 pi frac(k (q + 1) g), c_q = 2 pi frac(k (n + q + 1) g),
 * g = 0.6180339887498949.  F_out (host, required) =
 * |tau|^2 / d_c^2; phases_out (host, 2 n_qubits, nullable): a then c;
 * tau_out (device complex128, nullable).  cotangent (nullable, as for
 * scp_fidelity) receives the costate of L = 1 - F at the optimum,
 * -(tau/d_c^2) T_ij e^{-i theta_i} e^{-i chi_j} (the phases are stationary
 * there, so scp_propagate_adjoint then gives dL/dtheta of the compensated
 * loss).  target is a device pointer as for scp_fidelity.  Synchronises the
 * stream.  n_qubits: 1..6.  Errors: SCP_EINVAL, SCP_ENONFINITE, SCP_EHIP. */
scp_status scp_fidelity_zcomp(const void* U, int64_t D, int32_t S, int32_t precision,
                              int32_t n_qubits, const int64_t* comp_rows, const int32_t* comp_cols,
                              const void* target, void* block_out, void* tau_out, double* F_out,
                              double* phases_out, void* cotangent, void* stream);

/* Multi-qubit eigenbasis (App. D, eq. for the basis transform U -> V^dag U V):
 * the static Hamiltonian H0 of scp_energy_tensor is diagonalised (FP64,
 * device) and each bare product state labels[j] (host int64, n of them) takes
 * the eigenvector v_j of largest overlap |<k|v>|^2, its phase fixed by
 * <labels[j]|v_j> > 0, with energy E_j (E_out, host, nullable).  The
 * eigenbasis unitary is read in the frame of the dressed energies,
 * M_ij = exp(i E_i T) <v_i|U_lab|v_j> = <w_i|psi_I,j(T)> for the columns
 * psi_j(0) = v_j propagated by scp_propagate, with
 * w_i = exp(i (H_f - E_i) T) v_i (H_f the frame of the propagation).
 * Outputs (device, caller-owned, D x n column-major): psi0_out, the v_j in
 * complex64 (precision 0) or complex128 (1), to propagate; W_out (complex128,
 * nullable) the w_i; phi_out (complex128, nullable; needs target, host
 * complex128 n x n row-major as (re, im) pairs) the target states
 * phi_j = sum_i T_ij w_i, so that scp_fidelity_states of the propagated
 * columns against phi is the eigenbasis gate fidelity |Tr(T^dag M)|^2 / n^2.
 * The basis and energies are those of the system as built (held fixed when
 * parameters move, like the frame).  Synchronises the stream; allocates
 * temporary device memory.  Errors: SCP_EINVAL (as scp_energy_tensor, a
 * label out of range), SCP_ENONFINITE, SCP_EHIP. */
scp_status scp_eigenbasis_states(const scp_system* sys, int32_t n, const int64_t* labels,
                                 const double* target, double T, int32_t precision,
                                 void* psi0_out, void* phi_out, void* W_out, double* E_out,
                                 void* stream);

/* Fidelity with error-free single-qubit gates before and after the gate
 * (App. D step 6), in the product basis or an eigenbasis.  The d_c x d_c
 * block (d_c = 2^n_qubits, qubit 0 most significant) is
 * M_ij = <w_i | U[:, cols[j]]> for W (device complex128, D x d_c: the w_i of
 * scp_eigenbasis_states), or M_ij = U[comp_rows[i], cols[j]] when W is NULL;
 * FP64 on the device.  On the host the gates maximising
 * |tau| = |Tr(T^dag A M B)| are sought by coordinate ascent from the
 * identity: mode 1, Z rotations (the phases of scp_fidelity_zcomp);
 * mode 2, arbitrary single-qubit unitaries A = (x)a_q, B = (x)b_q, each set
 * in turn to the polar optimum of its partial trace, sweeps until |tau| grows
 * by at most 1e-14 relative or 500 sweeps (a local search: it reaches the
 * maximum for CZ, CNOT and product targets, not always for generic entangling
 * ones).  F_out (host, required) = |tau|^2 / d_c^2; params_out (host,
 * nullable): mode 1, a then c phases (2 n doubles); mode 2, a_0..a_{n-1} then
 * b_0..b_{n-1}, each 2 x 2 row-major as (re, im) pairs (16 n doubles).
 * block_out (device complex128, 2 d_c^2, caller-owned): M, then the
 * compensated target T' = A^dag T B^dag.  cotangent (nullable, as U): the
 * costate of L = 1 - F at the optimum, -(tau/d_c^2) sum_i T'_ij w_i in column
 * cols[j] (at the computational rows without W), zero elsewhere; the gates
 * are stationary there, so scp_propagate_adjoint gives dL/dtheta of the
 * compensated loss.  target: device complex128 d_c x d_c.  Synchronises the
 * stream.  Errors: SCP_EINVAL (n_qubits outside 1..6, mode), SCP_ENONFINITE,
 * SCP_EHIP. */
scp_status scp_fidelity_local(const void* U, int64_t D, int32_t S, int32_t precision,
                              int32_t n_qubits, const int32_t* cols, const void* W,
                              const int64_t* comp_rows, const void* target, int32_t mode,
                              void* block_out, void* tau_out, double* F_out, double* params_out,
                              void* cotangent, void* stream);

/* Gradient of L w.r.t. every parameter (host FP64, n_params entries in the
 * order of scp_system_info), given the costate cotangent = dL/dU* of the final
 * state (D x S complex64, device).  The discrete adjoint of Sec. 2.5 (the
 * per-step derivative sum and the costate chain rule) walks the checkpoint
 * segments back, recomputing each segment's states, on the engine
 * scp_solve_engine(opts, with_grad = 1) names.  The gather engine walks one
 * segment per launch while other workgroups of the same launch recompute the
 * next segment's states (two stage-input buffers); its per-stage sums are
 * folded in a fixed order, so both engines' gradients are deterministic.
 *   psi0 != NULL: the checkpoints are first computed here by a forward
 *     propagation of psi0 (D x S complex64, device) into the workspace;
 *   psi0 == NULL: the checkpoints of the system's most recent scp_propagate
 *     are used; it must have run with with_ckpt = 1 on this workspace with the
 *     same n_cols and ckpt_every, and no propagate without checkpoints (nor a
 *     frame or engine switch) may have come after it on this system, nor a propagate of
 *     another system on this workspace pointer.  Otherwise SCP_EINVAL, before
 *     any launch.
 * The checkpoints stay valid, so several cotangents may follow one forward.
 * SCP_EINVAL if opts->workspace_bytes is below scp_workspace_size(opts,
 * with_grad = 1).  Synchronises ``stream``.  SCP_ENONFINITE if any gradient
 * entry is not finite. */
scp_status scp_propagate_adjoint(scp_system* sys, const scp_solve_opts* opts, void* workspace,
                                 const void* psi0, const void* cotangent, double* grad_out,
                                 void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * gradient of scp_propagate_adjoint with psi0 given, with the workspace taken
 * from a static device array of SCP_NOALLOC_SCRATCH_BYTES = 64 MiB (each GPU
 * holds its own copy until the process ends) instead of a caller buffer.
 * psi0 (D x S complex64) and cotangent (D x S complex64) are device pointers;
 * opts->workspace_bytes is ignored.  The forward with checkpoints, the
 * segment recomputations and the reverse walk all run in the static array;
 * no device memory is allocated.  SCP_EINVAL if scp_workspace_size(opts,
 * with_grad = 1) exceeds 64 MiB (e.g. the 4-fluxonium chain, D = 625,
 * 16 columns, 5000 steps, needs about 35 MB; 256 columns of D = 6561 do not
 * fit).  Every call on one GPU uses that GPU's one array, so calls that
 * overlap on one GPU (other streams or threads) race and must be serialised
 * by the caller.  It always runs the register-layout engine (engine 1 of
 * scp_system_set_engine).  Synchronises ``stream``; results are bitwise those
 * of scp_propagate_adjoint with psi0 on that engine. */
scp_status scp_propagate_adjoint_noalloc(scp_system* sys, const scp_solve_opts* opts,
                                         const void* psi0, const void* cotangent,
                                         double* grad_out, void* stream);

/* Contraction probe (measurement only; no solve uses it).  The inner
 * operation of the register-layout stepper at d = 3 -- a uniform complex 3 x 3
 * operator applied to the 9 fibres of the 27 amplitudes each lane holds, the
 * result accumulated -- in form 0 (VALU FMAs with the operator in scalar
 * registers: the stepper's form), form 1 (v_mfma_f32_4x4x1f32 on the real
 * 6 x 6 form padded to two 4-row blocks, with the per-application operand
 * builds and register moves the stepper's layout would need) or form 2 (the
 * same MFMAs with the operands built once and the accumulators left in
 * place).  n_wg workgroups of 256 threads each run `iters` applications;
 * application i uses operator i % nop of ops (device, nop x 18 floats: the
 * real parts of the 9 entries row-major, then the imaginary parts; form 2
 * uses operator 0 throughout).  out (device, n_wg * 256 floats) receives each
 * lane's sum of its outputs (real parts + imaginary parts / 2).  Asynchronous
 * on stream.  Errors: SCP_EINVAL, SCP_EHIP. */
scp_status scp_probe_contraction(int32_t form, int32_t n_wg, int32_t iters, int32_t nop,
                                 const void* ops, void* out, void* stream);

/* ------------------------------------------------------------------------
 * Suzuki-Trotter product formulas (Sec. 2.3 Trotterization solver, App. A).
 *
 * The step propagator is a product of exponentials of local terms, in this
 * order: one single-mode term per mode (lab frame),
 *   H_m(t) = diag(eps_m) + sum_{drives k on m} c_k(t) O_k,
 * then one two-body term g_e A_i (x) B_j per coupling.  Q1 applies
 * exp(-i H_k dt) for k = 1..K; the symmetric piece Q2(a dt) applies
 * exp(-i a H_k dt/2) for k = 1..K and then k = K..1; Q2 is one piece with
 * a = 1, Q4 the pieces a = (p, 1-2p, p) with p = 1/(2 - 2^(1/3)), Q4J the
 * pieces a = (p, conj p) with p = (3 - i sqrt 3)/6.  Time-dependent terms
 * are frozen at the middle of their piece (Q4J: of the step).  Q4J is not
 * unitary; as printed it is third order for static terms and second order
 * for driven ones (Q1: first, Q2: second, Q4: fourth).
 * ------------------------------------------------------------------------ */
enum { SCP_TROTTER_Q1 = 0, SCP_TROTTER_Q2 = 1, SCP_TROTTER_Q4 = 2, SCP_TROTTER_Q4J = 3 };

/* Device workspace bytes of scp_propagate_trotter: inputs, the pair gates
 * of every (piece, coupling), the single-mode gates of every (step, piece,
 * mode) and the fused operations (adjacent couplings on one mode pair, and
 * for small D the single-mode gates joined to them) of every (step, piece,
 * pass), all complex FP64.  Grows linearly with n_steps.  SCP_EINVAL for an unknown order or a
 * system outside the path's limits (d = 2..5, 16 D bytes <= 160 KiB,
 * <= 48 couplings, <= 32 drives). */
scp_status scp_trotter_workspace_size(const scp_system* sys, int32_t order, size_t* bytes);

/* Propagate the n_cols columns psi0 (device, complex128, D x n_cols
 * column-major) over the system's n_steps steps of dt = T / n_steps with
 * the product formula ``order`` into psiT (same layout; may alias psi0).
 * Everything is complex FP64 on the device: the gates are formed by Taylor
 * scaling and squaring and fused (the result is the same product up to
 * rounding), and one workgroup per column keeps the column in LDS.  The result is rotated into the frame of scp_propagate,
 * psi_I(T) = exp(i H_f T) psi_lab(T), so both paths compare directly.
 * workspace: device, scp_trotter_workspace_size bytes, caller-owned.
 * Synchronises the stream once, before the first kernel (upload of the
 * inputs).  Errors: SCP_EINVAL, SCP_EHIP. */
scp_status scp_propagate_trotter(scp_system* sys, int32_t order, int32_t n_cols, void* workspace,
                                 const void* psi0, void* psiT, void* stream);

/* Local continuous adjoint method (LCAM) of the product formulas (Sec. 2.5,
 * continuous adjoint method: eqs. for the derivative sum and its i-th term,
 * the costate chain rule a_i = U_{i+1}^T a_{i+1}).  The gradient of L w.r.t.
 * every parameter (host FP64, n_params entries in the order of
 * scp_system_info) for the costate cotangent = dL/dpsi_I(T)* (device,
 * complex128, D x n_cols) of the columns psi0 (device, complex128, D x
 * n_cols) propagated by scp_propagate_trotter with the same order.  Only the
 * final state of the forward is kept: the walk back recovers every earlier
 * state by evolving backward in time (G^-1 of each gate) while the costate
 * moves by G^dag, and every gate contributes 2 Re <mu, dG/dtheta phi>
 * through its local reduced matrix and the Frechet derivative of its
 * exponential.  Complex FP64 throughout; the frame and the carriers are held
 * fixed.  The result is bitwise reproducible (no atomics).
 * workspace: device, scp_trotter_adjoint_workspace_size(order, n_cols) bytes
 * (the forward's gate tables, one column state and costate per column, the
 * inverse and adjoint gate tables, per-column local sums for a chunk of 128
 * steps); workspace_bytes is its size.  Synchronises the stream.
 * SCP_EINVAL (as scp_trotter_workspace_size, and for 16 (2 D + 512) bytes >
 * 160 KiB: a column and its costate live in LDS), SCP_ENONFINITE, SCP_EHIP. */
scp_status scp_trotter_adjoint_workspace_size(const scp_system* sys, int32_t order, int32_t n_cols,
                                              size_t* bytes);
scp_status scp_propagate_trotter_adjoint(scp_system* sys, int32_t order, int32_t n_cols,
                                         void* workspace, size_t workspace_bytes, const void* psi0,
                                         const void* cotangent, double* grad_out, void* stream);

/* The same LCAM gradient (Sec. 2.5) started from the forward's final state
 * instead of its initial one: psiT (device, complex128, D x n_cols) is what
 * scp_propagate_trotter returned for these columns with the same order, and
 * the walk back begins there (the method needs only psi(T) and the costate at
 * T).  The internal forward of scp_propagate_trotter_adjoint is skipped; the
 * gate tables are rebuilt.  With psiT equal to that forward's result, the
 * gradient is bitwise that of scp_propagate_trotter_adjoint.  Arguments,
 * workspace size, synchronisation and errors as scp_propagate_trotter_adjoint;
 * psiT is only read. */
scp_status scp_propagate_trotter_adjoint_final(scp_system* sys, int32_t order, int32_t n_cols,
                                               void* workspace, size_t workspace_bytes,
                                               const void* psiT, const void* cotangent,
                                               double* grad_out, void* stream);

void scp_destroy(scp_system* sys);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of propagation / gradient requests.
 *
 * Requests queue on the host and are admitted in arrival order while their
 * device footprint (stage tables, states, checkpoints, adjoint buffers) fits
 * hbm_budget_bytes and fewer than max_active requests run.  Each
 * scp_server_step is one tick: admit, advance every running request by one
 * chunk (forward steps, then adjoint segments) with one batched launch per
 * size class (d, register modes, pair terms per position), reduce fidelities,
 * finish gradients, release memory.  With scp_server_set_engine(sv, 0 or 2),
 * requests the gather engine would run (few columns of a small device, as for
 * scp_system_set_engine) are batched per (d, modes) on the gather engine
 * instead, when their workspace fits the budget beside what is admitted: per
 * tick one launch of every such request's step range of the forward (its
 * compensated state saved between chunks) and per round one launch of the
 * next segment of every such request's reverse walk.  The server starts with
 * engine 1 (the register-layout kernels), which gives the higher throughput
 * on a saturated mix.  Work per tick
 * per workgroup is about chunk_work cost units (0 = default).  A request's
 * result is bitwise the same whether it runs alone or among others, and the
 * same as scp_propagate / scp_propagate_adjoint on the same engine.  The server allocates device memory
 * (at admission); it is not for callers that cannot allocate.
 * ------------------------------------------------------------------------ */
typedef struct scp_server scp_server;

enum { SCP_REQ_QUEUED = 0, SCP_REQ_RUNNING = 1, SCP_REQ_DONE = 2, SCP_REQ_FAILED = 3 };

scp_status scp_server_create(size_t hbm_budget_bytes, int32_t max_active, double chunk_work,
                             void* stream, scp_server** out);

/* Queue one request: the system description (deep-copied), the basis index of
 * each propagated column (host, n_cols), the computational rows (host int64,
 * d_c) and columns (host int32 positions in [0, n_cols), d_c), the target
 * (host complex128, d_c x d_c row-major as (re, im) pairs) and whether the
 * gradient is wanted.  SCP_EBUSY if the request alone exceeds the budget. */
scp_status scp_server_submit(scp_server* sv, const scp_system_desc* desc, const int64_t* columns,
                             int32_t n_cols, const int64_t* comp_rows, const int32_t* comp_cols,
                             int32_t d_c, const double* target, int32_t want_grad,
                             int64_t* id_out);

/* Device footprint the server reserves for a request (admission unit). */
scp_status scp_request_bytes(const scp_system_desc* desc, int32_t n_cols, int32_t want_grad,
                             size_t* bytes);

/* One tick.  Size classes run concurrently on the server's four worker
 * streams (created with the server, default priority); the tick ends by
 * synchronising them.  Admission builds run on the stream given at creation. */
scp_status scp_server_step(scp_server* sv, int32_t* n_active, int32_t* n_queued);

/* State (SCP_REQ_*), fidelity, gradient (n_params entries when done, order
 * as scp_system_info; nullable) and the submit / admit / completion times in
 * seconds since the server was created. */
scp_status scp_server_result(scp_server* sv, int64_t id, int32_t* state, double* F, double* grad,
                             int32_t* n_params, double* t_submit, double* t_admit,
                             double* t_done);

/* Engine of later admissions: 0 automatic (as scp_system_set_engine), 1 the
 * register-layout kernels only (the default), 2 the gather engine wherever it
 * runs.  SCP_EINVAL otherwise. */
scp_status scp_server_set_engine(scp_server* sv, int32_t engine);

void scp_server_destroy(scp_server* sv);

/* ------------------------------------------------------------------------
 * Open systems: the vectorised Lindblad master equation (the superoperator
 * of App. D's closing remark on the average fidelity; the LindbladObj
 * component of Sec. 2).
 *
 * A density matrix rho (D x D) evolves in the interaction picture of the
 * system's frame under
 *   d rho/dt = -i [V(t), rho] + sum_m gamma1_m D[a_m(t)] rho
 *                             + 2 gammaphi_m D[n_m] rho,
 * D[L] rho = L rho L^dag - {L^dag L, rho}/2, V(t) the generator of
 * scp_propagate, a_m = sum_k sqrt(k) |k-1><k| and n_m = diag(0..d-1) in mode
 * m's dressed basis (a_m rotated into the frame), so an idle mode's excited
 * population decays as exp(-gamma1 t) and its 0-1 coherence as
 * exp(-gammaphi t).  Classical RK4 on the system's step grid, complex FP32
 * with a compensated (two-word) state, one workgroup per matrix with the
 * matrix resident in LDS: D^2 <= 6561 (d = 2: N <= 5, d = 3: N <= 4,
 * d = 4: N <= 3, d = 5: N <= 2), d the largest truncation (see
 * scp_mode_desc).
 * ------------------------------------------------------------------------ */

/* Device workspace bytes of scp_propagate_lindblad (a small argument block
 * and the relaxation phases of every half-step). */
scp_status scp_lindblad_workspace_size(const scp_system* sys, size_t* bytes);

/* Propagate n_cols density matrices rho0 (device, complex64, n_cols x D x D,
 * each row-major: element (A, B) at A * D + B, A the ket and B the bra
 * index in the system's basis order) over the system's steps into rhoT (same
 * layout, must not alias rho0).  gamma1, gammaphi: host, n_modes rates in
 * 1/ns each (nullable: zero), finite and >= 0.  workspace: device,
 * scp_lindblad_workspace_size bytes, caller-owned.  Asynchronous on stream.
 * Errors: SCP_EINVAL (unsupported shape, bad rates, small workspace), SCP_EHIP. */
scp_status scp_propagate_lindblad(scp_system* sys, const double* gamma1, const double* gammaphi,
                                  int32_t n_cols, void* workspace, size_t workspace_bytes,
                                  const void* rho0, void* rhoT, void* stream);

/* Device workspace bytes of scp_lindblad_adjoint for n_cols matrices: the
 * stage tables, checkpoints (hi and lo words) every ceil(sqrt(n_steps))
 * steps, one segment of stage inputs and the costate, per matrix. */
scp_status scp_lindblad_adjoint_workspace_size(const scp_system* sys, int32_t n_cols,
                                               size_t* bytes);

/* Gradient of a loss of the propagated density matrices by the discrete
 * adjoint of the Lindblad RK4 steps (the closed system's adjoint, Sec. 2.5,
 * carried over to open systems as App. D's closing remark says): given the
 * cotangent of rhoT (device, complex64, as rho0; convention
 * dLoss = 2 Re sum conj(cotangent) d rhoT, e.g. scp_fidelity_channel's),
 * grad_out (host) receives dLoss/dtheta for, in this order, the drive
 * parameters (drive order, then parameter order), the coupling strengths,
 * then (gamma1_m, gammaphi_m) of every mode: n_pulse + n_couplings + 2 n_modes
 * values.  The device parameters (E_J, E_C, E_L) are not differentiated here.
 * The forward is recomputed from rho0 with checkpoints, then each
 * checkpoint segment is recomputed (its stage inputs stored) and walked in
 * reverse, one workgroup per matrix; per-matrix FP64 partial sums are added
 * on the host in a fixed order.  rho0, gamma1, gammaphi as for
 * scp_propagate_lindblad.  Synchronises the stream.  Errors: SCP_EINVAL
 * (shape, rates, workspace, more than 10 drive operators, 16 drives or 16
 * couplings), SCP_ENONFINITE, SCP_EHIP. */
scp_status scp_lindblad_adjoint(scp_system* sys, const double* gamma1, const double* gammaphi,
                                int32_t n_cols, void* workspace, size_t workspace_bytes,
                                const void* rho0, const void* cotangent, double* grad_out,
                                void* stream);

/* Average gate fidelity of a channel on the computational subspace (App. D,
 * eq. for the average fidelity, with a unitary operator basis normalised to
 * tr(U_j^dag U_k) = d_c delta_jk): rhoT (device, complex64, d_c^2 x D x D)
 * holds the images of the matrix units |s_a><s_b| of the d_c input states
 * in the order a * d_c + b;
 *   ov = sum_ab sum_ij conj(T_ia) T_jb rhoT_ab[comp_rows[i], comp_rows[j]]
 * is accumulated in FP64 by one workgroup in a fixed order and
 * F = (Re ov + d_c) / (d_c (d_c + 1)); for a unitary channel W this is
 * (|Tr(T^dag W)|^2 + d_c) / (d_c (d_c + 1)).  comp_rows (int64, d_c), target
 * (complex128, d_c x d_c row-major T[i][a]) and overlap_out (complex128, 1)
 * are device pointers.  cotangent (nullable, complex64, as rhoT) receives the
 * costate of L = 1 - F, -T_ia conj(T_jb) / (2 d_c (d_c + 1)) at
 * (a * d_c + b, comp_rows[i], comp_rows[j]) and zero elsewhere.  F_out (host,
 * nullable) synchronises the stream.  Errors: SCP_EINVAL, SCP_ENONFINITE,
 * SCP_EHIP. */
scp_status scp_fidelity_channel(const void* rhoT, int64_t D, int32_t d_c, const int64_t* comp_rows,
                                const void* target, void* overlap_out, void* cotangent,
                                double* F_out, void* stream);

/* Message of the last failing call on this thread ("" if none); valid until
 * the next call on this thread. */
const char* scp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SCPROP_H */
