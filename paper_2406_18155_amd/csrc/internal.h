// Internal structures of libscprop (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/scprop.h"

namespace scp {

using cplx = std::complex<double>;

constexpr int MAXL = 8;        // layouts per stage
constexpr int MAXRB = 64;      // register block (complex amplitudes per thread per vector)
constexpr int MAXSLOTS = 48;   // (mode, op) slots
constexpr int MAXPAIRS = 48;   // (first slot, partner mode) pairs
constexpr int MAXGROUPS = 48;
constexpr int MAXPULSE = 256;  // pulse parameters
constexpr int WG_THREADS = 256;

// Canonical per-layout term list: every pair term has its first factor at
// register position p and its partner at p + 1 (layouts are ordered along
// paths of the coupling graph).  Absent entries point at a zero operator.
struct CPair {
  int32_t slot, pair, cidx, mode_i, mode_j;   // cidx < 0: no drive attached
  int32_t hsign;   // real frame: kappa^2 of the item's kind (the first-factor folds' sign)
};
struct CSingle {
  int32_t slot, cidx;
};

struct DriveDev {          // one drive in the device plan
  int32_t slot, cidx, par0, npar;   // slot of its operator, c-table column, first pulse param
};

struct Plan {
  int32_t d, N, NR, RB, TPC, CPW, WG, D, L, NT;
  int32_t nslots, npairs, ngroups, ndrives, npulse, ncoup;
  int32_t nsteps;
  float h;
  int32_t block_q;       // floats2 per half-step block in the op table
  int32_t off_pair;      // offset (complex) of pair ops inside a half-step block
  int32_t off_dslot;     // offset of slot derivative ops (3 per slot)
  int32_t has_delta;
  int32_t reg_off[MAXL][MAXRB];
  int32_t reg_stride[MAXL][8];   // natural-order stride of the mode at each register position
  int32_t tstride[MAXL][16];
  float delta[17][8];          // eps - frame per mode (FP32); row 16 is zero
  int32_t slot_mode[MAXSLOTS];
  int32_t slot_op[MAXSLOTS];
  float coup_g[MAXPAIRS];
  int32_t coup_slot_i[MAXPAIRS], coup_slot_j[MAXPAIRS];
  DriveDev drives[MAXGROUPS];
  int32_t layout_of_mode[16];  // a layout whose register modes contain the mode
  int32_t pos_of_mode[16];     // its register position there
  int32_t pair_ncoup[MAXPAIRS];
  int32_t pair_coup[MAXPAIRS][4];  // couplings summed into each pair operator
  int32_t pair_pslot[MAXPAIRS][4]; // their partner-side operator slots
  int32_t MP;                      // pair terms per position pair (compile-time variant)
  CPair cpair[MAXL][4][2];         // [layout][p][m]
  int32_t has_single[MAXL];
  CSingle csingle[MAXL][8];        // drive-only terms at position p
  int32_t has_diag[MAXL];
  int32_t cdiag[MAXL][8];          // mode of the diagonal term at position p (16: none)
  int32_t has_mode_pass[MAXL];
  int32_t mode_pass[MAXL][8];      // adjoint: single-mode sensitivities of this mode at p (-1: none)
  float deps[16][3][8];            // d eps / d(EJ, EC, EL) per mode
  int32_t lmode[MAXL][8];          // mode at each register position of each layout (-1: none)
  int32_t mdrv_off[17];            // drives of mode m: mdrv[mdrv_off[m] .. mdrv_off[m+1])
  int32_t mdrv[MAXGROUPS];         // drive indices grouped by mode
  int32_t mdrv_first[MAXGROUPS];   // 1: first drive on its operator slot
  int32_t nacc;                    // gradient accumulators: npulse + 3 N + ncoup
  // Real frame (every term a real operator: each operator is real or i times
  // real, both factors of a pair term of one kind, drives on real operators):
  // the stepper applies the un-rotated real operators between the diagonal
  // frame rotations of y and k, whose phases come from a per-half-step table
  // with ph_row entries (a multiple of 8): the RB register phases of the base
  // layout, then from ph_thr the NT * d thread-position phases.
  int32_t real_frame;
  int32_t ph_row, ph_thr;
};

// Work descriptor of one workgroup of a (possibly batched) forward launch:
// CPW columns (column block cb) of one system for steps [n0, n1).
struct FwdItem {
  const Plan* P;
  const float2* optab;
  const float* ctab;
  const float2* psi0;   // non-null: start from psi0 (natural order), lo = 0
  float2* psiT;         // non-null: write hi + lo (natural order) at the end
  float2* state_hi;     // register-order continuation state (nullable)
  float2* lo;           // register-order compensation slices
  float4* ckpt;         // nullable
  const float4* ckin;   // recompute: start from this checkpoint slab (hi, lo; register order)
  float2* ystore;       // recompute: stage inputs, natural order, 4 S D per step
  const float2* ph;     // real frame: phase table [2N+1][ph_row] (else unused)
  const float* rops;    // real frame: the un-rotated operators (real parts, block layout)
  int ce, S, cb, n0, n1, pad;
};

// Work descriptor of one workgroup of a (possibly batched) adjoint launch:
// segment seg_hi (= seg_lo) of column block cb, whose stage inputs a recompute
// launch has just written to segbuf.
struct AdjItem {
  const Plan* P;
  const float2* optab;
  const float* ctab;
  const float* dctab;
  const float4* ckpt;
  const float2* lamT;   // cotangent (natural order), read when first != 0
  float2* segbuf;
  float2* lamlo;        // register-order compensation word of the costate
  float2* sum;
  float2* lamstate;     // register-order costate carried between launches
  double* part;         // [column block][4 waves][nacc] FP64 accumulators
  const float2* ph;     // real frame: phase table (as in FwdItem)
  const float* rops;    // real frame: un-rotated operators and their derivatives
  int ce, nckpt, S, cb, seg_hi, seg_lo, first, pad;
};

struct ModeData {
  int kind = 0, K = 0, d = 0;
  double EC = 0, EJ = 0, EL = 0, ng = 0, phiext = 0;
  bool has_phi = false;
  std::vector<double> H;             // K*K row-major basis Hamiltonian
  std::vector<double> dH[3];         // d/d(EJ, EC, EL)
  std::vector<cplx> opB[2];          // basis operators n, phi (K*K)
  std::vector<cplx> dopB[3][2];      // their derivatives
  std::vector<double> w, V;          // eigenvalues (K), eigenvectors column a at V[k*K + a]
  double eps[SCP_MAX_TRUNC] = {0}, frame[SCP_MAX_TRUNC] = {0};
  cplx ops[2][SCP_MAX_TRUNC * SCP_MAX_TRUNC];
  double deps[3][SCP_MAX_TRUNC] = {{0}};
  cplx dops[3][2][SCP_MAX_TRUNC * SCP_MAX_TRUNC];
};

struct Coupling { int i, j, op_i, op_j; double g; };

// Basis function i of a drive envelope at time t of step n (App. C pulse
// shapes): the envelope is sum_i par_i * envelope_basis(.., i, ..).
__host__ __device__ inline double envelope_basis(int env, int i, int npar, long n, int nsteps,
                                                 double t, double T, double sigma) {
  if (env == SCP_ENV_GAUSS) {
    const double u = (t - 0.5 * T) / sigma;
    return exp(-0.5 * u * u);
  }
  if (env == SCP_ENV_GAUSS_BASIS) {
    const double u = (t - (i + 0.5) * T / npar) / sigma;
    return exp(-0.5 * u * u);
  }
  if (env == SCP_ENV_COS_RAMP) return 0.5 * (1.0 - cos(6.283185307179586476925286766559 * t / T));
  if (env == SCP_ENV_CONST) return 1.0;
  const long piece = (n * npar) / nsteps;   // SCP_ENV_PWC: the piece of step n
  return (piece == i) ? 1.0 : 0.0;
}
struct Drive {
  int mode, op, env;
  double omega, phase, sigma;
  std::vector<double> par;
};

}  // namespace scp

struct scp_system {
  int n_modes = 0, d = 0, n_steps = 0;
  int64_t D = 0;
  double T = 0, h = 0;
  std::vector<scp::ModeData> modes;
  std::vector<scp::Coupling> coup;
  std::vector<scp::Drive> drives;
  int n_params = 0, n_pulse = 0;
  // slots / pairs / groups (host copies used by gradient assembly)
  std::vector<int> slot_mode, slot_op;
  std::vector<scp::cplx> pairW_host;   // static pair operators sum g O_j (d*d each)
  std::vector<int> pair_mode_host;
  std::vector<int> slot_imag;          // real frame: slot operator (and derivatives) i * real
  std::vector<int> pair_imag;          // real frame: pair operator i * real (table sign -1)
  scp::Plan plan;
  // device
  scp::Plan* d_plan = nullptr;
  float2* d_ops = nullptr;      // [2N+1][block_q] rotated ops per half-step
  float* d_ctab = nullptr;      // [3N][ngroups] drive coefficients (per group = per drive)
  float* d_dctab = nullptr;     // [3N][npulse] dc/dpar
  double* d_dctab64 = nullptr;
  double* d_ctab64 = nullptr;   // [3N][n_drives] c(t) per drive, FP64 (plain path)
  float2* d_ph = nullptr;       // real frame: [2N+1][ph_row] frame phases (cos, sin)
  float* d_rops = nullptr;      // real frame: [block_q] un-rotated operators (real parts)
  void* d_scratch = nullptr;    // small per-system scratch (adjoint partial sums)
  size_t scratch_bytes = 0;
  int device = 0;
  bool real_ok = false;         // the real frame is allowed (tables built)
  // checkpoints of the most recent propagate with with_ckpt = 1 (for an
  // adjoint called without psi0): where, for which opts, and its stamp
  const void* ck_ws = nullptr;
  int ck_S = 0, ck_ce = 0, ck_N = 0;
  uint64_t ck_gen = 0;          // 0: no valid checkpoints
  // kernel timing (scp_system_set_timing): HIP events recorded on the launch
  // stream around each forward, recompute and reverse launch
  bool timing = false;
  // engine of the FP32 solves (scp_system_set_engine): 0 automatic, 1 the
  // register-layout stepper, 2 the gather engine where it runs
  int engine = 0;
  mutable std::vector<hipEvent_t> tev;   // recorded events (start, stop pairs)
  mutable std::vector<int> tkind;        // kind of each pair: 0 forward, 1 recompute, 2 reverse
};

namespace scp {

void set_error(const std::string& msg);
scp_status fail(scp_status st, const std::string& msg);

// Return SCP_EHIP with the failing call's text from a function returning scp_status.
#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(SCP_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// Kernel timing: a start event before a launch (nullptr when timing is off
// or no event could be made) and the stop event after it.
hipEvent_t timing_start(const scp_system* sys, hipStream_t s);
void timing_stop(const scp_system* sys, hipEvent_t start, int kind, hipStream_t s);

// host single-mode builders (single_mode.cpp)
void build_transmon(ModeData& m);
void build_fluxonium(ModeData& m);
scp_status finish_mode(ModeData& m);   // sign convention, truncation, dressed ops, derivatives

// kernels
hipError_t launch_jacobi(double* A, double* V, double* w, const int* K, const int64_t* offs,
                         int n_mat, hipStream_t s);
hipError_t launch_jacobi_big(double* A, double* V, int Dp, void* work, hipStream_t s);
hipError_t launch_tables(scp_system* sys, hipStream_t s);
scp_status launch_rk4(scp_system* sys, const float2* psi0, float2* psiT, float2* lo, float4* ckpt,
                      int ckpt_every, int S, hipStream_t s);
scp_status launch_apply(const scp_system* sys, int step, int stage, const float2* y, float2* out,
                        int S, hipStream_t s);
scp_status launch_adjoint(scp_system* sys, const float4* ckpt, const float2* lamT, float2* segbuf,
                          double* partial, int ckpt_every, int S, hipStream_t s);
scp_status launch_fidelity(const void* U, int64_t D, int S, int prec, int dc, const int64_t* rows,
                           const int32_t* cols, const void* target, void* tau, void* cot,
                           hipStream_t s);
scp_status launch_fidelity_states(const void* U, int64_t D, int S, int prec, int nt,
                                  const int32_t* cols, const void* phi, void* tau, void* cot,
                                  hipStream_t s);
scp_status launch_fidelity_local(const void* U, int64_t D, int S, int prec, int nq,
                                 const int32_t* cols, const void* W, const int64_t* rows,
                                 const void* target, int mode, void* block, void* tau_out,
                                 double* F_out, double* params_out, void* cot, hipStream_t s);
scp_status launch_plain64(scp_system* sys, const double2* psi0, double2* psiT, void* work, int S,
                          hipStream_t s);
scp_status trotter_check(const scp_system* sys, int order);
size_t trotter_workspace_bytes(const scp_system* sys, int order);
size_t trotter_adjoint_workspace_bytes(const scp_system* sys, int order, int S);
scp_status trotter_adjoint_check(const scp_system* sys, int order);
scp_status launch_trotter_adjoint(scp_system* sys, int order, int S, void* ws, const double2* psi0,
                                  const double2* cot, double* grad, hipStream_t st);
scp_status launch_trotter(scp_system* sys, int order, int S, void* ws, const double2* psi0,
                          double2* psiT, hipStream_t st);
size_t lindblad_workspace_bytes(const scp_system* sys);
scp_status lindblad_check(const scp_system* sys);
scp_status launch_lindblad(scp_system* sys, const double* gamma1, const double* gammaphi, int S,
                           void* ws, size_t ws_bytes, const float2* rho0, float2* rhoT,
                           hipStream_t st);
scp_status launch_fidelity_channel(const void* rhoT, int64_t D, int dc, const int64_t* rows,
                                   const void* target, void* ov, void* cot, hipStream_t st);
scp_status lindblad_adjoint_workspace_bytes(const scp_system* sys, int S, size_t* bytes);
scp_status launch_lindblad_adjoint(scp_system* sys, const double* gamma1, const double* gammaphi,
                                   int S, void* ws, size_t ws_bytes, const float2* rho0,
                                   const float2* cot, double* grad, hipStream_t st);
bool gather_preferred(const scp_system* sys, int S);
bool gather_supported(const scp_system* sys);
size_t gather_workspace_bytes(const scp_system* sys);
scp_status launch_gather_forward(scp_system* sys, int S, void* ws, size_t ws_bytes,
                                 const float2* psi0, float2* psiT, hipStream_t st);
scp_status gather_grad_check(const scp_system* sys);
size_t gather_grad_workspace_bytes(const scp_system* sys, int S, int ce, bool with_grad);
scp_status launch_gather_ckpt_forward(scp_system* sys, int S, int ce, void* ws, size_t ws_bytes,
                                      const float2* psi0, float2* psiT, hipStream_t st);
scp_status launch_gather_adjoint(scp_system* sys, int S, int ce, void* ws, size_t ws_bytes,
                                 const float2* cot, double* grad, hipStream_t st);
// A workgroup's work item of a batched gather-engine launch (serving).
struct GItem {
  const void* A;          // the request's description (device GArgs)
  const void* B;          // its adjoint description (device GAdj; nullptr: no checkpoints)
  const float4* st_in;    // forward: the saved state (nullptr: start from the columns)
  float4* st_out;         // forward: where the state is saved
  int col, n_lo, n_hi;    // forward: column and step range; reverse: col = block of 2S
  int gseg;               // reverse: segment
};
// Device pointers and LDS needs of a request prepared by gather_serve_prepare.
struct GServeInfo {
  const void* A;
  const void* B;
  float4* state;
  size_t lds_fwd, lds_adj;
  int nck;
};
scp_status gather_serve_info(const scp_system* sys, int S, int ce, bool grad, void* ws,
                             GServeInfo& out);
scp_status gather_launch_fwd_batched(int d, int N, bool ck, const GItem* items, int n, size_t lds,
                                     hipStream_t st);
scp_status gather_launch_adj_batched(int d, int N, const GItem* items, int n, size_t lds,
                                     hipStream_t st);
size_t gather_serve_bytes(const scp_system* sys, int S, int ce, bool grad);
scp_status gather_serve_prepare(scp_system* sys, int S, int ce, bool grad, void* ws, size_t bytes,
                                const float2* psi0, float2* psiT, const float2* cot, hipStream_t st);
scp_status gather_serve_forward(scp_system* sys, int S, int ce, bool grad, void* ws, int n0, int n1,
                                hipStream_t st);
scp_status gather_serve_adjoint(scp_system* sys, int S, int ce, void* ws, int gs, hipStream_t st);
int gather_serve_nckpt(const scp_system* sys, int ce);
scp_status gather_serve_gradient(scp_system* sys, int S, int ce, void* ws, std::vector<double>& grad,
                                 hipStream_t st);

}  // namespace scp
