/* A C11 program that drives libscprop through its C ABI alone (no Python,
 * no torch): two coupled, driven transmons (d = 3, D = 9) and their four
 * computational columns.
 *
 * It checks what the ABI promises, not parity (the parity tests compare the
 * same calls with the FP64 oracle):
 *   - the FP32 RK4 forward and the FP64 product formula (Q2) keep every
 *     column's norm (unitary evolution, Sec. 2.3).  Q2 is unitary to
 *     rounding (1e-12).  RK4 is not: at this step of 0.01 ns the FP64
 *     oracle's RK4 drifts by 1.2e-6 (at 0.05 ns by 2.7e-3, from the
 *     interaction picture's fast phases), so FP32 gets 2e-5;
 *   - the RK4 gradient of the infidelity against the identity is finite;
 *   - the LCAM gradient (Sec. 2.5) from psi0 and the one from the forward's
 *     psi_I(T) are bitwise equal;
 *   - a short workspace and a null pointer are refused with SCP_EINVAL and
 *     a message.
 * Prints "c abi ok" and exits 0, or names the failed check and exits 1. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "scprop.h"

#define TWO_PI 6.283185307179586

static int failures = 0;

static void check(int ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "FAILED: %s (last error: %s)\n", what, scp_last_error());
    ++failures;
  }
}

#define HIP_OK(x)                                                      \
  do {                                                                 \
    hipError_t e_ = (x);                                               \
    if (e_ != hipSuccess) {                                            \
      fprintf(stderr, "HIP error %s at %s\n", hipGetErrorString(e_), #x); \
      return 1;                                                        \
    }                                                                  \
  } while (0)

int main(void) {
  const int n_modes = 2, d = 3, S = 4, n_steps = 2000;
  const double T = 20.0;
  scp_mode_desc modes[2];
  memset(modes, 0, sizeof modes);
  for (int m = 0; m < n_modes; ++m) {
    modes[m].kind = SCP_MODE_TRANSMON;
    modes[m].basis_dim = 21;
    modes[m].trunc = d;
    modes[m].EC = (0.24 + 0.02 * m) * TWO_PI;
    modes[m].EJ = modes[m].EC * (48.0 + 4.0 * m);
  }
  scp_coupling_desc coup = {0, 1, SCP_OP_N, SCP_OP_N, 0.01 * TWO_PI};
  double amp[2] = {0.03 * TWO_PI, 0.02 * TWO_PI};
  scp_drive_desc drv[2];
  memset(drv, 0, sizeof drv);
  for (int k = 0; k < 2; ++k) {
    drv[k].mode = k;
    drv[k].op = SCP_OP_N;
    drv[k].env = SCP_ENV_GAUSS;
    drv[k].n_par = 1;
    drv[k].sigma = T / 4.0;
    drv[k].par = &amp[k];
  }
  scp_system_desc desc = {n_modes, 1, 2, n_steps, T, modes, &coup, drv};

  hipStream_t st;
  HIP_OK(hipStreamCreate(&st));
  scp_system* sys = NULL;
  if (scp_build_system(&desc, st, &sys) != SCP_OK) {
    fprintf(stderr, "FAILED: scp_build_system: %s\n", scp_last_error());
    return 1;
  }
  int64_t D = 0;
  int32_t n_params = 0, nm = 0;
  check(scp_system_info(sys, &D, &n_params, &nm, NULL) == SCP_OK, "scp_system_info");
  check(D == 9 && nm == 2 && n_params == 2 + 3 * 2 + 1, "system sizes");

  /* computational columns |00>, |01>, |10>, |11> at a0 d + a1 */
  const int cols[4] = {0, 1, 3, 4};

  /* FP32 RK4 forward with checkpoints, then the gradient of 1 - F */
  float* h32 = calloc((size_t)S * D * 2, sizeof(float));
  for (int s = 0; s < S; ++s) h32[((size_t)s * D + cols[s]) * 2] = 1.f;
  void *psi32, *U32, *cot32, *ws;
  HIP_OK(hipMalloc(&psi32, (size_t)S * D * 8));
  HIP_OK(hipMalloc(&U32, (size_t)S * D * 8));
  HIP_OK(hipMalloc(&cot32, (size_t)S * D * 8));
  HIP_OK(hipMemcpy(psi32, h32, (size_t)S * D * 8, hipMemcpyHostToDevice));
  scp_solve_opts opts = {S, 0, 0, 1, 0};
  size_t wsb = 0;
  check(scp_workspace_size(sys, &opts, 1, &wsb) == SCP_OK, "scp_workspace_size");
  opts.workspace_bytes = wsb;
  HIP_OK(hipMalloc(&ws, wsb));
  check(scp_propagate(sys, &opts, ws, psi32, U32, st) == SCP_OK, "scp_propagate");
  HIP_OK(hipStreamSynchronize(st));
  HIP_OK(hipMemcpy(h32, U32, (size_t)S * D * 8, hipMemcpyDeviceToHost));
  for (int s = 0; s < S; ++s) {
    double nrm = 0.0;
    for (int64_t i = 0; i < D; ++i) {
      const double re = h32[(s * D + i) * 2], im = h32[(s * D + i) * 2 + 1];
      nrm += re * re + im * im;
    }
    check(fabs(nrm - 1.0) <= 2e-5, "FP32 RK4 column norm");
  }
  /* identity target on the four columns; indices, target and tau on the device */
  int64_t rows[4];
  int32_t ccols[4];
  double target[4 * 4 * 2];
  memset(target, 0, sizeof target);
  for (int i = 0; i < 4; ++i) {
    rows[i] = cols[i];
    ccols[i] = i;
    target[(i * 4 + i) * 2] = 1.0;
  }
  void *d_rows, *d_cols, *d_target, *d_tau;
  HIP_OK(hipMalloc(&d_rows, sizeof rows));
  HIP_OK(hipMalloc(&d_cols, sizeof ccols));
  HIP_OK(hipMalloc(&d_target, sizeof target));
  HIP_OK(hipMalloc(&d_tau, 2 * sizeof(double)));
  HIP_OK(hipMemcpy(d_rows, rows, sizeof rows, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_cols, ccols, sizeof ccols, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_target, target, sizeof target, hipMemcpyHostToDevice));
  double F = -1.0;
  check(scp_fidelity(U32, D, S, 0, 4, (const int64_t*)d_rows, (const int32_t*)d_cols, d_target,
                     d_tau, cot32, &F, st) == SCP_OK,
        "scp_fidelity");
  check(F >= 0.0 && F <= 1.0 + 1e-6, "fidelity in [0, 1]");
  double* g = calloc((size_t)n_params, sizeof(double));
  check(scp_propagate_adjoint(sys, &opts, ws, psi32, cot32, g, st) == SCP_OK,
        "scp_propagate_adjoint");
  int finite = 1;
  for (int i = 0; i < n_params; ++i) finite &= isfinite(g[i]) != 0;
  check(finite, "RK4 gradient finite");

  /* refused calls: each call against its own workspace size (the forward's
     without the gradient's regions, the adjoint's with them) */
  size_t wsf = 0;
  check(scp_workspace_size(sys, &opts, 0, &wsf) == SCP_OK, "scp_workspace_size (forward)");
  check(wsf > 0 && wsf <= wsb, "forward workspace within the gradient's");
  scp_solve_opts small = opts;
  small.workspace_bytes = wsf - 1;
  check(scp_propagate(sys, &small, ws, psi32, U32, st) == SCP_EINVAL,
        "short forward workspace refused");
  small.workspace_bytes = wsb - 1;
  check(scp_propagate_adjoint(sys, &small, ws, psi32, cot32, g, st) == SCP_EINVAL,
        "short gradient workspace refused");
  check(scp_propagate(sys, &opts, NULL, psi32, U32, st) == SCP_EINVAL, "null workspace refused");
  check(strlen(scp_last_error()) > 0, "refusal leaves a message");

  /* FP64 product formula (Q2) and its LCAM gradient two ways */
  double* h64 = calloc((size_t)S * D * 2, sizeof(double));
  for (int s = 0; s < S; ++s) h64[((size_t)s * D + cols[s]) * 2] = 1.0;
  void *psi64, *UT, *cot64, *wt, *wa;
  HIP_OK(hipMalloc(&psi64, (size_t)S * D * 16));
  HIP_OK(hipMalloc(&UT, (size_t)S * D * 16));
  HIP_OK(hipMalloc(&cot64, (size_t)S * D * 16));
  HIP_OK(hipMemcpy(psi64, h64, (size_t)S * D * 16, hipMemcpyHostToDevice));
  size_t wtb = 0, wab = 0;
  check(scp_trotter_workspace_size(sys, SCP_TROTTER_Q2, &wtb) == SCP_OK,
        "scp_trotter_workspace_size");
  check(scp_trotter_adjoint_workspace_size(sys, SCP_TROTTER_Q2, S, &wab) == SCP_OK,
        "scp_trotter_adjoint_workspace_size");
  HIP_OK(hipMalloc(&wt, wtb));
  HIP_OK(hipMalloc(&wa, wab));
  check(scp_propagate_trotter(sys, SCP_TROTTER_Q2, S, wt, psi64, UT, st) == SCP_OK,
        "scp_propagate_trotter");
  HIP_OK(hipStreamSynchronize(st));
  HIP_OK(hipMemcpy(h64, UT, (size_t)S * D * 16, hipMemcpyDeviceToHost));
  for (int s = 0; s < S; ++s) {
    double nrm = 0.0;
    for (int64_t i = 0; i < D; ++i) {
      const double re = h64[(s * D + i) * 2], im = h64[(s * D + i) * 2 + 1];
      nrm += re * re + im * im;
    }
    check(fabs(nrm - 1.0) <= 1e-12, "FP64 Q2 column norm");
  }
  /* costate: a fixed pattern of unit-order entries */
  for (int64_t i = 0; i < (int64_t)S * D; ++i) {
    h64[2 * i] = 0.5 + 0.25 * (double)(i % 7) / 7.0;
    h64[2 * i + 1] = -0.25 + 0.5 * (double)(i % 5) / 5.0;
  }
  HIP_OK(hipMemcpy(cot64, h64, (size_t)S * D * 16, hipMemcpyHostToDevice));
  double* ga = calloc((size_t)n_params, sizeof(double));
  double* gb = calloc((size_t)n_params, sizeof(double));
  check(scp_propagate_trotter_adjoint(sys, SCP_TROTTER_Q2, S, wa, wab, psi64, cot64, ga, st) ==
            SCP_OK,
        "scp_propagate_trotter_adjoint");
  check(scp_propagate_trotter_adjoint_final(sys, SCP_TROTTER_Q2, S, wa, wab, UT, cot64, gb, st) ==
            SCP_OK,
        "scp_propagate_trotter_adjoint_final");
  check(memcmp(ga, gb, (size_t)n_params * sizeof(double)) == 0,
        "LCAM gradient from psi0 and from psi_I(T) bitwise equal");
  double gmax = 0.0;
  for (int i = 0; i < n_params; ++i) gmax = fmax(gmax, fabs(ga[i]));
  check(gmax > 0.0 && isfinite(gmax), "LCAM gradient nonzero and finite");

  scp_destroy(sys);
  hipFree(psi32);
  hipFree(U32);
  hipFree(cot32);
  hipFree(ws);
  hipFree(psi64);
  hipFree(UT);
  hipFree(cot64);
  hipFree(wt);
  hipFree(wa);
  hipFree(d_rows);
  hipFree(d_cols);
  hipFree(d_target);
  hipFree(d_tau);
  hipStreamDestroy(st);
  free(h32);
  free(h64);
  free(g);
  free(ga);
  free(gb);
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("c abi ok: D = %lld, %d parameters, F = %.6f\n", (long long)D, n_params, F);
  return 0;
}
