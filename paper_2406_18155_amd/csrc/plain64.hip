// Plain complex FP64 propagation (the unfused baseline of the fused FP32 path).
//
// Same discrete method as the fused stepper: classical RK4 on
// d psi_I/dt = -i V(t) psi_I in the interaction picture of the frame
// (Sec. 2.3 step grid; App. B one-mode contractions), with
//   V(t) = sum_e g_e A~_i(t) (x) B~_j(t)            (Sec. 2.1 local terms)
//        + sum_k c_k(t) O~_k(t)                     (App. C drives)
//        + sum_m diag(eps_m - frame_m)              (zero at the build point)
// but in the textbook form: every local term is its own kernel launch that
// reads its input from HBM and accumulates into the stage derivative in HBM,
// and one more launch per stage combines the RK4 stages.  Everything is
// complex FP64; the rotated operators O_ab exp(i (f_a - f_b) t) are formed on
// the host in FP64 (angle reduced modulo 2 pi) and passed by value, the drive
// coefficients come from the FP64 table built with the system.
//
// Workspace: four D x S complex128 buffers (stage accumulator, stage input,
// stage derivative, first-factor product).
#include <cmath>

#include "internal.h"

namespace scp {

namespace {

struct TermArgs {
  const double2* in;
  double2* out;
  int64_t total;     // D * S
  int64_t stride;    // stride of the contracted mode
  int d;
  int accumulate;    // 0: out = op in, 1: out += op in
  const double* coef;  // nullable: multiply by *coef (FP64 drive coefficient)
  double2 op[SCP_MAX_TRUNC * SCP_MAX_TRUNC];  // row-major d x d
};

// out[idx] (+)= coef * sum_b op[a][b] in[idx + (b - a) stride], a = digit of idx
__global__ void __launch_bounds__(256) term64_kernel(TermArgs A) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= A.total) return;
  const int a = (int)((idx / A.stride) % A.d);
  const int64_t base = idx - (int64_t)a * A.stride;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < A.d; ++b) {
    const double2 o = A.op[a * A.d + b];
    const double2 x = A.in[base + (int64_t)b * A.stride];
    re += o.x * x.x - o.y * x.y;
    im += o.x * x.y + o.y * x.x;
  }
  if (A.coef) {
    const double c = *A.coef;
    re *= c;
    im *= c;
  }
  if (A.accumulate) {
    const double2 v = A.out[idx];
    re += v.x;
    im += v.y;
  }
  A.out[idx] = make_double2(re, im);
}

struct DiagArgs {
  const double2* in;
  double2* out;
  int64_t total, D;
  int d, n_modes;
  double delta[SCP_MAX_MODES][SCP_MAX_TRUNC];   // eps - frame per mode and level
};

// out += -i sum_m delta_m[a_m] in
__global__ void __launch_bounds__(256) diag64_kernel(DiagArgs A) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= A.total) return;
  int64_t r = idx % A.D;
  double w = 0.0;
  for (int m = A.n_modes - 1; m >= 0; --m) {
    w += A.delta[m][r % A.d];
    r /= A.d;
  }
  const double2 x = A.in[idx];
  const double2 v = A.out[idx];
  A.out[idx] = make_double2(v.x + w * x.y, v.y - w * x.x);
}

// RK4 combination after stage s with derivative k:
//   s=0: acc = psi + h/6 k, y = psi + h/2 k
//   s=1: acc += h/3 k,      y = psi + h/2 k
//   s=2: acc += h/3 k,      y = psi + h k
//   s=3: psi = acc + h/6 k
__global__ void __launch_bounds__(256) combine64_kernel(double2* psi, double2* acc, double2* y,
                                                        const double2* k, int64_t total, int s,
                                                        double h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const double2 kv = k[i];
  if (s == 3) {
    const double2 a = acc[i];
    psi[i] = make_double2(a.x + (h / 6) * kv.x, a.y + (h / 6) * kv.y);
    return;
  }
  const double2 p = psi[i];
  const double wa = (s == 0) ? h / 6 : h / 3;
  const double wy = (s == 2) ? h : h / 2;
  if (s == 0) {
    acc[i] = make_double2(p.x + wa * kv.x, p.y + wa * kv.y);
  } else {
    const double2 a = acc[i];
    acc[i] = make_double2(a.x + wa * kv.x, a.y + wa * kv.y);
  }
  y[i] = make_double2(p.x + wy * kv.x, p.y + wy * kv.y);
}

double reduce_angle_host(double x) {
  const double twopi = 6.283185307179586476925286766559;
  return x - twopi * std::nearbyint(x / twopi);
}

// op(t) = scale * O_ab exp(i (f_a - f_b) t), FP64
void rotated(const ModeData& M, int op, double t, cplx scale, int d, double2* out) {
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      const double th = reduce_angle_host((M.frame[a] - M.frame[b]) * t);
      const cplx v = scale * M.ops[op][a * d + b] * cplx(std::cos(th), std::sin(th));
      out[a * d + b] = make_double2(v.real(), v.imag());
    }
}

}  // namespace

scp_status launch_plain64(scp_system* sys, const double2* psi0, double2* psiT, void* work, int S,
                          hipStream_t s) {
  if (!work) return fail(SCP_EINVAL, "the FP64 path needs a workspace (scp_workspace_size)");
  const int d = sys->d, nm = sys->n_modes, N = sys->n_steps;
  const int64_t D = sys->D, total = D * (int64_t)S;
  const double h = sys->h;
  double2* acc = static_cast<double2*>(work);
  double2* y = acc + total;
  double2* k = y + total;
  double2* tmp = k + total;
  if (psiT != psi0)
    HIPCHK(hipMemcpyAsync(psiT, psi0, total * sizeof(double2), hipMemcpyDeviceToDevice, s));
  std::vector<int64_t> stride(nm);
  for (int m = nm - 1, st = 1; m >= 0; --m, st *= d) stride[m] = st;
  DiagArgs dg{};
  bool has_diag = false;
  dg.total = total;
  dg.D = D;
  dg.d = d;
  dg.n_modes = nm;
  for (int m = 0; m < nm; ++m)
    for (int a = 0; a < d; ++a) {
      dg.delta[m][a] = sys->modes[m].eps[a] - sys->modes[m].frame[a];
      if (dg.delta[m][a] != 0.0) has_diag = true;
    }
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  const cplx mi(0.0, -1.0);
  const int ndr = (int)sys->drives.size();
  const double c_frac[4] = {0.0, 0.5, 0.5, 1.0};
  const int c_col[4] = {0, 1, 1, 2};
  TermArgs A{};
  A.total = total;
  A.d = d;
  for (int n = 0; n < N; ++n) {
    for (int st = 0; st < 4; ++st) {
      const double t = (n + c_frac[st]) * h;
      const double2* yin = (st == 0) ? psiT : y;
      bool first = true;
      for (const Coupling& e : sys->coup) {
        A.in = yin;
        A.out = tmp;
        A.stride = stride[e.i];
        A.accumulate = 0;
        A.coef = nullptr;
        rotated(sys->modes[e.i], e.op_i, t, cplx(1.0, 0.0), d, A.op);
        hipLaunchKernelGGL(term64_kernel, grid, block, 0, s, A);
        A.in = tmp;
        A.out = k;
        A.stride = stride[e.j];
        A.accumulate = first ? 0 : 1;
        rotated(sys->modes[e.j], e.op_j, t, mi * e.g, d, A.op);
        hipLaunchKernelGGL(term64_kernel, grid, block, 0, s, A);
        first = false;
      }
      for (int q = 0; q < ndr; ++q) {
        const Drive& R = sys->drives[q];
        A.in = yin;
        A.out = k;
        A.stride = stride[R.mode];
        A.accumulate = first ? 0 : 1;
        A.coef = sys->d_ctab64 + (size_t)(3 * n + c_col[st]) * ndr + q;
        rotated(sys->modes[R.mode], R.op, t, mi, d, A.op);
        hipLaunchKernelGGL(term64_kernel, grid, block, 0, s, A);
        first = false;
      }
      if (first) HIPCHK(hipMemsetAsync(k, 0, total * sizeof(double2), s));
      if (has_diag) {
        dg.in = yin;
        dg.out = k;
        hipLaunchKernelGGL(diag64_kernel, grid, block, 0, s, dg);
      }
      hipLaunchKernelGGL(combine64_kernel, grid, block, 0, s, psiT, acc, y, k, total, st, h);
    }
    if ((n & 255) == 255) HIPCHK(hipGetLastError());
  }
  HIPCHK(hipGetLastError());
  return SCP_OK;
}

}  // namespace scp
