// Stage tables, computed in FP64 on the device and stored in FP32.
//
// Half-step q (t_q = q h / 2, q = 0..2N) block of rotated operators in the
// interaction picture of the frame: O~_ab(t) = O_ab exp(i (f_a - f_b) t)
// (App. C microwave drives and Sec. 2.1 local terms, expressed in the frame
// rotating at the frame energies f).  The phase (f_a - f_b) t reaches
// ~1e4 rad, so it is reduced modulo 2 pi in FP64 before the sine/cosine.
// Block layout: [slot ops][pair ops][slot derivative ops (3 per slot)],
// d*d complex each.
//
// Drive coefficient tables at the three time points of every step
// (t_n, t_n + h/2, t_n + h): c(t) = E(t) cos(omega_d t + phase) summed per
// drive group, c(t) of every drive in FP64 (plain FP64 path), and dc/d(par)
// for every pulse parameter.
#include "internal.h"

namespace scp {

namespace {

struct TabStatic {
  int d, nslots, npairs, nd, ndrives, ngroups, npulse, nsteps;
  double h, T;
};

__device__ inline double reduce_angle(double x) {
  const double twopi = 6.283185307179586476925286766559;
  return x - twopi * rint(x / twopi);
}

// data: frames [n_modes][8], slot ops [nslots][d*d] (re,im), pair ops
// [npairs][d*d], slot dops [nslots][3][d*d]; slot_mode [nslots], pair_mode
// [npairs] as int arrays.
__global__ void optable_kernel(TabStatic ts, const double* __restrict__ frames,
                               const double2* __restrict__ sops, const double2* __restrict__ pops,
                               const double2* __restrict__ dops, const int* __restrict__ smode,
                               const int* __restrict__ pmode, float2* __restrict__ out,
                               int block_q) {
  const int q = blockIdx.x;
  const double t = q * (0.5 * ts.h);
  const int dd = ts.d * ts.d;
  for (int e = threadIdx.x; e < block_q / dd * dd; e += blockDim.x) {
    const int ent = e / dd, ab = e % dd, a = ab / ts.d, b = ab % ts.d;
    double2 v;
    int mode;
    if (ent < ts.nslots) {
      v = sops[ent * dd + ab];
      mode = smode[ent];
    } else if (ent < ts.nslots + ts.npairs) {
      v = pops[(ent - ts.nslots) * dd + ab];
      mode = pmode[ent - ts.nslots];
    } else {
      const int k = ent - ts.nslots - ts.npairs;   // slot*3 + theta
      v = dops[k * dd + ab];
      mode = smode[k / 3];
    }
    const double th = reduce_angle((frames[mode * 8 + a] - frames[mode * 8 + b]) * t);
    double sn, cs;
    sincos(th, &sn, &cs);
    out[(size_t)q * block_q + e] = make_float2((float)(v.x * cs - v.y * sn), (float)(v.x * sn + v.y * cs));
  }
}

// Frame phases of the real-frame stepper, row q (t_q = q h / 2): entry r < RB
// is exp(i sum_p f_{a_p} t) over the register positions p of register r
// (position 0 most significant); entry thr + k*d + a is exp(i f_a t) of the
// mode at base-layout thread position k; the rest is padding.  Angles summed
// and reduced in FP64.
__global__ void phase_kernel(int d, int NT, int NR, int RB, int thr, int row, double h,
                             const double* __restrict__ frames, const int* __restrict__ tmode,
                             const int* __restrict__ rmode, float2* __restrict__ out) {
  const int q = blockIdx.x;
  const double t = q * (0.5 * h);
  for (int e = threadIdx.x; e < row; e += blockDim.x) {
    double f = 0.0;
    if (e < RB) {
      int rr = e;
      for (int p = NR - 1; p >= 0; --p) {
        f += frames[rmode[p] * 8 + rr % d];
        rr /= d;
      }
    } else if (e >= thr && e < thr + NT * d) {
      f = frames[tmode[(e - thr) / d] * 8 + (e - thr) % d];
    }
    double sn, cs;
    sincos(reduce_angle(f * t), &sn, &cs);
    out[(size_t)q * row + e] = make_float2((float)cs, (float)sn);
  }
}

struct DriveStatic {
  int env, npar, par0, group;
  double omega, phase, sigma;
};

__global__ void ctable_kernel(TabStatic ts, const DriveStatic* __restrict__ dr,
                              const double* __restrict__ par, float* __restrict__ ctab,
                              float* __restrict__ dctab, double* __restrict__ dctab64,
                              double* __restrict__ ctab64) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= 3 * ts.nsteps) return;
  const int n = p / 3, j = p - 3 * n;
  const double t = (n + 0.5 * j) * ts.h;
  for (int g = 0; g < ts.ngroups; ++g) ctab[(size_t)p * ts.ngroups + g] = 0.f;
  double csum[64];
  for (int g = 0; g < ts.ngroups && g < 64; ++g) csum[g] = 0.0;
  for (int k = 0; k < ts.ndrives; ++k) {
    const DriveStatic D = dr[k];
    const double carrier = cos(reduce_angle(D.omega * t + D.phase));
    const double* pp = par + D.par0;
    double val = 0.0;
    for (int i = 0; i < D.npar; ++i) {
      const double basis = envelope_basis(D.env, i, D.npar, n, ts.nsteps, t, ts.T, D.sigma);
      val += pp[i] * basis;
      dctab[(size_t)p * ts.npulse + D.par0 + i] = (float)(basis * carrier);
      dctab64[(size_t)p * ts.npulse + D.par0 + i] = basis * carrier;
    }
    csum[D.group] += val * carrier;
    ctab64[(size_t)p * ts.ndrives + k] = val * carrier;
  }
  for (int g = 0; g < ts.ngroups && g < 64; ++g) ctab[(size_t)p * ts.ngroups + g] = (float)csum[g];
}

}  // namespace

hipError_t launch_tables_impl(int d, int nslots, int npairs, int ndrives, int ngroups, int npulse,
                              int nsteps, double h, double T, const double* frames,
                              const double2* sops, const double2* pops, const double2* dops,
                              const int* smode, const int* pmode, float2* optab, int block_q,
                              const void* drives, const double* par, float* ctab, float* dctab,
                              double* dctab64, double* ctab64, hipStream_t s) {
  TabStatic ts{d, nslots, npairs, d * d, ndrives, ngroups, npulse, nsteps, h, T};
  hipLaunchKernelGGL(optable_kernel, dim3(2 * nsteps + 1), dim3(256), 0, s, ts, frames, sops, pops,
                     dops, smode, pmode, optab, block_q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ndrives > 0) {
    const int n = 3 * nsteps;
    hipLaunchKernelGGL(ctable_kernel, dim3((n + 127) / 128), dim3(128), 0, s, ts,
                       static_cast<const DriveStatic*>(drives), par, ctab, dctab, dctab64, ctab64);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_phase_table(int d, int NT, int NR, int RB, int thr, int row, int nsteps,
                              double h, const double* frames, const int* tmode, const int* rmode,
                              float2* ph, hipStream_t s) {
  hipLaunchKernelGGL(phase_kernel, dim3(2 * nsteps + 1), dim3(64), 0, s, d, NT, NR, RB, thr, row,
                     h, frames, tmode, rmode, ph);
  return hipGetLastError();
}

size_t drive_static_size() { return sizeof(DriveStatic); }

void pack_drive_static(void* dst, int k, int env, int npar, int par0, int group, double omega,
                       double phase, double sigma) {
  DriveStatic* D = static_cast<DriveStatic*>(dst) + k;
  D->env = env;
  D->npar = npar;
  D->par0 = par0;
  D->group = group;
  D->omega = omega;
  D->phase = phase;
  D->sigma = sigma;
}

}  // namespace scp
