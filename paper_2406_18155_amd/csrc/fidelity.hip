// Gate fidelity on the computational subspace and its cotangent.
//
// tau = sum_ij conj(T_ij) U[comp_rows[i], comp_cols[j]] (Sec. 4.1 composite
// state-transfer cost with the target's columns as target states),
// accumulated in FP64: per-thread partial sums in a fixed order, then a
// fixed-shape LDS tree (deterministic).  The cotangent of L = 1 - |tau|^2/d_c^2
// with dL = 2 Re <lambda, dU> is lambda = -(tau / d_c^2) T_ij at the
// computational entries and zero elsewhere.
//
// The composite state cost with full target states (Sec. 4.1, S target
// states instead of a computational block) is reduced the same way.
//
// With single-qubit phase compensation (App. D compensation, restricted to Z
// rotations before and after the gate): the d_c x d_c block is gathered in
// FP64, the phases maximising |tau| are found on the host (a few hundred
// FP64 operations per phase update), and the cotangent is that of the target
// rephased by the optimal phases (they are stationary at the optimum).
#include <array>
#include <complex>
#include <vector>

#include "internal.h"

namespace scp {

namespace {

constexpr int FID_THREADS = 256;

template <typename T2>
__device__ inline double2 ld(const T2* U, size_t i) {
  T2 v = U[i];
  return make_double2((double)v.x, (double)v.y);
}

template <typename T2>
__global__ void __launch_bounds__(FID_THREADS)
tau_kernel(const T2* __restrict__ U, int64_t D, int S, int dc, const int64_t* __restrict__ rows,
           const int32_t* __restrict__ cols, const double2* __restrict__ target,
           double2* __restrict__ tau) {
  __shared__ double sre[FID_THREADS], sim[FID_THREADS];
  double ar = 0.0, ai = 0.0;
  const int n = dc * dc;
  for (int e = threadIdx.x; e < n; e += FID_THREADS) {
    const int i = e / dc, j = e - i * dc;
    const double2 t = target[e];
    const int64_t r = rows[i];
    const int c = cols[j];
    if (r < 0 || r >= D || c < 0 || c >= S) {   // out-of-range index: poison the result
      ar = __builtin_nan("");
      continue;
    }
    const double2 u = ld(U, (size_t)c * D + r);
    // conj(t) * u
    ar += t.x * u.x + t.y * u.y;
    ai += t.x * u.y - t.y * u.x;
  }
  sre[threadIdx.x] = ar;
  sim[threadIdx.x] = ai;
  __syncthreads();
  for (int s = FID_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sre[threadIdx.x] += sre[threadIdx.x + s];
      sim[threadIdx.x] += sim[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *tau = make_double2(sre[0], sim[0]);
}

template <typename T2>
__global__ void fill_zero_kernel(T2* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    T2 z;
    z.x = 0;
    z.y = 0;
    p[i] = z;
  }
}

template <typename T2>
__global__ void cot_kernel(T2* __restrict__ cot, int64_t D, int S, int dc,
                           const int64_t* __restrict__ rows,
                           const int32_t* __restrict__ cols, const double2* __restrict__ target,
                           const double2* __restrict__ tau) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dc * dc) return;
  const int i = e / dc, j = e - i * dc;
  if (rows[i] < 0 || rows[i] >= D || cols[j] < 0 || cols[j] >= S) return;
  const double2 tt = *tau;
  const double2 t = target[e];
  const double sc = -1.0 / ((double)dc * dc);
  // -(tau/dc^2) * T_ij
  const double re = sc * (tt.x * t.x - tt.y * t.y);
  const double im = sc * (tt.x * t.y + tt.y * t.x);
  T2 v;
  v.x = re;
  v.y = im;
  cot[(size_t)cols[j] * D + rows[i]] = v;
}

template <typename T2>
hipError_t run(const void* U, int64_t D, int S, int dc, const int64_t* rows, const int32_t* cols,
               const void* target, void* tau, void* cot, hipStream_t s) {
  hipLaunchKernelGGL(tau_kernel<T2>, dim3(1), dim3(FID_THREADS), 0, s, (const T2*)U, D, S, dc,
                     rows, cols, (const double2*)target, (double2*)tau);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || cot == nullptr) return e;
  const size_t n = (size_t)D * S;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_zero_kernel<T2>, dim3(blocks), dim3(256), 0, s, (T2*)cot, n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cot_kernel<T2>, dim3((dc * dc + 255) / 256), dim3(256), 0, s, (T2*)cot, D, S,
                     dc, rows, cols, (const double2*)target, (const double2*)tau);
  return hipGetLastError();
}

// Composite state cost (Sec. 4.1): tau = sum_j sum_i conj(phi[i, j]) U[i, cols[j]]
// over n_t full target states phi (D x n_t, complex128), one workgroup,
// per-thread partial sums in a fixed order (column by column, rows strided by
// the block), then a fixed-shape LDS tree: deterministic, FP64 throughout.
constexpr int ST_THREADS = 1024;

template <typename T2>
__global__ void __launch_bounds__(ST_THREADS)
tau_states_kernel(const T2* __restrict__ U, int64_t D, int S, int nt,
                  const int32_t* __restrict__ cols, const double2* __restrict__ phi,
                  double2* __restrict__ tau) {
  __shared__ double sre[ST_THREADS], sim[ST_THREADS];
  double ar = 0.0, ai = 0.0;
  for (int j = 0; j < nt; ++j) {
    const int c = cols[j];
    if (c < 0 || c >= S) {   // out-of-range column: poison the result
      ar = __builtin_nan("");
      continue;
    }
    const T2* u = U + (size_t)c * D;
    const double2* f = phi + (size_t)j * D;
    for (int64_t i = threadIdx.x; i < D; i += ST_THREADS) {
      const double2 t = f[i];
      const double2 v = ld(u, (size_t)i);
      ar += t.x * v.x + t.y * v.y;
      ai += t.x * v.y - t.y * v.x;
    }
  }
  sre[threadIdx.x] = ar;
  sim[threadIdx.x] = ai;
  __syncthreads();
  for (int s = ST_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sre[threadIdx.x] += sre[threadIdx.x + s];
      sim[threadIdx.x] += sim[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *tau = make_double2(sre[0], sim[0]);
}

// cotangent of L = 1 - |tau|^2/n_t^2: -(tau/n_t^2) phi[:, j] into column cols[j]
template <typename T2>
__global__ void cot_states_kernel(T2* __restrict__ cot, int64_t D, int S, int nt,
                                  const int32_t* __restrict__ cols,
                                  const double2* __restrict__ phi,
                                  const double2* __restrict__ tau) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)D * nt) return;
  const int j = (int)(e / (size_t)D);
  const int64_t i = (int64_t)(e - (size_t)j * D);
  const int c = cols[j];
  if (c < 0 || c >= S) return;
  const double2 tt = *tau;
  const double2 f = phi[e];
  const double sc = -1.0 / ((double)nt * nt);
  T2 v;
  v.x = sc * (tt.x * f.x - tt.y * f.y);
  v.y = sc * (tt.x * f.y + tt.y * f.x);
  cot[(size_t)c * D + i] = v;
}

template <typename T2>
hipError_t run_states(const void* U, int64_t D, int S, int nt, const int32_t* cols,
                      const void* phi, void* tau, void* cot, hipStream_t s) {
  hipLaunchKernelGGL(tau_states_kernel<T2>, dim3(1), dim3(ST_THREADS), 0, s, (const T2*)U, D, S,
                     nt, cols, (const double2*)phi, (double2*)tau);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || cot == nullptr) return e;
  const size_t n = (size_t)D * S;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_zero_kernel<T2>, dim3(blocks), dim3(256), 0, s, (T2*)cot, n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t m = (size_t)D * nt;
  hipLaunchKernelGGL(cot_states_kernel<T2>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                     (T2*)cot, D, S, nt, cols, (const double2*)phi, (const double2*)tau);
  return hipGetLastError();
}

// M_ij = U[comp_rows[i], comp_cols[j]] (FP64, row-major) for the host-side
// phase compensation.
template <typename T2>
__global__ void block_kernel(const T2* __restrict__ U, int64_t D, int S, int dc,
                             const int64_t* __restrict__ rows, const int32_t* __restrict__ cols,
                             double2* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dc * dc) return;
  const int i = e / dc, j = e - i * dc;
  const int64_t r = rows[i];
  const int c = cols[j];
  out[e] = (r < 0 || r >= D || c < 0 || c >= S) ? make_double2(__builtin_nan(""), 0.0)
                                                 : ld(U, (size_t)c * D + r);
}

// Compensation phases of the computational rows (after the gate) and
// columns (before it), passed by value.
struct ZPhases {
  double th[64], ch[64];
};

// cotangent at the optimum: -(tau/dc^2) T_ij e^{-i th_i} e^{-i ch_j}
template <typename T2>
__global__ void cot_zcomp_kernel(T2* __restrict__ cot, int64_t D, int S, int dc,
                                 const int64_t* __restrict__ rows,
                                 const int32_t* __restrict__ cols,
                                 const double2* __restrict__ target, ZPhases ph, double2 tau) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dc * dc) return;
  const int i = e / dc, j = e - i * dc;
  if (rows[i] < 0 || rows[i] >= D || cols[j] < 0 || cols[j] >= S) return;
  const double2 t = target[e];
  double sn, cs;
  sincos(-(ph.th[i] + ph.ch[j]), &sn, &cs);
  const double tr = t.x * cs - t.y * sn, ti = t.x * sn + t.y * cs;   // T'_ij
  const double sc = -1.0 / ((double)dc * dc);
  T2 v;
  v.x = sc * (tau.x * tr - tau.y * ti);
  v.y = sc * (tau.x * ti + tau.y * tr);
  cot[(size_t)cols[j] * D + rows[i]] = v;
}

template <typename T2>
hipError_t run_zcomp_block(const void* U, int64_t D, int S, int dc, const int64_t* rows,
                           const int32_t* cols, void* block, hipStream_t s) {
  hipLaunchKernelGGL(block_kernel<T2>, dim3((dc * dc + 255) / 256), dim3(256), 0, s,
                     (const T2*)U, D, S, dc, rows, cols, (double2*)block);
  return hipGetLastError();
}

template <typename T2>
hipError_t run_zcomp_cot(void* cot, int64_t D, int S, int dc, const int64_t* rows,
                         const int32_t* cols, const void* target, const ZPhases& ph,
                         double2 tau, hipStream_t s) {
  const size_t n = (size_t)D * S;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_zero_kernel<T2>, dim3(blocks), dim3(256), 0, s, (T2*)cot, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cot_zcomp_kernel<T2>, dim3((dc * dc + 255) / 256), dim3(256), 0, s, (T2*)cot,
                     D, S, dc, rows, cols, (const double2*)target, ph, tau);
  return hipGetLastError();
}

using cd = std::complex<double>;

// tau(a, c) = sum_ij W_ij e^{i theta_i} e^{i chi_j}, W_ij = conj(T_ij) M_ij
cd zcomp_tau(const std::vector<cd>& W, int nq, const std::vector<double>& a,
             const std::vector<double>& c) {
  const int dc = 1 << nq;
  cd t = 0.0;
  for (int i = 0; i < dc; ++i) {
    double th = 0.0;
    for (int q = 0; q < nq; ++q) th += ((i >> (nq - 1 - q)) & 1) ? a[q] : 0.0;
    for (int j = 0; j < dc; ++j) {
      double ch = 0.0;
      for (int q = 0; q < nq; ++q) ch += ((j >> (nq - 1 - q)) & 1) ? c[q] : 0.0;
      t += W[(size_t)i * dc + j] * std::polar(1.0, th + ch);
    }
  }
  return t;
}

}  // namespace

namespace {

// Coordinate ascent from the phases in a, c (in place): over a_0..a_{n-1}
// (after the gate), then c_0..c_{n-1} (before it); each phase goes to
// arg A - arg B, where tau = A + e^{i p} B with B the terms whose bit of that
// qubit is set and the other phases fixed (left unchanged if A or B is zero);
// sweeps end when |tau| grows by at most 1e-14 relative, or after 200.
void zcomp_ascend(const std::vector<cd>& W, int nq, std::vector<double>& a,
                  std::vector<double>& c) {
  const int dc = 1 << nq;
  double best = std::abs(zcomp_tau(W, nq, a, c));
  auto bit = [&](int i, int q) { return (i >> (nq - 1 - q)) & 1; };
  for (int sweep = 0; sweep < 200; ++sweep) {
    for (int side = 0; side < 2; ++side)
      for (int q = 0; q < nq; ++q) {
        cd A = 0.0, B = 0.0;
        for (int i = 0; i < dc; ++i) {
          double th = 0.0;
          for (int k = 0; k < nq; ++k)
            if (bit(i, k) && !(side == 0 && k == q)) th += a[k];
          for (int j = 0; j < dc; ++j) {
            double ch = 0.0;
            for (int k = 0; k < nq; ++k)
              if (bit(j, k) && !(side == 1 && k == q)) ch += c[k];
            const cd x = W[(size_t)i * dc + j] * std::polar(1.0, th + ch);
            if ((side == 0 ? bit(i, q) : bit(j, q)) != 0)
              B += x;
            else
              A += x;
          }
        }
        if (A != 0.0 && B != 0.0) (side == 0 ? a : c)[q] = std::arg(A) - std::arg(B);
      }
    const double t = std::abs(zcomp_tau(W, nq, a, c));
    const bool done = t - best <= 1e-14 * std::max(1.0, t);
    best = std::max(best, t);
    if (done) break;
  }
}

}  // namespace

// Phase compensation on the host (FP64): the coordinate ascent (zcomp_ascend)
// from each of a fixed set of starts, keeping the largest |tau| (the earliest
// start on a tie).  One start (zero) for one qubit, 16 otherwise; start k has
// a_q = 2 pi frac(k (q + 1) g) and c_q = 2 pi frac(k (nq + q + 1) g), g the
// fractional part of the golden ratio: one ascent from zero stalls below the
// maximum on many three-qubit blocks far from their target.
void zcomp_optimise(const std::vector<cd>& W, int nq, std::vector<double>& a,
                    std::vector<double>& c, cd& tau) {
  const double g = 0.6180339887498949, twopi = 2.0 * 3.141592653589793;
  const int K = nq == 1 ? 1 : 16;
  double best = -1.0;
  std::vector<double> ak(nq), ck(nq);
  for (int k = 0; k < K; ++k) {
    for (int q = 0; q < nq; ++q) {
      ak[q] = twopi * std::fmod((double)(k * (q + 1)) * g, 1.0);
      ck[q] = twopi * std::fmod((double)(k * (nq + q + 1)) * g, 1.0);
    }
    zcomp_ascend(W, nq, ak, ck);
    const double t = std::abs(zcomp_tau(W, nq, ak, ck));
    if (t > best) {
      best = t;
      a = ak;
      c = ck;
    }
  }
  tau = zcomp_tau(W, nq, a, c);
}

scp_status launch_zcomp(const void* U, int64_t D, int S, int prec, int nq, const int64_t* rows,
                        const int32_t* cols, const void* target, void* block, void* tau_out,
                        double* F_out, double* phases_out, void* cot, hipStream_t s) {
  const int dc = 1 << nq;
  hipError_t e = prec == 0 ? run_zcomp_block<float2>(U, D, S, dc, rows, cols, block, s)
                           : run_zcomp_block<double2>(U, D, S, dc, rows, cols, block, s);
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("zcomp block: ") + hipGetErrorString(e));
  std::vector<cd> M((size_t)dc * dc), T((size_t)dc * dc), W((size_t)dc * dc);
  HIPCHK(hipMemcpyAsync(M.data(), block, M.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(T.data(), target, T.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (size_t k = 0; k < W.size(); ++k) W[k] = std::conj(T[k]) * M[k];
  std::vector<double> a, c;
  cd tau;
  zcomp_optimise(W, nq, a, c, tau);
  *F_out = std::norm(tau) / ((double)dc * dc);
  if (!std::isfinite(*F_out)) return fail(SCP_ENONFINITE, "fidelity is not finite");
  if (phases_out) {
    for (int q = 0; q < nq; ++q) {
      phases_out[q] = a[q];
      phases_out[nq + q] = c[q];
    }
  }
  const double2 t2 = make_double2(tau.real(), tau.imag());
  if (tau_out) {
    HIPCHK(hipMemcpyAsync(tau_out, &t2, sizeof(double2), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  if (cot) {
    ZPhases ph;
    for (int i = 0; i < dc; ++i) {
      double th = 0.0, ch = 0.0;
      for (int q = 0; q < nq; ++q)
        if ((i >> (nq - 1 - q)) & 1) {
          th += a[q];
          ch += c[q];
        }
      ph.th[i] = th;
      ph.ch[i] = ch;
    }
    e = prec == 0 ? run_zcomp_cot<float2>(cot, D, S, dc, rows, cols, target, ph, t2, s)
                  : run_zcomp_cot<double2>(cot, D, S, dc, rows, cols, target, ph, t2, s);
    if (e != hipSuccess) return fail(SCP_EHIP, std::string("zcomp cotangent: ") + hipGetErrorString(e));
  }
  return SCP_OK;
}

// ---------------------------------------------------------------------------
// Compensated fidelity in a given basis (App. D): the block
// M_ij = <w_i | U[:, cols[j]]> (W: D x d_c device, complex128) or, without W,
// M_ij = U[comp_rows[i], cols[j]]; on the host the single-qubit compensation
// (Z phases, or arbitrary SU(2) unitaries by coordinate ascent with polar
// factors); the compensated target T' and the costate
// -(tau/d_c^2) sum_i T'_ij w_i (or at the computational rows).
// ---------------------------------------------------------------------------
namespace {

constexpr int PB_THREADS = 256;

// one workgroup per block entry (i, j): sum_k conj(W[k, i]) U[k, cols[j]] in FP64
template <typename T2>
__global__ void __launch_bounds__(PB_THREADS)
proj_block_kernel(const T2* __restrict__ U, int64_t D, int S, int dc,
                  const int32_t* __restrict__ cols, const double2* __restrict__ W,
                  double2* __restrict__ out) {
  __shared__ double sre[PB_THREADS], sim[PB_THREADS];
  const int e = blockIdx.x, i = e / dc, j = e - i * dc;
  const int c = cols[j];
  double ar = 0.0, ai = 0.0;
  if (c < 0 || c >= S) {
    ar = __builtin_nan("");
  } else {
    const T2* u = U + (size_t)c * D;
    const double2* w = W + (size_t)i * D;
    for (int64_t k = threadIdx.x; k < D; k += PB_THREADS) {
      const double2 x = w[k];
      const double2 v = ld(u, (size_t)k);
      ar += x.x * v.x + x.y * v.y;
      ai += x.x * v.y - x.y * v.x;
    }
  }
  sre[threadIdx.x] = ar;
  sim[threadIdx.x] = ai;
  __syncthreads();
  for (int st = PB_THREADS / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sre[threadIdx.x] += sre[threadIdx.x + st];
      sim[threadIdx.x] += sim[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[e] = make_double2(sre[0], sim[0]);
}

// cot[:, cols[j]] = -(tau/dc^2) sum_i T'_ij w_i
template <typename T2>
__global__ void cot_proj_kernel(T2* __restrict__ cot, int64_t D, int S, int dc,
                                const int32_t* __restrict__ cols, const double2* __restrict__ W,
                                const double2* __restrict__ Tp, double2 tau) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)D * dc) return;
  const int j = (int)(e / (size_t)D);
  const int64_t k = (int64_t)(e - (size_t)j * D);
  const int c = cols[j];
  if (c < 0 || c >= S) return;
  double re = 0.0, im = 0.0;
  for (int i = 0; i < dc; ++i) {
    const double2 t = Tp[(size_t)i * dc + j], w = W[(size_t)i * D + k];
    re += t.x * w.x - t.y * w.y;
    im += t.x * w.y + t.y * w.x;
  }
  const double sc = -1.0 / ((double)dc * dc);
  T2 v;
  v.x = sc * (tau.x * re - tau.y * im);
  v.y = sc * (tau.x * im + tau.y * re);
  cot[(size_t)c * D + k] = v;
}

// cot[comp_rows[i], cols[j]] = -(tau/dc^2) T'_ij
template <typename T2>
__global__ void cot_rows_kernel(T2* __restrict__ cot, int64_t D, int S, int dc,
                                const int64_t* __restrict__ rows, const int32_t* __restrict__ cols,
                                const double2* __restrict__ Tp, double2 tau) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dc * dc) return;
  const int i = e / dc, j = e - i * dc;
  if (rows[i] < 0 || rows[i] >= D || cols[j] < 0 || cols[j] >= S) return;
  const double2 t = Tp[e];
  const double sc = -1.0 / ((double)dc * dc);
  T2 v;
  v.x = sc * (tau.x * t.x - tau.y * t.y);
  v.y = sc * (tau.x * t.y + tau.y * t.x);
  cot[(size_t)cols[j] * D + rows[i]] = v;
}

using cmat = std::vector<cd>;

// (x)_q mats[q] (qubit 0 most significant), dc x dc
cmat kron_all(const std::vector<std::array<cd, 4>>& mats) {
  cmat K(1, 1.0);
  int n = 1;
  for (const auto& m : mats) {
    cmat R((size_t)4 * n * n);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c)
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            R[(size_t)(r * 2 + a) * (2 * n) + (c * 2 + b)] = K[(size_t)r * n + c] * m[a * 2 + b];
    K.swap(R);
    n *= 2;
  }
  return K;
}

cmat matmul(const cmat& A, const cmat& B, int n) {
  cmat C((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const cd a = A[(size_t)i * n + k];
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += a * B[(size_t)k * n + j];
    }
  return C;
}

cmat dagger(const cmat& A, int n) {
  cmat B((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[(size_t)j * n + i] = std::conj(A[(size_t)i * n + j]);
  return B;
}

cd trace(const cmat& A, int n) {
  cd t = 0.0;
  for (int i = 0; i < n; ++i) t += A[(size_t)i * n + i];
  return t;
}

// X with Tr(a X) = Tr((I (x) .. a at qubit q .. (x) I) Y): the partial trace of
// Y over every other qubit, X[r][c] = sum_rest Y[(r, rest), (c, rest)]
std::array<cd, 4> partial_trace(const cmat& Y, int nq, int q) {
  const int dc = 1 << nq, sh = nq - 1 - q;
  std::array<cd, 4> X{0.0, 0.0, 0.0, 0.0};
  for (int row = 0; row < dc; ++row) {
    const int r = (row >> sh) & 1;
    for (int c = 0; c < 2; ++c) {
      const int col = (row & ~(1 << sh)) | (c << sh);
      X[r * 2 + c] += Y[(size_t)row * dc + col];
    }
  }
  return X;
}

// The unitary u maximising |Tr(u X)| for a 2 x 2 X: with X = P S Q^dag,
// u = Q P^dag (then Tr(u X) = sum of the singular values).  The right
// singular vectors come from the Hermitian X^dag X in closed form; a zero
// singular value takes the unit vector orthogonal to the other.
std::array<cd, 4> polar_opt(const std::array<cd, 4>& X) {
  // H = X^dag X = [[p, q], [conj q, r]]
  const double p = std::norm(X[0]) + std::norm(X[2]);
  const double r = std::norm(X[1]) + std::norm(X[3]);
  const cd q = std::conj(X[0]) * X[1] + std::conj(X[2]) * X[3];
  const double m = 0.5 * (p + r), h = std::sqrt(0.25 * (p - r) * (p - r) + std::norm(q));
  const double l1 = m + h;
  // eigenvector of l1: (q, l1 - p) or (l1 - r, conj q), whichever is longer
  cd v0, v1;
  {
    const cd a0 = q, a1 = l1 - p;
    const cd b0 = l1 - r, b1 = std::conj(q);
    const double na = std::norm(a0) + std::norm(a1), nb = std::norm(b0) + std::norm(b1);
    if (na == 0.0 && nb == 0.0) {
      v0 = 1.0;
      v1 = 0.0;
    } else if (na >= nb) {
      v0 = a0 / std::sqrt(na);
      v1 = a1 / std::sqrt(na);
    } else {
      v0 = b0 / std::sqrt(nb);
      v1 = b1 / std::sqrt(nb);
    }
  }
  const cd w0 = -std::conj(v1), w1 = std::conj(v0);   // the other right singular vector
  // left singular vectors u_k = X v_k / s_k
  cd u00 = X[0] * v0 + X[1] * v1, u10 = X[2] * v0 + X[3] * v1;
  double s1 = std::sqrt(std::norm(u00) + std::norm(u10));
  if (s1 == 0.0) return {1.0, 0.0, 0.0, 1.0};
  u00 /= s1;
  u10 /= s1;
  cd u01 = X[0] * w0 + X[1] * w1, u11 = X[2] * w0 + X[3] * w1;
  const double s2 = std::sqrt(std::norm(u01) + std::norm(u11));
  if (s2 > 1e-300) {
    u01 /= s2;
    u11 /= s2;
  } else {
    u01 = -std::conj(u10);
    u11 = std::conj(u00);
  }
  // u = Q P^dag, Q = [v w], P = [u_0 u_1]
  std::array<cd, 4> out;
  out[0] = v0 * std::conj(u00) + w0 * std::conj(u01);
  out[1] = v0 * std::conj(u10) + w0 * std::conj(u11);
  out[2] = v1 * std::conj(u00) + w1 * std::conj(u01);
  out[3] = v1 * std::conj(u10) + w1 * std::conj(u11);
  return out;
}

// tau(a, b) = Tr(T^dag (x)a M (x)b)
cd su2_tau(const cmat& M, const cmat& Th, const std::vector<std::array<cd, 4>>& a,
           const std::vector<std::array<cd, 4>>& b, int dc) {
  return trace(matmul(Th, matmul(matmul(kron_all(a), M, dc), kron_all(b), dc), dc), dc);
}

}  // namespace

// Arbitrary single-qubit compensation: coordinate ascent from identities over
// a_0..a_{n-1} (after the gate), then b_0..b_{n-1} (before it), each set to the
// polar optimum of its partial trace with the others fixed, until |tau| grows
// by at most 1e-14 relative or after 500 sweeps.
void su2_optimise(const cmat& M, const cmat& T, int nq, std::vector<std::array<cd, 4>>& a,
                  std::vector<std::array<cd, 4>>& b, cd& tau) {
  const int dc = 1 << nq;
  const std::array<cd, 4> id{1.0, 0.0, 0.0, 1.0};
  a.assign(nq, id);
  b.assign(nq, id);
  const cmat Th = dagger(T, dc);
  double best = std::abs(su2_tau(M, Th, a, b, dc));
  for (int sweep = 0; sweep < 500; ++sweep) {
    for (int side = 0; side < 2; ++side)
      for (int q = 0; q < nq; ++q) {
        std::vector<std::array<cd, 4>> rest = side == 0 ? a : b;
        rest[q] = id;
        cmat Y;
        if (side == 0)   // tau = Tr((x)a (M B T^dag))
          Y = matmul(kron_all(rest), matmul(matmul(M, kron_all(b), dc), Th, dc), dc);
        else             // tau = Tr((x)b (T^dag A M))
          Y = matmul(kron_all(rest), matmul(Th, matmul(kron_all(a), M, dc), dc), dc);
        (side == 0 ? a : b)[q] = polar_opt(partial_trace(Y, nq, q));
      }
    const double t = std::abs(su2_tau(M, Th, a, b, dc));
    const bool done = t - best <= 1e-14 * std::max(1.0, t);
    best = std::max(best, t);
    if (done) break;
  }
  tau = su2_tau(M, Th, a, b, dc);
}

scp_status launch_fidelity_local(const void* U, int64_t D, int S, int prec, int nq,
                                 const int32_t* cols, const void* W, const int64_t* rows,
                                 const void* target, int mode, void* block, void* tau_out,
                                 double* F_out, double* params_out, void* cot, hipStream_t s) {
  const int dc = 1 << nq;
  hipError_t e;
  if (W != nullptr) {
    if (prec == 0)
      hipLaunchKernelGGL(proj_block_kernel<float2>, dim3(dc * dc), dim3(PB_THREADS), 0, s,
                         (const float2*)U, D, S, dc, cols, (const double2*)W, (double2*)block);
    else
      hipLaunchKernelGGL(proj_block_kernel<double2>, dim3(dc * dc), dim3(PB_THREADS), 0, s,
                         (const double2*)U, D, S, dc, cols, (const double2*)W, (double2*)block);
    e = hipGetLastError();
  } else {
    e = prec == 0 ? run_zcomp_block<float2>(U, D, S, dc, rows, cols, block, s)
                  : run_zcomp_block<double2>(U, D, S, dc, rows, cols, block, s);
  }
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("compensated block: ") + hipGetErrorString(e));
  cmat M((size_t)dc * dc), T((size_t)dc * dc);
  HIPCHK(hipMemcpyAsync(M.data(), block, M.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(T.data(), target, T.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (const cd& x : M)
    if (!std::isfinite(x.real()) || !std::isfinite(x.imag()))
      return fail(SCP_ENONFINITE, "the compensated block is not finite");
  cmat Tp((size_t)dc * dc);
  cd tau;
  if (mode == 1) {
    std::vector<cd> Wz((size_t)dc * dc);
    for (size_t k = 0; k < Wz.size(); ++k) Wz[k] = std::conj(T[k]) * M[k];
    std::vector<double> a, c;
    zcomp_optimise(Wz, nq, a, c, tau);
    for (int i = 0; i < dc; ++i)
      for (int j = 0; j < dc; ++j) {
        double th = 0.0, ch = 0.0;
        for (int q = 0; q < nq; ++q) {
          if ((i >> (nq - 1 - q)) & 1) th += a[q];
          if ((j >> (nq - 1 - q)) & 1) ch += c[q];
        }
        Tp[(size_t)i * dc + j] = T[(size_t)i * dc + j] * std::polar(1.0, -(th + ch));
      }
    if (params_out)
      for (int q = 0; q < nq; ++q) {
        params_out[q] = a[q];
        params_out[nq + q] = c[q];
      }
  } else {
    std::vector<std::array<cd, 4>> a, b;
    su2_optimise(M, T, nq, a, b, tau);
    // T' = A^dag T B^dag
    Tp = matmul(matmul(dagger(kron_all(a), dc), T, dc), dagger(kron_all(b), dc), dc);
    if (params_out)
      for (int q = 0; q < nq; ++q)
        for (int k = 0; k < 4; ++k) {
          params_out[(q * 4 + k) * 2] = a[q][k].real();
          params_out[(q * 4 + k) * 2 + 1] = a[q][k].imag();
          params_out[((nq + q) * 4 + k) * 2] = b[q][k].real();
          params_out[((nq + q) * 4 + k) * 2 + 1] = b[q][k].imag();
        }
  }
  *F_out = std::norm(tau) / ((double)dc * dc);
  if (!std::isfinite(*F_out)) return fail(SCP_ENONFINITE, "fidelity is not finite");
  const double2 t2 = make_double2(tau.real(), tau.imag());
  double2* Tpd = (double2*)block + (size_t)dc * dc;
  HIPCHK(hipMemcpyAsync(Tpd, Tp.data(), Tp.size() * sizeof(cd), hipMemcpyHostToDevice, s));
  if (tau_out) HIPCHK(hipMemcpyAsync(tau_out, &t2, sizeof(double2), hipMemcpyHostToDevice, s));
  if (cot) {
    const size_t n = (size_t)D * S;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    if (prec == 0)
      hipLaunchKernelGGL(fill_zero_kernel<float2>, dim3(blocks), dim3(256), 0, s, (float2*)cot, n);
    else
      hipLaunchKernelGGL(fill_zero_kernel<double2>, dim3(blocks), dim3(256), 0, s, (double2*)cot, n);
    HIPCHK(hipGetLastError());
    if (W != nullptr) {
      const size_t m = (size_t)D * dc;
      if (prec == 0)
        hipLaunchKernelGGL(cot_proj_kernel<float2>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                           (float2*)cot, D, S, dc, cols, (const double2*)W, Tpd, t2);
      else
        hipLaunchKernelGGL(cot_proj_kernel<double2>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                           (double2*)cot, D, S, dc, cols, (const double2*)W, Tpd, t2);
    } else {
      if (prec == 0)
        hipLaunchKernelGGL(cot_rows_kernel<float2>, dim3((dc * dc + 255) / 256), dim3(256), 0, s,
                           (float2*)cot, D, S, dc, rows, cols, Tpd, t2);
      else
        hipLaunchKernelGGL(cot_rows_kernel<double2>, dim3((dc * dc + 255) / 256), dim3(256), 0, s,
                           (double2*)cot, D, S, dc, rows, cols, Tpd, t2);
    }
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(s));
  return SCP_OK;
}

scp_status launch_fidelity_states(const void* U, int64_t D, int S, int prec, int nt,
                                  const int32_t* cols, const void* phi, void* tau, void* cot,
                                  hipStream_t s) {
  hipError_t e = prec == 0 ? run_states<float2>(U, D, S, nt, cols, phi, tau, cot, s)
                           : run_states<double2>(U, D, S, nt, cols, phi, tau, cot, s);
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("state fidelity: ") + hipGetErrorString(e));
  return SCP_OK;
}

scp_status launch_fidelity(const void* U, int64_t D, int S, int prec, int dc, const int64_t* rows,
                           const int32_t* cols, const void* target, void* tau, void* cot,
                           hipStream_t s) {
  hipError_t e = prec == 0 ? run<float2>(U, D, S, dc, rows, cols, target, tau, cot, s)
                           : run<double2>(U, D, S, dc, rows, cols, target, tau, cot, s);
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("fidelity: ") + hipGetErrorString(e));
  return SCP_OK;
}

}  // namespace scp
