// Gate fidelity on the computational subspace and its cotangent.
//
// tau = sum_ij conj(T_ij) U[comp_rows[i], comp_cols[j]] (Sec. 4.1 composite
// state-transfer cost with the target's columns as target states),
// accumulated in FP64: per-thread partial sums in a fixed order, then a
// fixed-shape LDS tree (deterministic).  The cotangent of L = 1 - |tau|^2/d_c^2
// with dL = 2 Re <lambda, dU> is lambda = -(tau / d_c^2) T_ij at the
// computational entries and zero elsewhere.
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

}  // namespace

scp_status launch_fidelity(const void* U, int64_t D, int S, int prec, int dc, const int64_t* rows,
                           const int32_t* cols, const void* target, void* tau, void* cot,
                           hipStream_t s) {
  hipError_t e = prec == 0 ? run<float2>(U, D, S, dc, rows, cols, target, tau, cot, s)
                           : run<double2>(U, D, S, dc, rows, cols, target, tau, cot, s);
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("fidelity: ") + hipGetErrorString(e));
  return SCP_OK;
}

}  // namespace scp
