// FP64 symmetric eigensolver for the single-mode Hamiltonians: cyclic
// two-sided Jacobi with the round-robin (circle) ordering, one workgroup per
// matrix, the matrix and the eigenvector accumulator resident in LDS.  Each
// round rotates K/2 disjoint (p, q) planes in parallel; a sweep is K'-1
// rounds (K' = K rounded up to even); sweeps stop when the off-diagonal
// Frobenius norm is below 1e-15 of the full norm.  Deterministic: fixed
// rotation order, fixed-order reductions, no atomics.
#include "internal.h"

namespace scp {
namespace {

constexpr int JAC_THREADS = 256;
constexpr int JAC_MAXK = 96;

__device__ inline int player(int pos, int round, int Kp) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (Kp - 1);
}

__global__ void __launch_bounds__(JAC_THREADS)
jacobi_kernel(double* __restrict__ Aall, double* __restrict__ Vall, double* __restrict__ wall,
              const int* __restrict__ Ks, const int64_t* __restrict__ offs) {
  extern __shared__ double sm[];
  const int mat = blockIdx.x;
  const int K = Ks[mat];
  const int Kp = K + (K & 1);
  double* A = sm;                  // K*K
  double* V = A + K * K;           // K*K
  double* cs = V + K * K;          // Kp/2
  double* sn = cs + Kp / 2;        // Kp/2
  double* red = sn + Kp / 2;       // JAC_THREADS
  int* pq = reinterpret_cast<int*>(red + JAC_THREADS);   // Kp
  const int tid = threadIdx.x;
  double* Ag = Aall + offs[mat];
  for (int i = tid; i < K * K; i += JAC_THREADS) {
    A[i] = Ag[i];
    V[i] = (i / K == i % K) ? 1.0 : 0.0;
  }
  __syncthreads();
  // full norm
  double loc = 0;
  for (int i = tid; i < K * K; i += JAC_THREADS) loc += A[i] * A[i];
  red[tid] = loc;
  __syncthreads();
  for (int s = JAC_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double full = red[0];
  __syncthreads();
  const int npair = Kp / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    for (int round = 0; round < Kp - 1; ++round) {
      if (tid < npair) {
        int p = player(tid, round, Kp), q = player(Kp - 1 - tid, round, Kp);
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < K) {
          double apq = A[p * K + q];
          if (apq != 0.0) {
            double theta = (A[q * K + q] - A[p * K + p]) / (2.0 * apq);
            double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs[tid] = c;
        sn[tid] = s;
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
      }
      __syncthreads();
      // rows: A <- P^T A
      for (int it = tid; it < npair * K; it += JAC_THREADS) {
        int i = it / K, k = it % K;
        int p = pq[2 * i], q = pq[2 * i + 1];
        if (q < K) {
          double c = cs[i], s = sn[i];
          double ap = A[p * K + k], aq = A[q * K + k];
          A[p * K + k] = c * ap - s * aq;
          A[q * K + k] = s * ap + c * aq;
        }
      }
      __syncthreads();
      // columns: A <- A P, V <- V P
      for (int it = tid; it < npair * K; it += JAC_THREADS) {
        int i = it / K, k = it % K;
        int p = pq[2 * i], q = pq[2 * i + 1];
        if (q < K) {
          double c = cs[i], s = sn[i];
          double ap = A[k * K + p], aq = A[k * K + q];
          A[k * K + p] = c * ap - s * aq;
          A[k * K + q] = s * ap + c * aq;
          double vp = V[k * K + p], vq = V[k * K + q];
          V[k * K + p] = c * vp - s * vq;
          V[k * K + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
    loc = 0;
    for (int i = tid; i < K * K; i += JAC_THREADS)
      if (i / K != i % K) loc += A[i] * A[i];
    red[tid] = loc;
    __syncthreads();
    for (int s = JAC_THREADS / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const double off = red[0];
    __syncthreads();
    if (off <= 1e-30 * full) break;
  }
  double* Vg = Vall + offs[mat];
  for (int i = tid; i < K * K; i += JAC_THREADS) Vg[i] = V[i];
  double* wg = wall + offs[mat];   // first K entries of the matrix slot
  for (int i = tid; i < K; i += JAC_THREADS) wg[i] = A[i * K + i];
}

}  // namespace

hipError_t launch_jacobi(double* A, double* V, double* w, const int* K, const int64_t* offs,
                         int n_mat, hipStream_t s) {
  const int Kp = JAC_MAXK;
  size_t shmem = sizeof(double) * (2 * JAC_MAXK * JAC_MAXK + Kp + JAC_THREADS) + sizeof(int) * Kp;
  hipFuncSetAttribute((const void*)jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shmem);
  hipLaunchKernelGGL(jacobi_kernel, dim3(n_mat), dim3(JAC_THREADS), shmem, s, A, V, w, K, offs);
  return hipGetLastError();
}

}  // namespace scp
