// FP64 symmetric eigensolvers.  For the single-mode Hamiltonians: cyclic
// two-sided Jacobi with the round-robin (circle) ordering, one workgroup per
// matrix, the matrix and the eigenvector accumulator resident in LDS.  Each
// round rotates K/2 disjoint (p, q) planes in parallel; a sweep is K'-1
// rounds (K' = K rounded up to even); sweeps stop when the off-diagonal
// Frobenius norm is below 1e-15 of the full norm.  Deterministic: fixed
// rotation order, fixed-order reductions, no atomics.
#include <algorithm>

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

// ---------------------------------------------------------------------------
// Larger symmetric matrices (composite static Hamiltonians, D up to 2048): the
// same cyclic two-sided Jacobi with round-robin ordering, the matrix and the
// eigenvector accumulator in device memory.  A round is two launches: the
// rotations of the Dp/2 disjoint planes from the current matrix, then every
// 2 x 2 block of A (rows of one plane, columns of another) gets
// J_rows^T A J_cols and every pair of V columns J, all blocks disjoint.  A
// sweep is Dp - 1 rounds; after each sweep the off-diagonal norm is reduced
// (fixed order) and sweeps stop below 1e-30 of the full squared norm, as in
// the one-workgroup solver.  Dp = D rounded up to even; the padding row and
// column are zero and never rotate (their off-diagonal entries stay 0).
// ---------------------------------------------------------------------------
__global__ void jac_rot_kernel(const double* __restrict__ A, int Dp, int round,
                               double* __restrict__ cs, int* __restrict__ pq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int npair = Dp / 2;
  if (i >= npair) return;
  int p = player(i, round, Dp), q = player(Dp - 1 - i, round, Dp);
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
  double c = 1.0, s = 0.0;
  const double apq = A[(size_t)p * Dp + q];
  if (apq != 0.0) {
    const double theta = (A[(size_t)q * Dp + q] - A[(size_t)p * Dp + p]) / (2.0 * apq);
    const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    c = 1.0 / sqrt(t * t + 1.0);
    s = t * c;
  }
  cs[2 * i] = c;
  cs[2 * i + 1] = s;
  pq[2 * i] = p;
  pq[2 * i + 1] = q;
}

// blocks (i, k) of A for i, k < npair, then V pairs (row r, plane k)
__global__ void jac_apply_kernel(double* __restrict__ A, double* __restrict__ V, int Dp,
                                 const double* __restrict__ cs, const int* __restrict__ pq) {
  const int npair = Dp / 2;
  const size_t nA = (size_t)npair * npair, nV = (size_t)Dp * npair;
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < nA + nV;
       w += (size_t)gridDim.x * blockDim.x) {
    if (w < nA) {
      const int i = (int)(w / npair), k = (int)(w % npair);
      const int p = pq[2 * i], q = pq[2 * i + 1], r = pq[2 * k], t = pq[2 * k + 1];
      const double ci = cs[2 * i], si = cs[2 * i + 1], ck = cs[2 * k], sk = cs[2 * k + 1];
      double* xpr = A + (size_t)p * Dp + r;
      double* xpt = A + (size_t)p * Dp + t;
      double* xqr = A + (size_t)q * Dp + r;
      double* xqt = A + (size_t)q * Dp + t;
      const double a = *xpr, b = *xpt, c = *xqr, dd = *xqt;
      // rows (plane i) then columns (plane k)
      const double ypr = ci * a - si * c, yqr = si * a + ci * c;
      const double ypt = ci * b - si * dd, yqt = si * b + ci * dd;
      *xpr = ck * ypr - sk * ypt;
      *xpt = sk * ypr + ck * ypt;
      *xqr = ck * yqr - sk * yqt;
      *xqt = sk * yqr + ck * yqt;
    } else {
      const size_t u = w - nA;
      const int row = (int)(u / npair), k = (int)(u % npair);
      const int p = pq[2 * k], q = pq[2 * k + 1];
      const double c = cs[2 * k], s = cs[2 * k + 1];
      double* vp = V + (size_t)row * Dp + p;
      double* vq = V + (size_t)row * Dp + q;
      const double x = *vp, y = *vq;
      *vp = c * x - s * y;
      *vq = s * x + c * y;
    }
  }
}

// sum of squares of the off-diagonal (offdiag = 1) or of all entries, one
// workgroup, fixed order
__global__ void __launch_bounds__(1024) jac_norm_kernel(const double* __restrict__ A, int Dp,
                                                        int offdiag, double* __restrict__ out) {
  __shared__ double red[1024];
  double loc = 0.0;
  const size_t n = (size_t)Dp * Dp;
  for (size_t i = threadIdx.x; i < n; i += 1024) {
    if (offdiag && i / Dp == i % Dp) continue;
    loc += A[i] * A[i];
  }
  red[threadIdx.x] = loc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void jac_init_kernel(double* __restrict__ V, int Dp) {
  const size_t n = (size_t)Dp * Dp;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    V[i] = (i / Dp == i % Dp) ? 1.0 : 0.0;
}

}  // namespace

// A: Dp x Dp row-major on the device (the matrix in its leading D x D block,
// zero elsewhere), overwritten; V: Dp x Dp eigenvectors (column a, leading D
// rows); work: 2 Dp doubles + Dp ints + 2 doubles.  Eigenvalue a is A[a][a].
// Synchronises the stream once per sweep (convergence test).
hipError_t launch_jacobi_big(double* A, double* V, int Dp, void* work, hipStream_t s) {
  double* cs = static_cast<double*>(work);
  int* pq = reinterpret_cast<int*>(cs + Dp);
  double* nrm = reinterpret_cast<double*>(pq + Dp + (Dp & 1)) ;
  hipLaunchKernelGGL(jac_init_kernel, dim3(256), dim3(256), 0, s, V, Dp);
  hipLaunchKernelGGL(jac_norm_kernel, dim3(1), dim3(1024), 0, s, A, Dp, 0, nrm);
  double full = 0.0;
  hipError_t e = hipMemcpyAsync(&full, nrm, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const int npair = Dp / 2;
  const size_t items = (size_t)npair * npair + (size_t)Dp * npair;
  const int blocks = (int)std::min<size_t>((items + 255) / 256, 4096);
  for (int sweep = 0; sweep < 40; ++sweep) {
    for (int round = 0; round < Dp - 1; ++round) {
      hipLaunchKernelGGL(jac_rot_kernel, dim3((npair + 127) / 128), dim3(128), 0, s, A, Dp, round, cs,
                         pq);
      hipLaunchKernelGGL(jac_apply_kernel, dim3(blocks), dim3(256), 0, s, A, V, Dp, cs, pq);
    }
    hipLaunchKernelGGL(jac_norm_kernel, dim3(1), dim3(1024), 0, s, A, Dp, 1, nrm + 1);
    double off = 0.0;
    e = hipMemcpyAsync(&off, nrm + 1, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (off <= 1e-30 * full) break;
  }
  return hipGetLastError();
}

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
