// Contraction probe (measurement only; no solve uses it).
//
// The inner operation of the register-layout stepper at d = 3: a uniform
// complex 3 x 3 operator applied to every fibre of the RB = 27 amplitudes a
// lane holds (9 fibres along the last register position) and accumulated,
// out += O in.  Three forms of the same arithmetic:
//   form 0: VALU FMAs with the operator in scalar registers (the stepper's
//           form: 36 FMAs per fibre);
//   form 1: v_mfma_f32_4x4x1f32 (16 blocks of 4 lanes, each lane its own
//           fibre as the B operand): the real 6 x 6 form of O padded to two
//           4-row blocks, one MFMA per block and input component (12 per
//           fibre).  The A operand (row m of a block in lane 4b + m) is built
//           from the uniform operator at every application, and each fibre's
//           outputs are moved from and back to the accumulator registers, as
//           the stepper's register layout would need;
//   form 2: as form 1 with the A operands built once and the accumulators
//           kept in the MFMA's consecutive registers (issue and padding only).
// Application it uses operator it % nop of the table.  Every lane writes the
// sum of its outputs, so no work is removed and the forms can be compared.
#include "internal.h"
#include "kernel_common.h"

namespace scp {

namespace {

constexpr int PB_THREADS = 256;
constexpr int PB_D = 3, PB_RB = 27, PB_NF = 9;

typedef float f4 __attribute__((ext_vector_type(4)));

// value of row (4 rb + q) of the real 6 x 6 form [[Or, -Oi], [Oi, Or]] at
// column k (rows 6, 7 zero)
__device__ __forceinline__ float real_form(const float (&Or)[9], const float (&Oi)[9], int m, int k) {
  if (m >= 6) return 0.f;
  const int a = m % 3, b = k % 3;
  const bool mi = m >= 3, ki = k >= 3;
  const float re = Or[a * 3 + b], im = Oi[a * 3 + b];
  return mi ? (ki ? re : im) : (ki ? -im : re);
}

// the A operand of block row rb and column k for this lane: row 4 rb + (lane & 3)
__device__ __forceinline__ float a_operand(const float (&Or)[9], const float (&Oi)[9], int rb, int k,
                                           int q) {
  const float v0 = real_form(Or, Oi, 4 * rb + 0, k), v1 = real_form(Or, Oi, 4 * rb + 1, k);
  const float v2 = real_form(Or, Oi, 4 * rb + 2, k), v3 = real_form(Or, Oi, 4 * rb + 3, k);
  return q == 0 ? v0 : (q == 1 ? v1 : (q == 2 ? v2 : v3));
}

template <int FORM>
__global__ void __launch_bounds__(PB_THREADS) probe_kernel(const float* __restrict__ opg, int nop,
                                                           int iters, float* __restrict__ out) {
  kptr<float> ops = kconst(opg);
  const int gid = blockIdx.x * PB_THREADS + threadIdx.x;
  const int q = threadIdx.x & 3;
  float xr[PB_RB], xi[PB_RB], yr[PB_RB], yi[PB_RB];
#pragma unroll
  for (int r = 0; r < PB_RB; ++r) {
    const uint32_t h = (uint32_t)(gid * 131 + r * 7919) * 2654435761u;
    xr[r] = (float)(h & 0xffff) * (1.0f / 65536.0f) - 0.5f;
    xi[r] = (float)((h >> 16) & 0xffff) * (1.0f / 65536.0f) - 0.5f;
    yr[r] = yi[r] = 0.f;
  }
  if constexpr (FORM == 0) {
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
      const int o = uni(it % nop) * 18;
      float Or[9], Oi[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        Or[i] = ops[o + i];
        Oi[i] = ops[o + 9 + i];
      }
#pragma unroll
      for (int f = 0; f < PB_NF; ++f)
#pragma unroll
        for (int a = 0; a < PB_D; ++a) {
          float sr = yr[f * 3 + a], si = yi[f * 3 + a];
#pragma unroll
          for (int b = 0; b < PB_D; ++b) {
            sr = fmaf(Or[a * 3 + b], xr[f * 3 + b], sr);
            sr = fmaf(-Oi[a * 3 + b], xi[f * 3 + b], sr);
            si = fmaf(Or[a * 3 + b], xi[f * 3 + b], si);
            si = fmaf(Oi[a * 3 + b], xr[f * 3 + b], si);
          }
          yr[f * 3 + a] = sr;
          yi[f * 3 + a] = si;
        }
    }
  } else if constexpr (FORM == 1) {
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
      const int o = uni(it % nop) * 18;
      float Or[9], Oi[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        Or[i] = ops[o + i];
        Oi[i] = ops[o + 9 + i];
      }
      float A[2][6];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int k = 0; k < 6; ++k) A[rb][k] = a_operand(Or, Oi, rb, k, q);
#pragma unroll
      for (int f = 0; f < PB_NF; ++f) {
        f4 c0 = {yr[f * 3], yr[f * 3 + 1], yr[f * 3 + 2], yi[f * 3]};
        f4 c1 = {yi[f * 3 + 1], yi[f * 3 + 2], 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const float b = k < 3 ? xr[f * 3 + k] : xi[f * 3 + k - 3];
          c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(A[0][k], b, c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(A[1][k], b, c1, 0, 0, 0);
        }
        yr[f * 3] = c0[0];
        yr[f * 3 + 1] = c0[1];
        yr[f * 3 + 2] = c0[2];
        yi[f * 3] = c0[3];
        yi[f * 3 + 1] = c1[0];
        yi[f * 3 + 2] = c1[1];
      }
    }
  } else {
    float Or[9], Oi[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      Or[i] = ops[i];
      Oi[i] = ops[9 + i];
    }
    float A[2][6];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int k = 0; k < 6; ++k) A[rb][k] = a_operand(Or, Oi, rb, k, q);
    f4 c0[PB_NF], c1[PB_NF];
#pragma unroll
    for (int f = 0; f < PB_NF; ++f) {
      c0[f] = f4{0.f, 0.f, 0.f, 0.f};
      c1[f] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int f = 0; f < PB_NF; ++f)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const float b = k < 3 ? xr[f * 3 + k] : xi[f * 3 + k - 3];
          c0[f] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[0][k], b, c0[f], 0, 0, 0);
          c1[f] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[1][k], b, c1[f], 0, 0, 0);
        }
    }
#pragma unroll
    for (int f = 0; f < PB_NF; ++f) {
      yr[f * 3] = c0[f][0];
      yr[f * 3 + 1] = c0[f][1];
      yr[f * 3 + 2] = c0[f][2];
      yi[f * 3] = c0[f][3];
      yi[f * 3 + 1] = c1[f][0];
      yi[f * 3 + 2] = c1[f][1];
    }
  }
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < PB_RB; ++r) s += yr[r] + 0.5f * yi[r];
  out[gid] = s;
}

}  // namespace

scp_status launch_probe_contraction(int form, int n_wg, int iters, int nop, const float* ops,
                                    float* out, hipStream_t st) {
  if (form < 0 || form > 2 || n_wg < 1 || iters < 1 || nop < 1 || !ops || !out)
    return fail(SCP_EINVAL, "probe: form 0..2, n_wg, iters, nop >= 1 and device buffers");
  if (form == 0)
    hipLaunchKernelGGL(probe_kernel<0>, dim3(n_wg), dim3(PB_THREADS), 0, st, ops, nop, iters, out);
  else if (form == 1)
    hipLaunchKernelGGL(probe_kernel<1>, dim3(n_wg), dim3(PB_THREADS), 0, st, ops, nop, iters, out);
  else
    hipLaunchKernelGGL(probe_kernel<2>, dim3(n_wg), dim3(PB_THREADS), 0, st, ops, nop, iters, out);
  HIPCHK(hipGetLastError());
  return SCP_OK;
}

}  // namespace scp

extern "C" scp_status scp_probe_contraction(int32_t form, int32_t n_wg, int32_t iters, int32_t nop,
                                            const void* ops, void* out, void* stream) {
  scp::set_error("");
  return scp::launch_probe_contraction(form, n_wg, iters, nop, (const float*)ops, (float*)out,
                                       (hipStream_t)stream);
}
