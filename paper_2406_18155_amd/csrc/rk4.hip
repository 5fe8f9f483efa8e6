// Fused RK4 stepper in the interaction picture (complex FP32, state on chip).
//
// One workgroup owns CPW columns for the whole run (columns evolve
// independently under the same H(t), so no inter-workgroup traffic).  Each
// column's state stays in registers: psi as a compensated (hi, lo) pair, the
// RK accumulator, the stage input y and the generator output k.  Per stage
// the generator V(t) y = sum of local terms (App. B: one mode's local
// operator contracted at a time) is evaluated layout by layout; between
// layouts y and k pass through LDS.  Classical RK4 (nodes 0, 1/2, 1/2, 1;
// weights 1/6, 1/3, 1/3, 1/6) on psi' = -i V(t) psi; the psi update is a
// two-sum so that 10^4 steps do not drift in FP32.  Rotated operators and
// drive coefficients come from tables reduced in FP64 at build.
#include "kernel_common.h"

namespace scp {

namespace {

template <int d>
__device__ __forceinline__ int thread_base(const Plan* __restrict__ P, int l, int tc) {
  int b = 0, t = tc;
  const int NT = P->NT;
  for (int k = 0; k < NT; ++k) {
    const int q = t / d;
    b += (t - q * d) * P->tstride[l][k];
    t = q;
  }
  return b;
}

// Layout switch of one or two vectors (WAR barrier, write, RAW barrier, read).
template <int d, int RB>
__device__ __forceinline__ void switch1(const Plan* __restrict__ P, c32* lds, int cbase,
                                        bool lds_ok, int tc, int from, int to, Vec<RB>& v) {
  __syncthreads();
  if (lds_ok) lds_put<RB>(lds, cbase + thread_base<d>(P, from, tc), P->reg_off[from], v);
  __syncthreads();
  if (lds_ok) lds_get<RB>(lds, cbase + thread_base<d>(P, to, tc), P->reg_off[to], v);
}

template <int d, int RB>
__device__ __forceinline__ void switch2(const Plan* __restrict__ P, c32* lds, int cbase,
                                        int vstride, bool lds_ok, int tc, int from, int to,
                                        Vec<RB>& v, Vec<RB>& w) {
  __syncthreads();
  if (lds_ok) {
    const int b = cbase + thread_base<d>(P, from, tc);
    lds_put<RB>(lds, b, P->reg_off[from], v);
    lds_put<RB>(lds + vstride, b, P->reg_off[from], w);
  }
  __syncthreads();
  if (lds_ok) {
    const int b = cbase + thread_base<d>(P, to, tc);
    lds_get<RB>(lds, b, P->reg_off[to], v);
    lds_get<RB>(lds + vstride, b, P->reg_off[to], w);
  }
}

}  // namespace

// k = V(t) y for one stage; y enters and k leaves in the base layout (L-1);
// y is left in an unspecified layout.
template <int d, int NR, int RB>
__device__ __forceinline__ void stage_apply(const Plan* __restrict__ P, c32* lds, int cbase,
                                            int vstride, bool lds_ok, int tc,
                                            const c32* __restrict__ ops,
                                            const float* __restrict__ cq, Vec<RB>& y, Vec<RB>& k) {
  const int L = P->L;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    k.re[r] = 0.f;
    k.im[r] = 0.f;
  }
  for (int l = 0; l < L; ++l) {
    if (l == 0) {
      if (L > 1) switch1<d, RB>(P, lds, cbase, lds_ok, tc, L - 1, 0, y);
    } else {
      switch2<d, RB>(P, lds, cbase, vstride, lds_ok, tc, l - 1, l, y, k);
    }
    apply_layout<d, NR, RB>(P, l, ops, cq, y, k);
  }
}

__device__ __forceinline__ int stage_q(int n, int s) { return 2 * n + (s == 0 ? 0 : (s == 3 ? 2 : 1)); }
__device__ __forceinline__ int stage_c(int n, int s) { return 3 * n + (s == 0 ? 0 : (s == 3 ? 2 : 1)); }

template <int d, int NR>
__global__ void __launch_bounds__(WG_THREADS)
rk4_kernel(const Plan* __restrict__ P, const c32* __restrict__ optab,
           const float* __restrict__ ctab, const c32* __restrict__ psi0,
           c32* __restrict__ psiT, c32x2* __restrict__ state, c32x2* __restrict__ ckpt,
           int ckpt_every, int S, int n0, int n1) {
  constexpr int RB = Cfg<d, NR>::RB;
  extern __shared__ c32 lds[];
  const int TPC = P->TPC, CPW = P->CPW, D = P->D, L = P->L;
  const int cw = threadIdx.x / TPC;
  const int tc = threadIdx.x - cw * TPC;
  const int col = blockIdx.x * CPW + cw;
  const bool lds_ok = cw < CPW;
  const bool active = lds_ok && col < S;
  const int cbase = cw * D;
  const int vstride = CPW * D;
  const int base = L - 1;
  const float h = P->h;
  const int ng = P->ngroups;
  const int bq = P->block_q;

  Vec<RB> hi, lo, acc, y, k;
  // load the initial state in the base layout
  if (active) {
    if (psi0 != nullptr) {
      const int tb = thread_base<d>(P, base, tc);
      const c32* src = psi0 + (size_t)col * D + tb;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        c32 v = src[P->reg_off[base][r]];
        hi.re[r] = v.x;
        hi.im[r] = v.y;
        lo.re[r] = 0.f;
        lo.im[r] = 0.f;
      }
    } else {
      const c32x2* src = state + (size_t)col * RB * TPC + tc;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        c32x2 v = src[(size_t)r * TPC];
        hi.re[r] = v.x;
        hi.im[r] = v.y;
        lo.re[r] = v.z;
        lo.im[r] = v.w;
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      hi.re[r] = hi.im[r] = lo.re[r] = lo.im[r] = 0.f;
    }
  }

  for (int n = n0; n < n1; ++n) {
    if (ckpt != nullptr && n % ckpt_every == 0 && active) {
      c32x2* dst = ckpt + ((size_t)(n / ckpt_every) * S + col) * RB * TPC + tc;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        c32x2 v;
        v.x = hi.re[r]; v.y = hi.im[r]; v.z = lo.re[r]; v.w = lo.im[r];
        dst[(size_t)r * TPC] = v;
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      acc.re[r] = 0.f;
      acc.im[r] = 0.f;
      y.re[r] = hi.re[r] + lo.re[r];
      y.im[r] = hi.im[r] + lo.im[r];
    }
#pragma unroll 1
    for (int s = 0; s < 4; ++s) {
      const c32* ops = optab + (size_t)stage_q(n, s) * bq;
      const float* cq = ctab + (size_t)stage_c(n, s) * ng;
      stage_apply<d, NR, RB>(P, lds, cbase, vstride, lds_ok, tc, ops, cq, y, k);
      // k_s = -i V y
      const float w = (s == 0 || s == 3) ? 1.f : 2.f;
      const float ch = (s == 2) ? h : 0.5f * h;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const float kr = k.im[r], ki = -k.re[r];
        acc.re[r] = fmaf(w, kr, acc.re[r]);
        acc.im[r] = fmaf(w, ki, acc.im[r]);
        if (s < 3) {
          y.re[r] = hi.re[r] + fmaf(ch, kr, lo.re[r]);
          y.im[r] = hi.im[r] + fmaf(ch, ki, lo.im[r]);
        }
      }
    }
    // psi <- psi + h/6 acc, compensated
    const float h6 = h * (1.0f / 6.0f);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      {
        const float dx = h6 * acc.re[r];
        const float sx = hi.re[r] + dx;
        const float bp = sx - hi.re[r];
        const float err = (hi.re[r] - (sx - bp)) + (dx - bp);
        const float l2 = lo.re[r] + err;
        const float s2 = sx + l2;
        lo.re[r] = l2 - (s2 - sx);
        hi.re[r] = s2;
      }
      {
        const float dx = h6 * acc.im[r];
        const float sx = hi.im[r] + dx;
        const float bp = sx - hi.im[r];
        const float err = (hi.im[r] - (sx - bp)) + (dx - bp);
        const float l2 = lo.im[r] + err;
        const float s2 = sx + l2;
        lo.im[r] = l2 - (s2 - sx);
        hi.im[r] = s2;
      }
    }
  }
  if (!active) return;
  if (state != nullptr) {
    c32x2* dst = state + (size_t)col * RB * TPC + tc;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      c32x2 v;
      v.x = hi.re[r]; v.y = hi.im[r]; v.z = lo.re[r]; v.w = lo.im[r];
      dst[(size_t)r * TPC] = v;
    }
  }
  if (psiT != nullptr) {
    const int tb = thread_base<d>(P, base, tc);
    c32* dst = psiT + (size_t)col * D + tb;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      c32 v;
      v.x = hi.re[r] + lo.re[r];
      v.y = hi.im[r] + lo.im[r];
      dst[P->reg_off[base][r]] = v;
    }
  }
}

// out = V(t) y at one stage time, through the same stage_apply as the stepper.
template <int d, int NR>
__global__ void __launch_bounds__(WG_THREADS)
apply_kernel(const Plan* __restrict__ P, const c32* __restrict__ ops,
             const float* __restrict__ cq, const c32* __restrict__ yin, c32* __restrict__ out,
             int S) {
  constexpr int RB = Cfg<d, NR>::RB;
  extern __shared__ c32 lds[];
  const int TPC = P->TPC, CPW = P->CPW, D = P->D, L = P->L;
  const int cw = threadIdx.x / TPC;
  const int tc = threadIdx.x - cw * TPC;
  const int col = blockIdx.x * CPW + cw;
  const bool lds_ok = cw < CPW;
  const bool active = lds_ok && col < S;
  const int base = L - 1;
  Vec<RB> y, k;
  if (active) {
    const int tb = thread_base<d>(P, base, tc);
    const c32* src = yin + (size_t)col * D + tb;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      c32 v = src[P->reg_off[base][r]];
      y.re[r] = v.x;
      y.im[r] = v.y;
    }
  } else {
#pragma unroll
    for (int r = 0; r < RB; ++r) y.re[r] = y.im[r] = 0.f;
  }
  stage_apply<d, NR, RB>(P, lds, cw * D, CPW * D, lds_ok, tc, ops, cq, y, k);
  if (!active) return;
  const int tb = thread_base<d>(P, base, tc);
  c32* dst = out + (size_t)col * D + tb;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    c32 v;
    v.x = k.re[r];
    v.y = k.im[r];
    dst[P->reg_off[base][r]] = v;
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
namespace {

template <int d, int NR>
struct Launch {
  static hipError_t rk4(const scp_system* sys, const float2* psi0, float2* psiT, float4* state,
                        float4* ckpt, int ce, int S, int n0, int n1, hipStream_t s) {
    const Plan& P = sys->plan;
    const int nwg = (S + P.CPW - 1) / P.CPW;
    const size_t sh = sizeof(c32) * 2 * (size_t)P.CPW * P.D;
    hipFuncSetAttribute((const void*)rk4_kernel<d, NR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)sh);
    hipLaunchKernelGGL((rk4_kernel<d, NR>), dim3(nwg), dim3(P.WG), sh, s, sys->d_plan,
                       (const c32*)sys->d_ops, sys->d_ctab, (const c32*)psi0, (c32*)psiT,
                       (c32x2*)state, (c32x2*)ckpt, ce, S, n0, n1);
    return hipGetLastError();
  }
  static hipError_t apply(const scp_system* sys, const float2* ops, const float* cq,
                          const float2* y, float2* out, int S, hipStream_t s) {
    const Plan& P = sys->plan;
    const int nwg = (S + P.CPW - 1) / P.CPW;
    const size_t sh = sizeof(c32) * 2 * (size_t)P.CPW * P.D;
    hipFuncSetAttribute((const void*)apply_kernel<d, NR>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((apply_kernel<d, NR>), dim3(nwg), dim3(P.WG), sh, s, sys->d_plan,
                       (const c32*)ops, cq, (const c32*)y, (c32*)out, S);
    return hipGetLastError();
  }
};

template <typename F>
hipError_t dispatch(int d, int NR, F&& f) {
#define SCP_CASE(D_, NR_) \
  if (d == D_ && NR == NR_) return f(Launch<D_, NR_>());
  SCP_CASE(2, 1) SCP_CASE(2, 2) SCP_CASE(2, 3) SCP_CASE(2, 4)
  SCP_CASE(3, 1) SCP_CASE(3, 2) SCP_CASE(3, 3)
  SCP_CASE(4, 1) SCP_CASE(4, 2)
  SCP_CASE(5, 1) SCP_CASE(5, 2)
#undef SCP_CASE
  return hipErrorInvalidValue;
}

}  // namespace

scp_status launch_rk4_range(const scp_system* sys, const float2* psi0, float2* psiT, float4* state,
                            float4* ckpt, int ce, int S, int n0, int n1, hipStream_t s) {
  hipError_t e = dispatch(sys->plan.d, sys->plan.NR, [&](auto L) {
    return decltype(L)::rk4(sys, psi0, psiT, state, ckpt, ce, S, n0, n1, s);
  });
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("rk4 launch: ") + hipGetErrorString(e));
  return SCP_OK;
}

scp_status launch_rk4(scp_system* sys, const float2* psi0, float2* psiT, float4* ckpt,
                      int ckpt_every, int S, hipStream_t s) {
  return launch_rk4_range(sys, psi0, psiT, nullptr, ckpt, ckpt_every, S, 0, sys->n_steps, s);
}

scp_status launch_apply(const scp_system* sys, int step, int stage, const float2* y, float2* out,
                        int S, hipStream_t s) {
  const int q = 2 * step + (stage == 0 ? 0 : (stage == 3 ? 2 : 1));
  const int c = 3 * step + (stage == 0 ? 0 : (stage == 3 ? 2 : 1));
  const float2* ops = sys->d_ops + (size_t)q * sys->plan.block_q;
  const float* cq = sys->d_ctab + (size_t)c * sys->plan.ngroups;
  hipError_t e = dispatch(sys->plan.d, sys->plan.NR, [&](auto L) {
    return decltype(L)::apply(sys, ops, cq, y, out, S, s);
  });
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("apply launch: ") + hipGetErrorString(e));
  return SCP_OK;
}

}  // namespace scp
