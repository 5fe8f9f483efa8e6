// Fused RK4 stepper in the interaction picture (complex FP32, state on chip).
//
// One workgroup owns CPW columns for the whole run (columns evolve
// independently under the same H(t), so no inter-workgroup traffic).  Each
// column's state stays on chip: psi as a compensated (hi, lo) pair and the RK
// accumulator in registers, the stage input y in natural order in LDS.  Per
// stage the generator V(t) y = sum of local terms (App. B: one mode's local
// operator contracted at a time) is evaluated layout by layout; the
// accumulating k moves between layouts through LDS.  Classical RK4 (nodes 0,
// 1/2, 1/2, 1; weights 1/6, 1/3, 1/3, 1/6) on psi' = -i V(t) psi; the psi
// update is a two-sum so that 10^4 steps do not drift in FP32.  Rotated
// operators and drive coefficients come from tables reduced in FP64 at build.
// The same kernel, started from a checkpoint and recording every stage input
// (REC), is the adjoint's recompute of one segment.  When every term is real
// (transmons: the dressed charge operator is real symmetric; fluxoniums: n is
// i times a real antisymmetric matrix and phi is real, so n(x)n and
// phi(x)phi terms are real) the real-frame variant (RF) applies the un-rotated
// real operators between diagonal frame rotations of the stage input and of k,
// which halves the FMAs of every contraction.
#include "kernel_common.h"

namespace scp {

// Whole-run (or chunked) propagation of CPW columns per workgroup.
// psi0 != nullptr: start from psi0 (natural order), lo = 0; else continue from
// state_hi / lo (register order).  At the end: state_hi and lo (if state_hi is
// given) and psiT (natural order, hi + lo, if given).  lo: S x D
// register-order slices, touched only at the start and the end of a run.
// REC: the adjoint's recompute of one segment: start from the checkpoint slab
// ckin and write the four stage inputs of every step to ystore.
// RF: the real-frame stepper (all terms real; frame phases from I.ph).
template <int d, int NR, int MP, bool REC, bool RF>
__device__ __forceinline__ void rk4_block(const FwdItem& I) {
  constexpr int RB = Cfg<d, NR>::RB;
  extern __shared__ c32 lds[];
  kptr<Plan> P = kconst(I.P);
  kptr<c32> optab = kconst((const c32*)I.optab);
  kptr<float> ctab = kconst(I.ctab);
  kptr<c32> ph = kconst((const c32*)I.ph);
  kptr<float> rops = kconst(I.rops);
  const c32* __restrict__ psi0 = (const c32*)I.psi0;
  c32* __restrict__ psiT = (c32*)I.psiT;
  c32* __restrict__ state_hi = (c32*)I.state_hi;
  c32* __restrict__ lo_buf = (c32*)I.lo;
  c32x2* __restrict__ ckpt = (c32x2*)I.ckpt;
  const int ckpt_every = I.ce, S = I.S, n0 = I.n0, n1 = I.n1;
  const int TPC = P->TPC, CPW = P->CPW, D = P->D, L = P->L;
  const int cw = threadIdx.x / TPC;
  const int tc = threadIdx.x - cw * TPC;
  const int col = I.cb * CPW + cw;
  const bool lds_ok = cw < CPW;
  const bool active = lds_ok && col < S;
  const int cbase = cw * D;
  const int vstride = CPW * D;
  const int base = L - 1;
  const size_t colreg = (size_t)(active ? col : 0) * D + tc;   // register-order slice

  Vec<RB> hi, lo;   // psi = hi + lo, both kept in registers for the whole run
#pragma unroll
  for (int r = 0; r < RB; ++r) hi.re[r] = hi.im[r] = lo.re[r] = lo.im[r] = 0.f;
  if (REC && active) {
    const c32x2* src = (const c32x2*)I.ckin + (size_t)col * D + tc;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const c32x2 v = src[(size_t)r * TPC];
      hi.re[r] = v.x;
      hi.im[r] = v.y;
      lo.re[r] = v.z;
      lo.im[r] = v.w;
    }
  } else if (active) {
    if (psi0 != nullptr) {
      const int tb = thread_base<d>(P, base, tc);
      const c32* src = psi0 + (size_t)col * D + tb;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const c32 v = src[P->reg_off[base][r]];
        hi.re[r] = v.x;
        hi.im[r] = v.y;
      }
    } else {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const c32 v = state_hi[colreg + (size_t)r * TPC];
        const c32 l = lo_buf[colreg + (size_t)r * TPC];
        hi.re[r] = v.x;
        hi.im[r] = v.y;
        lo.re[r] = l.x;
        lo.im[r] = l.y;
      }
    }
  }
  int iy = 0, ka = 1, kb = 2;   // LDS regions: stage input, k moves
  int pq = -1;                  // real frame: half-step row of the cached thread phase
  c32 pt_q{1.f, 0.f};
  for (int n = n0; n < n1; ++n) {
    if (ckpt != nullptr && n % ckpt_every == 0 && active) {
      c32x2* dst = ckpt + ((size_t)(n / ckpt_every) * S + col) * D + tc;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        c32x2 v;
        v.x = hi.re[r];
        v.y = hi.im[r];
        v.z = lo.re[r];
        v.w = lo.im[r];
        dst[(size_t)r * TPC] = v;
      }
    }
    if (REC)
      rk4_step<d, NR, MP, RB, RF>(P, lds, cbase, vstride, lds_ok, active, tc, TPC, optab, rops,
                                  ctab, ph, n, hi, lo, iy, ka, kb,
                                  (c32*)I.ystore + (size_t)(active ? col : 0) * D +
                                      (size_t)(n - n0) * 4 * S * D,
                                  (size_t)S * D, pq, pt_q);
    else
      rk4_step<d, NR, MP, RB, RF>(P, lds, cbase, vstride, lds_ok, active, tc, TPC, optab, rops,
                                  ctab, ph, n, hi, lo, iy, ka, kb, nullptr, 0, pq, pt_q);
  }
  if (!active) return;
  if (state_hi != nullptr) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      c32 v, l;
      v.x = hi.re[r];
      v.y = hi.im[r];
      l.x = lo.re[r];
      l.y = lo.im[r];
      state_hi[colreg + (size_t)r * TPC] = v;
      lo_buf[colreg + (size_t)r * TPC] = l;
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

template <int d, int NR, int MP, bool REC, bool RF>
__global__ void __launch_bounds__(WG_THREADS) rk4_kernel(FwdItem I) {
  I.cb = blockIdx.x;
  rk4_block<d, NR, MP, REC, RF>(I);
}

// Batched launch: workgroup b runs items[b] (requests of one size class).
template <int d, int NR, int MP, bool REC, bool RF>
__global__ void __launch_bounds__(WG_THREADS) rk4_batched_kernel(const FwdItem* __restrict__ items) {
  rk4_block<d, NR, MP, REC, RF>(items[blockIdx.x]);
}

// out = V(t) y at one stage time, through the same stage_apply as the stepper.
template <int d, int NR, int MP>
__global__ void __launch_bounds__(WG_THREADS)
apply_kernel(const Plan* __restrict__ Pg, const c32* __restrict__ opsg,
             const float* __restrict__ cqg, const c32* __restrict__ yin, c32* __restrict__ out,
             int S) {
  kptr<Plan> P = kconst(Pg);
  kptr<c32> ops = kconst(opsg);
  kptr<float> cq = kconst(cqg);
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
  if (lds_ok) {
    const int tb = thread_base<d>(P, base, tc);
    lds_put<d, NR, RB>(lds, cw * D + tb, reg_off_of<d, NR>(P, base), y);
  }
  __syncthreads();
  int ka = 1, kb = 2;
  stage_apply<d, NR, MP, RB>(P, lds, cw * D, CPW * D, lds_ok, tc, ops, kconst((const float*)nullptr),
                             cq, 0, ka, kb, k);
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

template <int d, int NR, int MP>
struct Launch {
  template <bool REC, bool RF>
  static hipError_t run1(const scp_system* sys, const FwdItem& I, int S, hipStream_t s) {
    const Plan& P = sys->plan;
    const int nwg = (S + P.CPW - 1) / P.CPW;
    const size_t sh = sizeof(c32) * 3 * (size_t)P.CPW * P.D;
    hipFuncSetAttribute((const void*)rk4_kernel<d, NR, MP, REC, RF>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((rk4_kernel<d, NR, MP, REC, RF>), dim3(nwg), dim3(P.WG), sh, s, I);
    return hipGetLastError();
  }
  template <bool REC>
  static hipError_t run(const scp_system* sys, const FwdItem& I, int S, hipStream_t s) {
    if (sys->plan.real_frame) return run1<REC, true>(sys, I, S, s);
    return run1<REC, false>(sys, I, S, s);
  }
  static hipError_t rk4(const scp_system* sys, const float2* psi0, float2* psiT, float2* state,
                        float2* lo, float4* ckpt, int ce, int S, int n0, int n1, hipStream_t s) {
    FwdItem I{sys->d_plan, sys->d_ops, sys->d_ctab, psi0, psiT, state, lo, ckpt, nullptr, nullptr,
              sys->d_ph, sys->d_rops, ce, S, 0, n0, n1, 0};
    return run<false>(sys, I, S, s);
  }
  static hipError_t recompute(const scp_system* sys, const float4* ckin, float2* lo,
                              float2* ystore, int S, int n0, int n1, hipStream_t s) {
    FwdItem I{sys->d_plan, sys->d_ops, sys->d_ctab, nullptr, nullptr, nullptr, lo, nullptr, ckin,
              ystore, sys->d_ph, sys->d_rops, 1, S, 0, n0, n1, 0};
    return run<true>(sys, I, S, s);
  }
  template <bool REC, bool RF>
  static void batched1(const FwdItem* items, int nitems, int wg, size_t sh, hipStream_t s) {
    hipFuncSetAttribute((const void*)rk4_batched_kernel<d, NR, MP, REC, RF>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((rk4_batched_kernel<d, NR, MP, REC, RF>), dim3(nitems), dim3(wg), sh, s,
                       items);
  }
  static hipError_t batched(const FwdItem* items, int nitems, int wg, size_t sh, bool rec,
                            bool rf, hipStream_t s) {
    if (rf) {
      if (rec)
        batched1<true, true>(items, nitems, wg, sh, s);
      else
        batched1<false, true>(items, nitems, wg, sh, s);
      return hipGetLastError();
    }
    if (rec)
      batched1<true, false>(items, nitems, wg, sh, s);
    else
      batched1<false, false>(items, nitems, wg, sh, s);
    return hipGetLastError();
  }
  static hipError_t apply(const scp_system* sys, const float2* ops, const float* cq,
                          const float2* y, float2* out, int S, hipStream_t s) {
    const Plan& P = sys->plan;
    const int nwg = (S + P.CPW - 1) / P.CPW;
    const size_t sh = sizeof(c32) * 3 * (size_t)P.CPW * P.D;
    hipFuncSetAttribute((const void*)apply_kernel<d, NR, MP>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((apply_kernel<d, NR, MP>), dim3(nwg), dim3(P.WG), sh, s, sys->d_plan,
                       (const c32*)ops, cq, (const c32*)y, (c32*)out, S);
    return hipGetLastError();
  }
};

template <typename F>
hipError_t dispatch(int d, int NR, int MP, F&& f) {
#define SCP_CASE(D_, NR_)                                        \
  if (d == D_ && NR == NR_ && MP == 1) return f(Launch<D_, NR_, 1>()); \
  if (d == D_ && NR == NR_ && MP == 2) return f(Launch<D_, NR_, 2>());
  SCP_CASE(2, 1) SCP_CASE(2, 2) SCP_CASE(2, 3) SCP_CASE(2, 4)
  SCP_CASE(3, 1) SCP_CASE(3, 2) SCP_CASE(3, 3)
  SCP_CASE(4, 1) SCP_CASE(4, 2)
  SCP_CASE(5, 1) SCP_CASE(5, 2)
#undef SCP_CASE
  return hipErrorInvalidValue;
}

}  // namespace

scp_status launch_rk4_range(const scp_system* sys, const float2* psi0, float2* psiT, float2* state,
                            float2* lo, float4* ckpt, int ce, int S, int n0, int n1, hipStream_t s) {
  hipError_t e = dispatch(sys->plan.d, sys->plan.NR, sys->plan.MP, [&](auto L) {
    return decltype(L)::rk4(sys, psi0, psiT, state, lo, ckpt, ce, S, n0, n1, s);
  });
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("rk4 launch: ") + hipGetErrorString(e));
  return SCP_OK;
}

scp_status launch_rk4(scp_system* sys, const float2* psi0, float2* psiT, float2* lo, float4* ckpt,
                      int ckpt_every, int S, hipStream_t s) {
  hipEvent_t t0 = timing_start(sys, s);
  scp_status st =
      launch_rk4_range(sys, psi0, psiT, nullptr, lo, ckpt, ckpt_every, S, 0, sys->n_steps, s);
  if (st == SCP_OK) timing_stop(sys, t0, 0, s);
  return st;
}

scp_status launch_rk4_recompute(const scp_system* sys, const float4* ckin, float2* lo,
                                float2* ystore, int S, int n0, int n1, hipStream_t s) {
  hipError_t e = dispatch(sys->plan.d, sys->plan.NR, sys->plan.MP, [&](auto L) {
    return decltype(L)::recompute(sys, ckin, lo, ystore, S, n0, n1, s);
  });
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("recompute launch: ") + hipGetErrorString(e));
  return SCP_OK;
}

scp_status launch_apply(const scp_system* sys, int step, int stage, const float2* y, float2* out,
                        int S, hipStream_t s) {
  const int q = 2 * step + (stage == 0 ? 0 : (stage == 3 ? 2 : 1));
  const int c = 3 * step + (stage == 0 ? 0 : (stage == 3 ? 2 : 1));
  const float2* ops = sys->d_ops + (size_t)q * sys->plan.block_q;
  auto cq = sys->d_ctab + (size_t)c * sys->plan.ngroups;
  hipError_t e = dispatch(sys->plan.d, sys->plan.NR, sys->plan.MP, [&](auto L) {
    return decltype(L)::apply(sys, ops, cq, y, out, S, s);
  });
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("apply launch: ") + hipGetErrorString(e));
  return SCP_OK;
}

}  // namespace scp

namespace scp {
scp_status launch_rk4_batched(int d, int NR, int MP, bool rf, const FwdItem* items, int nitems,
                              int wg, size_t sh, bool recompute, hipStream_t s) {
  hipError_t e = dispatch(d, NR, MP, [&](auto L) {
    return decltype(L)::batched(items, nitems, wg, sh, recompute, rf, s);
  });
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("batched rk4 launch: ") + hipGetErrorString(e));
  return SCP_OK;
}
}  // namespace scp
