// Device building blocks shared by the fused stepper, the applicator and the
// adjoint: register-resident state in a mode layout, LDS layout switches,
// and the per-mode contractions of one term item.
//
// State of one column: D = d^N complex amplitudes.  In layout l a thread
// holds RB = d^NR of them in registers: the digits of the NR "register
// modes" of layout l index the registers (position 0 most significant), the
// digits of the other modes index the thread inside the column.  Element of
// register r of thread t: tb[l](t) + reg_off[l][r] in the natural (mode-0
// slowest) order.  A contraction on a register mode is local to the thread;
// switching layouts goes through LDS in natural order.
#pragma once

#include <utility>
#include <type_traits>

#include "internal.h"

namespace scp {

template <int d, int NR>
struct Cfg {
  static constexpr int RB = (NR == 1) ? d : (NR == 2) ? d * d : (NR == 3) ? d * d * d
                          : (NR == 4) ? d * d * d * d : d * d * d * d * d;
  static constexpr int stride(int p) {
    int s = 1;
    for (int q = p + 1; q < NR; ++q) s *= d;
    return s;
  }
  static constexpr int digit(int r, int p) { return (r / stride(p)) % d; }
};

// Vector of RB complex amplitudes in registers.
template <int RB>
struct Vec {
  float re[RB];
  float im[RB];
};

// Plain complex storage types for device memory (no vector-type punning).
struct c32 {
  float x, y;
};
struct c32x2 {   // compensated pair (hi.re, hi.im, lo.re, lo.im)
  float x, y, z, w;
};

// ----------------------------------------------------------------------------
// layout switches through LDS
// ----------------------------------------------------------------------------
template <int RB>
__device__ __forceinline__ void lds_put(c32* lds, int base, const int* __restrict__ roff,
                                        const Vec<RB>& v) {
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    c32 t;
    t.x = v.re[r];
    t.y = v.im[r];
    lds[base + roff[r]] = t;
  }
}

template <int RB>
__device__ __forceinline__ void lds_get(const c32* lds, int base, const int* __restrict__ roff,
                                        Vec<RB>& v) {
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    c32 t = lds[base + roff[r]];
    v.re[r] = t.x;
    v.im[r] = t.y;
  }
}

// ----------------------------------------------------------------------------
// operators (uniform, read through the scalar path)
// ----------------------------------------------------------------------------
template <int d>
struct Op {
  float re[d * d];
  float im[d * d];
};

template <int d>
__device__ __forceinline__ void load_op(const c32* __restrict__ p, Op<d>& o) {
#pragma unroll
  for (int i = 0; i < d * d; ++i) {
    c32 t = p[i];
    o.re[i] = t.x;
    o.im[i] = t.y;
  }
}

// Compile-time loop (guaranteed expansion; register arrays stay in VGPRs).
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Register index of the b-th fiber base (digit 0 at the excluded positions X1, X2).
template <int d, int NR, int X1, int X2>
constexpr int fiber_base(int b) {
  int r = 0;
  for (int p = NR - 1; p >= 0; --p) {
    if (p == X1 || p == X2) continue;
    r += (b % d) * Cfg<d, NR>::stride(p);
    b /= d;
  }
  return r;
}

// out += (O at position P) in, for all fibers along P
template <int d, int NR, int P, int RB>
__device__ __forceinline__ void contract_acc(const Op<d>& O, const Vec<RB>& in, Vec<RB>& out) {
  using C = Cfg<d, NR>;
  constexpr int st = C::stride(P);
  static_for<RB / d>([&](auto B) {
    constexpr int r0 = fiber_base<d, NR, P, -1>(decltype(B)::value);
#pragma unroll
    for (int a = 0; a < d; ++a) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int b = 0; b < d; ++b) {
        const float orr = O.re[a * d + b], oi = O.im[a * d + b];
        const float xr = in.re[r0 + b * st], xi = in.im[r0 + b * st];
        sr = fmaf(orr, xr, sr);
        sr = fmaf(-oi, xi, sr);
        si = fmaf(orr, xi, si);
        si = fmaf(oi, xr, si);
      }
      out.re[r0 + a * st] += sr;
      out.im[r0 + a * st] += si;
    }
  });
}

// Group item with one partner: out += W(at PJ) O(at PI) in + c O(at PI) in,
// evaluated block by block over the (PI, PJ) plane to keep temporaries small.
template <int d, int NR, int PI, int PJ, int RB>
__device__ __forceinline__ void group_pair(const Op<d>& O, const Op<d>& W, float c,
                                           const Vec<RB>& in, Vec<RB>& out) {
  using C = Cfg<d, NR>;
  constexpr int si_ = C::stride(PI);
  constexpr int sj_ = C::stride(PJ);
  static_for<RB / (d * d)>([&](auto B) {
    constexpr int r0 = fiber_base<d, NR, PI, PJ>(decltype(B)::value);
    float tr[d][d], ti[d][d];   // T[a_i][a_j] = sum_b O[a_i][b] in[b, a_j]
#pragma unroll
    for (int aj = 0; aj < d; ++aj)
#pragma unroll
      for (int ai = 0; ai < d; ++ai) {
        float sr = 0.f, sim = 0.f;
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float orr = O.re[ai * d + b], oi = O.im[ai * d + b];
          const float xr = in.re[r0 + b * si_ + aj * sj_], xi = in.im[r0 + b * si_ + aj * sj_];
          sr = fmaf(orr, xr, sr);
          sr = fmaf(-oi, xi, sr);
          sim = fmaf(orr, xi, sim);
          sim = fmaf(oi, xr, sim);
        }
        tr[ai][aj] = sr;
        ti[ai][aj] = sim;
      }
#pragma unroll
    for (int ai = 0; ai < d; ++ai)
#pragma unroll
      for (int aj = 0; aj < d; ++aj) {
        float sr = c * tr[ai][aj], sim = c * ti[ai][aj];
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float wr = W.re[aj * d + b], wi = W.im[aj * d + b];
          sr = fmaf(wr, tr[ai][b], sr);
          sr = fmaf(-wi, ti[ai][b], sr);
          sim = fmaf(wr, ti[ai][b], sim);
          sim = fmaf(wi, tr[ai][b], sim);
        }
        out.re[r0 + ai * si_ + aj * sj_] += sr;
        out.im[r0 + ai * si_ + aj * sj_] += sim;
      }
  });
}

template <int d, int NR, int P, int RB>
__device__ __forceinline__ void diag_acc(const float* __restrict__ dl, const Vec<RB>& in,
                                         Vec<RB>& out) {
  using C = Cfg<d, NR>;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const float v = dl[C::digit(r, P)];
    out.re[r] = fmaf(v, in.re[r], out.re[r]);
    out.im[r] = fmaf(v, in.im[r], out.im[r]);
  }
}

// Dispatch on runtime register positions (uniform branches).
template <int d, int NR, int RB>
__device__ __forceinline__ void dispatch_single(int pi, const Op<d>& O, const Vec<RB>& in,
                                                Vec<RB>& out) {
  if constexpr (NR >= 1) if (pi == 0) { contract_acc<d, NR, 0>(O, in, out); return; }
  if constexpr (NR >= 2) if (pi == 1) { contract_acc<d, NR, 1>(O, in, out); return; }
  if constexpr (NR >= 3) if (pi == 2) { contract_acc<d, NR, 2>(O, in, out); return; }
  if constexpr (NR >= 4) if (pi == 3) { contract_acc<d, NR, 3>(O, in, out); return; }
  if constexpr (NR >= 5) if (pi == 4) { contract_acc<d, NR, 4>(O, in, out); return; }
}

template <int d, int NR, int PI, int RB>
__device__ __forceinline__ void dispatch_pair_j(int pj, const Op<d>& O, const Op<d>& W, float c,
                                                const Vec<RB>& in, Vec<RB>& out) {
  if constexpr (NR >= 1 && PI != 0) if (pj == 0) { group_pair<d, NR, PI, 0>(O, W, c, in, out); return; }
  if constexpr (NR >= 2 && PI != 1) if (pj == 1) { group_pair<d, NR, PI, 1>(O, W, c, in, out); return; }
  if constexpr (NR >= 3 && PI != 2) if (pj == 2) { group_pair<d, NR, PI, 2>(O, W, c, in, out); return; }
  if constexpr (NR >= 4 && PI != 3) if (pj == 3) { group_pair<d, NR, PI, 3>(O, W, c, in, out); return; }
  if constexpr (NR >= 5 && PI != 4) if (pj == 4) { group_pair<d, NR, PI, 4>(O, W, c, in, out); return; }
}

template <int d, int NR, int RB>
__device__ __forceinline__ void dispatch_pair(int pi, int pj, const Op<d>& O, const Op<d>& W,
                                              float c, const Vec<RB>& in, Vec<RB>& out) {
  if constexpr (NR >= 1) if (pi == 0) { dispatch_pair_j<d, NR, 0>(pj, O, W, c, in, out); return; }
  if constexpr (NR >= 2) if (pi == 1) { dispatch_pair_j<d, NR, 1>(pj, O, W, c, in, out); return; }
  if constexpr (NR >= 3) if (pi == 2) { dispatch_pair_j<d, NR, 2>(pj, O, W, c, in, out); return; }
  if constexpr (NR >= 4) if (pi == 3) { dispatch_pair_j<d, NR, 3>(pj, O, W, c, in, out); return; }
  if constexpr (NR >= 5) if (pi == 4) { dispatch_pair_j<d, NR, 4>(pj, O, W, c, in, out); return; }
}

template <int d, int NR, int RB>
__device__ __forceinline__ void dispatch_diag(int pi, const float* dl, const Vec<RB>& in,
                                              Vec<RB>& out) {
  if constexpr (NR >= 1) if (pi == 0) { diag_acc<d, NR, 0>(dl, in, out); return; }
  if constexpr (NR >= 2) if (pi == 1) { diag_acc<d, NR, 1>(dl, in, out); return; }
  if constexpr (NR >= 3) if (pi == 2) { diag_acc<d, NR, 2>(dl, in, out); return; }
  if constexpr (NR >= 4) if (pi == 3) { diag_acc<d, NR, 3>(dl, in, out); return; }
  if constexpr (NR >= 5) if (pi == 4) { diag_acc<d, NR, 4>(dl, in, out); return; }
}

// Apply all items of layout l: out += V_l(t) in, for the half-step block
// `ops` (rotated operators) and the drive coefficients `cq` of this stage.
template <int d, int NR, int RB>
__device__ __forceinline__ void apply_layout(const Plan* __restrict__ P, int l,
                                             const c32* __restrict__ ops,
                                             const float* __restrict__ cq, const Vec<RB>& in,
                                             Vec<RB>& out) {
  const int ni = P->n_items[l];
  for (int it = 0; it < ni; ++it) {
    const Item& I = P->items[l][it];
    if (I.kind == 2) continue;
    if (I.kind == 0) {
      dispatch_diag<d, NR>(I.pos, P->delta[I.mode], in, out);
      continue;
    }
    Op<d> O;
    load_op<d>(ops + I.slot * d * d, O);
    const float c = I.cidx >= 0 ? cq[I.cidx] : 0.f;
    if (I.n_part == 0) {
      // c * O~ y
#pragma unroll
      for (int i = 0; i < d * d; ++i) {
        O.re[i] *= c;
        O.im[i] *= c;
      }
      dispatch_single<d, NR>(I.pos, O, in, out);
    } else {
      Op<d> W;
      load_op<d>(ops + P->off_pair + I.pair[0] * d * d, W);
      dispatch_pair<d, NR>(I.pos, I.pos_j[0], O, W, c, in, out);
    }
  }
}

}  // namespace scp
