// Discrete adjoint of the fused RK4 propagation (complex FP32) with
// checkpoints every ce steps.
//
// The gradient is the sum over steps of the per-step terms (Sec. 2.5): the
// costate is carried backward by the transposed step map (for RK4 with
// A_s = -i V(t_s), A_s^dag = i V(t_s)):
//   kb3 = h/6 l',  kb2 = h/3 l' + h yb3,  kb1 = h/3 l' + h/2 yb2,
//   kb0 = h/6 l' + h/2 yb1,  yb_s = i V_s kb_s,  l = l' + sum_s yb_s,
// and every stage adds dL/dtheta += 2 Im <kb_s, dV_s/dtheta y_s>, with y_s the
// stage input of the forward step.  The derivative of V w.r.t. a parameter
// is a sum of local terms, so only local reductions are needed (the paper's
// local adjoint idea): for a coupling g A_i (x) B_j the d x d matrices
//   G_ab = <A~_i kb, E_ab on j  y>   and   H_ab = <W~_j kb, E_ab on i  y>
// give the coupling and the dressed-operator sensitivities of both modes,
// and per mode K_ab = <kb, E_ab y> gives the drive and diagonal ones.  They
// are formed block by block inside the adjoint applicator, folded with the
// rotated operators / operator derivatives of the stage (FP64-built tables)
// into scalars (summed per lane over a layout where they share a target),
// wave-reduced, and accumulated in FP64 per wave, one target per lane.
// No atomics: the result is bitwise reproducible.
//
// Real frame (every term real: each operator real or i times real, both
// factors of a pair term of one kind, drives on real operators): kb and y are
// rotated by D(t)^dag at each stage, the items use the un-rotated real
// operators (a pair term of imaginary factors carries i^2 = -1 in its pair
// table), and the folds with the real derivative tables need only the
// imaginary parts of G, H and K (the first factor's folds of an imaginary
// term take the sign -1); yb is rotated back by D(t).  The frame is held
// fixed, so <kb, D dR D^dag y> = <D^dag kb, dR D^dag y> and the
// sensitivities are unchanged.
//
// Per segment, last to first, a recompute launch (the forward stepper started
// from the segment's checkpoint) writes the four stage inputs of every step
// to the segment buffer, then one launch of the kernel here walks the segment
// back.  Within a stage kb and y sit in LDS in natural order and every layout
// gathers its elements; yb passes from layout to layout in natural order.
// The costate (a compensated hi + lo pair: its per-step increments are small
// against it), the running sum of yb and the FP64 accumulators live in device
// memory and carry between launches exactly.
#include <algorithm>

#include "kernel_common.h"

namespace scp {

namespace {

template <int d>
struct Mat {
  float re[d * d];
  float im[d * d];
};

template <int d>
__device__ __forceinline__ void zero(Mat<d>& m) {
#pragma unroll
  for (int i = 0; i < d * d; ++i) m.re[i] = m.im[i] = 0.f;
}

// Adjoint pair item: ybar += W(at PJ) T + c T with T = O(at PI) kb, and the
// local sensitivities G (along PJ, left factor T) and H (along PI, left
// factor X' = W(at PJ) kb), both against y.
template <int d, int NR, int PI, int PJ, int RB>
__device__ __forceinline__ void group_pair_adj(const Op<d>& O, const Op<d>& W, float c,
                                               const Vec<RB>& kb, const Vec<RB>& y,
                                               Vec<RB>& yb, Mat<d>& G, Mat<d>& H) {
  using C = Cfg<d, NR>;
  constexpr int si_ = C::stride(PI);
  constexpr int sj_ = C::stride(PJ);
  static_for<RB / (d * d)>([&](auto B) {
    constexpr int r0 = fiber_base<d, NR, PI, PJ>(decltype(B)::value);
    float tr[d][d], ti[d][d];
#pragma unroll
    for (int aj = 0; aj < d; ++aj)
#pragma unroll
      for (int ai = 0; ai < d; ++ai) {
        float sr = 0.f, sim = 0.f;
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float orr = O.re[ai * d + b], oi = O.im[ai * d + b];
          const float xr = kb.re[r0 + b * si_ + aj * sj_], xi = kb.im[r0 + b * si_ + aj * sj_];
          sr = fmaf(orr, xr, sr);
          sr = fmaf(-oi, xi, sr);
          sim = fmaf(orr, xi, sim);
          sim = fmaf(oi, xr, sim);
        }
        tr[ai][aj] = sr;
        ti[ai][aj] = sim;
      }
    // apply
#pragma unroll
    for (int ai = 0; ai < d; ++ai)
#pragma unroll
      for (int aj = 0; aj < d; ++aj) {
        float sr = fmaf(c, tr[ai][aj], yb.re[r0 + ai * si_ + aj * sj_]);
        float sim = fmaf(c, ti[ai][aj], yb.im[r0 + ai * si_ + aj * sj_]);
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float wr = W.re[aj * d + b], wi = W.im[aj * d + b];
          sr = fmaf(wr, tr[ai][b], sr);
          sr = fmaf(-wi, ti[ai][b], sr);
          sim = fmaf(wr, ti[ai][b], sim);
          sim = fmaf(wi, tr[ai][b], sim);
        }
        yb.re[r0 + ai * si_ + aj * sj_] = sr;
        yb.im[r0 + ai * si_ + aj * sj_] = sim;
      }
    // G_ab += sum_ai conj(T[ai][a]) y[ai][b]
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) {
        float gr = G.re[a * d + b], gi = G.im[a * d + b];
#pragma unroll
        for (int ai = 0; ai < d; ++ai) {
          const float yr = y.re[r0 + ai * si_ + b * sj_], yi = y.im[r0 + ai * si_ + b * sj_];
          gr = fmaf(tr[ai][a], yr, gr);
          gr = fmaf(ti[ai][a], yi, gr);
          gi = fmaf(tr[ai][a], yi, gi);
          gi = fmaf(-ti[ai][a], yr, gi);
        }
        G.re[a * d + b] = gr;
        G.im[a * d + b] = gi;
      }
    // X'[ai][aj] = sum_b W[aj][b] kb[ai][b]; H_ab += sum_aj conj(X'[a][aj]) y[b][aj]
#pragma unroll
    for (int ai = 0; ai < d; ++ai)
#pragma unroll
      for (int aj = 0; aj < d; ++aj) {
        float sr = 0.f, sim = 0.f;
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float wr = W.re[aj * d + b], wi = W.im[aj * d + b];
          const float xr = kb.re[r0 + ai * si_ + b * sj_], xi = kb.im[r0 + ai * si_ + b * sj_];
          sr = fmaf(wr, xr, sr);
          sr = fmaf(-wi, xi, sr);
          sim = fmaf(wr, xi, sim);
          sim = fmaf(wi, xr, sim);
        }
        tr[ai][aj] = sr;
        ti[ai][aj] = sim;
      }
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) {
        float hr = H.re[a * d + b], hi = H.im[a * d + b];
#pragma unroll
        for (int aj = 0; aj < d; ++aj) {
          const float yr = y.re[r0 + b * si_ + aj * sj_], yi = y.im[r0 + b * si_ + aj * sj_];
          hr = fmaf(tr[a][aj], yr, hr);
          hr = fmaf(ti[a][aj], yi, hr);
          hi = fmaf(tr[a][aj], yi, hi);
          hi = fmaf(-ti[a][aj], yr, hi);
        }
        H.re[a * d + b] = hr;
        H.im[a * d + b] = hi;
      }
  });
}

// K_ab += sum over fibers along P of conj(kb[a]) y[b]
template <int d, int NR, int P, int RB>
__device__ __forceinline__ void mode_reduce(const Vec<RB>& kb, const Vec<RB>& y, Mat<d>& K) {
  using C = Cfg<d, NR>;
  constexpr int st = C::stride(P);
  static_for<RB / d>([&](auto B) {
    constexpr int r0 = fiber_base<d, NR, P, -1>(decltype(B)::value);
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) {
        const float kr = kb.re[r0 + a * st], ki = kb.im[r0 + a * st];
        const float yr = y.re[r0 + b * st], yi = y.im[r0 + b * st];
        K.re[a * d + b] = fmaf(kr, yr, fmaf(ki, yi, K.re[a * d + b]));
        K.im[a * d + b] = fmaf(kr, yi, fmaf(-ki, yr, K.im[a * d + b]));
      }
  });
}

// Real frame (real operators, vectors rotated by D(t)^dag): the same items
// with real O and W; the folds with real tables need only Im G, Im H, Im K.
template <int d, int NR, int PI, int PJ, int RB>
__device__ __forceinline__ void group_pair_adj_real(const ROp<d>& O, const ROp<d>& W, float c,
                                                    const Vec<RB>& kb, const Vec<RB>& y,
                                                    Vec<RB>& yb, Mat<d>& G, Mat<d>& H) {
  using C = Cfg<d, NR>;
  constexpr int si_ = C::stride(PI);
  constexpr int sj_ = C::stride(PJ);
  static_for<RB / (d * d)>([&](auto B) {
    constexpr int r0 = fiber_base<d, NR, PI, PJ>(decltype(B)::value);
    float tr[d][d], ti[d][d];
#pragma unroll
    for (int aj = 0; aj < d; ++aj)
#pragma unroll
      for (int ai = 0; ai < d; ++ai) {
        float sr = 0.f, sim = 0.f;
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float o = O.v[ai * d + b];
          sr = fmaf(o, kb.re[r0 + b * si_ + aj * sj_], sr);
          sim = fmaf(o, kb.im[r0 + b * si_ + aj * sj_], sim);
        }
        tr[ai][aj] = sr;
        ti[ai][aj] = sim;
      }
#pragma unroll
    for (int ai = 0; ai < d; ++ai)
#pragma unroll
      for (int aj = 0; aj < d; ++aj) {
        float sr = fmaf(c, tr[ai][aj], yb.re[r0 + ai * si_ + aj * sj_]);
        float sim = fmaf(c, ti[ai][aj], yb.im[r0 + ai * si_ + aj * sj_]);
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float w = W.v[aj * d + b];
          sr = fmaf(w, tr[ai][b], sr);
          sim = fmaf(w, ti[ai][b], sim);
        }
        yb.re[r0 + ai * si_ + aj * sj_] = sr;
        yb.im[r0 + ai * si_ + aj * sj_] = sim;
      }
    // Im G_ab += sum_ai Im(conj(T[ai][a]) y[ai][b])
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) {
        float gi = G.im[a * d + b];
#pragma unroll
        for (int ai = 0; ai < d; ++ai) {
          gi = fmaf(tr[ai][a], y.im[r0 + ai * si_ + b * sj_], gi);
          gi = fmaf(-ti[ai][a], y.re[r0 + ai * si_ + b * sj_], gi);
        }
        G.im[a * d + b] = gi;
      }
    // X'[ai][aj] = sum_b W[aj][b] kb[ai][b]; Im H_ab += sum_aj Im(conj(X'[a][aj]) y[b][aj])
#pragma unroll
    for (int ai = 0; ai < d; ++ai)
#pragma unroll
      for (int aj = 0; aj < d; ++aj) {
        float sr = 0.f, sim = 0.f;
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float w = W.v[aj * d + b];
          sr = fmaf(w, kb.re[r0 + ai * si_ + b * sj_], sr);
          sim = fmaf(w, kb.im[r0 + ai * si_ + b * sj_], sim);
        }
        tr[ai][aj] = sr;
        ti[ai][aj] = sim;
      }
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) {
        float hi = H.im[a * d + b];
#pragma unroll
        for (int aj = 0; aj < d; ++aj) {
          hi = fmaf(tr[a][aj], y.im[r0 + b * si_ + aj * sj_], hi);
          hi = fmaf(-ti[a][aj], y.re[r0 + b * si_ + aj * sj_], hi);
        }
        H.im[a * d + b] = hi;
      }
  });
}

// Im K_ab += sum over fibers along P of Im(conj(kb[a]) y[b])
template <int d, int NR, int P, int RB>
__device__ __forceinline__ void mode_reduce_real(const Vec<RB>& kb, const Vec<RB>& y, Mat<d>& K) {
  using C = Cfg<d, NR>;
  constexpr int st = C::stride(P);
  static_for<RB / d>([&](auto B) {
    constexpr int r0 = fiber_base<d, NR, P, -1>(decltype(B)::value);
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b)
        K.im[a * d + b] = fmaf(kb.re[r0 + a * st], y.im[r0 + b * st],
                               fmaf(-kb.im[r0 + a * st], y.re[r0 + b * st], K.im[a * d + b]));
  });
}

// Im( sum_ab X_ab M_ab ) for a uniform operator X from the table
template <int d>
__device__ __forceinline__ float im_dot(kptr<c32> X, const Mat<d>& M) {
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < d * d; ++i) {
    s = fmaf(X[i].x, M.im[i], fmaf(X[i].y, M.re[i], s));
  }
  return s;
}

// Im( sum_ab X_ab M_ab ) with X at element offset off of the stage's complex
// table, or (real frame) of the real table.
template <int d, bool RF>
__device__ __forceinline__ float tdot(kptr<c32> ops, kptr<float> rops, int off, const Mat<d>& M) {
  if constexpr (RF) {
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < d * d; ++i) s = fmaf(rops[off + i], M.im[i], s);
    return s;
  } else {
    return im_dot<d>(ops + off, M);
  }
}

// Sum over the 64 lanes (the result is uniform): a butterfly inside each row
// of 16 lanes with DPP (quad xor 1, quad xor 2, half-row mirror, row mirror),
// then row broadcasts 15 and 31 gather the four row sums into lane 63.  No LDS
// round trips; the order is fixed, so the result is deterministic.
template <int ctrl, int row_mask>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, row_mask, 0xF, false));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_f<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_f<0x141, 0xF>(v);   // row_half_mirror
  v += dpp_f<0x140, 0xF>(v);   // row_mirror: every lane holds its row's sum
  v += dpp_f<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_f<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// FP64 gradient accumulators of one wave.  Target t < 128 is held by lane
// t & 63 of a[t >> 6] (every lane owns one target per register, so adding to
// a target is a masked add, with no branch and no LDS round trip); targets
// from 128 on live in this wave's LDS row.  Each target receives the same
// sequence of FP64 additions in either place.
struct LaneAcc {
  double a0, a1;
};

__device__ __forceinline__ void acc_add(LaneAcc& A, double* accw, int target, double x,
                                        int lane) {
  if (target < 64) {
    A.a0 += (lane == target) ? x : 0.0;
  } else if (target < 128) {
    A.a1 += (lane == target - 64) ? x : 0.0;
  } else if (lane == 0) {
    accw[target] += x;
  }
}

// target += sum over the wave of v
__device__ __forceinline__ void fold(LaneAcc& A, double* accw, int target, float v, int lane) {
  acc_add(A, accw, target, (double)wave_sum(v), lane);
}


// A device-memory pointer the compiler cannot see through: the addresses
// derived from it are formed where they are used instead of being hoisted out
// of the step loop (27 live 64-bit addresses per array otherwise).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> fresh(T* p) {
  uintptr_t u = (uintptr_t)p;
  asm volatile("" : "+v"(u));
  return (gptr<T>)u;
}

// One adjoint stage: yb = i V(t) kb (base layout out), with the parameter
// folds of this stage.  kb and y are in natural order in LDS regions 0 and 1
// (read only during the stage), and every layout gathers its elements from
// there; yb accumulates layout by layout and passes to the next layout in
// natural order through region 2.
template <int d, int NR, int MP, int RB, bool RF>
__device__ __forceinline__ void adj_stage(kptr<Plan> P, c32* lds, int cbase,
                                          int vstride, bool lds_ok, int tc, int lane,
                                          LaneAcc& A, double* accw, kptr<c32> ops,
                                          kptr<float> rops, kptr<float> cq,
                                          kptr<float> dcq, Vec<RB>& yb) {
  constexpr int dd = d * d;
  const int L = P->L;
  const int npulse = P->npulse, N = P->N;
#pragma unroll
  for (int r = 0; r < RB; ++r) yb.re[r] = yb.im[r] = 0.f;
  // per-lane derivative sums of a mode shared by the last register position
  // of one layout and the first of the next are carried across the boundary
  float carry[3] = {0.f, 0.f, 0.f};
  for (int lv = 0; lv < L; ++lv) {
    const int l = __builtin_amdgcn_readfirstlane(lv);
    const int tb = cbase + thread_base<d>(P, l, tc);
    const RegOff<d, NR> R = reg_off_of<d, NR>(P, l);
    if (l > 0) {
      // the previous layout's yb (natural order in region 2) is visible
      __syncthreads();
      if (lds_ok) lds_get<d, NR, RB>(lds + 2 * vstride, tb, R, yb);
    }
    Vec<RB> kb, y;
    if (lds_ok) {
      lds_get<d, NR, RB>(lds, tb, R, kb);
      lds_get<d, NR, RB>(lds + vstride, tb, R, y);
    } else {
#pragma unroll
      for (int r = 0; r < RB; ++r) kb.re[r] = kb.im[r] = y.re[r] = y.im[r] = 0.f;
    }
    // derivative contributions to the (EJ, EC, EL) of the mode at each register
    // position, summed per lane over this layout's terms and reduced once
    float dacc[NR * 3];
#pragma unroll
    for (int i = 0; i < NR * 3; ++i) dacc[i] = i < 3 ? carry[i] : 0.f;
    // pair terms
    static_for<NR - 1>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      static_for<MP>([&](auto Mm) {
        constexpr int m = decltype(Mm)::value;
        const auto& C = P->cpair[l][p][m];
        const int c_slot = uni(C.slot), c_pair = uni(C.pair);
        Mat<d> G, H;
        zero(G);
        zero(H);
        if constexpr (RF) {
          ROp<d> O, W;
          load_rop<d>(rops + c_slot * dd, O);
          load_rop<d>(rops + uni(P->off_pair + c_pair * dd), W);
          group_pair_adj_real<d, NR, p, p + 1>(O, W, coef(cq, uni(C.cidx)), kb, y, yb, G, H);
        } else {
          Op<d> O, W;
          load_op<d>(ops + c_slot * dd, O);
          load_op<d>(ops + uni(P->off_pair + c_pair * dd), W);
          group_pair_adj<d, NR, p, p + 1>(O, W, coef(cq, uni(C.cidx)), kb, y, yb, G, H);
        }
        const int mi = uni(C.mode_i);
        if (mi >= 0) {
          // couplings of this pair term; the partner's (position p + 1) and the
          // first factor's (position p) operator derivatives
          const int pr = c_pair;
          const int nq = uni(P->pair_ncoup[pr]);
          const int offd = uni(P->off_dslot);
          for (int q = 0; q < nq; ++q) {
            const int e = uni(P->pair_coup[pr][q]);
            const int sj = uni(P->pair_pslot[pr][q]);
            fold(A, accw, npulse + 3 * N + e, tdot<d, RF>(ops, rops, sj * dd, G), lane);
            const float ge = unif(P->coup_g[e]);
#pragma unroll
            for (int th = 0; th < 3; ++th)
              dacc[(p + 1) * 3 + th] += ge * tdot<d, RF>(ops, rops, offd + (sj * 3 + th) * dd, G);
          }
          // real frame, first factor i times real: its folds change sign (i^2)
          const float hs = RF ? (float)uni(C.hsign) : 1.f;
#pragma unroll
          for (int th = 0; th < 3; ++th)
            dacc[p * 3 + th] += hs * tdot<d, RF>(ops, rops, offd + (c_slot * 3 + th) * dd, H);
        }
      });
    });
    if (uni(P->has_single[l])) {
      static_for<NR>([&](auto Pp) {
        constexpr int p = decltype(Pp)::value;
        const auto& C1 = P->csingle[l][p];
        const float c = coef(cq, uni(C1.cidx));
        if constexpr (RF) {
          ROp<d> O;
          load_rop<d>(rops + uni(C1.slot) * dd, O);
#pragma unroll
          for (int i = 0; i < dd; ++i) O.v[i] *= c;
          contract_acc_real<d, NR, p>(O, kb, yb);
        } else {
          Op<d> O;
          load_op<d>(ops + uni(C1.slot) * dd, O);
#pragma unroll
          for (int i = 0; i < dd; ++i) {
            O.re[i] *= c;
            O.im[i] *= c;
          }
          contract_acc<d, NR, p>(O, kb, yb);
        }
      });
    }
    if (uni(P->has_diag[l])) {
      static_for<NR>([&](auto Pp) {
        constexpr int p = decltype(Pp)::value;
        diag_acc<d, NR, p>(P->delta[uni(P->cdiag[l][p])], kb, yb);
      });
    }
    // yb is complete for this layout: hand it to the next one (each element has
    // one owner per layout, so one barrier per layout boundary suffices)
    if (l + 1 < L && lds_ok) lds_put<d, NR, RB>(lds + 2 * vstride, tb, R, yb);
    // single-mode sensitivities (drives and the diagonal) of the modes owned here
    if (uni(P->has_mode_pass[l])) {
      static_for<NR>([&](auto Pp) {
        constexpr int p = decltype(Pp)::value;
        const int m = uni(P->mode_pass[l][p]);
        if (m >= 0) {
          Mat<d> K;
          zero(K);
          if constexpr (RF)
            mode_reduce_real<d, NR, p>(kb, y, K);
          else
            mode_reduce<d, NR, p>(kb, y, K);
          float dev[3] = {0.f, 0.f, 0.f};
#pragma unroll
          for (int th = 0; th < 3; ++th)
#pragma unroll
            for (int a = 0; a < d; ++a) dev[th] = fmaf(unif(P->deps[m][th][a]), K.im[a * d + a], dev[th]);
          const int offd = uni(P->off_dslot);
          const int k0 = uni(P->mdrv_off[m]), k1 = uni(P->mdrv_off[m + 1]);
          for (int kk = k0; kk < k1; ++kk) {
            const auto& R = P->drives[uni(P->mdrv[kk])];
            const int rslot = uni(R.slot);
            const float s_im = wave_sum(tdot<d, RF>(ops, rops, rslot * dd, K));
            const int par0 = uni(R.par0), npar = uni(R.npar);
            for (int q = 0; q < npar; ++q)
              acc_add(A, accw, par0 + q, (double)dcq[par0 + q] * (double)s_im, lane);
            if (uni(P->mdrv_first[kk])) {   // one c(t) per slot: count the slot once
              const float c = cq[uni(R.cidx)];
#pragma unroll
              for (int th = 0; th < 3; ++th)
                dev[th] = fmaf(c, tdot<d, RF>(ops, rops, offd + (rslot * 3 + th) * dd, K), dev[th]);
            }
          }
#pragma unroll
          for (int th = 0; th < 3; ++th) dacc[p * 3 + th] += dev[th];
        }
      });
    }
    // the last position's mode continues as the next layout's first one?
    const bool pass_on = (NR > 1) && l + 1 < L &&
                         uni(P->lmode[l][NR - 1]) == uni(P->lmode[l + 1][0]) &&
                         uni(P->lmode[l][NR - 1]) >= 0;
    static_for<NR>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      const int m = uni(P->lmode[l][p]);
      if (m >= 0 && !(p == NR - 1 && pass_on)) {
#pragma unroll
        for (int th = 0; th < 3; ++th) fold(A, accw, npulse + 3 * m + th, dacc[p * 3 + th], lane);
      }
    });
#pragma unroll
    for (int th = 0; th < 3; ++th) carry[th] = pass_on ? dacc[(NR - 1) * 3 + th] : 0.f;
  }
  // yb <- i * yb
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const float t = yb.re[r];
    yb.re[r] = -yb.im[r];
    yb.im[r] = t;
  }
}

}  // namespace

// Segments I.seg_hi down to I.seg_lo of column block I.cb.  first != 0: the
// costate starts from the cotangent and the accumulators from zero; else both
// continue from lamstate / part exactly (chunked runs are bitwise identical to
// one launch).
// RF: the real frame (vectors rotated by D(t)^dag at every stage, real
// operator and derivative tables; yb rotated back).
template <int d, int NR, int MP, bool RF>
__device__ __forceinline__ void adjoint_block(const AdjItem& I) {
  constexpr int RB = Cfg<d, NR>::RB;
  extern __shared__ c32 lds[];
  kptr<Plan> P = kconst(I.P);
  kptr<c32> optab = kconst((const c32*)I.optab);
  kptr<c32> ph = kconst((const c32*)I.ph);
  kptr<float> rops = kconst(I.rops);
  const int NT = uni(P->NT);
  const int prow = RF ? uni(P->ph_row) : 0;
  const int pthr = RF ? uni(P->ph_thr) : 0;
  kptr<float> ctab = kconst(I.ctab);
  kptr<float> dctab = kconst(I.dctab);
  const c32x2* __restrict__ ckpt = (const c32x2*)I.ckpt;
  c32* __restrict__ segbuf = (c32*)I.segbuf;
  const int ce = I.ce, S = I.S;
  const int TPC = P->TPC, CPW = P->CPW, D = P->D, L = P->L, N = P->nsteps;
  const int cw = threadIdx.x / TPC;
  const int tc = threadIdx.x - cw * TPC;
  const int col = I.cb * CPW + cw;
  const bool lds_ok = cw < CPW;
  const bool active = lds_ok && col < S;
  const int cbase = cw * D;
  const int vstride = CPW * D;
  const int base = L - 1;
  const float h = P->h;
  const int ng = P->ngroups, npl = P->npulse, nacc = P->nacc;
  const int bq = P->block_q;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  // LDS: [CPW D] kb and [CPW D] y of the stage in natural order | [CPW D] the
  // layout moves of yb | FP64 accumulators of the waves (targets >= 128, and
  // the hand-over to part).
  double* acc = reinterpret_cast<double*>(lds + 3 * (size_t)CPW * D);
  double* accw = acc + wave * nacc;
  double* partb = I.part + (size_t)I.cb * 4 * nacc;
  for (int i = threadIdx.x; i < nwaves * nacc; i += blockDim.x)
    acc[i] = (I.first || i >= 4 * nacc) ? 0.0 : partb[i];
  __syncthreads();
  LaneAcc A;
  A.a0 = lane < nacc ? accw[lane] : 0.0;
  A.a1 = lane + 64 < nacc ? accw[lane + 64] : 0.0;

  const size_t colreg = (size_t)(active ? col : 0) * D + tc;   // register-order slice
  c32* ysum = (c32*)I.sum + colreg;            // per-step sum of yb (device memory)
  c32* lst = (c32*)I.lamstate + colreg;        // costate lambda (device memory)
  c32* lsl = (c32*)I.lamlo + colreg;           // its compensation word
  const size_t ystride = (size_t)S * D;        // between stages in the segment buffer
  c32* ycol0 = segbuf + (size_t)(active ? col : 0) * D;   // this column, natural order
  const int tbB = thread_base<d>(P, base, tc);            // base-layout addressing
  const RegOff<d, NR> RB_ = reg_off_of<d, NR>(P, base);
  // the costate starts from the cotangent (natural order) on the first launch
  if (active && I.first) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      lst[(size_t)r * TPC] = ((const c32*)I.lamT)[(size_t)col * D + tbB + RB_(r)];
      lsl[(size_t)r * TPC] = c32{0.f, 0.f};
    }
  }

  float pf_sink = 0.f;
  {
    const int seg = I.seg_hi;
    const int start = seg * ce;
    const int stop = min(start + ce, N);
    // walk the segment back.  As in the stepper, one stage ahead the first
    // threads of each column touch every 64-byte line of the next (earlier)
    // stage's operator block, so its scalar reads find the lines in L2.
    const int pf_lines = RF ? (prow * (int)sizeof(c32) + 63) / 64 : (bq * (int)sizeof(c32) + 63) / 64;
    const kptr<c32> pf_base = RF ? ph : optab;
    const int pf_stride = RF ? prow : bq;
    for (int n = stop - 1; n >= start; --n) {
      Vec<RB> yb;
#pragma unroll
      for (int r = 0; r < RB; ++r) yb.re[r] = yb.im[r] = 0.f;
#pragma unroll 1
      for (int sv = 3; sv >= 0; --sv) {
        const int s = __builtin_amdgcn_readfirstlane(sv);
        const float bs = (s == 0 || s == 3) ? h * (1.0f / 6.0f) : h * (1.0f / 3.0f);
        const float as = (s == 2) ? h : 0.5f * h;   // coefficient of yb_{s+1}; unused for s = 3
        // kb = bs lambda + as yb_{s+1} and the stage input y (base layout)
        Vec<RB> kb, y;
        {
          const gptr<c32> lm_p = fresh(lst);
          const gptr<c32> y_p = fresh(ycol0 + (size_t)((n - start) * 4 + s) * ystride + tbB);
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            float lx = 0.f, ly = 0.f, vx = 0.f, vy = 0.f;
            if (active) {
              lx = lm_p[(size_t)r * TPC].x;
              ly = lm_p[(size_t)r * TPC].y;
              vx = y_p[RB_(r)].x;
              vy = y_p[RB_(r)].y;
            }
            kb.re[r] = s == 3 ? bs * lx : fmaf(as, yb.re[r], bs * lx);
            kb.im[r] = s == 3 ? bs * ly : fmaf(as, yb.im[r], bs * ly);
            y.re[r] = vx;
            y.im[r] = vy;
          }
        }
        kptr<c32> prw = ph + (size_t)stage_q(n, s) * prow;
        // thread part of the stage's frame phase (also for yb at the end)
        c32 pt{1.f, 0.f};
        if constexpr (RF) pt = thread_phase<d>(prw + pthr, NT, tc);
        if constexpr (RF) {
          // into the frame: kb <- D^dag kb, y <- D^dag y
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            const c32 e = elem_phase<true>(pt, (kptr<c32x8>)prw, r);
            float xr = kb.re[r], xi = kb.im[r];
            kb.re[r] = e.x * xr - e.y * xi;
            kb.im[r] = fmaf(e.x, xi, e.y * xr);
            xr = y.re[r];
            xi = y.im[r];
            y.re[r] = e.x * xr - e.y * xi;
            y.im[r] = fmaf(e.x, xi, e.y * xr);
          }
        }
        // regions 0 and 1 were last read before this barrier (previous stage)
        __syncthreads();
        if (lds_ok) {
          lds_put<d, NR, RB>(lds, cbase + tbB, RB_, kb);
          lds_put<d, NR, RB>(lds + vstride, cbase + tbB, RB_, y);
        }
        __syncthreads();
        auto ops = optab + (RF ? 0 : (size_t)stage_q(n, s) * bq);
        auto cq = ctab + (size_t)stage_c(n, s) * ng;
        auto dcq = dctab + (size_t)stage_c(n, s) * npl;
        float pf = 0.f;
        if (tc < pf_lines) {
          const int qn = s > 0 ? stage_q(n, s - 1) : stage_q(n - 1, 3);   // >= 0
          pf = ((const float*)(uintptr_t)(pf_base + (size_t)qn * pf_stride))[tc * 16];
        }
        adj_stage<d, NR, MP, RB, RF>(P, lds, cbase, vstride, lds_ok, tc, lane, A, accw, ops, rops,
                                     cq, dcq, yb);
        if constexpr (RF) {
          // back to the interaction picture: yb <- D yb
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            const c32 e = elem_phase<false>(pt, (kptr<c32x8>)prw, r);
            const float xr = yb.re[r], xi = yb.im[r];
            yb.re[r] = e.x * xr - e.y * xi;
            yb.im[r] = fmaf(e.x, xi, e.y * xr);
          }
        }
        pf_sink += pf;
        if (active) {
          // sum of the yb of this step; after its last stage lambda <- lambda + sum
          const gptr<c32> ys_p = fresh(ysum);
          const gptr<c32> lm_p = fresh(lst);
          const gptr<c32> ll_p = fresh(lsl);
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            float vx = yb.re[r], vy = yb.im[r];
            if (s != 3) {
              vx = ys_p[(size_t)r * TPC].x + vx;
              vy = ys_p[(size_t)r * TPC].y + vy;
            }
            if (s == 0) {
              // lambda (hi + lo) += the step's sum, compensated: the per-step
              // increments are O(h |V|) of lambda, so plain FP32 accumulation
              // would drift over thousands of steps
              float hx = lm_p[(size_t)r * TPC].x, hy = lm_p[(size_t)r * TPC].y;
              float lx = ll_p[(size_t)r * TPC].x, ly = ll_p[(size_t)r * TPC].y;
              comp_add(hx, lx, vx);
              comp_add(hy, ly, vy);
              lm_p[(size_t)r * TPC].x = hx;
              lm_p[(size_t)r * TPC].y = hy;
              ll_p[(size_t)r * TPC].x = lx;
              ll_p[(size_t)r * TPC].y = ly;
            } else {
              ys_p[(size_t)r * TPC].x = vx;
              ys_p[(size_t)r * TPC].y = vy;
            }
          }
        }
      }
    }
  }
  // keeps the prefetch loads alive; the sum of table values is never this NaN pattern
  if (__float_as_uint(pf_sink) == 0xffffffffu && I.seg_hi < 0) A.a0 += pf_sink;
  // hand the lane accumulators back to the LDS rows
  if (lane < nacc) accw[lane] = A.a0;
  if (lane + 64 < nacc) accw[lane + 64] = A.a1;
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * nacc; i += blockDim.x) partb[i] = i < nwaves * nacc ? acc[i] : 0.0;
}

template <int d, int NR, int MP, bool RF>
__global__ void __launch_bounds__(WG_THREADS) adjoint_kernel(AdjItem I) {
  I.cb = blockIdx.x;
  adjoint_block<d, NR, MP, RF>(I);
}

template <int d, int NR, int MP, bool RF>
__global__ void __launch_bounds__(WG_THREADS) adjoint_batched_kernel(const AdjItem* __restrict__ items) {
  adjoint_block<d, NR, MP, RF>(items[blockIdx.x]);
}

namespace {

size_t adj_lds_bytes(const Plan& P) {
  return sizeof(c32) * 3 * (size_t)P.CPW * P.D + sizeof(double) * 4 * (size_t)P.nacc;
}

template <int d, int NR, int MP, bool RF>
hipError_t run_adj1(const AdjItem& I0, int nwg, int wg, size_t sh, hipStream_t s) {
  hipFuncSetAttribute((const void*)adjoint_kernel<d, NR, MP, RF>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((adjoint_kernel<d, NR, MP, RF>), dim3(nwg), dim3(wg), sh, s, I0);
  return hipGetLastError();
}

template <int d, int NR, int MP>
hipError_t run_adj(const AdjItem& I0, int nwg, int wg, size_t sh, bool rf, hipStream_t s) {
  if (sh > 160 * 1024) return hipErrorInvalidValue;
  if (rf) return run_adj1<d, NR, MP, true>(I0, nwg, wg, sh, s);
  return run_adj1<d, NR, MP, false>(I0, nwg, wg, sh, s);
}

template <int d, int NR, int MP, bool RF>
hipError_t run_adj_batched1(const AdjItem* items, int nitems, int wg, size_t sh, hipStream_t s) {
  hipFuncSetAttribute((const void*)adjoint_batched_kernel<d, NR, MP, RF>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((adjoint_batched_kernel<d, NR, MP, RF>), dim3(nitems), dim3(wg), sh, s, items);
  return hipGetLastError();
}

template <int d, int NR, int MP>
hipError_t run_adj_batched(const AdjItem* items, int nitems, int wg, size_t sh, bool rf,
                           hipStream_t s) {
  if (sh > 160 * 1024) return hipErrorInvalidValue;
  if (rf) return run_adj_batched1<d, NR, MP, true>(items, nitems, wg, sh, s);
  return run_adj_batched1<d, NR, MP, false>(items, nitems, wg, sh, s);
}

}  // namespace

#define SCP_ADJ_ALL(X)                                                      \
  X(2, 1, 1) X(2, 1, 2) X(2, 2, 1) X(2, 2, 2) X(2, 3, 1) X(2, 3, 2) X(2, 4, 1) X(2, 4, 2) \
  X(3, 1, 1) X(3, 1, 2) X(3, 2, 1) X(3, 2, 2) X(3, 3, 1) X(3, 3, 2)                       \
  X(4, 1, 1) X(4, 1, 2) X(4, 2, 1) X(4, 2, 2) X(5, 1, 1) X(5, 1, 2) X(5, 2, 1) X(5, 2, 2)

scp_status launch_rk4_recompute(const scp_system* sys, const float4* ckin, float2* lo,
                                float2* ystore, int S, int n0, int n1, hipStream_t s);

scp_status launch_adjoint_impl(const scp_system* sys, const void* ckpt, const void* lamT,
                               void* segbuf, void* lo, void* sum, void* lamstate, double* part,
                               int ce, int nckpt, int S, hipStream_t s) {
  const Plan& P = sys->plan;
  const int d = P.d, NR = P.NR, MP = P.MP, N = P.nsteps;
  const int nwg = (S + P.CPW - 1) / P.CPW;
  const size_t sh = adj_lds_bytes(P);
  for (int seg = nckpt - 1; seg >= 0; --seg) {
    const int n0 = seg * ce, n1 = std::min(n0 + ce, N);
    hipEvent_t t0 = timing_start(sys, s);
    scp_status st = launch_rk4_recompute(sys, (const float4*)ckpt + (size_t)seg * S * P.D,
                                         (float2*)lo, (float2*)segbuf, S, n0, n1, s);
    if (st != SCP_OK) return st;
    timing_stop(sys, t0, 1, s);
    t0 = timing_start(sys, s);
    AdjItem I{sys->d_plan, sys->d_ops, sys->d_ctab, sys->d_dctab, (const float4*)ckpt,
              (const float2*)lamT, (float2*)segbuf, (float2*)lo, (float2*)sum,
              (float2*)lamstate, part, sys->d_ph, sys->d_rops, ce, nckpt, S, 0, seg, seg,
              seg == nckpt - 1 ? 1 : 0, 0};
    hipError_t e = hipErrorInvalidValue;
    const bool rf = P.real_frame != 0;
#define X(D_, NR_, MP_) \
  if (d == D_ && NR == NR_ && MP == MP_) e = run_adj<D_, NR_, MP_>(I, nwg, P.WG, sh, rf, s);
    SCP_ADJ_ALL(X)
#undef X
    if (e != hipSuccess) return fail(SCP_EHIP, std::string("adjoint launch: ") + hipGetErrorString(e));
    timing_stop(sys, t0, 2, s);
  }
  return SCP_OK;
}

scp_status launch_adjoint_batched(int d, int NR, int MP, bool rf, const AdjItem* items, int nitems,
                                  int wg, size_t sh, hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
#define X(D_, NR_, MP_) \
  if (d == D_ && NR == NR_ && MP == MP_) e = run_adj_batched<D_, NR_, MP_>(items, nitems, wg, sh, rf, s);
  SCP_ADJ_ALL(X)
#undef X
  if (e != hipSuccess)
    return fail(SCP_EHIP, std::string("batched adjoint launch: ") + hipGetErrorString(e));
  return SCP_OK;
}

size_t adjoint_lds_bytes(const Plan& P) { return adj_lds_bytes(P); }

}  // namespace scp
