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
// into scalars, wave-reduced, and accumulated in FP64 per wave in LDS.
// No atomics: the result is bitwise reproducible.
//
// One workgroup owns its columns for the whole adjoint: for each segment,
// last to first, it recomputes the segment's steps from the checkpoint
// (storing the four stage inputs of every step) and then walks them back.
#include "kernel_common.h"

namespace scp {

namespace {

template <int d>
__device__ __forceinline__ int thread_base_a(const Plan* __restrict__ P, int l, int tc) {
  int b = 0, t = tc;
  const int NT = P->NT;
  for (int k = 0; k < NT; ++k) {
    const int q = t / d;
    b += (t - q * d) * P->tstride[l][k];
    t = q;
  }
  return b;
}

template <int d, int RB>
__device__ __forceinline__ void xswitch1(const Plan* __restrict__ P, c32* lds, int cbase,
                                         bool lds_ok, int tc, int from, int to, Vec<RB>& v) {
  __syncthreads();
  if (lds_ok) lds_put<RB>(lds, cbase + thread_base_a<d>(P, from, tc), P->reg_off[from], v);
  __syncthreads();
  if (lds_ok) lds_get<RB>(lds, cbase + thread_base_a<d>(P, to, tc), P->reg_off[to], v);
}

template <int d, int RB>
__device__ __forceinline__ void xswitch2(const Plan* __restrict__ P, c32* lds, int cbase,
                                         int vstride, bool lds_ok, int tc, int from, int to,
                                         Vec<RB>& v, Vec<RB>& w) {
  __syncthreads();
  if (lds_ok) {
    const int b = cbase + thread_base_a<d>(P, from, tc);
    lds_put<RB>(lds, b, P->reg_off[from], v);
    lds_put<RB>(lds + vstride, b, P->reg_off[from], w);
  }
  __syncthreads();
  if (lds_ok) {
    const int b = cbase + thread_base_a<d>(P, to, tc);
    lds_get<RB>(lds, b, P->reg_off[to], v);
    lds_get<RB>(lds + vstride, b, P->reg_off[to], w);
  }
}

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
        float sr = c * tr[ai][aj], sim = c * ti[ai][aj];
#pragma unroll
        for (int b = 0; b < d; ++b) {
          const float wr = W.re[aj * d + b], wi = W.im[aj * d + b];
          sr = fmaf(wr, tr[ai][b], sr);
          sr = fmaf(-wi, ti[ai][b], sr);
          sim = fmaf(wr, ti[ai][b], sim);
          sim = fmaf(wi, tr[ai][b], sim);
        }
        yb.re[r0 + ai * si_ + aj * sj_] += sr;
        yb.im[r0 + ai * si_ + aj * sj_] += sim;
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

template <int d, int NR, int PI, int RB>
__device__ __forceinline__ void dispatch_pair_adj_j(int pj, const Op<d>& O, const Op<d>& W, float c,
                                                    const Vec<RB>& kb, const Vec<RB>& y,
                                                    Vec<RB>& yb, Mat<d>& G, Mat<d>& H) {
  if constexpr (NR >= 1 && PI != 0) if (pj == 0) { group_pair_adj<d, NR, PI, 0>(O, W, c, kb, y, yb, G, H); return; }
  if constexpr (NR >= 2 && PI != 1) if (pj == 1) { group_pair_adj<d, NR, PI, 1>(O, W, c, kb, y, yb, G, H); return; }
  if constexpr (NR >= 3 && PI != 2) if (pj == 2) { group_pair_adj<d, NR, PI, 2>(O, W, c, kb, y, yb, G, H); return; }
  if constexpr (NR >= 4 && PI != 3) if (pj == 3) { group_pair_adj<d, NR, PI, 3>(O, W, c, kb, y, yb, G, H); return; }
}

template <int d, int NR, int RB>
__device__ __forceinline__ void dispatch_pair_adj(int pi, int pj, const Op<d>& O, const Op<d>& W,
                                                  float c, const Vec<RB>& kb, const Vec<RB>& y,
                                                  Vec<RB>& yb, Mat<d>& G, Mat<d>& H) {
  if constexpr (NR >= 1) if (pi == 0) { dispatch_pair_adj_j<d, NR, 0>(pj, O, W, c, kb, y, yb, G, H); return; }
  if constexpr (NR >= 2) if (pi == 1) { dispatch_pair_adj_j<d, NR, 1>(pj, O, W, c, kb, y, yb, G, H); return; }
  if constexpr (NR >= 3) if (pi == 2) { dispatch_pair_adj_j<d, NR, 2>(pj, O, W, c, kb, y, yb, G, H); return; }
  if constexpr (NR >= 4) if (pi == 3) { dispatch_pair_adj_j<d, NR, 3>(pj, O, W, c, kb, y, yb, G, H); return; }
}

template <int d, int NR, int RB>
__device__ __forceinline__ void dispatch_mode_reduce(int p, const Vec<RB>& kb, const Vec<RB>& y,
                                                     Mat<d>& K) {
  if constexpr (NR >= 1) if (p == 0) { mode_reduce<d, NR, 0>(kb, y, K); return; }
  if constexpr (NR >= 2) if (p == 1) { mode_reduce<d, NR, 1>(kb, y, K); return; }
  if constexpr (NR >= 3) if (p == 2) { mode_reduce<d, NR, 2>(kb, y, K); return; }
  if constexpr (NR >= 4) if (p == 3) { mode_reduce<d, NR, 3>(kb, y, K); return; }
}

// Im( sum_ab X_ab M_ab ) for a uniform operator X from the table
template <int d>
__device__ __forceinline__ float im_dot(const c32* __restrict__ X, const Mat<d>& M) {
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < d * d; ++i) {
    const c32 x = X[i];
    s = fmaf(x.x, M.im[i], fmaf(x.y, M.re[i], s));
  }
  return s;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// acc (this wave's LDS row) [target] += weight * sum over the wave of v
__device__ __forceinline__ void fold(double* accw, int target, float v, int lane, double weight = 1.0) {
  const float s = wave_sum(v);
  if (lane == 0) accw[target] += weight * (double)s;
}

// One adjoint stage: yb = i V(t) kb (base layout out), with the parameter
// folds of this stage.  kb and y enter in the base layout.
template <int d, int NR, int RB>
__device__ __forceinline__ void adj_stage(const Plan* __restrict__ P, c32* lds, int cbase,
                                          int vstride, bool lds_ok, int tc, int lane,
                                          double* accw, const c32* __restrict__ ops,
                                          const float* __restrict__ cq,
                                          const float* __restrict__ dcq, Vec<RB>& kb, Vec<RB>& y,
                                          Vec<RB>& yb) {
  const int L = P->L;
  const int dd = d * d;
  const int npulse = P->npulse, N = P->N;
#pragma unroll
  for (int r = 0; r < RB; ++r) yb.re[r] = yb.im[r] = 0.f;
  for (int l = 0; l < L; ++l) {
    if (l == 0) {
      if (L > 1) xswitch2<d, RB>(P, lds, cbase, vstride, lds_ok, tc, L - 1, 0, kb, y);
    } else {
      xswitch2<d, RB>(P, lds, cbase, vstride, lds_ok, tc, l - 1, l, kb, y);
      xswitch1<d, RB>(P, lds, cbase, lds_ok, tc, l - 1, l, yb);
    }
    const int ni = P->n_items[l];
    for (int it = 0; it < ni; ++it) {
      const Item& I = P->items[l][it];
      if (I.kind == 0) {
        dispatch_diag<d, NR>(I.pos, P->delta[I.mode], kb, yb);
      } else if (I.kind == 1) {
        Op<d> O;
        load_op<d>(ops + I.slot * dd, O);
        const float c = I.cidx >= 0 ? cq[I.cidx] : 0.f;
        if (I.n_part == 0) {
#pragma unroll
          for (int i = 0; i < d * d; ++i) {
            O.re[i] *= c;
            O.im[i] *= c;
          }
          dispatch_single<d, NR>(I.pos, O, kb, yb);
        } else {
          Op<d> W;
          const int p = I.pair[0];
          load_op<d>(ops + P->off_pair + p * dd, W);
          Mat<d> G, H;
          zero(G);
          zero(H);
          dispatch_pair_adj<d, NR>(I.pos, I.pos_j[0], O, W, c, kb, y, yb, G, H);
          // folds: couplings of this pair and the dressed operators of both modes
          const int mi = I.mode, mj = I.mode_j[0];
          for (int q = 0; q < P->pair_ncoup[p]; ++q) {
            const int e = P->pair_coup[p][q];
            const int sj = P->coup_slot_j[e];
            fold(accw, npulse + 3 * N + e, im_dot<d>(ops + sj * dd, G), lane);
            for (int th = 0; th < 3; ++th)
              fold(accw, npulse + 3 * mj + th,
                   P->coup_g[e] * im_dot<d>(ops + P->off_dslot + (sj * 3 + th) * dd, G), lane);
          }
          for (int th = 0; th < 3; ++th)
            fold(accw, npulse + 3 * mi + th,
                 im_dot<d>(ops + P->off_dslot + (I.slot * 3 + th) * dd, H), lane);
        }
      } else {
        // single-mode sensitivities of mode I.mode: drives and the diagonal
        Mat<d> K;
        zero(K);
        dispatch_mode_reduce<d, NR>(I.pos, kb, y, K);
        const int m = I.mode;
        float dev[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int th = 0; th < 3; ++th)
#pragma unroll
          for (int a = 0; a < d; ++a) dev[th] = fmaf(P->deps[m][th][a], K.im[a * d + a], dev[th]);
        for (int k = 0; k < P->ndrives; ++k) {
          const DriveDev& R = P->drives[k];
          if (P->slot_mode[R.slot] != m) continue;
          const float s_im = wave_sum(im_dot<d>(ops + R.slot * dd, K));
          if (lane == 0)
            for (int q = 0; q < R.npar; ++q) accw[R.par0 + q] += (double)dcq[R.par0 + q] * (double)s_im;
          bool first = true;   // one c(t) per slot: count the slot once
          for (int k2 = 0; k2 < k; ++k2) first &= P->drives[k2].slot != R.slot;
          if (first) {
            const float c = cq[R.cidx];
#pragma unroll
            for (int th = 0; th < 3; ++th)
              dev[th] = fmaf(c, im_dot<d>(ops + P->off_dslot + (R.slot * 3 + th) * dd, K), dev[th]);
          }
        }
#pragma unroll
        for (int th = 0; th < 3; ++th) fold(accw, npulse + 3 * m + th, dev[th], lane);
      }
    }
  }
  // yb <- i * yb
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const float t = yb.re[r];
    yb.re[r] = -yb.im[r];
    yb.im[r] = t;
  }
}

__device__ __forceinline__ int sq(int n, int s) { return 2 * n + (s == 0 ? 0 : (s == 3 ? 2 : 1)); }
__device__ __forceinline__ int sc(int n, int s) { return 3 * n + (s == 0 ? 0 : (s == 3 ? 2 : 1)); }

}  // namespace

// forward step helper shared with the recompute: defined in rk4.hip's style
template <int d, int NR, int RB>
__device__ __forceinline__ void fwd_apply(const Plan* __restrict__ P, c32* lds, int cbase,
                                          int vstride, bool lds_ok, int tc,
                                          const c32* __restrict__ ops, const float* __restrict__ cq,
                                          Vec<RB>& y, Vec<RB>& k) {
  const int L = P->L;
#pragma unroll
  for (int r = 0; r < RB; ++r) k.re[r] = k.im[r] = 0.f;
  for (int l = 0; l < L; ++l) {
    if (l == 0) {
      if (L > 1) xswitch1<d, RB>(P, lds, cbase, lds_ok, tc, L - 1, 0, y);
    } else {
      xswitch2<d, RB>(P, lds, cbase, vstride, lds_ok, tc, l - 1, l, y, k);
    }
    apply_layout<d, NR, RB>(P, l, ops, cq, y, k);
  }
}

template <int d, int NR>
__global__ void __launch_bounds__(WG_THREADS)
adjoint_kernel(const Plan* __restrict__ P, const c32* __restrict__ optab,
               const float* __restrict__ ctab, const float* __restrict__ dctab,
               const c32x2* __restrict__ ckpt, const c32* __restrict__ lamT,
               c32* __restrict__ segbuf, c32* __restrict__ lamsave, double* __restrict__ part,
               int ce, int nckpt, int S) {
  constexpr int RB = Cfg<d, NR>::RB;
  extern __shared__ c32 lds[];
  const int TPC = P->TPC, CPW = P->CPW, D = P->D, L = P->L, N = P->nsteps;
  const int cw = threadIdx.x / TPC;
  const int tc = threadIdx.x - cw * TPC;
  const int col = blockIdx.x * CPW + cw;
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
  double* acc = reinterpret_cast<double*>(lds + 2 * (size_t)CPW * D);
  double* accw = acc + wave * nacc;
  for (int i = threadIdx.x; i < nwaves * nacc; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();

  const size_t colreg = (size_t)col * RB * TPC + tc;   // register-order offset of this thread
  Vec<RB> lam;
  if (active) {
    const int tb = thread_base_a<d>(P, base, tc);
    const c32* src = lamT + (size_t)col * D + tb;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const c32 v = src[P->reg_off[base][r]];
      lam.re[r] = v.x;
      lam.im[r] = v.y;
    }
  } else {
#pragma unroll
    for (int r = 0; r < RB; ++r) lam.re[r] = lam.im[r] = 0.f;
  }

  for (int seg = nckpt - 1; seg >= 0; --seg) {
    const int start = seg * ce;
    const int stop = min(start + ce, N);
    // park the costate while the segment is recomputed
    if (active) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        c32 v;
        v.x = lam.re[r];
        v.y = lam.im[r];
        lamsave[colreg + (size_t)r * TPC] = v;
      }
    }
    {
      Vec<RB> hi, lo, ac, y, k;
      if (active) {
        const c32x2* src = ckpt + ((size_t)seg * S + col) * RB * TPC + tc;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const c32x2 v = src[(size_t)r * TPC];
          hi.re[r] = v.x;
          hi.im[r] = v.y;
          lo.re[r] = v.z;
          lo.im[r] = v.w;
        }
      } else {
#pragma unroll
        for (int r = 0; r < RB; ++r) hi.re[r] = hi.im[r] = lo.re[r] = lo.im[r] = 0.f;
      }
      for (int n = start; n < stop; ++n) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          ac.re[r] = ac.im[r] = 0.f;
          y.re[r] = hi.re[r] + lo.re[r];
          y.im[r] = hi.im[r] + lo.im[r];
        }
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
          if (active) {
            c32* dst = segbuf + ((size_t)((n - start) * 4 + s) * S) * RB * TPC + colreg;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
              c32 v;
              v.x = y.re[r];
              v.y = y.im[r];
              dst[(size_t)r * TPC] = v;
            }
          }
          const c32* ops = optab + (size_t)sq(n, s) * bq;
          const float* cq = ctab + (size_t)sc(n, s) * ng;
          fwd_apply<d, NR, RB>(P, lds, cbase, vstride, lds_ok, tc, ops, cq, y, k);
          const float w = (s == 0 || s == 3) ? 1.f : 2.f;
          const float ch = (s == 2) ? h : 0.5f * h;
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            const float kr = k.im[r], ki = -k.re[r];
            ac.re[r] = fmaf(w, kr, ac.re[r]);
            ac.im[r] = fmaf(w, ki, ac.im[r]);
            if (s < 3) {
              y.re[r] = hi.re[r] + fmaf(ch, kr, lo.re[r]);
              y.im[r] = hi.im[r] + fmaf(ch, ki, lo.im[r]);
            }
          }
        }
        const float h6 = h * (1.0f / 6.0f);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          {
            const float dx = h6 * ac.re[r];
            const float sx = hi.re[r] + dx;
            const float bp = sx - hi.re[r];
            const float err = (hi.re[r] - (sx - bp)) + (dx - bp);
            const float l2 = lo.re[r] + err;
            const float s2 = sx + l2;
            lo.re[r] = l2 - (s2 - sx);
            hi.re[r] = s2;
          }
          {
            const float dx = h6 * ac.im[r];
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
    }
    if (active) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const c32 v = lamsave[colreg + (size_t)r * TPC];
        lam.re[r] = v.x;
        lam.im[r] = v.y;
      }
    }
    // walk the segment back
    for (int n = stop - 1; n >= start; --n) {
      Vec<RB> lsum, kb, y, yb;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        lsum.re[r] = lsum.im[r] = 0.f;
        yb.re[r] = yb.im[r] = 0.f;
      }
#pragma unroll 1
      for (int s = 3; s >= 0; --s) {
        const float bs = (s == 0 || s == 3) ? h * (1.0f / 6.0f) : h * (1.0f / 3.0f);
        const float as = (s == 2) ? h : 0.5f * h;   // coefficient of yb_{s+1}; unused for s = 3
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          kb.re[r] = s == 3 ? bs * lam.re[r] : fmaf(as, yb.re[r], bs * lam.re[r]);
          kb.im[r] = s == 3 ? bs * lam.im[r] : fmaf(as, yb.im[r], bs * lam.im[r]);
        }
        if (active) {
          const c32* src = segbuf + ((size_t)((n - start) * 4 + s) * S) * RB * TPC + colreg;
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            const c32 v = src[(size_t)r * TPC];
            y.re[r] = v.x;
            y.im[r] = v.y;
          }
        } else {
#pragma unroll
          for (int r = 0; r < RB; ++r) y.re[r] = y.im[r] = 0.f;
        }
        const c32* ops = optab + (size_t)sq(n, s) * bq;
        const float* cq = ctab + (size_t)sc(n, s) * ng;
        const float* dcq = dctab + (size_t)sc(n, s) * npl;
        adj_stage<d, NR, RB>(P, lds, cbase, vstride, lds_ok, tc, lane, accw, ops, cq, dcq, kb, y, yb);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          lsum.re[r] += yb.re[r];
          lsum.im[r] += yb.im[r];
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        lam.re[r] += lsum.re[r];
        lam.im[r] += lsum.im[r];
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nacc; i += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += acc[w * nacc + i];
    part[(size_t)blockIdx.x * nacc + i] = s;
  }
}

namespace {

template <int d, int NR>
hipError_t run_adj(const scp_system* sys, const c32x2* ckpt, const c32* lamT, c32* segbuf,
                   c32* lamsave, double* part, int ce, int nckpt, int S, hipStream_t s) {
  const Plan& P = sys->plan;
  const int nwg = (S + P.CPW - 1) / P.CPW;
  const size_t sh = sizeof(c32) * 2 * (size_t)P.CPW * P.D + sizeof(double) * (P.WG / 64) * P.nacc;
  if (sh > 160 * 1024) return hipErrorInvalidValue;
  hipFuncSetAttribute((const void*)adjoint_kernel<d, NR>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((adjoint_kernel<d, NR>), dim3(nwg), dim3(P.WG), sh, s, sys->d_plan,
                     (const c32*)sys->d_ops, sys->d_ctab, sys->d_dctab, ckpt, lamT, segbuf,
                     lamsave, part, ce, nckpt, S);
  return hipGetLastError();
}

}  // namespace

scp_status launch_adjoint_impl(const scp_system* sys, const void* ckpt, const void* lamT,
                               void* segbuf, void* lamsave, double* part, int ce, int nckpt, int S,
                               hipStream_t s) {
  const int d = sys->plan.d, NR = sys->plan.NR;
  hipError_t e = hipErrorInvalidValue;
#define SCP_ADJ(D_, NR_) \
  if (d == D_ && NR == NR_) e = run_adj<D_, NR_>(sys, (const c32x2*)ckpt, (const c32*)lamT, (c32*)segbuf, (c32*)lamsave, part, ce, nckpt, S, s);
  SCP_ADJ(2, 1) SCP_ADJ(2, 2) SCP_ADJ(2, 3) SCP_ADJ(2, 4)
  SCP_ADJ(3, 1) SCP_ADJ(3, 2) SCP_ADJ(3, 3)
  SCP_ADJ(4, 1) SCP_ADJ(4, 2)
  SCP_ADJ(5, 1) SCP_ADJ(5, 2)
#undef SCP_ADJ
  if (e != hipSuccess) return fail(SCP_EHIP, std::string("adjoint launch: ") + hipGetErrorString(e));
  return SCP_OK;
}

}  // namespace scp
