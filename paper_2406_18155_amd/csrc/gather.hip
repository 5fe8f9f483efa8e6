// Gather engine: classical RK4 with one column per workgroup, the column held
// in LDS for the whole propagation and every thread evaluating the generator
// on its own elements by gathering their neighbours along the contracted
// digits.  Two uses:
//
// Closed systems (OPEN = false): a state column psi of D = d^N amplitudes
// (element A, the multi-index of the N modes, mode 0 slowest) under the
// interaction-picture generator of Sec. 2.1's local decomposition,
//   k_A = -i [ delta(A) y_A + sum (one- and two-mode contractions of V) ],
// for devices whose columns are too few to fill the chip with the register-
// layout stepper (the 4-fluxonium chain: 16 columns of 625).
//
// Open systems (OPEN = true): the vectorised Lindblad master equation (the
// superoperator form of App. D's closing remark; the LindbladObj component of
// Sec. 2).  rho (D x D) is the rank-2N tensor rho[a_0..a_{N-1}, b_0..b_{N-1}]
// stored row-major: element A*D + B, A the ket and B the bra multi-index.  In
// the interaction picture of the frame,
//   d rho/dt = -i (V rho - rho V) + sum_m g1_m D[a_m(t)] rho + 2 gphi_m D[n_m] rho,
// D[L] rho = L rho L^dag - {L^dag L, rho}/2, a the ladder and n the number
// operator of mode m in its dressed basis.  Per element (A, B):
//   k_AB = dg_AB rho_AB                                       static diagonal
//        + sum_m g1_m J_m(t)[a_m][b_m] rho_{A+e_m, B+e_m}      relaxation jump
//        - i (ket contractions of V) + i (bra contractions of conj V),
//   dg_AB = -i sum_m (delta_m[a_m] - delta_m[b_m]) - sum_m g1_m (a_m + b_m)/2
//           - sum_m gphi_m (a_m - b_m)^2,
//   J_m(t)[a][b] = sqrt((a+1)(b+1)) exp(i (f_a - f_{a+1} - f_b + f_{b+1}) t),
// delta = eps - f the diagonal left by the frame f.
//
// The Hamiltonian enters as one-mode contractions (per driven mode the sum of
// c_k(t) O_k(t) of its drives) and two-mode contractions (per coupled pair of
// modes the d^2 x d^2 operator sum_e g_e O_i(t) (x) O_j(t)), along the ket
// digits with the operator and (open systems) along the bra digits with its
// complex conjugate.  These stage tables are precomputed for every stage row
// of the step grid (3 per step, as the drive coefficients) by one kernel; the
// stepper loads the next stage's table into registers while the current stage
// runs and stores it into LDS after.  LDS holds two stage-input buffers (a
// stage reads y_s from one and writes y_{s+1} into the other), the static
// diagonal and two stage tables; each thread keeps its elements' state
// (compensated hi + lo) and the RK4 accumulator in registers.  One barrier
// per stage.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>
#include <string>

#include "internal.h"
#include "kernel_common.h"

namespace scp {

constexpr int GA_MAXM = 10;      // modes (three-bit digits, 2N (open) or N in one word)
constexpr int GA_MAXDM = 5;      // driven modes
constexpr int GA_MAXPR = 10;     // coupled mode pairs
constexpr int GA_MAXC = 4;       // operators summed into one table entry
constexpr int GA_MAXTAB = 4096;  // complex entries of a stage table
constexpr int GA_PRE = 4;        // table entries each thread prefetches per stage
constexpr int GA_MAXSL = 16;     // slots in a gradient table
constexpr int GA_MAXDS = 10;     // distinct drive slots (gradient)
constexpr int GA_MAXDR = 16;     // drives (gradient)
constexpr int GA_MAXCP = 16;     // couplings (gradient)
constexpr int GA_MAXME = 24;     // coupling ends (closed-system gradient)
// per-wave partial sums of one stage: drive slots | 3 per mode | couplings
constexpr int GA_NV = GA_MAXDS + 3 * GA_MAXM + GA_MAXCP;

// Static description of one gather-engine propagation (device copy in the
// workspace, read through the scalar path where uniform).
struct GArgs {
  const float2* optab;   // [2N+1][block_q] rotated slot operators of the system
  const float* ctab;     // [3N][ngroups] drive coefficients
  const float2* jtab;    // [2N+1][N][d*d] unit-rate relaxation band (open systems)
  const float2* gtab;    // [3N][ntab] stage tables (built by gtab_kernel)
  const float2* x0;      // [S][L] input columns
  float2* xT;            // [S][L] output columns
  int block_q, ngroups, nsteps, S;
  float h;
  int ndm, npr, ntab, has_jump, off_p, off_j;
  int prow;   // stride of a pair-operator row: d^2 rounded up to even
  int orow;   // stride of a driven-mode operator row: d rounded up to even
  int kst[GA_MAXM], bst[GA_MAXM];                    // strides of ket / bra digits in a column
  int dm_mode[GA_MAXDM], dm_n[GA_MAXDM];
  int dm_slot[GA_MAXDM][GA_MAXC], dm_cidx[GA_MAXDM][GA_MAXC];
  int pr_i[GA_MAXPR], pr_j[GA_MAXPR], pr_n[GA_MAXPR];
  int pr_si[GA_MAXPR][GA_MAXC], pr_sj[GA_MAXPR][GA_MAXC];
  float pr_g[GA_MAXPR][GA_MAXC];
  float g1[GA_MAXM], gp[GA_MAXM];
  float delta[GA_MAXM][8];
  // gradient (open systems): the table gains the rotated slot operators and
  // the unit-rate relaxation bands
  int grad, ntabg, off_s, off_u, nsl;
  int sl_slot[GA_MAXSL];                             // system slot of each table slot
  int nds, ds_sl[GA_MAXDS], ds_mode[GA_MAXDS];       // distinct drive slots
  int ndr, dr_ds[GA_MAXDR], dr_par0[GA_MAXDR], dr_npar[GA_MAXDR];
  int ncp, cp_i[GA_MAXCP], cp_j[GA_MAXCP], cp_si[GA_MAXCP], cp_sj[GA_MAXCP];
  // gradient (closed systems, grad = 2): the table gains the rotated slot
  // operators, per mode and device parameter the one-mode derivative operator
  // (sum_k c_k dO_k + d delta), and the derivative slot operators
  int off_m, off_d, off_dslot;
  int mdm[GA_MAXM];                                  // driven-mode index of a mode (-1: none)
  float deps[GA_MAXM][3][8];                         // d delta / d(EJ, EC, EL)
  float cp_g[GA_MAXCP];
  // coupling ends grouped by mode and own table slot: me_beg[m] .. me_beg[m+1]
  // packed (coupling | own slot << 5 | partner slot << 10 | partner mode << 15 |
  // first side << 20 | last of its own-slot group << 21)
  int me_beg[GA_MAXM + 1];
  int me[GA_MAXME];
};

// Checkpoints, costate and gradient buffers of an open-system adjoint.
struct GAdj {
  float4* ck;            // [S][nck][L] (hi re, hi im, lo re, lo im) at steps g * ce
  const float2* cot;     // [S][L] cotangent of the final columns
  float2* seg;           // [S][ce][4][L] stage inputs of the current segment
  const double* dctab;   // [3N][npulse] dc/dpar
  double* part;          // [S][nacc] gradient partial sums
  float4* lam;           // [S][L] costate (hi, lo) between reverse walks
  int ce, nck, npulse, nacc;
};

#define SCP_TRY(expr)                  \
  do {                                 \
    const scp_status st_ = (expr);     \
    if (st_ != SCP_OK) return st_;     \
  } while (0)

namespace {

constexpr int cpow(int b, int e) { return e == 0 ? 1 : b * cpow(b, e - 1); }

// Geometry of one column: N modes of dimension d; a state (L = D) or a
// vectorised density matrix (L = D^2).
template <int d, int N, bool OPEN>
struct GShape {
  static constexpr int D = cpow(d, N);
  static constexpr int L = OPEN ? D * D : D;
  static constexpr int T = L >= 1024 ? 1024 : ((L + 63) / 64) * 64;   // threads
  static constexpr int E = (L + T - 1) / T;                           // elements per thread
  static constexpr int st(int m) { return cpow(d, N - 1 - m); }       // stride in A or B
};

__device__ __forceinline__ int ket_digit(uint32_t pk, int m) { return (pk >> (3 * m)) & 7; }
__device__ __forceinline__ int bra_digit(uint32_t pk, int m, int N) {
  return (pk >> (3 * (N + m))) & 7;
}

__device__ __forceinline__ void cmac(float& sr, float& si, c32 a, c32 b) {
  sr = fmaf(a.x, b.x, sr);
  sr = fmaf(-a.y, b.y, sr);
  si = fmaf(a.x, b.y, si);
  si = fmaf(a.y, b.x, si);
}
// s += conj(a) b
__device__ __forceinline__ void cmac_conj(float& sr, float& si, c32 a, c32 b) {
  sr = fmaf(a.x, b.x, sr);
  sr = fmaf(a.y, b.y, sr);
  si = fmaf(a.x, b.y, si);
  si = fmaf(-a.y, b.x, si);
}

// Row of the drive table of step-grid row r (3 per step: t_n, t_n + h/2,
// t_n + h) and the half-step of its operators.
__device__ __forceinline__ int row_q(int r) { return 2 * (r / 3) + r % 3; }

// Stage table of step-grid row r: [driven-mode operators sum_k c_k O_k]
// [pair operators sum_e g_e O_i (x) O_j][relaxation bands g1_m J_m], from the
// FP32 rotated operators and coefficients.
__global__ void gtab_kernel(const GArgs* __restrict__ Ag, int d, int N, float2* __restrict__ out) {
  const GArgs& A = *Ag;
  const int r = blockIdx.x;
  const int q = row_q(r);
  const int dd = d * d;
  const c32* ops = (const c32*)A.optab + (size_t)q * A.block_q;
  const float* cq = A.ctab + (size_t)r * A.ngroups;
  const int ntot = A.grad ? A.ntabg : A.ntab;
  for (int t = threadIdx.x; t < ntot; t += blockDim.x) {
    float vr = 0.f, vi = 0.f;
    if (t >= A.ntab) {
      if (t < A.off_s + A.nsl * dd) {   // rotated slot operator
        const int u = t - A.off_s;
        const int k = u / dd, ab = u - k * dd;
        const c32 o = ops[A.sl_slot[k] * dd + ab];
        vr = o.x;
        vi = o.y;
      } else if (A.grad == 1) {         // unit-rate relaxation band (then row padding)
        if (t - A.off_u < N * dd) {
          const c32 j = ((const c32*)A.jtab)[((size_t)q * N) * dd + (t - A.off_u)];
          vr = j.x;
          vi = j.y;
        }
      } else if (t < A.off_d) {         // d/dtheta of mode m's one-mode terms
        const int u = t - A.off_m;
        const int m = u / (3 * dd), th = (u / dd) % 3, ab = u % dd;
        const int a = ab / d, b = ab - a * d;
        if (a == b) vr = A.deps[m][th][a];
        const int dm = A.mdm[m];
        if (dm >= 0)
          for (int k = 0; k < A.dm_n[dm]; ++k) {
            const float c = cq[A.dm_cidx[dm][k]];
            const c32 o = ops[A.off_dslot + (A.dm_slot[dm][k] * 3 + th) * dd + ab];
            vr = fmaf(c, o.x, vr);
            vi = fmaf(c, o.y, vi);
          }
      } else if (t < A.off_d + 3 * A.nsl * dd) {   // derivative slot operator
        const int u = t - A.off_d;
        const int k = u / (3 * dd), th = (u / dd) % 3, ab = u % dd;
        const c32 o = ops[A.off_dslot + (A.sl_slot[k] * 3 + th) * dd + ab];
        vr = o.x;
        vi = o.y;
      }
    } else if (t < A.off_p) {
      const int dm = t / (d * A.orow), rr = t - dm * d * A.orow;
      const int ra = rr / A.orow, rb = rr - ra * A.orow;   // rb >= d: row padding
      const int ab = ra * d + rb;
      for (int k = 0; k < (dm < A.ndm && rb < d ? A.dm_n[dm] : 0); ++k) {
        const float c = cq[A.dm_cidx[dm][k]];
        const c32 o = ops[A.dm_slot[dm][k] * dd + ab];
        vr = fmaf(c, o.x, vr);
        vi = fmaf(c, o.y, vi);
      }
    } else if (t < A.off_j) {
      const int u = t - A.off_p;
      const int p = u / (dd * A.prow), rr = u - p * dd * A.prow;
      const int row = rr / A.prow, col = rr - row * A.prow;   // col >= dd: row padding
      const int ai = row / d, aj = row - ai * d, x = col / d, z = col - x * d;
      for (int k = 0; k < (col < dd ? A.pr_n[p] : 0); ++k) {
        const c32 oi = ops[A.pr_si[p][k] * dd + ai * d + x];
        const c32 oj = ops[A.pr_sj[p][k] * dd + aj * d + z];
        const float g = A.pr_g[p][k];
        vr = fmaf(g, oi.x * oj.x - oi.y * oj.y, vr);
        vi = fmaf(g, oi.x * oj.y + oi.y * oj.x, vi);
      }
    } else if (A.has_jump && t - A.off_j < N * dd) {   // relaxation bands (then row padding)
      const int u = t - A.off_j;
      const int m = u / dd;
      const c32 j = ((const c32*)A.jtab)[((size_t)q * N) * dd + u];
      vr = A.g1[m] * j.x;
      vi = A.g1[m] * j.y;
    }
    out[(size_t)r * ntot + t] = make_float2(vr, vi);
  }
}

// Stride of a pair-operator row in the stage table: the d^2 entries padded to
// an even count so that a row starts 16-byte aligned and is read two entries
// per LDS instruction.
template <int d, bool OPEN>
__host__ __device__ constexpr int pair_row() {
  return d * d + ((d * d) & 1);
}

template <int d, bool OPEN>
__host__ __device__ constexpr int one_row() {
  return d + (d & 1);
}

// sum_x row[x] y0[x sm] (CONJ: conj(row[x])) over one driven-mode operator
// row; the row is 16-byte aligned and read two entries at a time
template <int d, bool CONJ>
__device__ __forceinline__ void one_dot(const c32* __restrict__ row, const c32* __restrict__ y0,
                                        int sm, float& sr, float& si) {
  const float4* r4 = reinterpret_cast<const float4*>(row);
#pragma unroll
  for (int k = 0; k < (d + 1) / 2; ++k) {
    const float4 q = r4[k];
    c32 a;
    a.x = q.x;
    a.y = q.y;
    if (CONJ)
      cmac_conj(sr, si, a, y0[(2 * k) * sm]);
    else
      cmac(sr, si, a, y0[(2 * k) * sm]);
    if (2 * k + 1 < d) {
      c32 b;
      b.x = q.z;
      b.y = q.w;
      if (CONJ)
        cmac_conj(sr, si, b, y0[(2 * k + 1) * sm]);
      else
        cmac(sr, si, b, y0[(2 * k + 1) * sm]);
    }
  }
}

// sum_{x,z} row[x d + z] y0[x si + z sj] (CONJ: conj(row[...])) over one
// pair-operator row, read two entries at a time
template <int d, bool CONJ>
__device__ __forceinline__ void pair_dot(const c32* __restrict__ row, const c32* __restrict__ y0,
                                         int si_, int sj_, float& sr, float& si) {
  constexpr int dd = d * d;
  const float4* r4 = reinterpret_cast<const float4*>(row);
#pragma unroll
  for (int k = 0; k < (dd + 1) / 2; ++k) {
    const float4 q = r4[k];
    c32 a;
    a.x = q.x;
    a.y = q.y;
    const c32 ya = y0[((2 * k) / d) * si_ + ((2 * k) % d) * sj_];
    if (CONJ)
      cmac_conj(sr, si, a, ya);
    else
      cmac(sr, si, a, ya);
    if (2 * k + 1 < dd) {
      c32 b;
      b.x = q.z;
      b.y = q.w;
      const c32 yb_ = y0[((2 * k + 1) / d) * si_ + ((2 * k + 1) % d) * sj_];
      if (CONJ)
        cmac_conj(sr, si, b, yb_);
      else
        cmac(sr, si, b, yb_);
    }
  }
}

// k = G(t) y for one element; y read from LDS (neighbours), the own value
// from the caller.
template <int d, int N, bool OPEN>
__device__ __forceinline__ void g_apply(kptr<GArgs> A, const c32* __restrict__ yb,
                                        const c32* __restrict__ tab, int e, uint32_t pk,
                                        float dgr, float dgi, float yr, float yi, float& kr,
                                        float& ki) {
  using Sh = GShape<d, N, OPEN>;
  constexpr int D = Sh::D, dd = d * d;
  kr = dgr * yr - dgi * yi;
  ki = fmaf(dgr, yi, dgi * yr);
  if (OPEN && uni(A->has_jump)) {
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int am = ket_digit(pk, m), bm = bra_digit(pk, m, N);
      if (am < d - 1 && bm < d - 1) {
        const c32 J = tab[A->off_j + m * dd + am * d + bm];
        const c32 v = yb[e + (D + 1) * Sh::st(m)];
        cmac(kr, ki, J, v);
      }
    }
  }
  // driven modes: ket -i Hd y, bra +i y Hd
  const int ndm = uni(A->ndm);
  for (int dmv = 0; dmv < ndm; ++dmv) {
    const int dm = uni(dmv);
    const int m = uni(A->dm_mode[dm]);
    {
      const int sm = uni(A->kst[m]);
      const int am = ket_digit(pk, m);
      constexpr int RD = one_row<d, OPEN>();
      const c32* row = tab + dm * d * RD + am * RD;
      const c32* y0 = yb + e - am * sm;
      float sr = 0.f, si = 0.f;
      one_dot<d, false>(row, y0, sm, sr, si);
      kr += si;
      ki -= sr;
    }
    if (OPEN) {
      const int sm = uni(A->bst[m]);
      const int bm = bra_digit(pk, m, N);
      constexpr int RD = one_row<d, OPEN>();
      const c32* row = tab + dm * d * RD + bm * RD;
      const c32* y0 = yb + e - bm * sm;
      float sr = 0.f, si = 0.f;
      one_dot<d, true>(row, y0, sm, sr, si);
      kr -= si;
      ki += sr;
    }
  }
  // coupled pairs
  const int npr = uni(A->npr);
  for (int pv = 0; pv < npr; ++pv) {
    const int p = uni(pv);
    const int i = uni(A->pr_i[p]), j = uni(A->pr_j[p]);
    constexpr int PR = pair_row<d, OPEN>();
    const c32* P = tab + A->off_p + p * dd * PR;
    {
      const int si_ = uni(A->kst[i]), sj_ = uni(A->kst[j]);
      const int ai = ket_digit(pk, i), aj = ket_digit(pk, j);
      const c32* row = P + (ai * d + aj) * PR;
      const c32* y0 = yb + e - (ai * si_ + aj * sj_);
      float sr = 0.f, si = 0.f;
      pair_dot<d, false>(row, y0, si_, sj_, sr, si);
      kr += si;
      ki -= sr;
    }
    if (OPEN) {
      const int si_ = uni(A->bst[i]), sj_ = uni(A->bst[j]);
      const int bi = bra_digit(pk, i, N), bj = bra_digit(pk, j, N);
      const c32* row = P + (bi * d + bj) * PR;
      const c32* y0 = yb + e - (bi * si_ + bj * sj_);
      float sr = 0.f, si = 0.f;
      pair_dot<d, true>(row, y0, si_, sj_, sr, si);
      kr -= si;
      ki += sr;
    }
  }
}

// One column (col) of a propagation: the body of the stepper kernels.
template <int d, int N, bool OPEN, bool CK>
__device__ __forceinline__ void g_rk4_body(const GArgs* __restrict__ Ag, const GAdj* __restrict__ Bg,
                                           int col, int n_lo, int n_hi,
                                           const float4* __restrict__ st_in,
                                           float4* __restrict__ st_out) {
  using Sh = GShape<d, N, OPEN>;
  constexpr int L = Sh::L, T = Sh::T, E = Sh::E;
  // LDS: two stage-input buffers, the static diagonal, two stage tables
  extern __shared__ __align__(16) c32 lds[];
  kptr<GArgs> A = kconst(Ag);
  const int ntab = A->ntab;
  const int nrow = A->grad ? A->ntabg : ntab;   // table row stride in gtab
  c32* dgb = lds + 2 * L;
  const c32* gtab = (const c32*)A->gtab;
  const int tid = threadIdx.x;
  const float h = A->h;
  const int nsteps = A->nsteps;
  // steps n_lo .. n_hi - 1; the compensated state comes from st_in (else the
  // columns x0, lo = 0) and goes to st_out (a later call continues exactly)
  uint32_t pk[E];
  float hr[E], hm[E], lr[E], lm[E], ar[E], am_[E];
  float dgr_[E], dgi_[E];   // the element's static diagonal (closed systems: in registers)
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = tid + r * T;
    const bool ok = e < L;
    const int Ai = OPEN ? e / Sh::D : e, Bi = OPEN ? e - Ai * Sh::D : 0;
    uint32_t p = 0;
    float gr = 0.f, gi = 0.f;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int a = (Ai / Sh::st(m)) % d;
      p |= (uint32_t)a << (3 * m);
      if (OPEN) {
        const int b = (Bi / Sh::st(m)) % d;
        p |= (uint32_t)b << (3 * (N + m));
        gi -= A->delta[m][a] - A->delta[m][b];
        gr -= 0.5f * A->g1[m] * (float)(a + b) + A->gp[m] * (float)((a - b) * (a - b));
      } else {
        gi -= A->delta[m][a];
      }
    }
    pk[r] = p;
    c32 v;
    v.x = v.y = 0.f;
    lr[r] = lm[r] = 0.f;
    if (ok) {
      if (st_in != nullptr) {
        const float4 q = st_in[(size_t)col * L + e];
        v.x = q.x;
        v.y = q.y;
        lr[r] = q.z;
        lm[r] = q.w;
      } else {
        v = ((const c32*)A->x0)[(size_t)col * L + e];
      }
    }
    hr[r] = v.x;
    hm[r] = v.y;
    ar[r] = am_[r] = 0.f;
    dgr_[r] = gr;
    dgi_[r] = gi;
    if (ok) {
      lds[e] = v;
      if (OPEN) {
        c32 g;
        g.x = gr;
        g.y = gi;
        dgb[e] = g;
      }
    }
  }
  // the stage tables start 16-byte aligned (operator rows are read two
  // entries at a time)
  constexpr int TB = 3 * L + ((3 * L) & 1);
  for (int t = tid; t < ntab; t += T) lds[TB + t] = gtab[(size_t)stage_c(n_lo, 0) * nrow + t];
  __syncthreads();
  // closed systems move table rows two entries (16 bytes) at a time: the
  // tables' rows and LDS buffers are 16-byte aligned and of even length
  constexpr int GP4 = GA_PRE / 2;
  int cur = 0;
#pragma unroll 1
  for (int n = n_lo; n < n_hi; ++n) {
    if (CK) {
      kptr<GAdj> B = kconst(Bg);
      const int ce = B->ce;
      if (n % ce == 0) {
        float4* ck = B->ck + ((size_t)col * B->nck + n / ce) * L;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int e = tid + r * T;
          if (e < L) ck[e] = make_float4(hr[r], hm[r], lr[r], lm[r]);
        }
      }
    }
#pragma unroll 1
    for (int s = 0; s < 4; ++s) {
      const float w = (s == 0 || s == 3) ? 1.f : 2.f;
      const float ch = (s == 2) ? h : 0.5f * h;
      const c32* yc = lds + cur * L;
      const c32* tc = lds + TB + cur * ntab;
      c32* yn = lds + (cur ^ 1) * L;
      // the next stage's table, loaded now and stored after this stage
      const int n2 = s < 3 ? n : n + 1, s2 = s < 3 ? s + 1 : 0;
      const bool more = n2 < n_hi;
      const c32* gnext = gtab + (size_t)stage_c(n2, s2) * nrow;
      c32 pre[OPEN ? GA_PRE : 1];
      float4 pre4[OPEN ? 1 : GP4];
      if constexpr (OPEN) {
#pragma unroll
        for (int k = 0; k < GA_PRE; ++k) {
          const int t = tid + k * T;
          if (more && t < ntab) pre[k] = gnext[t];
        }
      } else {
#pragma unroll
        for (int k = 0; k < GP4; ++k) {
          const int t = tid + k * T;
          pre4[k] = (more && 2 * t < ntab) ? reinterpret_cast<const float4*>(gnext)[t]
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
#pragma unroll
      for (int r = 0; r < E; ++r) {
        int e = tid + r * T;
        uint32_t p = pk[r];
        // opaque per stage: the element's LDS offsets are then formed inside
        // the stage instead of being hoisted out of the step loop (which
        // would hold E sets of them in registers)
        asm volatile("" : "+v"(e), "+v"(p));
        if (e < L) {
          c32 g;
          if (OPEN) {
            g = dgb[e];
          } else {
            g.x = dgr_[r];
            g.y = dgi_[r];
          }
          const c32 ye = yc[e];
          float kr, ki;
          g_apply<d, N, OPEN>(A, yc, tc, e, p, g.x, g.y, ye.x, ye.y, kr, ki);
          if (s == 0) {
            ar[r] = kr;
            am_[r] = ki;
          } else {
            ar[r] = fmaf(w, kr, ar[r]);
            am_[r] = fmaf(w, ki, am_[r]);
          }
          c32 v;
          if (s < 3) {
            v.x = fmaf(ch, kr, hr[r]);
            v.y = fmaf(ch, ki, hm[r]);
          } else {
            const float h6 = h * (1.0f / 6.0f);
            comp_add(hr[r], lr[r], h6 * ar[r]);
            comp_add(hm[r], lm[r], h6 * am_[r]);
            v.x = hr[r];
            v.y = hm[r];
          }
          yn[e] = v;
        }
        // one element at a time: keeps the live registers of the unrolled
        // element loop from piling up across elements
        __builtin_amdgcn_sched_barrier(0);
      }
      if (more) {
        c32* tn = lds + TB + (cur ^ 1) * ntab;
        if constexpr (OPEN) {
#pragma unroll
          for (int k = 0; k < GA_PRE; ++k) {
            const int t = tid + k * T;
            if (t < ntab) tn[t] = pre[k];
          }
          for (int t = tid + GA_PRE * T; t < ntab; t += T) tn[t] = gnext[t];
        } else {
          float4* tn4 = reinterpret_cast<float4*>(tn);
          const float4* gn4 = reinterpret_cast<const float4*>(gnext);
#pragma unroll
          for (int k = 0; k < GP4; ++k) {
            const int t = tid + k * T;
            if (2 * t < ntab) tn4[t] = pre4[k];
          }
          for (int t = tid + GP4 * T; 2 * t < ntab; t += T) tn4[t] = gn4[t];
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  if (st_out != nullptr) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = tid + r * T;
      if (e < L) st_out[(size_t)col * L + e] = make_float4(hr[r], hm[r], lr[r], lm[r]);
    }
  }
  if (A->xT == nullptr || n_hi < nsteps) return;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = tid + r * T;
    if (e < L) {
      c32 v;
      v.x = hr[r] + lr[r];
      v.y = hm[r] + lm[r];
      ((c32*)A->xT)[(size_t)col * L + e] = v;
    }
  }
}

template <int d, int N, bool OPEN, bool CK>
__global__ void __launch_bounds__((GShape<d, N, OPEN>::T))
g_rk4_kernel(const GArgs* __restrict__ Ag, const GAdj* __restrict__ Bg, int n_lo, int n_hi,
             const float4* __restrict__ st_in, float4* __restrict__ st_out) {
  g_rk4_body<d, N, OPEN, CK>(Ag, Bg, blockIdx.x, n_lo, n_hi, st_in, st_out);
}

// Batched (serving): every workgroup reads its own work item -- its request's
// description, column, step range and state buffers.
template <int d, int N, bool CK>
__global__ void __launch_bounds__((GShape<d, N, false>::T))
g_rk4_batched_kernel(const GItem* __restrict__ items) {
  kptr<GItem> it = kconst(items) + blockIdx.x;
  g_rk4_body<d, N, false, CK>((const GArgs*)it->A, (const GAdj*)it->B, it->col, it->n_lo,
                              it->n_hi, it->st_in, it->st_out);
}

// ---------------------------------------------------------------------------
// open-system adjoint (discrete adjoint of the RK4 steps, as the closed
// system's: kb_s from the costate, yb_s = L_s^dag kb_s, lambda += sum yb_s,
// dLoss/dtheta += 2 Re <kb_s, dL_s/dtheta y_s>), one workgroup per column
// walking the checkpoint segments backwards: each segment is recomputed from
// its checkpoint with its stage inputs stored, then walked in reverse.
// ---------------------------------------------------------------------------

// L^dag x for one element: the Hamiltonian part with the opposite sign, the
// static diagonal conjugated, the relaxation jump transposed
// (conj(J[a-1][b-1]) x_{A-e_m, B-e_m}).  Closed systems: G^dag = i (delta + H).
template <int d, int N, bool OPEN>
__device__ __forceinline__ void g_apply_adj(kptr<GArgs> A, const c32* __restrict__ xb,
                                            const c32* __restrict__ tab, int e, uint32_t pk,
                                            float dgr, float dgi, float xr, float xi, float& yr,
                                            float& yi) {
  using Sh = GShape<d, N, OPEN>;
  constexpr int D = Sh::D, dd = d * d;
  yr = dgr * xr + dgi * xi;
  yi = dgr * xi - dgi * xr;
  if (OPEN && uni(A->has_jump)) {
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int am = ket_digit(pk, m), bm = bra_digit(pk, m, N);
      if (am > 0 && bm > 0) {
        const c32 J = tab[A->off_j + m * dd + (am - 1) * d + (bm - 1)];
        const c32 v = xb[e - (D + 1) * Sh::st(m)];
        cmac_conj(yr, yi, J, v);
      }
    }
  }
  const int ndm = uni(A->ndm);
  for (int dmv = 0; dmv < ndm; ++dmv) {
    const int dm = uni(dmv);
    const int m = uni(A->dm_mode[dm]);
    {
      const int sm = uni(A->kst[m]);
      const int am = ket_digit(pk, m);
      constexpr int RD = one_row<d, OPEN>();
      const c32* row = tab + dm * d * RD + am * RD;
      const c32* x0 = xb + e - am * sm;
      float sr = 0.f, si = 0.f;
      one_dot<d, false>(row, x0, sm, sr, si);
      yr -= si;
      yi += sr;
    }
    if (OPEN) {
      const int sm = uni(A->bst[m]);
      const int bm = bra_digit(pk, m, N);
      constexpr int RD = one_row<d, OPEN>();
      const c32* row = tab + dm * d * RD + bm * RD;
      const c32* x0 = xb + e - bm * sm;
      float sr = 0.f, si = 0.f;
      one_dot<d, true>(row, x0, sm, sr, si);
      yr += si;
      yi -= sr;
    }
  }
  const int npr = uni(A->npr);
  for (int pv = 0; pv < npr; ++pv) {
    const int p = uni(pv);
    const int i = uni(A->pr_i[p]), j = uni(A->pr_j[p]);
    constexpr int PR = pair_row<d, OPEN>();
    const c32* P = tab + A->off_p + p * dd * PR;
    {
      const int si_ = uni(A->kst[i]), sj_ = uni(A->kst[j]);
      const int ai = ket_digit(pk, i), aj = ket_digit(pk, j);
      const c32* row = P + (ai * d + aj) * PR;
      const c32* x0 = xb + e - (ai * si_ + aj * sj_);
      float sr = 0.f, si = 0.f;
      pair_dot<d, false>(row, x0, si_, sj_, sr, si);
      yr -= si;
      yi += sr;
    }
    if (OPEN) {
      const int si_ = uni(A->bst[i]), sj_ = uni(A->bst[j]);
      const int bi = bra_digit(pk, i, N), bj = bra_digit(pk, j, N);
      const c32* row = P + (bi * d + bj) * PR;
      const c32* x0 = xb + e - (bi * si_ + bj * sj_);
      float sr = 0.f, si = 0.f;
      pair_dot<d, true>(row, x0, si_, sj_, sr, si);
      yr += si;
      yi -= sr;
    }
  }
}

// z = (O kb - kb O) at one element for a one-mode operator O (table rows at
// `rows`, O Hermitian): the commutator's ket gather minus its bra gather.
template <int d, int N>
__device__ __forceinline__ c32 comm1(const c32* __restrict__ kb, const c32* __restrict__ rows,
                                     int e, int am, int bm, int ks, int bs) {
  float kr = 0.f, ki = 0.f, br = 0.f, bi = 0.f;
  const c32* k0 = kb + e - am * ks;
  const c32* b0 = kb + e - bm * bs;
#pragma unroll
  for (int x = 0; x < d; ++x) {
    cmac(kr, ki, rows[am * d + x], k0[x * ks]);
    cmac_conj(br, bi, rows[bm * d + x], b0[x * bs]);
  }
  c32 z;
  z.x = kr - br;
  z.y = ki - bi;
  return z;
}

// z = (P kb - kb P) at one element for P = Oi (x) Oj on modes (i, j).
template <int d, int N>
__device__ __forceinline__ c32 comm2(const c32* __restrict__ kb, const c32* __restrict__ Ri,
                                     const c32* __restrict__ Rj, int e, int ai, int aj, int bi,
                                     int bj, int ksi, int ksj, int bsi, int bsj) {
  float kr = 0.f, ki = 0.f, br = 0.f, bim = 0.f;
  const c32* k0 = kb + e - ai * ksi - aj * ksj;
  const c32* b0 = kb + e - bi * bsi - bj * bsj;
#pragma unroll
  for (int x = 0; x < d; ++x) {
    float ir = 0.f, ii = 0.f, jr = 0.f, ji = 0.f;
#pragma unroll
    for (int z = 0; z < d; ++z) {
      cmac(ir, ii, Rj[aj * d + z], k0[x * ksi + z * ksj]);
      cmac_conj(jr, ji, Rj[bj * d + z], b0[x * bsi + z * bsj]);
    }
    c32 u, w;
    u.x = ir;
    u.y = ii;
    w.x = jr;
    w.y = ji;
    cmac(kr, ki, Ri[ai * d + x], u);
    cmac_conj(br, bim, Ri[bi * d + x], w);
  }
  c32 z;
  z.x = kr - br;
  z.y = ki - bim;
  return z;
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Sum over the wave (all 64 lanes active), the same in every lane, in a fixed
// order: within each row of 16 lanes by DPP (quad exchanges, then the half-row
// and row mirrors), then the four row sums.  DPP stays on the vector ALU
// (a shuffle would use the LDS crossbar these kernels are bound by).
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_f<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_f<0x141>(v);   // row_half_mirror
  v += dpp_f<0x140>(v);   // row_mirror
  return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}

// s = sum_x row[x] v[x]
template <int d>
__device__ __forceinline__ c32 rowdot(const c32* __restrict__ row, const c32 (&v)[d]) {
  float sr = 0.f, si = 0.f;
#pragma unroll
  for (int x = 0; x < d; ++x) cmac(sr, si, row[x], v[x]);
  c32 z;
  z.x = sr;
  z.y = si;
  return z;
}

// Im(conj(a) b)
__device__ __forceinline__ float im_conj(c32 a, c32 b) { return a.x * b.y - a.y * b.x; }

// w[x] = conj(v[x]) b
template <int d>
__device__ __forceinline__ void conj_scale(const c32 (&v)[d], c32 b, c32 (&w)[d]) {
#pragma unroll
  for (int x = 0; x < d; ++x) {
    w[x].x = fmaf(v[x].x, b.x, v[x].y * b.y);
    w[x].y = fmaf(v[x].x, b.y, -v[x].y * b.x);
  }
}

// Im(conj(sum_x row[x] v[x]) b) = sum_x Im(conj(row[x]) w[x]) with w = conj(v) b
template <int d>
__device__ __forceinline__ float im_rowdot(const c32* __restrict__ row, const c32 (&w)[d]) {
  float s = 0.f;
#pragma unroll
  for (int x = 0; x < d; ++x) {
    s = fmaf(row[x].x, w[x].y, s);
    s = fmaf(-row[x].y, w[x].x, s);
  }
  return s;
}

// Block blk of a reverse-walk launch for segment gseg (see g_adj_kernel).
template <int d, int N, bool OPEN>
__device__ __forceinline__ void g_adj_body(const GArgs* __restrict__ Ag, const GAdj* __restrict__ Bg,
                                           int gseg, int blk) {
  using Sh = GShape<d, N, OPEN>;
  constexpr int L = Sh::L, T = Sh::T, E = Sh::E, D = Sh::D, dd = d * d;
  constexpr int NW = T / 64;
  constexpr int WS = OPEN ? GA_MAXDS : GA_NV;   // per-wave sums of one stage
  extern __shared__ __align__(16) c32 lds[];
  kptr<GArgs> A = kconst(Ag);
  kptr<GAdj> B = kconst(Bg);
  const int ntab = A->ntab, ntabg = A->ntabg;
  const int nacc = B->nacc, npulse = B->npulse;
  // LDS: two column buffers (stage inputs while recomputing, kb while
  // reversing), for closed systems two more (y while reversing), two stage
  // tables (gradient width), FP64 accumulators, and per-wave partial sums of
  // a stage (two stage parities)
  c32* yb0 = lds + 2 * L;
  c32* tb0 = lds + (OPEN ? 2 : 4) * L;
  double* acc = (double*)(tb0 + 2 * ntabg);
  float* wsum = (float*)(acc + ((nacc + 1) & ~1));
  const c32* gtab = (const c32*)A->gtab;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float h = A->h;
  const int nsteps = A->nsteps, ce = B->ce, nck = B->nck;
  // Open systems: one launch walks every segment (recompute, then reverse).
  // Closed systems: one launch per segment, 2S workgroups: the first S walk
  // segment gseg back while the other S recompute segment gseg - 1 into the
  // other stage-input buffer, so the recompute hides behind the reverse walk.
  const int S = A->S;
  const bool rev_role = OPEN || blk < S;
  const int col = (OPEN || rev_role) ? blk : blk - S;
  const int g_hi = OPEN ? nck - 1 : (rev_role ? gseg : gseg - 1);
  const int g_lo = OPEN ? 0 : g_hi;
  if (!OPEN && (g_hi < 0 || g_hi >= nck)) return;
  const int nds = uni(A->nds), ncp = uni(A->ncp), ndr = uni(A->ndr);
  const int nv = OPEN ? 0 : 3 * N + ncp;   // closed: device-parameter and coupling sums
  // closed systems continue the accumulators of the later segments
  const bool resume = !OPEN && rev_role && g_hi < nck - 1;
  for (int t = tid; t < nacc; t += T) acc[t] = resume ? B->part[(size_t)col * nacc + t] : 0.0;
  uint32_t pk[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = tid + r * T;
    const int Ai = OPEN ? e / D : e, Bi = OPEN ? e - Ai * D : 0;
    uint32_t p = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      p |= (uint32_t)((Ai / Sh::st(m)) % d) << (3 * m);
      if (OPEN) p |= (uint32_t)((Bi / Sh::st(m)) % d) << (3 * (N + m));
    }
    pk[r] = p;
  }
  // the costate lives in registers only during the reverse walks; between
  // them (while a segment is recomputed) it waits in device memory
  float4* lsave = B->lam + (size_t)col * L;
  int prev_row = -1;   // step-grid row of the stage whose sums wait in wsum
  int par = 0;         // parity of the wsum buffer being filled
  // fold the previous stage's per-wave sums in a fixed order: the drive slots
  // into the pulse parameters (one thread per drive, times dc/dpar of that
  // stage), closed systems' device-parameter and coupling sums as they are
  auto fold_prev = [&]() {
    for (int t = tid; t < ndr + nv; t += T) {
      if (t < ndr) {
        const int ds = A->dr_ds[t];
        double G = 0.0;
        for (int w = 0; w < NW; ++w) G += (double)wsum[((par ^ 1) * NW + w) * WS + ds];
        const double* dct = B->dctab + (size_t)prev_row * npulse;
        for (int p = A->dr_par0[t]; p < A->dr_par0[t] + A->dr_npar[t]; ++p) acc[p] += dct[p] * G;
      } else {
        const int k = t - ndr;
        double G = 0.0;
        for (int w = 0; w < NW; ++w) G += (double)wsum[((par ^ 1) * NW + w) * WS + GA_MAXDS + k];
        acc[npulse + k] += G;
      }
    }
  };
  __syncthreads();
#pragma unroll 1
  for (int g = g_hi; g >= g_lo; --g) {
    const int n0 = g * ce, n1 = min(nsteps, n0 + ce);
    // stage inputs of the segment: one buffer per column (open systems), two
    // alternating by segment (closed systems)
    c32* segc = (c32*)B->seg + ((size_t)col * (OPEN ? 1 : 2) + (OPEN ? 0 : (g & 1))) * ce * 4 * L;
    // ---- recompute the segment from its checkpoint, storing the stage inputs
    if (OPEN || !rev_role) {
      float hr[E], hm[E], lr[E], lm[E], ar[E], am_[E];
      const float4* ck = B->ck + ((size_t)col * nck + g) * L;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int e = tid + r * T;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < L) v = ck[e];
        hr[r] = v.x;
        hm[r] = v.y;
        lr[r] = v.z;
        lm[r] = v.w;
        ar[r] = am_[r] = 0.f;
        if (e < L) {
          c32 u;
          u.x = v.x;
          u.y = v.y;
          lds[e] = u;
        }
      }
      {
        const c32* g0 = gtab + (size_t)stage_c(n0, 0) * ntabg;
        for (int t = tid; t < ntab; t += T) tb0[t] = g0[t];
      }
      __syncthreads();
      int cur = 0;
#pragma unroll 1
      for (int n = n0; n < n1; ++n) {
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
          const float w = (s == 0 || s == 3) ? 1.f : 2.f;
          const float ch = (s == 2) ? h : 0.5f * h;
          const c32* yc = lds + cur * L;
          const c32* tc = tb0 + cur * ntabg;
          c32* yn = lds + (cur ^ 1) * L;
          c32* ys = segc + ((size_t)(n - n0) * 4 + s) * L;
          const int n2 = s < 3 ? n : n + 1, s2 = s < 3 ? s + 1 : 0;
          const bool more = n2 < n1;
          const c32* gnext = gtab + (size_t)stage_c(n2, s2) * ntabg;
          c32 pre[GA_PRE];
#pragma unroll
          for (int k = 0; k < GA_PRE; ++k) {
            const int t = tid + k * T;
            if (more && t < ntab) pre[k] = gnext[t];
          }
#pragma unroll
          for (int r = 0; r < E; ++r) {
            int e = tid + r * T;
            uint32_t p = pk[r];
            asm volatile("" : "+v"(e), "+v"(p));
            if (e < L) {
              float gr = 0.f, gi = 0.f;
#pragma unroll
              for (int m = 0; m < N; ++m) {
                const int a = ket_digit(p, m);
                if (OPEN) {
                  const int b = bra_digit(p, m, N);
                  gi -= A->delta[m][a] - A->delta[m][b];
                  gr -= 0.5f * A->g1[m] * (float)(a + b) + A->gp[m] * (float)((a - b) * (a - b));
                } else {
                  gi -= A->delta[m][a];
                }
              }
              const c32 ye = yc[e];
              ys[e] = ye;
              float kr, ki;
              g_apply<d, N, OPEN>(A, yc, tc, e, p, gr, gi, ye.x, ye.y, kr, ki);
              if (s == 0) {
                ar[r] = kr;
                am_[r] = ki;
              } else {
                ar[r] = fmaf(w, kr, ar[r]);
                am_[r] = fmaf(w, ki, am_[r]);
              }
              c32 v;
              if (s < 3) {
                v.x = fmaf(ch, kr, hr[r]);
                v.y = fmaf(ch, ki, hm[r]);
              } else {
                const float h6 = h * (1.0f / 6.0f);
                comp_add(hr[r], lr[r], h6 * ar[r]);
                comp_add(hm[r], lm[r], h6 * am_[r]);
                v.x = hr[r];
                v.y = hm[r];
              }
              yn[e] = v;
            }
            __builtin_amdgcn_sched_barrier(0);
          }
          if (more) {
            c32* tn = tb0 + (cur ^ 1) * ntabg;
#pragma unroll
            for (int k = 0; k < GA_PRE; ++k) {
              const int t = tid + k * T;
              if (t < ntab) tn[t] = pre[k];
            }
            for (int t = tid + GA_PRE * T; t < ntab; t += T) tn[t] = gnext[t];
          }
          __syncthreads();
          cur ^= 1;
        }
      }
    }
    if (!OPEN && !rev_role) return;
    // ---- reverse walk of the segment
    float lhr[E], lhm[E], llr[E], llm[E];   // costate (hi, lo)
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = tid + r * T;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < L) {
        if (g == nck - 1) {
          const c32 c = ((const c32*)B->cot)[(size_t)col * L + e];
          v = make_float4(c.x, c.y, 0.f, 0.f);
        } else {
          v = lsave[e];
        }
      }
      lhr[r] = v.x;
      lhm[r] = v.y;
      llr[r] = v.z;
      llm[r] = v.w;
    }
    int cur = 0;
    // closed systems: the next stage's y and the first GP table entries per
    // thread are loaded into registers while the current stage runs
    constexpr int GP = OPEN ? 1 : 8;
    c32 pre_t[GP], pre_y[OPEN ? 1 : E];
    if constexpr (!OPEN) {   // the walk's first stage: (n1 - 1, 3)
      const c32* ysn = segc + ((size_t)(n1 - 1 - n0) * 4 + 3) * L;
      const c32* grn = gtab + (size_t)stage_c(n1 - 1, 3) * ntabg;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int e = tid + r * T;
        if (e < L) pre_y[r] = ysn[e];
      }
#pragma unroll
      for (int k = 0; k < GP; ++k) {
        const int t = tid + k * T;
        if (t < ntabg) pre_t[k] = grn[t];
      }
    }
#pragma unroll 1
    for (int n = n1 - 1; n >= n0; --n) {
      // yb_{s+1}; the step's increments sum_s yb_s gather in the costate's lo
      // word (kb_s reads only hi) and are folded into hi at the step's end
      float ybr[E], ybm[E];
#pragma unroll
      for (int r = 0; r < E; ++r) ybr[r] = ybm[r] = 0.f;
#pragma unroll 1
      for (int s = 3; s >= 0; --s) {
        const float cs = (s == 0 || s == 3) ? h * (1.0f / 6.0f) : h * (1.0f / 3.0f);
        const float cy = (s == 3) ? 0.f : (s == 2 ? h : 0.5f * h);
        const int row = stage_c(n, s);
        c32* kbw = lds + cur * L;
        c32* ybw = yb0 + cur * L;   // closed systems
        c32* tw = tb0 + cur * ntabg;
        const c32* ys = segc + ((size_t)(n - n0) * 4 + s) * L;
        const c32* gr_ = gtab + (size_t)row * ntabg;
        // kb_s (own elements), closed systems y_s too, and the stage table
        // into this stage's buffers
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int e = tid + r * T;
          if (e < L) {
            c32 v;
            v.x = fmaf(cs, lhr[r], cy * ybr[r]);
            v.y = fmaf(cs, lhm[r], cy * ybm[r]);
            kbw[e] = v;
            if (!OPEN) ybw[e] = pre_y[OPEN ? 0 : r];
          }
        }
        if (!OPEN) {
#pragma unroll
          for (int k = 0; k < GP; ++k) {
            const int t = tid + k * T;
            if (t < ntabg) tw[t] = pre_t[k];
          }
          for (int t = tid + GP * T; t < ntabg; t += T) tw[t] = gr_[t];
        } else {
          for (int t = tid; t < ntabg; t += T) tw[t] = gr_[t];
        }
        __syncthreads();
        if constexpr (!OPEN) {
          // the next stage of the walk: (n, s - 1), else (n - 1, 3) within the segment
          const int nn = s > 0 ? n : n - 1, sn = s > 0 ? s - 1 : 3;
          if (nn >= n0) {
            const c32* ysn = segc + ((size_t)(nn - n0) * 4 + sn) * L;
            const c32* grn = gtab + (size_t)stage_c(nn, sn) * ntabg;
#pragma unroll
            for (int r = 0; r < E; ++r) {
              const int e = tid + r * T;
              if (e < L) pre_y[r] = ysn[e];
            }
#pragma unroll
            for (int k = 0; k < GP; ++k) {
              const int t = tid + k * T;
              if (t < ntabg) pre_t[k] = grn[t];
            }
          }
        }
        // the previous stage's sums are complete
        if (prev_row >= 0) fold_prev();
#pragma unroll
        for (int r = 0; r < E; ++r) {
          int e = tid + r * T;
          uint32_t p = pk[r];
          asm volatile("" : "+v"(e), "+v"(p));
          if (e < L) {
            float gr = 0.f, gi = 0.f;
#pragma unroll
            for (int m = 0; m < N; ++m) {
              const int a = ket_digit(p, m);
              if (OPEN) {
                const int b = bra_digit(p, m, N);
                gi -= A->delta[m][a] - A->delta[m][b];
                gr -= 0.5f * A->g1[m] * (float)(a + b) + A->gp[m] * (float)((a - b) * (a - b));
              } else {
                gi -= A->delta[m][a];
              }
            }
            const c32 kbe = kbw[e];
            float yr_, yi_;
            g_apply_adj<d, N, OPEN>(A, kbw, tw, e, p, gr, gi, kbe.x, kbe.y, yr_, yi_);
            ybr[r] = yr_;
            ybm[r] = yi_;
            llr[r] += yr_;
            llm[r] += yi_;
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (OPEN) {
          // drive slots: 2 Im <O kb - kb O, y>, one sum per wave
#pragma unroll 1
          for (int k = 0; k < nds; ++k) {
            const int m = uni(A->ds_mode[k]);
            const c32* rows = tw + A->off_s + uni(A->ds_sl[k]) * dd;
            const int ks = uni(A->kst[m]), bs = uni(A->bst[m]);
            float v = 0.f;
#pragma unroll
            for (int r = 0; r < E; ++r) {
              const int e = tid + r * T;
              if (e < L) {
                const c32 z =
                    comm1<d, N>(kbw, rows, e, ket_digit(pk[r], m), bra_digit(pk[r], m, N), ks, bs);
                v += 2.f * im_conj(z, ys[e]);
              }
            }
            v = wave_sum(v);
            if (lane == 0) wsum[(par * NW + wave) * WS + k] = v;
          }
          // couplings: 2 Im <P kb - kb P, y>, added to the FP64 sums per wave
#pragma unroll 1
          for (int c = 0; c < ncp; ++c) {
            const int i = uni(A->cp_i[c]), j = uni(A->cp_j[c]);
            const c32* Ri = tw + A->off_s + uni(A->cp_si[c]) * dd;
            const c32* Rj = tw + A->off_s + uni(A->cp_sj[c]) * dd;
            const int ksi = uni(A->kst[i]), ksj = uni(A->kst[j]);
            const int bsi = uni(A->bst[i]), bsj = uni(A->bst[j]);
            float v = 0.f;
#pragma unroll
            for (int r = 0; r < E; ++r) {
              const int e = tid + r * T;
              if (e < L) {
                const uint32_t p = pk[r];
                const c32 z = comm2<d, N>(kbw, Ri, Rj, e, ket_digit(p, i), ket_digit(p, j),
                                          bra_digit(p, i, N), bra_digit(p, j, N), ksi, ksj, bsi,
                                          bsj);
                const c32 y = ys[e];
                v += 2.f * (z.x * y.y - z.y * y.x);
              }
            }
            v = wave_sum(v);
            if (lane == 0) atomicAdd(&acc[npulse + c], (double)v);
          }
          // rates: 2 Re <D[a_m]^dag kb, y> and 2 Re <-(a - b)^2 kb, y>
#pragma unroll 1
          for (int m = 0; m < N; ++m) {
            const int sm = (D + 1) * uni(A->bst[m]);
            const c32* Ju = tw + A->off_u + m * dd;
            float v1 = 0.f, v2 = 0.f;
#pragma unroll
            for (int r = 0; r < E; ++r) {
              const int e = tid + r * T;
              if (e < L) {
                const int a = ket_digit(pk[r], m), b = bra_digit(pk[r], m, N);
                const c32 kbe = kbw[e];
                float zr = -0.5f * (float)(a + b) * kbe.x, zi = -0.5f * (float)(a + b) * kbe.y;
                if (a > 0 && b > 0) cmac_conj(zr, zi, Ju[(a - 1) * d + (b - 1)], kbw[e - sm]);
                const c32 y = ys[e];
                v1 += 2.f * (zr * y.x + zi * y.y);
                v2 -= 2.f * (float)((a - b) * (a - b)) * (kbe.x * y.x + kbe.y * y.y);
              }
            }
            v1 = wave_sum(v1);
            v2 = wave_sum(v2);
            if (lane == 0) {
              atomicAdd(&acc[npulse + ncp + 2 * m], (double)v1);
              atomicAdd(&acc[npulse + ncp + 2 * m + 1], (double)v2);
            }
          }
        } else {
          // Device parameters of mode m and couplings.  <kb, dH y> with dH a
          // one-mode operator Q on m: 2 Im <Q kb, y> from kb gathered along m.
          // A two-mode term P_i (x) P_j factors as <(P_i (x) 1) kb, (1 (x) P_j) y>,
          // so each coupling end needs kb gathered along its own mode and y
          // along the partner's; the device derivative on the own side is
          // g (dP_own (x) P_partner), summed over the ends sharing dP_own.
#pragma unroll 1
          for (int mv = 0; mv < N; ++mv) {
            const int m = uni(mv);
            const int ks = uni(A->kst[m]);
            const c32* Dm = tw + uni(A->off_m) + m * 3 * dd;
            // kb along m: kept in registers for the whole mode when small,
            // else gathered again at each use (keeps the E = 4 shapes out of
            // scratch)
            constexpr bool KC = E * d <= 12;
            c32 kv[KC ? E : 1][d];
            c32 C[E];
            float v0 = 0.f, v1 = 0.f, v2 = 0.f;
#pragma unroll
            for (int r = 0; r < E; ++r) {
              const int e = tid + r * T;
              C[r].x = C[r].y = 0.f;
              if (e < L) {
                const int am = ket_digit(pk[r], m);
                c32 kt[d];
#pragma unroll
                for (int x = 0; x < d; ++x) kt[x] = kbw[e + (x - am) * ks];
                if constexpr (KC) {
#pragma unroll
                  for (int x = 0; x < d; ++x) kv[r][x] = kt[x];
                }
                c32 w[d];
                conj_scale<d>(kt, ybw[e], w);
                v0 += 2.f * im_rowdot<d>(Dm + am * d, w);
                v1 += 2.f * im_rowdot<d>(Dm + dd + am * d, w);
                v2 += 2.f * im_rowdot<d>(Dm + 2 * dd + am * d, w);
              }
              __builtin_amdgcn_sched_barrier(0);
            }
            // kb along m of element r (registers or LDS)
            auto kb_of = [&](int r, int e, int am, c32(&kt)[d]) {
              if constexpr (KC) {
#pragma unroll
                for (int x = 0; x < d; ++x) kt[x] = kv[KC ? r : 0][x];
              } else {
#pragma unroll
                for (int x = 0; x < d; ++x) kt[x] = kbw[e + (x - am) * ks];
              }
            };
            // drive slots on this mode: 2 Im <O kb, y>, one sum per wave (the
            // large shapes take them in a loop of their own, below)
#pragma unroll 1
            for (int k = 0; k < (KC ? nds : 0); ++k) {
              if (uni(A->ds_mode[k]) != m) continue;
              const c32* rows = tw + A->off_s + uni(A->ds_sl[k]) * dd;
              float v = 0.f;
#pragma unroll
              for (int r = 0; r < E; ++r) {
                const int e = tid + r * T;
                if (e < L) {
                  const int am = ket_digit(pk[r], m);
                  c32 kt[d];
                  kb_of(r, e, am, kt);
                  v += 2.f * im_conj(rowdot<d>(rows + am * d, kt), ybw[e]);
                }
              }
              v = wave_sum(v);
              if (lane == 0) wsum[(par * NW + wave) * WS + k] = v;
            }
            const int k0 = uni(A->me_beg[m]), k1 = uni(A->me_beg[m + 1]);
#pragma unroll 1
            for (int kq = k0; kq < k1; ++kq) {
              const int pkd = uni(A->me[kq]);
              const int c = pkd & 31, own = (pkd >> 5) & 31, psl = (pkd >> 10) & 31;
              const int pm = (pkd >> 15) & 31;
              const bool first = (pkd >> 20) & 1, last = (pkd >> 21) & 1;
              const float gc = unif(A->cp_g[c]);
              const int ps = uni(A->kst[pm]);
              const c32* Ro = tw + A->off_s + own * dd;
              const c32* Rp = tw + A->off_s + psl * dd;
              const c32* dR = tw + A->off_d + own * 3 * dd;
              float vc = 0.f;
#pragma unroll
              for (int r = 0; r < E; ++r) {
                const int e = tid + r * T;
                if (e < L) {
                  const int am = ket_digit(pk[r], m), ap = ket_digit(pk[r], pm);
                  c32 yv[d];
#pragma unroll
                  for (int z = 0; z < d; ++z) yv[z] = ybw[e + (z - ap) * ps];
                  const c32 cp = rowdot<d>(Rp + ap * d, yv);
                  C[r].x = fmaf(gc, cp.x, C[r].x);
                  C[r].y = fmaf(gc, cp.y, C[r].y);
                  if (first || last) {
                    c32 kt[d];
                    kb_of(r, e, am, kt);
                    if (first) vc += 2.f * im_conj(rowdot<d>(Ro + am * d, kt), cp);
                    if (last) {
                      c32 w[d];
                      conj_scale<d>(kt, C[r], w);
                      v0 += 2.f * im_rowdot<d>(dR + am * d, w);
                      v1 += 2.f * im_rowdot<d>(dR + dd + am * d, w);
                      v2 += 2.f * im_rowdot<d>(dR + 2 * dd + am * d, w);
                      C[r].x = C[r].y = 0.f;
                    }
                  }
                }
              }
              if (first) {
                vc = wave_sum(vc);
                if (lane == 0) wsum[(par * NW + wave) * WS + GA_MAXDS + 3 * N + c] = vc;
              }
            }
            v0 = wave_sum(v0);
            v1 = wave_sum(v1);
            v2 = wave_sum(v2);
            if (lane == 0) {
              float* wv = wsum + (par * NW + wave) * WS + GA_MAXDS + 3 * m;
              wv[0] = v0;
              wv[1] = v1;
              wv[2] = v2;
            }
          }
          if constexpr (E * d > 12) {
#pragma unroll 1
            for (int k = 0; k < nds; ++k) {
              const int m = uni(A->ds_mode[k]);
              const int ks = uni(A->kst[m]);
              const c32* rows = tw + A->off_s + uni(A->ds_sl[k]) * dd;
              float v = 0.f;
#pragma unroll
              for (int r = 0; r < E; ++r) {
                const int e = tid + r * T;
                if (e < L) {
                  const int am = ket_digit(pk[r], m);
                  c32 kt[d];
#pragma unroll
                  for (int x = 0; x < d; ++x) kt[x] = kbw[e + (x - am) * ks];
                  v += 2.f * im_conj(rowdot<d>(rows + am * d, kt), ybw[e]);
                }
              }
              v = wave_sum(v);
              if (lane == 0) wsum[(par * NW + wave) * WS + k] = v;
            }
          }
        }
        prev_row = row;
        par ^= 1;
        cur ^= 1;
      }
      // lambda_n = lambda_{n+1} + sum_s yb_s: fold lo (holding the old lo and
      // the increments, small next to hi) into hi exactly (fast two-sum)
#pragma unroll
      for (int r = 0; r < E; ++r) {
        float t = lhr[r] + llr[r];
        llr[r] -= t - lhr[r];
        lhr[r] = t;
        t = lhm[r] + llm[r];
        llm[r] -= t - lhm[r];
        lhm[r] = t;
      }
    }
    if (g > 0) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int e = tid + r * T;
        if (e < L) lsave[e] = make_float4(lhr[r], lhm[r], llr[r], llm[r]);
      }
    }
    __syncthreads();
  }
  // the last stage's sums
  if (prev_row >= 0) fold_prev();
  __syncthreads();
  for (int t = tid; t < nacc; t += T) B->part[(size_t)col * nacc + t] = acc[t];
}

template <int d, int N, bool OPEN>
__global__ void __launch_bounds__((GShape<d, N, OPEN>::T))
g_adj_kernel(const GArgs* __restrict__ Ag, const GAdj* __restrict__ Bg, int gseg) {
  g_adj_body<d, N, OPEN>(Ag, Bg, gseg, blockIdx.x);
}

// Batched (serving, closed systems): item.col is the block of the request's
// 2S-block launch, item.gseg its segment.
template <int d, int N>
__global__ void __launch_bounds__((GShape<d, N, false>::T))
g_adj_batched_kernel(const GItem* __restrict__ items) {
  kptr<GItem> it = kconst(items) + blockIdx.x;
  g_adj_body<d, N, false>((const GArgs*)it->A, (const GAdj*)it->B, it->gseg, it->col);
}

// Unit-rate relaxation band of every mode at every half-step q (t = q h/2):
// sqrt((a+1)(b+1)) exp(i (f_a - f_{a+1} - f_b + f_{b+1}) t) for a, b < d - 1,
// zero otherwise; FP64 angle reduced modulo 2 pi, stored FP32.
struct JtabStatic {
  int d, N, nq;
  double h;
  double f[GA_MAXM][8];
};

__global__ void jtab_kernel(JtabStatic js, float2* __restrict__ out) {
  const int q = blockIdx.x;
  const int dd = js.d * js.d;
  const double t = q * (0.5 * js.h);
  const double twopi = 6.283185307179586476925286766559;
  for (int u = threadIdx.x; u < js.N * dd; u += blockDim.x) {
    const int m = u / dd, ab = u - m * dd, a = ab / js.d, b = ab - a * js.d;
    float2 v = make_float2(0.f, 0.f);
    if (a < js.d - 1 && b < js.d - 1) {
      double x = (js.f[m][a] - js.f[m][a + 1] - js.f[m][b] + js.f[m][b + 1]) * t;
      x -= twopi * rint(x / twopi);
      double sn, cs;
      sincos(x, &sn, &cs);
      const double r = sqrt((double)((a + 1) * (b + 1)));
      v = make_float2((float)(r * cs), (float)(r * sn));
    }
    out[(size_t)q * js.N * dd + u] = v;
  }
}

__global__ void store_args_kernel(GArgs a, GArgs* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = a;
}

template <int d, int N, bool OPEN>
size_t g_lds_bytes(int ntab) {
  constexpr size_t L = GShape<d, N, OPEN>::L;
  return sizeof(c32) * (3 * L + ((3 * L) & 1) + 2 * (size_t)ntab);
}

// Steps [n_lo, n_hi) with the state from st_in / to st_out (nullable; see the
// kernel); dadj != nullptr also writes the checkpoints.
template <int d, int N, bool OPEN>
hipError_t g_launch(const GArgs* dargs, const GAdj* dadj, int S, int ntab, int n_lo, int n_hi,
                    const float4* st_in, float4* st_out, hipStream_t s) {
  using Sh = GShape<d, N, OPEN>;
  const size_t sh = g_lds_bytes<d, N, OPEN>(ntab);
  if (dadj != nullptr) {
    (void)hipFuncSetAttribute((const void*)g_rk4_kernel<d, N, OPEN, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((g_rk4_kernel<d, N, OPEN, true>), dim3(S), dim3(Sh::T), sh, s, dargs, dadj,
                       n_lo, n_hi, st_in, st_out);
    return hipGetLastError();
  }
  {
    (void)hipFuncSetAttribute((const void*)g_rk4_kernel<d, N, OPEN, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((g_rk4_kernel<d, N, OPEN, false>), dim3(S), dim3(Sh::T), sh, s, dargs, dadj,
                       n_lo, n_hi, st_in, st_out);
  }
  return hipGetLastError();
}

// Shapes with a compiled stepper: open systems D^2 <= 6561, closed systems
// 64 <= D <= 4096 with at most 10 modes.
#define GA_OPEN_SHAPES(X) X(2, 1) X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(3, 1) X(3, 2) X(3, 3) X(3, 4) \
  X(4, 1) X(4, 2) X(4, 3) X(5, 1) X(5, 2)
#define GA_CLOSED_SHAPES(X) X(2, 6) X(2, 7) X(2, 8) X(2, 9) X(2, 10) X(3, 4) X(3, 5) X(3, 6) \
  X(3, 7) X(4, 3) X(4, 4) X(4, 5) X(4, 6) X(5, 3) X(5, 4) X(5, 5)

hipError_t g_dispatch(int d, int N, bool open, const GArgs* dargs, const GAdj* dadj, int S, int ntab,
                      int n_lo, int n_hi, const float4* st_in, float4* st_out, hipStream_t s) {
#define GA_CASE_O(dd_, nn_)          \
  if (open && d == dd_ && N == nn_) \
    return g_launch<dd_, nn_, true>(dargs, dadj, S, ntab, n_lo, n_hi, st_in, st_out, s);
#define GA_CASE_C(dd_, nn_)           \
  if (!open && d == dd_ && N == nn_) \
    return g_launch<dd_, nn_, false>(dargs, dadj, S, ntab, n_lo, n_hi, st_in, st_out, s);
  GA_OPEN_SHAPES(GA_CASE_O)
  GA_CLOSED_SHAPES(GA_CASE_C)
#undef GA_CASE_O
#undef GA_CASE_C
  return hipErrorInvalidValue;
}

bool g_supported(int d, int N, bool open) {
#define GA_HAS_O(dd_, nn_) if (open && d == dd_ && N == nn_) return true;
#define GA_HAS_C(dd_, nn_) if (!open && d == dd_ && N == nn_) return true;
  GA_OPEN_SHAPES(GA_HAS_O)
  GA_CLOSED_SHAPES(GA_HAS_C)
#undef GA_HAS_O
#undef GA_HAS_C
  return false;
}

__global__ void store_adj_kernel(GAdj a, GAdj* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = a;
}

template <int d, int N, bool OPEN>
size_t g_adj_lds_bytes(int ntabg, int nacc) {
  using Sh = GShape<d, N, OPEN>;
  return sizeof(c32) * ((OPEN ? 2 : 4) * (size_t)Sh::L + 2 * (size_t)ntabg) +
         sizeof(double) * (size_t)((nacc + 1) & ~1) +
         sizeof(float) * 2 * (Sh::T / 64) * (OPEN ? GA_MAXDS : GA_NV);
}

// Open systems: one launch (gseg unused).  Closed systems: launch gseg = nck
// down to 0 in order on one stream, 2S workgroups each (see the kernel).
template <int d, int N, bool OPEN>
hipError_t g_adj_launch(const GArgs* dargs, const GAdj* dadj, int S, int ntabg, int nacc,
                        int gseg, hipStream_t s) {
  using Sh = GShape<d, N, OPEN>;
  const size_t sh = g_adj_lds_bytes<d, N, OPEN>(ntabg, nacc);
  if (sh > 163840) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)g_adj_kernel<d, N, OPEN>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((g_adj_kernel<d, N, OPEN>), dim3(OPEN ? S : 2 * S), dim3(Sh::T), sh, s,
                     dargs, dadj, gseg);
  return hipGetLastError();
}

size_t g_adj_lds(int d, int N, bool open, int ntabg, int nacc) {
#define GA_ADJ_LDS_O(dd_, nn_) \
  if (open && d == dd_ && N == nn_) return g_adj_lds_bytes<dd_, nn_, true>(ntabg, nacc);
#define GA_ADJ_LDS_C(dd_, nn_) \
  if (!open && d == dd_ && N == nn_) return g_adj_lds_bytes<dd_, nn_, false>(ntabg, nacc);
  GA_OPEN_SHAPES(GA_ADJ_LDS_O)
  GA_CLOSED_SHAPES(GA_ADJ_LDS_C)
#undef GA_ADJ_LDS_O
#undef GA_ADJ_LDS_C
  return ~(size_t)0;
}

hipError_t g_adj_dispatch(int d, int N, bool open, const GArgs* dargs, const GAdj* dadj, int S,
                          int ntabg, int nacc, int gseg, hipStream_t s) {
#define GA_ADJ_CASE_O(dd_, nn_) \
  if (open && d == dd_ && N == nn_)  \
    return g_adj_launch<dd_, nn_, true>(dargs, dadj, S, ntabg, nacc, gseg, s);
#define GA_ADJ_CASE_C(dd_, nn_) \
  if (!open && d == dd_ && N == nn_)   \
    return g_adj_launch<dd_, nn_, false>(dargs, dadj, S, ntabg, nacc, gseg, s);
  GA_OPEN_SHAPES(GA_ADJ_CASE_O)
  GA_CLOSED_SHAPES(GA_ADJ_CASE_C)
#undef GA_ADJ_CASE_O
#undef GA_ADJ_CASE_C
  return hipErrorInvalidValue;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Fill the static description from the system and (open systems) the rates.
static scp_status g_args(const scp_system* sys, bool open, const double* gamma1,
                         const double* gammaphi, GArgs& A) {
  std::memset(&A, 0, sizeof(A));
  const Plan& P = sys->plan;
  const int N = sys->n_modes, d = sys->d, dd = d * d;
  if (N > GA_MAXM || (open && 2 * N > GA_MAXM) || d > 7)
    return fail(SCP_EINVAL, "gather engine: too many modes");
  const int D = (int)sys->D;
  A.block_q = P.block_q;
  A.ngroups = std::max(1, P.ngroups);
  A.nsteps = sys->n_steps;
  A.h = (float)sys->h;
  for (int m = 0; m < N; ++m) {
    int st = 1;
    for (int q = m + 1; q < N; ++q) st *= d;
    A.kst[m] = open ? st * D : st;
    A.bst[m] = st;
    const double g1 = (open && gamma1) ? gamma1[m] : 0.0;
    const double gp = (open && gammaphi) ? gammaphi[m] : 0.0;
    if (!(g1 >= 0.0) || !(gp >= 0.0) || !std::isfinite(g1) || !std::isfinite(gp))
      return fail(SCP_EINVAL, "decay rates must be finite and non-negative");
    A.g1[m] = (float)g1;
    A.gp[m] = (float)gp;
    A.has_jump |= g1 > 0.0;
    for (int a = 0; a < d; ++a) A.delta[m][a] = P.delta[m][a];
  }
  // driven modes: the distinct (slot, coefficient group) pairs of each mode
  for (int k = 0; k < P.ndrives; ++k) {
    const int s = P.drives[k].slot, g = P.drives[k].cidx, m = P.slot_mode[s];
    int dm = -1;
    for (int q = 0; q < A.ndm; ++q)
      if (A.dm_mode[q] == m) dm = q;
    if (dm < 0) {
      if (A.ndm >= GA_MAXDM) return fail(SCP_EINVAL, "gather engine: too many driven modes");
      dm = A.ndm++;
      A.dm_mode[dm] = m;
    }
    bool seen = false;
    for (int q = 0; q < A.dm_n[dm]; ++q) seen |= A.dm_slot[dm][q] == s;
    if (seen) continue;
    if (A.dm_n[dm] >= GA_MAXC)
      return fail(SCP_EINVAL, "gather engine: too many drive operators on one mode");
    A.dm_slot[dm][A.dm_n[dm]] = s;
    A.dm_cidx[dm][A.dm_n[dm]++] = g;
  }
  // coupled pairs (i < j)
  for (int e = 0; e < P.ncoup; ++e) {
    const int si = P.coup_slot_i[e], sj = P.coup_slot_j[e];
    int i = P.slot_mode[si], j = P.slot_mode[sj];
    int ssi = si, ssj = sj;
    if (i > j) {
      std::swap(i, j);
      std::swap(ssi, ssj);
    }
    int p = -1;
    for (int q = 0; q < A.npr; ++q)
      if (A.pr_i[q] == i && A.pr_j[q] == j) p = q;
    if (p < 0) {
      if (A.npr >= GA_MAXPR) return fail(SCP_EINVAL, "gather engine: too many coupled pairs");
      p = A.npr++;
      A.pr_i[p] = i;
      A.pr_j[p] = j;
    }
    if (A.pr_n[p] >= GA_MAXC) return fail(SCP_EINVAL, "gather engine: too many couplings on one pair");
    A.pr_si[p][A.pr_n[p]] = ssi;
    A.pr_sj[p][A.pr_n[p]] = ssj;
    A.pr_g[p][A.pr_n[p]++] = (float)sys->coup[e].g;
  }
  // operator rows padded to an even length, the pair block and
  // the table starting at even entries (16-byte aligned rows)
  auto even = [](int x) { return x + (x & 1); };
  A.prow = even(dd);
  A.orow = even(d);
  A.off_p = even(A.ndm * d * A.orow);
  A.off_j = A.off_p + A.npr * dd * A.prow;
  A.ntab = even(A.off_j + (A.has_jump ? N * dd : 0));
  if (A.ntab > GA_MAXTAB) return fail(SCP_EINVAL, "gather engine: stage table too large");
  const size_t L = open ? (size_t)D * D : (size_t)D;
  if ((3 * L + ((3 * L) & 1) + 2 * (size_t)A.ntab) * sizeof(float2) > 163840)
    return fail(SCP_EINVAL, "gather engine: column and stage tables exceed the LDS");
  A.ntabg = A.ntab;
  return SCP_OK;
}

// Gradient description: table slots, drive slots, drives and couplings.  Open
// systems: the table rows widen by the slot operators and the unit bands.
// Closed systems: by the slot operators, the one-mode derivative operators of
// every mode and the derivative slot operators; the coupling ends are grouped
// by mode and own slot.
static scp_status g_args_grad(const scp_system* sys, bool open, GArgs& A) {
  const Plan& P = sys->plan;
  const int N = sys->n_modes, d = sys->d, dd = d * d;
  auto tslot = [&](int s) -> int {
    for (int k = 0; k < A.nsl; ++k)
      if (A.sl_slot[k] == s) return k;
    if (A.nsl >= GA_MAXSL) return -1;
    A.sl_slot[A.nsl] = s;
    return A.nsl++;
  };
  if (P.ndrives > GA_MAXDR) return fail(SCP_EINVAL, "gather-engine gradient: too many drives");
  if (P.ncoup > GA_MAXCP) return fail(SCP_EINVAL, "gather-engine gradient: too many couplings");
  A.ndr = P.ndrives;
  for (int k = 0; k < P.ndrives; ++k) {
    const int s = P.drives[k].slot;
    int ds = -1;
    for (int q = 0; q < A.nds; ++q)
      if (A.sl_slot[A.ds_sl[q]] == s) ds = q;
    if (ds < 0) {
      if (A.nds >= GA_MAXDS)
        return fail(SCP_EINVAL, "gather-engine gradient: too many drive operators");
      const int t = tslot(s);
      if (t < 0) return fail(SCP_EINVAL, "gather-engine gradient: too many operator slots");
      ds = A.nds++;
      A.ds_sl[ds] = t;
      A.ds_mode[ds] = P.slot_mode[s];
    }
    A.dr_ds[k] = ds;
    A.dr_par0[k] = P.drives[k].par0;
    A.dr_npar[k] = P.drives[k].npar;
  }
  A.ncp = P.ncoup;
  for (int e = 0; e < P.ncoup; ++e) {
    const int si = P.coup_slot_i[e], sj = P.coup_slot_j[e];
    const int ti = tslot(si), tj = tslot(sj);
    if (ti < 0 || tj < 0) return fail(SCP_EINVAL, "gather-engine gradient: too many operator slots");
    A.cp_i[e] = P.slot_mode[si];
    A.cp_j[e] = P.slot_mode[sj];
    A.cp_si[e] = ti;
    A.cp_sj[e] = tj;
    A.cp_g[e] = (float)sys->coup[e].g;
  }
  A.off_s = A.ntab;
  if (open) {
    A.grad = 1;
    A.off_u = A.off_s + A.nsl * dd;
    A.ntabg = A.off_u + N * dd;
    A.ntabg += A.ntabg & 1;   // the second table buffer starts 16-byte aligned
  } else {
    A.grad = 2;
    A.off_dslot = P.off_dslot;
    for (int m = 0; m < N; ++m) A.mdm[m] = -1;
    for (int q = 0; q < A.ndm; ++q) A.mdm[A.dm_mode[q]] = q;
    for (int m = 0; m < N; ++m)
      for (int th = 0; th < 3; ++th)
        for (int a = 0; a < d; ++a) A.deps[m][th][a] = (float)sys->modes[m].deps[th][a];
    // coupling ends of each mode, grouped by the own table slot
    int k = 0;
    for (int m = 0; m < N; ++m) {
      A.me_beg[m] = k;
      struct End { int own, c, psl, pm, first; };
      std::vector<End> ends;
      for (int e = 0; e < P.ncoup; ++e) {
        if (A.cp_i[e] == m) ends.push_back({A.cp_si[e], e, A.cp_sj[e], A.cp_j[e], 1});
        if (A.cp_j[e] == m) ends.push_back({A.cp_sj[e], e, A.cp_si[e], A.cp_i[e], 0});
      }
      std::stable_sort(ends.begin(), ends.end(),
                       [](const End& x, const End& y) { return x.own < y.own; });
      for (size_t q = 0; q < ends.size(); ++q) {
        if (k >= GA_MAXME) return fail(SCP_EINVAL, "gather-engine gradient: too many coupling ends");
        const End& x = ends[q];
        const int last = (q + 1 == ends.size() || ends[q + 1].own != x.own) ? 1 : 0;
        A.me[k++] = x.c | (x.own << 5) | (x.psl << 10) | (x.pm << 15) | (x.first << 20) |
                    (last << 21);
      }
    }
    A.me_beg[N] = k;
    A.off_m = A.off_s + A.nsl * dd;
    A.off_d = A.off_m + 3 * N * dd;
    A.off_u = A.off_m;
    A.ntabg = A.off_d + 3 * A.nsl * dd;
    A.ntabg += A.ntabg & 1;   // the second table buffer starts 16-byte aligned
  }
  if (A.ntabg > GA_MAXTAB) return fail(SCP_EINVAL, "gather-engine gradient: stage table too large");
  return SCP_OK;
}

// Workspace: [GArgs][stage tables [3N][ntab]][open: jump bands [2N+1][N][d*d]].
static size_t g_ws_bytes(const scp_system* sys, bool open, int ntab) {
  const size_t dd = (size_t)sys->d * sys->d;
  size_t b = align256(sizeof(GArgs)) + align256(3 * (size_t)sys->n_steps * ntab * sizeof(float2));
  if (open) b += align256((2 * (size_t)sys->n_steps + 1) * sys->n_modes * dd * sizeof(float2));
  return b;
}

static scp_status g_run(scp_system* sys, bool open, const double* gamma1, const double* gammaphi,
                        int S, void* ws, size_t ws_bytes, const float2* x0, float2* xT,
                        hipStream_t st) {
  GArgs A;
  SCP_TRY(g_args(sys, open, gamma1, gammaphi, A));
  if (ws_bytes < g_ws_bytes(sys, open, A.ntab)) return fail(SCP_EINVAL, "workspace too small");
  char* w = static_cast<char*>(ws);
  GArgs* dargs = reinterpret_cast<GArgs*>(w);
  w += align256(sizeof(GArgs));
  float2* gtab = reinterpret_cast<float2*>(w);
  w += align256(3 * (size_t)sys->n_steps * A.ntab * sizeof(float2));
  float2* jtab = open ? reinterpret_cast<float2*>(w) : nullptr;
  A.optab = sys->d_ops;
  A.ctab = sys->d_ctab;
  A.jtab = jtab;
  A.gtab = gtab;
  A.x0 = x0;
  A.xT = xT;
  A.S = S;
  const int N = sys->n_modes, d = sys->d;
  if (A.has_jump) {
    JtabStatic js;
    std::memset(&js, 0, sizeof(js));
    js.d = d;
    js.N = N;
    js.nq = 2 * sys->n_steps + 1;
    js.h = sys->h;
    for (int m = 0; m < N; ++m)
      for (int a = 0; a < d; ++a) js.f[m][a] = sys->modes[m].frame[a];
    hipLaunchKernelGGL(jtab_kernel, dim3(js.nq), dim3(64), 0, st, js, jtab);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(store_args_kernel, dim3(1), dim3(64), 0, st, A, dargs);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(gtab_kernel, dim3(3 * sys->n_steps), dim3(256), 0, st, dargs, d, N, gtab);
  HIPCHK(hipGetLastError());
  if (S == 0) return SCP_OK;
  hipEvent_t t0 = timing_start(sys, st);
  HIPCHK(g_dispatch(d, N, open, dargs, nullptr, S, A.ntab, 0, sys->n_steps, nullptr, nullptr, st));
  timing_stop(sys, t0, 0, st);
  return SCP_OK;
}

// --- open systems ----------------------------------------------------------
scp_status lindblad_check(const scp_system* sys) {
  if (!g_supported(sys->d, sys->n_modes, true))
    return fail(SCP_EINVAL, "open-system path: the density matrix must fit in LDS (d=2: N<=5, "
                            "d=3: N<=4, d=4: N<=3, d=5: N<=2)");
  GArgs A;
  return g_args(sys, true, nullptr, nullptr, A);
}

size_t lindblad_workspace_bytes(const scp_system* sys) {
  GArgs A;
  std::vector<double> one(sys->n_modes, 1.0);   // the largest table: relaxation on
  if (g_args(sys, true, one.data(), nullptr, A) != SCP_OK) return 0;
  return g_ws_bytes(sys, true, A.ntab);
}

scp_status launch_lindblad(scp_system* sys, const double* gamma1, const double* gammaphi, int S,
                           void* ws, size_t ws_bytes, const float2* rho0, float2* rhoT,
                           hipStream_t st) {
  SCP_TRY(lindblad_check(sys));
  return g_run(sys, true, gamma1, gammaphi, S, ws, ws_bytes, rho0, rhoT, st);
}

// Open-system gradient.  Workspace: [GArgs][GAdj][stage tables [3N][ntabg]]
// [unit bands [2N+1][N][d*d]][checkpoints [S][nck][L] float4]
// [stage inputs [S][ce][4][L]][partial sums [S][nacc] double][costate [S][L] float4].
struct LbAdjLayout {
  size_t args, adj, gtab, jtab, ck, seg, part, lam, total;
  int ce, nck, nacc, ntabg;
};

static scp_status lb_adj_layout(const scp_system* sys, int S, LbAdjLayout& w, GArgs* Aout) {
  GArgs A;
  std::vector<double> one(sys->n_modes, 1.0);   // the widest table: relaxation on
  SCP_TRY(g_args(sys, true, one.data(), nullptr, A));
  SCP_TRY(g_args_grad(sys, true, A));
  const Plan& P = sys->plan;
  const size_t L = (size_t)sys->D * sys->D, dd = (size_t)sys->d * sys->d;
  const int N = sys->n_steps;
  w.ce = (int)std::ceil(std::sqrt((double)N));
  w.nck = (N + w.ce - 1) / w.ce;
  w.nacc = P.npulse + P.ncoup + 2 * sys->n_modes;
  w.ntabg = A.ntabg;
  size_t off = 0;
  w.args = off;
  off += align256(sizeof(GArgs));
  w.adj = off;
  off += align256(sizeof(GAdj));
  w.gtab = off;
  off += align256(3 * (size_t)N * A.ntabg * sizeof(float2));
  w.jtab = off;
  off += align256((2 * (size_t)N + 1) * sys->n_modes * dd * sizeof(float2));
  w.ck = off;
  off += align256((size_t)S * w.nck * L * sizeof(float4));
  w.seg = off;
  off += align256((size_t)S * w.ce * 4 * L * sizeof(float2));
  w.part = off;
  off += align256((size_t)S * w.nacc * sizeof(double));
  w.lam = off;
  off += align256((size_t)S * L * sizeof(float4));
  w.total = off;
  if (g_adj_lds(sys->d, sys->n_modes, true, A.ntabg, w.nacc) > 163840)
    return fail(SCP_EINVAL, "open-system gradient: column and tables exceed the LDS");
  if (Aout) *Aout = A;
  return SCP_OK;
}

scp_status lindblad_adjoint_workspace_bytes(const scp_system* sys, int S, size_t* bytes) {
  SCP_TRY(lindblad_check(sys));
  LbAdjLayout w;
  SCP_TRY(lb_adj_layout(sys, S, w, nullptr));
  *bytes = w.total;
  return SCP_OK;
}

scp_status launch_lindblad_adjoint(scp_system* sys, const double* gamma1, const double* gammaphi,
                                   int S, void* ws, size_t ws_bytes, const float2* rho0,
                                   const float2* cot, double* grad, hipStream_t st) {
  SCP_TRY(lindblad_check(sys));
  LbAdjLayout w;
  SCP_TRY(lb_adj_layout(sys, S, w, nullptr));
  if (ws_bytes < w.total) return fail(SCP_EINVAL, "workspace too small");
  GArgs A;
  SCP_TRY(g_args(sys, true, gamma1, gammaphi, A));
  SCP_TRY(g_args_grad(sys, true, A));
  char* base = static_cast<char*>(ws);
  GArgs* dargs = reinterpret_cast<GArgs*>(base + w.args);
  GAdj* dadj = reinterpret_cast<GAdj*>(base + w.adj);
  float2* gtab = reinterpret_cast<float2*>(base + w.gtab);
  float2* jtab = reinterpret_cast<float2*>(base + w.jtab);
  const int N = sys->n_modes, d = sys->d;
  A.optab = sys->d_ops;
  A.ctab = sys->d_ctab;
  A.jtab = jtab;
  A.gtab = gtab;
  A.x0 = rho0;
  A.xT = nullptr;
  A.S = S;
  GAdj B;
  std::memset(&B, 0, sizeof(B));
  B.ck = reinterpret_cast<float4*>(base + w.ck);
  B.cot = cot;
  B.seg = reinterpret_cast<float2*>(base + w.seg);
  B.dctab = sys->d_dctab64;
  B.part = reinterpret_cast<double*>(base + w.part);
  B.lam = reinterpret_cast<float4*>(base + w.lam);
  B.ce = w.ce;
  B.nck = w.nck;
  B.npulse = sys->plan.npulse;
  B.nacc = w.nacc;
  {
    JtabStatic js;
    std::memset(&js, 0, sizeof(js));
    js.d = d;
    js.N = N;
    js.nq = 2 * sys->n_steps + 1;
    js.h = sys->h;
    for (int m = 0; m < N; ++m)
      for (int a = 0; a < d; ++a) js.f[m][a] = sys->modes[m].frame[a];
    hipLaunchKernelGGL(jtab_kernel, dim3(js.nq), dim3(64), 0, st, js, jtab);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(store_args_kernel, dim3(1), dim3(64), 0, st, A, dargs);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(store_adj_kernel, dim3(1), dim3(64), 0, st, B, dadj);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(gtab_kernel, dim3(3 * sys->n_steps), dim3(256), 0, st, dargs, d, N, gtab);
  HIPCHK(hipGetLastError());
  hipEvent_t t0 = timing_start(sys, st);
  HIPCHK(g_dispatch(d, N, true, dargs, dadj, S, A.ntab, 0, sys->n_steps, nullptr, nullptr, st));
  timing_stop(sys, t0, 0, st);
  t0 = timing_start(sys, st);
  HIPCHK(g_adj_dispatch(d, N, true, dargs, dadj, S, A.ntabg, w.nacc, -1, st));
  timing_stop(sys, t0, 2, st);
  std::vector<double> part((size_t)S * w.nacc);
  HIPCHK(hipMemcpyAsync(part.data(), base + w.part, part.size() * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < w.nacc; ++k) {
    double v = 0.0;
    for (int c = 0; c < S; ++c) v += part[(size_t)c * w.nacc + k];   // fixed order
    if (!std::isfinite(v)) return fail(SCP_ENONFINITE, "non-finite gradient");
    grad[k] = v;
  }
  return SCP_OK;
}

// --- closed systems ----------------------------------------------------------
// The gather engine takes a closed-system forward (no checkpoints) when the
// system has a compiled shape and its columns would leave most of the chip
// idle in the register-layout stepper: fewer columns than 256 workgroups'
// worth (each gather workgroup holds one column).
bool gather_preferred(const scp_system* sys, int S) {
  if (!g_supported(sys->d, sys->n_modes, false) || S > 256) return false;
  GArgs A;
  if (g_args(sys, false, nullptr, nullptr, A) != SCP_OK) {
    set_error("");
    return false;
  }
  const int fused_wg = (S + sys->plan.CPW - 1) / sys->plan.CPW;
  return fused_wg < 64;
}

bool gather_supported(const scp_system* sys) {
  if (!g_supported(sys->d, sys->n_modes, false)) return false;
  GArgs A;
  if (g_args(sys, false, nullptr, nullptr, A) != SCP_OK) {
    set_error("");
    return false;
  }
  return true;
}

size_t gather_workspace_bytes(const scp_system* sys) {
  GArgs A;
  if (g_args(sys, false, nullptr, nullptr, A) != SCP_OK) {
    set_error("");
    return 0;
  }
  return g_ws_bytes(sys, false, A.ntab);
}

scp_status launch_gather_forward(scp_system* sys, int S, void* ws, size_t ws_bytes,
                                 const float2* psi0, float2* psiT, hipStream_t st) {
  return g_run(sys, false, nullptr, nullptr, S, ws, ws_bytes, psi0, psiT, st);
}

// Closed-system gradient on the gather engine.  Workspace: [GArgs][GAdj]
// [stage tables [3N][ntabg]][checkpoints [S][nck][D] float4] and, for the
// adjoint, [stage inputs [S][2][ce][4][D]][partial sums [S][nacc] double]
// [costate [S][D] float4].  The forward with checkpoints and the adjoint
// share the offsets of the first four.
struct GcLayout {
  size_t args, adj, gtab, ck, seg, part, lam, total;
  int nck, nacc;
};

static scp_status gc_layout(const scp_system* sys, int S, int ce, bool with_grad, GcLayout& w,
                            GArgs* Aout) {
  if (!g_supported(sys->d, sys->n_modes, false))
    return fail(SCP_EINVAL, "gather engine: no compiled stepper for this d and mode count");
  GArgs A;
  SCP_TRY(g_args(sys, false, nullptr, nullptr, A));
  SCP_TRY(g_args_grad(sys, false, A));
  const size_t L = (size_t)sys->D;
  const int N = sys->n_steps;
  w.nck = (N + ce - 1) / ce;
  w.nacc = sys->plan.npulse + 3 * sys->n_modes + sys->plan.ncoup;
  size_t off = 0;
  w.args = off;
  off += align256(sizeof(GArgs));
  w.adj = off;
  off += align256(sizeof(GAdj));
  w.gtab = off;
  off += align256(3 * (size_t)N * A.ntabg * sizeof(float2));
  w.ck = off;
  off += align256((size_t)S * w.nck * L * sizeof(float4));
  w.seg = w.part = w.lam = off;
  if (with_grad) {
    w.seg = off;   // two stage-input buffers per column (segments alternate)
    off += align256((size_t)S * 2 * ce * 4 * L * sizeof(float2));
    w.part = off;
    off += align256((size_t)S * w.nacc * sizeof(double));
    w.lam = off;
    off += align256((size_t)S * L * sizeof(float4));
  }
  w.total = off;
  if (g_adj_lds(sys->d, sys->n_modes, false, A.ntabg, w.nacc) > 163840)
    return fail(SCP_EINVAL, "gather-engine gradient: column and tables exceed the LDS");
  if (Aout) *Aout = A;
  return SCP_OK;
}

scp_status gather_grad_check(const scp_system* sys) {
  GcLayout w;
  return gc_layout(sys, 1, 1, true, w, nullptr);
}

size_t gather_grad_workspace_bytes(const scp_system* sys, int S, int ce, bool with_grad) {
  GcLayout w;
  if (gc_layout(sys, S, ce, with_grad, w, nullptr) != SCP_OK) {
    set_error("");
    return 0;
  }
  return w.total;
}

// Args and adjoint description into the workspace (and the stage tables when
// `tables`).
static scp_status gc_prepare(scp_system* sys, int S, int ce, bool with_grad, char* base,
                             size_t ws_bytes, const float2* x0, float2* xT, const float2* cot,
                             bool tables, GcLayout& w, GArgs& A, hipStream_t st) {
  SCP_TRY(gc_layout(sys, S, ce, with_grad, w, &A));
  if (ws_bytes < w.total) return fail(SCP_EINVAL, "workspace too small");
  GArgs* dargs = reinterpret_cast<GArgs*>(base + w.args);
  GAdj* dadj = reinterpret_cast<GAdj*>(base + w.adj);
  float2* gtab = reinterpret_cast<float2*>(base + w.gtab);
  A.optab = sys->d_ops;
  A.ctab = sys->d_ctab;
  A.jtab = nullptr;
  A.gtab = gtab;
  A.x0 = x0;
  A.xT = xT;
  A.S = S;
  GAdj B;
  std::memset(&B, 0, sizeof(B));
  B.ck = reinterpret_cast<float4*>(base + w.ck);
  B.cot = cot;
  B.seg = with_grad ? reinterpret_cast<float2*>(base + w.seg) : nullptr;
  B.dctab = sys->d_dctab64;
  B.part = with_grad ? reinterpret_cast<double*>(base + w.part) : nullptr;
  B.lam = with_grad ? reinterpret_cast<float4*>(base + w.lam) : nullptr;
  B.ce = ce;
  B.nck = w.nck;
  B.npulse = sys->plan.npulse;
  B.nacc = w.nacc;
  hipLaunchKernelGGL(store_args_kernel, dim3(1), dim3(64), 0, st, A, dargs);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(store_adj_kernel, dim3(1), dim3(64), 0, st, B, dadj);
  HIPCHK(hipGetLastError());
  if (tables) {
    hipLaunchKernelGGL(gtab_kernel, dim3(3 * sys->n_steps), dim3(256), 0, st, dargs, sys->d,
                       sys->n_modes, gtab);
    HIPCHK(hipGetLastError());
  }
  return SCP_OK;
}

scp_status launch_gather_ckpt_forward(scp_system* sys, int S, int ce, void* ws, size_t ws_bytes,
                                      const float2* psi0, float2* psiT, hipStream_t st) {
  char* base = static_cast<char*>(ws);
  GcLayout w;
  GArgs A;
  SCP_TRY(gc_prepare(sys, S, ce, false, base, ws_bytes, psi0, psiT, nullptr, true, w, A, st));
  hipEvent_t t0 = timing_start(sys, st);
  HIPCHK(g_dispatch(sys->d, sys->n_modes, false, reinterpret_cast<GArgs*>(base + w.args),
                    reinterpret_cast<GAdj*>(base + w.adj), S, A.ntab, 0, sys->n_steps, nullptr,
                    nullptr, st));
  timing_stop(sys, t0, 0, st);
  return SCP_OK;
}

// The reverse walk from the checkpoints (and stage tables) that
// launch_gather_ckpt_forward left in the same workspace; the gradient is the
// fixed-order sum of the columns' partial sums.
scp_status launch_gather_adjoint(scp_system* sys, int S, int ce, void* ws, size_t ws_bytes,
                                 const float2* cot, double* grad, hipStream_t st) {
  char* base = static_cast<char*>(ws);
  GcLayout w;
  GArgs A;
  SCP_TRY(gc_prepare(sys, S, ce, true, base, ws_bytes, nullptr, nullptr, cot, false, w, A, st));
  for (int gs = w.nck; gs >= 0; --gs) {
    hipEvent_t t0 = timing_start(sys, st);
    HIPCHK(g_adj_dispatch(sys->d, sys->n_modes, false, reinterpret_cast<GArgs*>(base + w.args),
                          reinterpret_cast<GAdj*>(base + w.adj), S, A.ntabg, w.nacc, gs, st));
    timing_stop(sys, t0, 2, st);
  }
  std::vector<double> part((size_t)S * w.nacc);
  HIPCHK(hipMemcpyAsync(part.data(), base + w.part, part.size() * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < w.nacc; ++k) {
    double v = 0.0;
    for (int c = 0; c < S; ++c) v += part[(size_t)c * w.nacc + k];   // fixed order
    if (!std::isfinite(v)) return fail(SCP_ENONFINITE, "gradient is not finite");
    grad[k] = v;
  }
  return SCP_OK;
}

// --- serving: a closed-system request on the gather engine, in chunks --------
// Workspace: the layout of gc_layout (the adjoint's when the gradient is
// wanted) followed by the compensated state [S][D] float4 between chunks.
size_t gather_serve_bytes(const scp_system* sys, int S, int ce, bool grad) {
  GcLayout w;
  if (gc_layout(sys, S, ce, grad, w, nullptr) != SCP_OK) {
    set_error("");
    return 0;
  }
  return w.total + align256((size_t)S * sys->D * sizeof(float4));
}

scp_status gather_serve_prepare(scp_system* sys, int S, int ce, bool grad, void* ws, size_t bytes,
                                const float2* psi0, float2* psiT, const float2* cot, hipStream_t st) {
  GcLayout w;
  GArgs A;
  return gc_prepare(sys, S, ce, grad, static_cast<char*>(ws), bytes, psi0, psiT, cot, true, w, A,
                    st);
}

// Forward steps [n0, n1): from psi0 when n0 = 0, else from the saved state;
// the state is saved after, psiT written when n1 = n_steps, checkpoints kept
// when the gradient is wanted.
scp_status gather_serve_forward(scp_system* sys, int S, int ce, bool grad, void* ws, int n0, int n1,
                                hipStream_t st) {
  GcLayout w;
  GArgs A;
  SCP_TRY(gc_layout(sys, S, ce, grad, w, &A));
  char* base = static_cast<char*>(ws);
  float4* state = reinterpret_cast<float4*>(base + w.total);
  HIPCHK(g_dispatch(sys->d, sys->n_modes, false, reinterpret_cast<GArgs*>(base + w.args),
                    grad ? reinterpret_cast<GAdj*>(base + w.adj) : nullptr, S, A.ntab, n0, n1,
                    n0 == 0 ? nullptr : state, state, st));
  return SCP_OK;
}

// One launch of the reverse walk (gs = nckpt down to 0, in order).
scp_status gather_serve_adjoint(scp_system* sys, int S, int ce, void* ws, int gs, hipStream_t st) {
  GcLayout w;
  GArgs A;
  SCP_TRY(gc_layout(sys, S, ce, true, w, &A));
  char* base = static_cast<char*>(ws);
  HIPCHK(g_adj_dispatch(sys->d, sys->n_modes, false, reinterpret_cast<GArgs*>(base + w.args),
                        reinterpret_cast<GAdj*>(base + w.adj), S, A.ntabg, w.nacc, gs, st));
  return SCP_OK;
}

int gather_serve_nckpt(const scp_system* sys, int ce) { return (sys->n_steps + ce - 1) / ce; }

scp_status gather_serve_info(const scp_system* sys, int S, int ce, bool grad, void* ws,
                             GServeInfo& out) {
  GcLayout w;
  GArgs A;
  SCP_TRY(gc_layout(sys, S, ce, grad, w, &A));
  char* base = static_cast<char*>(ws);
  out.A = base + w.args;
  out.B = base + w.adj;
  out.state = reinterpret_cast<float4*>(base + w.total);
  out.lds_fwd = sizeof(c32) * (3 * (size_t)sys->D + ((3 * (size_t)sys->D) & 1) + 2 * (size_t)A.ntab);
  out.lds_adj = g_adj_lds(sys->d, sys->n_modes, false, A.ntabg, w.nacc);
  out.nck = w.nck;
  return SCP_OK;
}

namespace {

template <int d, int N>
hipError_t g_fwd_batched_launch(bool ck, const GItem* items, int n, size_t sh, hipStream_t s) {
  using Sh = GShape<d, N, false>;
  if (sh > 163840) return hipErrorInvalidValue;
  if (ck) {
    (void)hipFuncSetAttribute((const void*)g_rk4_batched_kernel<d, N, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((g_rk4_batched_kernel<d, N, true>), dim3(n), dim3(Sh::T), sh, s, items);
  } else {
    (void)hipFuncSetAttribute((const void*)g_rk4_batched_kernel<d, N, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((g_rk4_batched_kernel<d, N, false>), dim3(n), dim3(Sh::T), sh, s, items);
  }
  return hipGetLastError();
}

template <int d, int N>
hipError_t g_adj_batched_launch(const GItem* items, int n, size_t sh, hipStream_t s) {
  using Sh = GShape<d, N, false>;
  if (sh > 163840) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)g_adj_batched_kernel<d, N>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((g_adj_batched_kernel<d, N>), dim3(n), dim3(Sh::T), sh, s, items);
  return hipGetLastError();
}

}  // namespace

scp_status gather_launch_fwd_batched(int d, int N, bool ck, const GItem* items, int n, size_t lds,
                                     hipStream_t st) {
#define GA_FWD_B(dd_, nn_) \
  if (d == dd_ && N == nn_) {                                                  \
    HIPCHK((g_fwd_batched_launch<dd_, nn_>(ck, items, n, lds, st)));          \
    return SCP_OK;                                                            \
  }
  GA_CLOSED_SHAPES(GA_FWD_B)
#undef GA_FWD_B
  return fail(SCP_EINVAL, "gather engine: no compiled stepper for this shape");
}

scp_status gather_launch_adj_batched(int d, int N, const GItem* items, int n, size_t lds,
                                     hipStream_t st) {
#define GA_ADJ_B(dd_, nn_) \
  if (d == dd_ && N == nn_) {                                                  \
    HIPCHK((g_adj_batched_launch<dd_, nn_>(items, n, lds, st)));              \
    return SCP_OK;                                                            \
  }
  GA_CLOSED_SHAPES(GA_ADJ_B)
#undef GA_ADJ_B
  return fail(SCP_EINVAL, "gather engine: no compiled stepper for this shape");
}

// The gradient after the last reverse launch (synchronises st).
scp_status gather_serve_gradient(scp_system* sys, int S, int ce, void* ws, std::vector<double>& grad,
                                 hipStream_t st) {
  GcLayout w;
  SCP_TRY(gc_layout(sys, S, ce, true, w, nullptr));
  std::vector<double> part((size_t)S * w.nacc);
  HIPCHK(hipMemcpyAsync(part.data(), static_cast<char*>(ws) + w.part, part.size() * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  grad.assign(w.nacc, 0.0);
  for (int k = 0; k < w.nacc; ++k) {
    double v = 0.0;
    for (int c = 0; c < S; ++c) v += part[(size_t)c * w.nacc + k];   // fixed order
    grad[k] = v;
  }
  return SCP_OK;
}

// ---------------------------------------------------------------------------
// average gate fidelity of the channel on the computational subspace
// ---------------------------------------------------------------------------
namespace {

// ov = sum_ab sum_ij conj(T_ia) T_jb rho_ab[r_i, r_j] in FP64 by one
// workgroup in a fixed order.
__global__ void __launch_bounds__(1024) chan_overlap_kernel(const c32* __restrict__ rho, int64_t D,
                                                            int dc, const int64_t* __restrict__ rows,
                                                            const double2* __restrict__ Tm,
                                                            double2* __restrict__ ov) {
  __shared__ double red[2][1024];
  const int64_t n = (int64_t)dc * dc * dc * dc;
  double sr = 0.0, si = 0.0;
  for (int64_t u = threadIdx.x; u < n; u += blockDim.x) {
    const int64_t ab = u / ((int64_t)dc * dc), ij = u - ab * dc * dc;
    const int a = (int)(ab / dc), b = (int)(ab - (int64_t)a * dc);
    const int i = (int)(ij / dc), j = (int)(ij - (int64_t)i * dc);
    const double2 ta = Tm[(size_t)i * dc + a], tb = Tm[(size_t)j * dc + b];
    // w = conj(ta) tb
    const double wr = ta.x * tb.x + ta.y * tb.y, wi = ta.x * tb.y - ta.y * tb.x;
    const c32 v = rho[(size_t)ab * D * D + (size_t)rows[i] * D + rows[j]];
    sr += wr * v.x - wi * v.y;
    si += wr * v.y + wi * v.x;
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = si;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) ov[0] = make_double2(red[0][0], red[1][0]);
}

// cotangent of 1 - F: -T_ia conj(T_jb) / (2 dc (dc + 1)) at (ab, r_i, r_j), zero elsewhere
__global__ void chan_cot_kernel(c32* __restrict__ cot, int64_t D, int dc,
                                const int64_t* __restrict__ rows, const double2* __restrict__ Tm) {
  const int64_t total = (int64_t)dc * dc * D * D;
  const double c = -1.0 / (2.0 * dc * (dc + 1.0));
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < total;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ab = u / (D * D), rem = u - ab * D * D;
    const int64_t R = rem / D, C = rem - R * D;
    const int a = (int)(ab / dc), b = (int)(ab - (int64_t)a * dc);
    int i = -1, j = -1;
    for (int q = 0; q < dc; ++q) {
      if (rows[q] == R) i = q;
      if (rows[q] == C) j = q;
    }
    c32 v;
    v.x = v.y = 0.f;
    if (i >= 0 && j >= 0) {
      const double2 ta = Tm[(size_t)i * dc + a], tb = Tm[(size_t)j * dc + b];
      // ta conj(tb)
      v.x = (float)(c * (ta.x * tb.x + ta.y * tb.y));
      v.y = (float)(c * (ta.y * tb.x - ta.x * tb.y));
    }
    cot[u] = v;
  }
}

}  // namespace

scp_status launch_fidelity_channel(const void* rhoT, int64_t D, int dc, const int64_t* rows,
                                   const void* target, void* ov, void* cot, hipStream_t st) {
  hipLaunchKernelGGL(chan_overlap_kernel, dim3(1), dim3(1024), 0, st, (const c32*)rhoT, D, dc, rows,
                     (const double2*)target, (double2*)ov);
  HIPCHK(hipGetLastError());
  if (cot) {
    const int64_t total = (int64_t)dc * dc * D * D;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(chan_cot_kernel, dim3(std::max(1, blocks)), dim3(256), 0, st, (c32*)cot, D,
                       dc, rows, (const double2*)target);
    HIPCHK(hipGetLastError());
  }
  return SCP_OK;
}

}  // namespace scp
