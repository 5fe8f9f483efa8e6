// Suzuki-Trotter product formulas in complex FP64 (Sec. 2.3 Trotterization
// solver, App. A higher-order decompositions, App. B local contractions).
//
// Local terms, in this order: one single-mode term per mode (lab frame),
//   H_m(t) = diag(eps_m) + sum_{drives k on m} c_k(t) O_k,
// then one two-body term g_e A_i (x) B_j per coupling.  A step is the
// sequence of pieces of the chosen formula.  Q1 applies exp(-i H_k dt) for
// k = 1..K; the symmetric piece Q2(a dt) applies exp(-i a H_k dt/2) for
// k = 1..K and then for k = K..1.
//   Q1, Q2: one piece, a = 1;
//   Q4:  a = (p, 1 - 2p, p), p = 1 / (2 - 2^(1/3));
//   Q4j: a = (p, conj p), p = (3 - i sqrt 3) / 6 (the printed value is
//        garbled; this one satisfies p + conj p = 1 and p^3 + conj p^3 = 0).
// A time-dependent term is frozen at the middle of its piece (real
// coefficients) or of the step (Q4j, whose complex pieces have no real
// middle).  The result is rotated into the frame of the RK4 path,
// psi_I(T) = exp(i H_f T) psi_lab(T), H_f = sum_m diag(frame_m).
//
// Device work, all FP64:
//   1. pair gates exp(-i a tau g A (x) B) for every (piece, coupling) and
//      single-mode gates exp(-i a tau H_m(t)) for every (step, piece, mode),
//      one workgroup per gate, by Taylor scaling and squaring in LDS (Moler
//      and Van Loan, "Nineteen dubious ways to compute the exponential of a
//      matrix, twenty-five years later", SIAM Review 2003, Sec. 3): halve
//      until the 1-norm is at most 1/2, sum the series to degree 18
//      (truncation below 1e-22 relative), square back;
//   2. fusion (build_plan, tr_fuse_kernel): adjacent couplings on the same
//      mode pair become one operation, and single-mode gates join pair
//      operations (as table products where pair gates run split, in
//      registers where they run in place);
//   3. the propagation: one workgroup per state column keeps the column in
//      LDS (16 D bytes) for all steps and applies the operations in
//      sequence, one barrier between operations.  An operation kind with at
//      least as many fibres as threads runs in place, a thread owning whole
//      fibres of the contracted mode(s).  With fewer fibres (small D) and
//      room for a second column buffer (32 D bytes <= 160 KiB), a work item
//      computes d output rows (pair operations, when that fills the block)
//      or one output row of one fibre from one buffer into the other, which
//      keeps up to d^2 times more threads busy; the buffers then swap.
#include <cmath>
#include <cstring>

#include "trotter.h"

namespace scp {

namespace {

constexpr int TR_MAXD = 5;        // largest d (pair gates of dimension d^2 <= 25)
constexpr int TR_MAXDRV = 32;
constexpr int TR_MAXE = 48;
constexpr int TR_MAXPIECE = 3;
constexpr int TR_THREADS = 512;   // propagation workgroup
constexpr int TR_MAXLDS = 160 * 1024;
constexpr int TR_MAXOPS = 64;     // fused operations per pass
constexpr int TR_MAXC = 8;        // gates fused into one operation

struct TrDrive {
  int mode, op, env, npar, par0;
  double omega, phase, sigma;
};

struct TrGen {
  int d, M, E, N, r, ndrives;
  double dt, T, tau;
  double a_re[TR_MAXPIECE], a_im[TR_MAXPIECE], mid[TR_MAXPIECE];
  TrDrive dr[TR_MAXDRV];
  int ci[TR_MAXE], cj[TR_MAXE], coi[TR_MAXE], coj[TR_MAXE];
  double g[TR_MAXE];
};

// Fused operations of one pass.  An operation acts on one mode pair
// (kind 1, digits (mi, mj)) or on one mode (kind 0, mi); its constituents
// act in the listed order: ctype 1 = pair gate e = cidx (same orientation),
// ctype 0 = single-mode gate of mode cidx on digit cdig (0: mi, 1: mj).
struct TrOp {
  int kind, mi, mj, nc;
  int stat;   // no single-mode factor: the same gate every step, in static slot sid
  int sid, own;   // own: this operation forms the slot (equal products share one)
  int s0, s1;     // register form: mode + 1 of the single-mode gate on digit 0 / 1 (0: none),
                  // applied before the pair product in the first pass, after it in the second
  int dix;        // pair operation with a single-mode factor: its index in the per-step
                  // fused-gate table (-1 otherwise)
  int ctype[TR_MAXC], cidx[TR_MAXC], cdig[TR_MAXC];
};
struct TrPlan {
  int nop[2], nslot;
  int ndyn;       // pair operations re-formed every step (fused-gate table width)
  TrOp op[2][TR_MAXOPS];
};

struct TrRun {
  int M, N, r, D, H, nopmax, nslot, ndyn;
  int nop[2];
  int opk[2][TR_MAXOPS], opi[2][TR_MAXOPS], opj[2][TR_MAXOPS];
  int ops[2][TR_MAXOPS];   // pair operations: static slot + 1, or -(fused-gate index + 1)
  int opa[2][TR_MAXOPS];   // register form: (s0) | (s1 << 8), see TrOp
  int mode1;                   // single-mode gates: 0 in place, 1 one output row per item
  int mode2;                   // pair gates: 0 in place, 1 one row, 2 d rows per item
  int stride[SCP_MAX_MODES];   // stride of mode m inside a column (mode 0 slowest)
  double fT[SCP_MAX_MODES][SCP_MAX_TRUNC];   // frame energy times T, reduced mod 2 pi
};

static_assert(sizeof(TrRun) <= 4000, "TrRun is passed by value as a kernel argument");

__device__ __forceinline__ double wrap_2pi(double x) {
  const double twopi = 6.283185307179586476925286766559;
  return x - twopi * rint(x / twopi);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// exp(X) for the n x n matrix X (row-major, LDS) into E; T and W are LDS
// scratch of n*n.  Every thread of the block takes part; X is overwritten.
__device__ void expm_taylor(int n, double2* X, double2* E, double2* T, double2* W) {
  const int nn = n * n;
  double nrm = 0.0;
  for (int c = 0; c < n; ++c) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += sqrt(X[r * n + c].x * X[r * n + c].x + X[r * n + c].y * X[r * n + c].y);
    nrm = fmax(nrm, s);
  }
  int sq = 0;
  while (nrm > 0.5 && sq < 64) {
    nrm *= 0.5;
    ++sq;
  }
  const double scale = ldexp(1.0, -sq);
  __syncthreads();   // every thread has read X
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    X[e].x *= scale;
    X[e].y *= scale;
    const double one = (e / n == e % n) ? 1.0 : 0.0;
    E[e] = make_double2(one, 0.0);
    T[e] = make_double2(one, 0.0);
  }
  __syncthreads();
  for (int k = 1; k <= 18; ++k) {
    const double inv = 1.0 / k;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
      const int r = e / n, c = e % n;
      double re = 0.0, im = 0.0;
      for (int l = 0; l < n; ++l) {
        const double2 a = T[r * n + l], b = X[l * n + c];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
      }
      W[e] = make_double2(re * inv, im * inv);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
      T[e] = W[e];
      E[e].x += W[e].x;
      E[e].y += W[e].y;
    }
    __syncthreads();
  }
  for (int q = 0; q < sq; ++q) {
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
      const int r = e / n, c = e % n;
      double re = 0.0, im = 0.0;
      for (int l = 0; l < n; ++l) {
        const double2 a = E[r * n + l], b = E[l * n + c];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
      }
      W[e] = make_double2(re, im);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nn; e += blockDim.x) E[e] = W[e];
    __syncthreads();
  }
}

// -i a tau (times g for a pair gate): the factor of the generator.
__device__ __forceinline__ double2 gate_factor(const TrGen& G, int j, double g) {
  return make_double2(G.a_im[j] * G.tau * g, -G.a_re[j] * G.tau * g);
}

// Pair gates: block b = j * E + e; row and column index (a_i d + a_j).
// ops: [mode][op][d*d] dressed operators.
__global__ void __launch_bounds__(256) tr_pair_gate_kernel(TrGen G, const double2* __restrict__ ops,
                                                           double2* __restrict__ out) {
  extern __shared__ double2 sh[];
  const int d = G.d, dd = d * d, n = dd, nn = n * n;
  double2 *X = sh, *E = sh + nn, *T = sh + 2 * nn, *W = sh + 3 * nn;
  const int b = blockIdx.x, j = b / G.E, e = b % G.E;
  const double2 w = gate_factor(G, j, G.g[e]);
  const double2* A = ops + (size_t)(G.ci[e] * 2 + G.coi[e]) * dd;
  const double2* B = ops + (size_t)(G.cj[e] * 2 + G.coj[e]) * dd;
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
    const int row = idx / n, col = idx % n;
    const double2 ab = cmul(A[(row / d) * d + col / d], B[(row % d) * d + col % d]);
    X[idx] = cmul(w, ab);
  }
  __syncthreads();
  expm_taylor(n, X, E, T, W);
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) out[(size_t)b * nn + idx] = E[idx];
}

// Single-mode gates: block b = (step * r + j) * M + m.
__global__ void __launch_bounds__(64) tr_single_gate_kernel(TrGen G, const double* __restrict__ eps,
                                                            const double2* __restrict__ ops,
                                                            const double* __restrict__ par,
                                                            double2* __restrict__ out) {
  extern __shared__ double2 sh[];
  const int d = G.d, n = d, nn = n * n;
  double2 *X = sh, *E = sh + nn, *T = sh + 2 * nn, *W = sh + 3 * nn;
  double* ck = reinterpret_cast<double*>(sh + 4 * nn);   // TR_MAXDRV drive values
  const int b = blockIdx.x, m = b % G.M, q = b / G.M, j = q % G.r;
  const long step = q / G.r;
  const double t = step * G.dt + G.mid[j];
  for (int k = threadIdx.x; k < G.ndrives; k += blockDim.x) {
    const TrDrive R = G.dr[k];
    double v = 0.0;
    if (R.mode == m) {
      for (int i = 0; i < R.npar; ++i)
        v += par[R.par0 + i] * envelope_basis(R.env, i, R.npar, step, G.N, t, G.T, R.sigma);
      v *= cos(wrap_2pi(R.omega * t + R.phase));
    }
    ck[k] = v;
  }
  __syncthreads();
  const double2 w = gate_factor(G, j, 1.0);
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
    const int row = idx / n, col = idx % n;
    double2 h = make_double2(row == col ? eps[m * d + row] : 0.0, 0.0);
    for (int k = 0; k < G.ndrives; ++k) {
      if (G.dr[k].mode != m) continue;
      const double2 o = ops[(size_t)(m * 2 + G.dr[k].op) * nn + idx];
      h.x += ck[k] * o.x;
      h.y += ck[k] * o.y;
    }
    X[idx] = cmul(w, h);
  }
  __syncthreads();
  expm_taylor(n, X, E, T, W);
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) out[(size_t)b * nn + idx] = E[idx];
}

// Fused gates: block b = ((step * r + j) * H + h) * nopmax + o multiplies the
// constituents of operation o of pass h, in action order, into a d^2 x d^2
// (pair) or d x d (single) matrix: a static operation into its slot of the
// static table (step 0 only), the others into [step][j][dix] of the per-step
// table (d^4 complex per slot).
__global__ void __launch_bounds__(256) tr_fuse_kernel(int d, int r, int H, int nopmax, int M, int E,
                                                      const TrPlan* __restrict__ plan,
                                                      const double2* __restrict__ sg,
                                                      const double2* __restrict__ pg,
                                                      double2* __restrict__ out,
                                                      double2* __restrict__ out_static) {
  extern __shared__ double2 sh[];
  const int b = blockIdx.x, o = b % nopmax, h = (b / nopmax) % H, q = b / (nopmax * H);
  const int j = q % r;
  const long step = q / r;
  const int dd = d * d;
  if (o >= plan->nop[h]) return;   // the whole block leaves together
  const TrOp& op = plan->op[h][o];
  // a lone single-mode operation reads the single-mode table directly; a
  // static operation is formed once, into the table of (piece, pass, operation)
  if (op.kind == 0 || (op.stat && (step > 0 || !op.own))) return;
  double2* slot = op.stat ? out_static + ((size_t)j * plan->nslot + op.sid) * dd * dd
                          : out + (((size_t)step * r + j) * plan->ndyn + op.dix) * dd * dd;
  const int n = op.kind ? dd : d, nn = n * n;
  double2 *A = sh, *W = sh + nn;
  for (int e = threadIdx.x; e < nn; e += blockDim.x)
    A[e] = make_double2((e / n == e % n) ? 1.0 : 0.0, 0.0);
  __syncthreads();
  for (int c = 0; c < op.nc; ++c) {
    const int ty = op.ctype[c], ix = op.cidx[c], dg = op.cdig[c];
    const double2* S = sg + ((size_t)step * r + j) * M * dd + (size_t)ix * dd;
    const double2* P = pg + ((size_t)j * E + ix) * dd * dd;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
      const int row = e / n, col = e % n;
      double re = 0.0, im = 0.0;
      if (ty == 1) {                       // pair gate times A
        for (int k = 0; k < n; ++k) {
          const double2 g = P[row * n + k], a = A[k * n + col];
          re += g.x * a.x - g.y * a.y;
          im += g.x * a.y + g.y * a.x;
        }
      } else if (!op.kind) {               // single on a single operation
        for (int k = 0; k < d; ++k) {
          const double2 g = S[row * d + k], a = A[k * n + col];
          re += g.x * a.x - g.y * a.y;
          im += g.x * a.y + g.y * a.x;
        }
      } else {                             // single embedded on digit dg of a pair
        const int ra = row / d, rb = row % d;
        for (int k = 0; k < d; ++k) {
          const double2 g = dg == 0 ? S[ra * d + k] : S[rb * d + k];
          const double2 a = dg == 0 ? A[(k * d + rb) * n + col] : A[(ra * d + k) * n + col];
          re += g.x * a.x - g.y * a.y;
          im += g.x * a.y + g.y * a.x;
        }
      }
      W[e] = make_double2(re, im);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nn; e += blockDim.x) A[e] = W[e];
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nn; e += blockDim.x) slot[e] = A[e];
}

// floor(x / n) for 0 <= x, n < 2^26 from inv = 1/n: (x + 1/2) / n lies at
// least 1/(2n) from an integer, far beyond the rounding of the product.
__device__ __forceinline__ int qdiv(int x, double inv) { return (int)(((double)x + 0.5) * inv); }

// Fibre f of a single-mode gate on the mode of stride s: the d amplitudes
// base + a*s, base = hi*s*d + lo with f = hi*s + lo.
template <int d>
__device__ __forceinline__ int fibre1(int f, int s, double inv_s) {
  const int hi = qdiv(f, inv_s);
  return hi * s * d + (f - hi * s);
}

// Fibre f of a pair gate on modes of strides si (row digit a) and sj (digit
// b), sp = max, sq = min, w = sp / (sq d): the d^2 amplitudes
// base + a*si + b*sj, base = hi*sp*d + mid*sq*d + lo with f = (hi*w + mid)*sq + lo.
template <int d>
__device__ __forceinline__ int fibre2(int f, int sp, int sq, int w, double inv_sq, double inv_w) {
  const int t = qdiv(f, inv_sq), hi = qdiv(t, inv_w);
  return hi * sp * d + (t - hi * w) * sq * d + (f - t * sq);
}

// (re, im) += g v as four fused multiply-adds (written as a difference of
// products the compiler keeps a separate multiply and add per component).
__device__ __forceinline__ void cmac(double& re, double& im, double2 g, double2 v) {
  re = fma(g.x, v.x, re);
  re = fma(-g.y, v.y, re);
  im = fma(g.x, v.y, im);
  im = fma(g.y, v.x, im);
}

// Row times a register vector of n entries (n compile-time: the vector stays
// in registers).
template <int n>
__device__ __forceinline__ double2 crow(const double2* __restrict__ g, const double2* x) {
  double re = 0.0, im = 0.0;
#pragma unroll
  for (int c = 0; c < n; ++c) {
    cmac(re, im, g[c], x[c]);
  }
  return make_double2(re, im);
}

// In place: a thread owns whole fibres of a single-mode gate.
template <int d>
__device__ __forceinline__ void tr_apply1(double2* L, int D, int s, const double2* __restrict__ Gt) {
  const int nf = D / d;
  const double is = 1.0 / s;
  for (int f = threadIdx.x; f < nf; f += blockDim.x) {
    const int base = fibre1<d>(f, s, is);
    double2 x[d];
#pragma unroll
    for (int a = 0; a < d; ++a) x[a] = L[base + a * s];
#pragma unroll
    for (int r = 0; r < d; ++r) L[base + r * s] = crow<d>(Gt + r * d, x);
  }
}

// A d x d gate on digit 0 (dg = 0) or digit 1 of a fibre x[a * d + b] in registers.
template <int d, int dg>
__device__ __forceinline__ void single_on_digit(const double2* __restrict__ S, double2* x) {
#pragma unroll
  for (int u = 0; u < d; ++u) {
    double2 t[d];
#pragma unroll
    for (int a = 0; a < d; ++a) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int k = 0; k < d; ++k) {
        cmac(re, im, S[a * d + k], dg == 0 ? x[k * d + u] : x[u * d + k]);
      }
      t[a] = make_double2(re, im);
    }
#pragma unroll
    for (int a = 0; a < d; ++a) (dg == 0 ? x[a * d + u] : x[u * d + a]) = t[a];
  }
}

// In place: a thread owns whole fibres of a pair gate.  For d <= 3 the
// single-mode gates S0 (digit 0) and S1 (digit 1), when not null, are
// applied in registers before the pair gate (post = 0) or after it.
template <int d, bool OPAQUE = false>
__device__ __forceinline__ void tr_apply2(double2* L, int D, int si, int sj, const double2* __restrict__ Gt,
                                 const double2* __restrict__ S0, const double2* __restrict__ S1,
                                 int post) {
  constexpr int dd = d * d;
  const int sp = si > sj ? si : sj, sq = si > sj ? sj : si, w = sp / (sq * d);
  const double isq = 1.0 / sq, iw = 1.0 / w;
  const int nf = D / dd;
  for (int f = threadIdx.x; f < nf; f += blockDim.x) {
    const int base = fibre2<d>(f, sp, sq, w, isq, iw);
    // OPAQUE: the gate pointer is made opaque per fibre, so that the d^4
    // gate entries are loaded where they are used instead of being hoisted
    // out of the fibre loop into registers (where the LCAM walk, with four
    // gate kinds in one loop, ran out of them); the forward keeps the
    // compiler's scalar loads of the read-only gate table
    const double2* G = Gt;
    if constexpr (OPAQUE) asm volatile("" : "+s"(G));
    double2 x[dd];
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) x[a * d + b] = L[base + a * si + b * sj];
    if constexpr (d <= 3) {
      if (!post) {
        if (S0) single_on_digit<d, 0>(S0, x);
        if (S1) single_on_digit<d, 1>(S1, x);
      } else if (S0 || S1) {
        double2 y[dd];
#pragma unroll
        for (int r = 0; r < dd; ++r) y[r] = crow<dd>(G + r * dd, x);
        if (S0) single_on_digit<d, 0>(S0, y);
        if (S1) single_on_digit<d, 1>(S1, y);
#pragma unroll
        for (int a = 0; a < d; ++a)
#pragma unroll
          for (int b = 0; b < d; ++b) L[base + a * si + b * sj] = y[a * d + b];
        continue;
      }
    }
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) L[base + a * si + b * sj] = crow<dd>(G + (a * d + b) * dd, x);
  }
}

// Split forms read ``in`` and write ``out`` (the other buffer).  Single-mode
// gate, one output row per work item w = r * nf + f.
template <int d>
__device__ __forceinline__ void tr_apply1_rows(const double2* in, double2* out, int D, int s,
                                      const double2* __restrict__ Gt) {
  const int nf = D / d;
  const double is = 1.0 / s, inf = 1.0 / nf;
  for (int w = threadIdx.x; w < D; w += blockDim.x) {
    const int r = qdiv(w, inf);
    const int base = fibre1<d>(w - r * nf, s, is);
    double2 x[d];
#pragma unroll
    for (int c = 0; c < d; ++c) x[c] = in[base + c * s];
    out[base + r * s] = crow<d>(Gt + r * d, x);
  }
}

// Pair gate, RPI output rows per work item: RPI = d computes the rows
// (a, 0..d-1) of one fibre (w = a * nf + f), RPI = 1 one row (w = r * nf + f).
// UNI: nf is a multiple of 64, so the 64 items of a wave (w from a multiple
// of 64, stepping by the block size) share their row group; taking it from
// the first lane makes the gate rows wave-uniform (scalar loads).
template <int d, int RPI, bool UNI>
__device__ __forceinline__ void tr_apply2_rows_as(const double2* in, double2* out, int D, int si, int sj,
                                         const double2* __restrict__ Gt) {
  constexpr int dd = d * d;
  const int sp = si > sj ? si : sj, sq = si > sj ? sj : si, w0 = sp / (sq * d);
  const double isq = 1.0 / sq, iw = 1.0 / w0;
  const int nf = D / dd;
  const double inf = 1.0 / nf;
  const int items = nf * (dd / RPI);
  for (int w = threadIdx.x; w < items; w += blockDim.x) {
    int g = qdiv(w, inf);                     // row group
    if constexpr (UNI) g = __builtin_amdgcn_readfirstlane(g);
    const int base = fibre2<d>(w - g * nf, sp, sq, w0, isq, iw);
    double2 x[dd];
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) x[a * d + b] = in[base + a * si + b * sj];
#pragma unroll
    for (int k = 0; k < RPI; ++k) {
      const int r = g * RPI + k;
      out[base + (r / d) * si + (r % d) * sj] = crow<dd>(Gt + r * dd, x);
    }
  }
}

template <int d, int RPI>
__device__ __forceinline__ void tr_apply2_rows(const double2* in, double2* out, int D, int si, int sj,
                                      const double2* __restrict__ Gt) {
  if ((D / (d * d)) % 64 == 0)
    tr_apply2_rows_as<d, RPI, true>(in, out, D, si, sj, Gt);
  else
    tr_apply2_rows_as<d, RPI, false>(in, out, D, si, sj, Gt);
}

// Workgroup = one column; fg: fused gates [N][r][ndyn][d^4] of pair
// operations with a single-mode factor, fs: [r][nslot][d^4] of the static
// ones, sg: [N][r][M][d^2] single-mode gates (lone single-mode operations).
template <int d>
__global__ void __launch_bounds__(TR_THREADS) trotter_kernel(TrRun R, const double2* __restrict__ psi0,
                                                             double2* __restrict__ psiT,
                                                             const double2* __restrict__ fg,
                                                             const double2* __restrict__ fs,
                                                             const double2* __restrict__ sg) {
  extern __shared__ double2 lds[];
  constexpr int dd = d * d;
  const size_t off = (size_t)blockIdx.x * R.D;
  double2* L = lds;                 // current buffer
  double2* Lo = lds + R.D;          // the other one (allocated only if a gate kind splits)
  for (int i = threadIdx.x; i < R.D; i += blockDim.x) L[i] = psi0[off + i];
  __syncthreads();
  for (int n = 0; n < R.N; ++n) {
    for (int j = 0; j < R.r; ++j) {
      for (int h = 0; h < R.H; ++h) {
        const double2* fgh = fg + ((size_t)n * R.r + j) * R.ndyn * dd * dd;
        const double2* fsj = fs + (size_t)j * R.nslot * dd * dd;
        const double2* sgj = sg + ((size_t)n * R.r + j) * R.M * dd;
        for (int o = 0; o < R.nop[h]; ++o) {
          const double2* gt = !R.opk[h][o]  ? sgj + (size_t)R.opi[h][o] * dd
                              : R.ops[h][o] > 0 ? fsj + (size_t)(R.ops[h][o] - 1) * dd * dd
                                                : fgh + (size_t)(-R.ops[h][o] - 1) * dd * dd;
          bool swap = false;
          if (!R.opk[h][o]) {
            const int sm = R.stride[R.opi[h][o]];
            if (R.mode1) {
              tr_apply1_rows<d>(L, Lo, R.D, sm, gt);
              swap = true;
            } else {
              tr_apply1<d>(L, R.D, sm, gt);
            }
          } else {
            const int si = R.stride[R.opi[h][o]], sj = R.stride[R.opj[h][o]];
            if (R.mode2 == 2) {
              tr_apply2_rows<d, d>(L, Lo, R.D, si, sj, gt);
              swap = true;
            } else if (R.mode2 == 1) {
              tr_apply2_rows<d, 1>(L, Lo, R.D, si, sj, gt);
              swap = true;
            } else {
              const int pa = R.opa[h][o], a0 = pa & 255, a1 = pa >> 8;
              tr_apply2<d>(L, R.D, si, sj, gt, a0 ? sgj + (size_t)(a0 - 1) * dd : nullptr,
                           a1 ? sgj + (size_t)(a1 - 1) * dd : nullptr, h);
            }
          }
          if (swap) {
            double2* t = L;
            L = Lo;
            Lo = t;
          }
          __syncthreads();
        }
      }
    }
  }
  for (int i = threadIdx.x; i < R.D; i += blockDim.x) {
    int r = i;
    double th = 0.0;
    for (int m = R.M - 1; m >= 0; --m) {
      th += R.fT[m][r % d];
      r /= d;
    }
    double sn, cs;
    sincos(wrap_2pi(th), &sn, &cs);
    const double2 v = L[i];
    psiT[off + i] = make_double2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
  }
}

template <int d>
hipError_t run_trotter(const TrRun& R, int S, const double2* psi0, double2* psiT, const double2* fg,
                       const double2* fs, const double2* sg, hipStream_t st) {
  const size_t sh = (size_t)R.D * sizeof(double2) * ((R.mode1 || R.mode2) ? 2 : 1);
  hipError_t e = hipFuncSetAttribute((const void*)trotter_kernel<d>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(trotter_kernel<d>, dim3(S), dim3(TR_THREADS), sh, st, R, psi0, psiT, fg, fs, sg);
  return hipGetLastError();
}

struct TrLayout {
  size_t eps, ops, par, plan, pg, sg, fg, fs, total;
  int r, sym, npar, H, nopmax, mode1, mode2;
  TrPlan P;
};

// Fusion plan.  Adjacent couplings on the same ordered mode pair form one
// operation.  With ``absorb``, in the first pass (terms in order) every
// single-mode gate commutes with the gates that do not touch its mode, so it
// moves forward to the first pair operation on its mode and joins it as its
// first factor; in the second pass (terms in reverse) it moves back to the
// last pair operation on its mode and joins it as its last factor.  Without
// it, or for a mode without a coupling, a single-mode gate stays an
// operation of its own, where the unfused sequence has it.  Absorbing halves
// the operations per step.  Formed into the fused tables it makes the pair
// operations step-dependent, which pays where a step is latency-bound (few
// fibres per gate); with ``regs`` the absorbed gates instead stay separate
// (TrOp::s0, s1) and are applied in registers next to a static pair product.
void build_plan(const scp_system* sys, int H, bool absorb, bool regs, TrPlan& P) {
  const int M = sys->n_modes, E = (int)sys->coup.size();
  for (int h = 0; h < H; ++h) {
    int nop = 0;
    TrOp lone[SCP_MAX_MODES];
    int nlone = 0;
    for (int q = 0; q < E; ++q) {
      const int e = h == 0 ? q : E - 1 - q;
      const Coupling& c = sys->coup[e];
      const bool join = nop > 0 && P.op[h][nop - 1].kind == 1 && P.op[h][nop - 1].mi == c.i &&
                        P.op[h][nop - 1].mj == c.j && P.op[h][nop - 1].nc < TR_MAXC - 2;
      if (!join) {
        TrOp& o = P.op[h][nop++];
        o = TrOp{};
        o.kind = 1;
        o.mi = c.i;
        o.mj = c.j;
      }
      TrOp& o = P.op[h][nop - 1];
      o.ctype[o.nc] = 1;
      o.cidx[o.nc] = e;
      o.cdig[o.nc] = 0;
      ++o.nc;
    }
    const int npair = nop;
    for (int m = 0; m < M; ++m) {
      int host = -1;
      for (int k = 0; absorb && k < npair; ++k) {
        const TrOp& o = P.op[h][k];
        if (o.mi == m || o.mj == m) {
          host = k;
          if (h == 0) break;                       // first operation on m (pass 1), else last
        }
      }
      if (host < 0) {
        TrOp& o = lone[nlone++];
        o = TrOp{};
        o.kind = 0;
        o.mi = o.mj = m;
        o.nc = 1;
        o.ctype[0] = 0;
        o.cidx[0] = m;
        continue;
      }
      TrOp& o = P.op[h][host];
      const int dg = o.mi == m ? 0 : 1;
      if (h == 0) {                                // acts first: prepend
        for (int c = o.nc; c > 0; --c) {
          o.ctype[c] = o.ctype[c - 1];
          o.cidx[c] = o.cidx[c - 1];
          o.cdig[c] = o.cdig[c - 1];
        }
        o.ctype[0] = 0;
        o.cidx[0] = m;
        o.cdig[0] = dg;
      } else {                                     // acts last: append
        o.ctype[o.nc] = 0;
        o.cidx[o.nc] = m;
        o.cdig[o.nc] = dg;
      }
      ++o.nc;
    }
    // register form: the absorbed single-mode gates leave the factor list
    for (int k = 0; regs && k < npair; ++k) {
      TrOp& o = P.op[h][k];
      int nc = 0;
      for (int c = 0; c < o.nc; ++c) {
        if (o.ctype[c] == 0) {
          (o.cdig[c] == 0 ? o.s0 : o.s1) = o.cidx[c] + 1;
          continue;
        }
        o.ctype[nc] = o.ctype[c];
        o.cidx[nc] = o.cidx[c];
        o.cdig[nc] = o.cdig[c];
        ++nc;
      }
      o.nc = nc;
    }
    // lone single-mode operations act first in the first pass, last in the
    // second, in the order of the unfused sequence
    for (int k = 0; k < npair; ++k) {
      TrOp& o = P.op[h][k];
      o.stat = 1;
      for (int c = 0; c < o.nc; ++c) o.stat &= o.ctype[c] == 1;
    }
    if (h == 0) {
      for (int k = npair - 1; k >= 0; --k) P.op[h][k + nlone] = P.op[h][k];
      for (int k = 0; k < nlone; ++k) P.op[h][k] = lone[k];
    } else {
      for (int k = 0; k < nlone; ++k) P.op[h][npair + k] = lone[nlone - 1 - k];
    }
    P.nop[h] = nop + nlone;
  }
  // static slots: operations with the same factors in the same order share one
  P.nslot = 0;
  for (int h = 0; h < H; ++h)
    for (int o = 0; o < P.nop[h]; ++o) {
      TrOp& a = P.op[h][o];
      if (!a.stat) continue;
      a.own = 1;
      a.sid = P.nslot;
      for (int h2 = 0; h2 <= h && a.own; ++h2)
        for (int o2 = 0; o2 < (h2 == h ? o : P.nop[h2]); ++o2) {
          const TrOp& b = P.op[h2][o2];
          bool same = b.stat && b.own && b.mi == a.mi && b.mj == a.mj && b.nc == a.nc;
          for (int c = 0; same && c < a.nc; ++c) same = b.cidx[c] == a.cidx[c];
          if (same) {
            a.own = 0;
            a.sid = b.sid;
            break;
          }
        }
      if (a.own) ++P.nslot;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

TrLayout tr_layout(const scp_system* sys, int order) {
  TrLayout L{};
  L.r = order == SCP_TROTTER_Q4 ? 3 : (order == SCP_TROTTER_Q4J ? 2 : 1);
  L.sym = order != SCP_TROTTER_Q1;
  L.H = L.sym ? 2 : 1;
  {
    // split forms need a second column buffer; single-mode gates are
    // absorbed into pair operations exactly when pair gates run split
    const int64_t D = sys->D, dg = sys->d, E0 = (int64_t)sys->coup.size();
    const bool two = 2 * D * (int64_t)sizeof(double2) <= TR_MAXLDS;
    const int64_t nf1 = D / dg, nf2 = D / (dg * dg);
    L.mode2 = (!two || E0 == 0 || nf2 >= TR_THREADS) ? 0 : (nf2 * dg >= TR_THREADS ? 2 : 1);
    // where pair gates run in place (large D, d <= 3) the single-mode gates
    // are absorbed in registers instead, next to static pair products
    const bool regs = L.mode2 == 0 && E0 > 0 && dg <= 3;
    L.P = TrPlan{};
    build_plan(sys, L.H, L.mode2 != 0 || regs, regs, L.P);
    bool any_single = false;
    for (int h = 0; h < L.H; ++h)
      for (int o = 0; o < L.P.nop[h]; ++o) any_single |= L.P.op[h][o].kind == 0;
    L.mode1 = (two && any_single && nf1 < TR_THREADS) ? 1 : 0;
  }
  L.nopmax = std::max(L.P.nop[0], L.H > 1 ? L.P.nop[1] : 0);
  // the per-step fused-gate table holds only the pair operations with a
  // single-mode factor (the static ones are formed once)
  L.P.ndyn = 0;
  for (int h = 0; h < L.H; ++h)
    for (int o = 0; o < L.P.nop[h]; ++o) {
      TrOp& op = L.P.op[h][o];
      op.dix = (op.kind == 1 && !op.stat) ? L.P.ndyn++ : -1;
    }
  L.npar = 0;
  for (const Drive& R : sys->drives) L.npar += (int)R.par.size();
  const size_t d = sys->d, M = sys->n_modes, E = sys->coup.size();
  size_t o = 0;
  L.eps = o;
  o = align256(o + M * d * sizeof(double));
  L.ops = o;
  o = align256(o + M * 2 * d * d * sizeof(double2));
  L.par = o;
  o = align256(o + std::max(1, L.npar) * sizeof(double));
  L.plan = o;
  o = align256(o + sizeof(TrPlan));
  L.pg = o;
  o = align256(o + (size_t)L.r * std::max<size_t>(1, E) * d * d * d * d * sizeof(double2));
  L.sg = o;
  o = align256(o + (size_t)sys->n_steps * L.r * M * d * d * sizeof(double2));
  L.fg = o;
  o = align256(o + (size_t)sys->n_steps * L.r * L.P.ndyn * d * d * d * d * sizeof(double2));
  L.fs = o;
  o = align256(o + (size_t)L.r * std::max(1, L.P.nslot) * d * d * d * d * sizeof(double2));
  L.total = o;
  return L;
}

}  // namespace

scp_status trotter_check(const scp_system* sys, int order) {
  if (order < SCP_TROTTER_Q1 || order > SCP_TROTTER_Q4J)
    return fail(SCP_EINVAL, "order must be one of SCP_TROTTER_Q1, Q2, Q4, Q4J");
  if (sys->d < 2 || sys->d > TR_MAXD) return fail(SCP_EINVAL, "the Trotter path takes d = 2..5");
  if (sys->D * (int64_t)sizeof(double2) > TR_MAXLDS)
    return fail(SCP_EINVAL, "the Trotter path keeps a column in LDS: 16 D bytes must be <= 160 KiB");
  if ((int)sys->coup.size() > TR_MAXE) return fail(SCP_EINVAL, "the Trotter path takes <= 48 couplings");
  if ((int)sys->drives.size() > TR_MAXDRV) return fail(SCP_EINVAL, "the Trotter path takes <= 32 drives");
  return SCP_OK;
}

size_t trotter_workspace_bytes(const scp_system* sys, int order) { return tr_layout(sys, order).total; }

namespace {

// The gate generator description of a system and order (pieces, frozen
// times, drives, couplings); the pulse parameters go to ipar in drive order.
TrGen make_gen(const scp_system* sys, int order, const TrLayout& W, double* ipar) {
  const int d = sys->d, M = sys->n_modes, E = (int)sys->coup.size(), N = sys->n_steps;
  TrGen G{};
  G.d = d;
  G.M = M;
  G.E = E;
  G.N = N;
  G.r = W.r;
  G.ndrives = (int)sys->drives.size();
  G.dt = sys->h;
  G.T = sys->T;
  G.tau = W.sym ? 0.5 * sys->h : sys->h;
  double are[3] = {1.0, 0.0, 0.0}, aim[3] = {0.0, 0.0, 0.0};
  if (order == SCP_TROTTER_Q4) {
    const double p = 1.0 / (2.0 - std::cbrt(2.0));
    are[0] = p;
    are[1] = 1.0 - 2.0 * p;
    are[2] = p;
  } else if (order == SCP_TROTTER_Q4J) {
    are[0] = are[1] = 0.5;
    aim[0] = -std::sqrt(3.0) / 6.0;
    aim[1] = std::sqrt(3.0) / 6.0;
  }
  double start = 0.0;
  for (int j = 0; j < W.r; ++j) {
    G.a_re[j] = are[j];
    G.a_im[j] = aim[j];
    G.mid[j] = order == SCP_TROTTER_Q4J ? 0.5 * sys->h : start + 0.5 * are[j] * sys->h;
    start += are[j] * sys->h;
  }
  int np = 0;
  for (int k = 0; k < G.ndrives; ++k) {
    const Drive& R = sys->drives[k];
    G.dr[k] = TrDrive{R.mode, R.op, R.env, (int)R.par.size(), np, R.omega, R.phase, R.sigma};
    for (double v : R.par) ipar[np++] = v;
  }
  for (int e = 0; e < E; ++e) {
    const Coupling& c = sys->coup[e];
    G.ci[e] = c.i;
    G.cj[e] = c.j;
    G.coi[e] = c.op_i;
    G.coj[e] = c.op_j;
    G.g[e] = c.g;
  }
  return G;
}

}  // namespace

// psi0 == nullptr: the gate tables only (single-mode and pair gates, what
// the adjoint reuses), no fusion and no propagation
scp_status launch_trotter(scp_system* sys, int order, int S, void* ws, const double2* psi0,
                          double2* psiT, hipStream_t st) {
  scp_status chk = trotter_check(sys, order);
  if (chk != SCP_OK) return chk;
  const TrLayout W = tr_layout(sys, order);
  const int d = sys->d, M = sys->n_modes, E = (int)sys->coup.size(), N = sys->n_steps;
  char* base = static_cast<char*>(ws);
  // inputs: energies, dressed operators, pulse parameters
  std::vector<char> in(W.pg, 0);
  double* ieps = reinterpret_cast<double*>(in.data() + W.eps);
  double2* iops = reinterpret_cast<double2*>(in.data() + W.ops);
  double* ipar = reinterpret_cast<double*>(in.data() + W.par);
  std::memcpy(in.data() + W.plan, &W.P, sizeof(TrPlan));
  for (int m = 0; m < M; ++m) {
    for (int a = 0; a < d; ++a) ieps[m * d + a] = sys->modes[m].eps[a];
    for (int op = 0; op < 2; ++op)
      for (int i = 0; i < d * d; ++i) {
        const cplx v = sys->modes[m].ops[op][i];
        iops[(m * 2 + op) * d * d + i] = make_double2(v.real(), v.imag());
      }
  }
  const TrGen G = make_gen(sys, order, W, ipar);
  HIPCHK(hipMemcpyAsync(base, in.data(), in.size(), hipMemcpyHostToDevice, st));
  // the staging vector must outlive the copy
  HIPCHK(hipStreamSynchronize(st));
  const double* deps = reinterpret_cast<const double*>(base + W.eps);
  const double2* dops = reinterpret_cast<const double2*>(base + W.ops);
  const double* dpar = reinterpret_cast<const double*>(base + W.par);
  double2* pg = reinterpret_cast<double2*>(base + W.pg);
  double2* sg = reinterpret_cast<double2*>(base + W.sg);
  if (E > 0) {
    const int n = d * d;
    hipLaunchKernelGGL(tr_pair_gate_kernel, dim3(W.r * E), dim3(256), 4 * n * n * sizeof(double2), st,
                       G, dops, pg);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(tr_single_gate_kernel, dim3((unsigned)((size_t)N * W.r * M)), dim3(64),
                     4 * d * d * sizeof(double2) + TR_MAXDRV * sizeof(double), st, G, deps, dops, dpar,
                     sg);
  HIPCHK(hipGetLastError());
  if (psi0 == nullptr) return SCP_OK;
  double2* fg = reinterpret_cast<double2*>(base + W.fg);
  double2* fs = reinterpret_cast<double2*>(base + W.fs);
  {
    // every step only where some pair operation is re-formed per step; else
    // step 0, which forms the static operations
    const size_t blocks = (size_t)(W.P.ndyn > 0 ? N : 1) * W.r * W.H * W.nopmax;
    const int n = d * d;
    hipLaunchKernelGGL(tr_fuse_kernel, dim3((unsigned)blocks), dim3(256), 2 * n * n * sizeof(double2), st,
                       d, W.r, W.H, W.nopmax, M, E, reinterpret_cast<const TrPlan*>(base + W.plan), sg,
                       pg, fg, fs);
    HIPCHK(hipGetLastError());
  }
  TrRun R{};
  R.M = M;
  R.N = N;
  R.r = W.r;
  R.H = W.H;
  R.nopmax = W.nopmax;
  R.nslot = W.P.nslot;
  R.ndyn = W.P.ndyn;
  for (int h = 0; h < W.H; ++h) {
    R.nop[h] = W.P.nop[h];
    for (int o = 0; o < W.P.nop[h]; ++o) {
      R.opk[h][o] = W.P.op[h][o].kind;
      R.opi[h][o] = W.P.op[h][o].mi;
      R.opj[h][o] = W.P.op[h][o].mj;
      R.ops[h][o] = W.P.op[h][o].stat ? W.P.op[h][o].sid + 1 : -(W.P.op[h][o].dix + 1);
      R.opa[h][o] = W.P.op[h][o].s0 | (W.P.op[h][o].s1 << 8);
    }
  }
  R.D = (int)sys->D;
  R.mode1 = W.mode1;
  R.mode2 = W.mode2;
  int s = 1;
  for (int m = M - 1; m >= 0; --m) {
    R.stride[m] = s;
    s *= d;
  }
  const double twopi = 6.283185307179586476925286766559;
  for (int m = 0; m < M; ++m)
    for (int a = 0; a < d; ++a) R.fT[m][a] = std::remainder(sys->modes[m].frame[a] * N * sys->h, twopi);
  hipError_t e;
  switch (d) {
    case 2: e = run_trotter<2>(R, S, psi0, psiT, fg, fs, sg, st); break;
    case 3: e = run_trotter<3>(R, S, psi0, psiT, fg, fs, sg, st); break;
    case 4: e = run_trotter<4>(R, S, psi0, psiT, fg, fs, sg, st); break;
    default: e = run_trotter<5>(R, S, psi0, psiT, fg, fs, sg, st); break;
  }
  HIPCHK(e);
  return SCP_OK;
}


// ---------------------------------------------------------------------------
// Local continuous adjoint method (LCAM) of the product formulas (Sec. 2.5).
//
// Only the final state of the forward is kept.  The walk goes back over the
// steps, and within a step over its gates in reverse order; at every gate
//   phi = G^-1 psi              (the state before the gate, recovered by
//                                evolving backward in time),
//   M_ab += sum_rest conj(mu[a, rest]) phi[b, rest]   (the gate's local
//                                reduced matrix; a, b its local indices),
//   mu  = G^dag mu              (the costate before the gate),
// which is the paper's i-th term a_i^T (dU_i/dtheta) psi_{i-1} with the step
// written as a product of local gates, so that every gate contributes through
// its own local derivative.  For G = exp(X), X = -i a tau h,
//   sum_ab (dG)_ab M_ab = Tr(L(X, M^T) dX),
// L the Frechet derivative of exp, taken from the block-triangular exponential
// exp([[X, M^T], [0, X]]) = [[e^X, L(X, M^T)], [0, e^X]] (Van Loan 1978) by
// the same Taylor scaling and squaring as the gates.  L is linear in M, so M
// can be summed first: over the columns for a single-mode gate (one h per
// step and piece), and over columns, steps and both passes for a pair gate
// (its h does not depend on time).  Then every parameter needs the traces of
// K = L(X, M^T) with dh/dtheta; the host forms
//   dL/dtheta = sum 2 Re(-i a tau Tr(K dh/dtheta))
// in FP64 in a fixed order.  For Q4j the gates are not unitary: the state is
// recovered with exp(-X), the costate uses G^dag.  Everything is FP64.
//
// The walk: one workgroup per column keeps psi and mu in LDS (in place, 32 D
// bytes plus a reduction scratch, or split into two buffers each when 64 D
// bytes and the gate tables fit, see the split walk); the single-mode reduced
// matrices of a chunk of steps go to a per-column buffer (the visits of a
// step summed in place, or one slot per visit in the split walk) that a
// second kernel reduces over the visits and columns in a fixed order; the
// pair sums accumulate per column.  No atomics: the result is bitwise
// reproducible.
// ---------------------------------------------------------------------------
namespace {

constexpr int LC_CHUNK = 128;     // steps per walk launch

struct LcRun {
  int M, E, N, r, H, D, S;
  int stride[SCP_MAX_MODES];
  int ci[TR_MAXE], cj[TR_MAXE];
  double fT[SCP_MAX_MODES][SCP_MAX_TRUNC];   // frame energy times T, reduced mod 2 pi
};

static_assert(sizeof(LcRun) <= 2048, "LcRun is passed by value as a kernel argument");

// G^dag of n x n gates (blocks of nn entries)
__global__ void lc_adjoint_table_kernel(const double2* __restrict__ G, double2* __restrict__ out,
                                        int n, size_t count) {
  const size_t nn = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count * nn;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t b = e / nn, w = e % nn;
    const int r = (int)(w / n), c = (int)(w % n);
    const double2 v = G[b * nn + (size_t)c * n + r];
    out[e] = make_double2(v.x, -v.y);
  }
}

// exp(-i f T) times x (the frame rotation of the output, undone)
__device__ __forceinline__ double2 unrotate(const LcRun& R, int d, int i, double2 v) {
  int r = i;
  double th = 0.0;
  for (int m = R.M - 1; m >= 0; --m) {
    th += R.fT[m][r % d];
    r /= d;
  }
  double sn, cs;
  sincos(-wrap_2pi(th), &sn, &cs);
  return make_double2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
}

// Walk of steps [n_lo, n_hi) backward for one column.  first: start from
// psi_I(T) and lambda_I(T) (un-rotated to the lab frame) and clear this
// column's pair sums; else continue from psi_st / mu_st.  Ms: [(step - n_lo)
// r + j) M + m][S][d^2] single-mode sums of this chunk; Mp: [S][r E][d^4].
// Gate applications of the walk (inverse and adjoint, one- and two-mode).
template <int d>
__device__ __forceinline__ void lc_apply1(double2* L, int D, int s, const double2* G) {
  tr_apply1<d>(L, D, s, G);
}
template <int d>
__device__ __forceinline__ void lc_apply2(double2* L, int D, int si, int sj, const double2* G) {
  tr_apply2<d, true>(L, D, si, sj, G, nullptr, nullptr, 0);
}

template <int d>
__global__ void __launch_bounds__(TR_THREADS)
lc_walk_kernel(LcRun R, int n_hi, int n_lo, int first, const double2* __restrict__ psiT,
               const double2* __restrict__ lamT, double2* __restrict__ psi_st,
               double2* __restrict__ mu_st, const double2* __restrict__ sg_inv,
               const double2* __restrict__ sg_adj, const double2* __restrict__ pg_inv,
               const double2* __restrict__ pg_adj, double2* __restrict__ Ms,
               double2* __restrict__ Mp) {
  extern __shared__ double2 lds[];
  constexpr int dd = d * d;
  const int col = blockIdx.x;
  const size_t off = (size_t)col * R.D;
  double2* L = lds;                   // psi (the state)
  double2* Lm = lds + R.D;            // mu (the costate)
  double2* scr = lds + 2 * R.D;       // TR_THREADS partial sums
  const size_t np_col = (size_t)R.r * R.E * dd * dd;
  if (first) {
    for (int i = threadIdx.x; i < R.D; i += blockDim.x) {
      L[i] = unrotate(R, d, i, psiT[off + i]);
      Lm[i] = unrotate(R, d, i, lamT[off + i]);
    }
    for (size_t e = threadIdx.x; e < np_col; e += blockDim.x) Mp[col * np_col + e] = make_double2(0, 0);
  } else {
    for (int i = threadIdx.x; i < R.D; i += blockDim.x) {
      L[i] = psi_st[off + i];
      Lm[i] = mu_st[off + i];
    }
  }
  const int nq = (n_hi - n_lo) * R.r * R.M;
  for (int e = threadIdx.x; e < nq * dd; e += blockDim.x)
    Ms[((size_t)(e / dd) * R.S + col) * dd + e % dd] = make_double2(0, 0);
  __syncthreads();
  const int K = R.M + R.E;
  const int len = R.H == 2 ? 2 * K : K;
  // the adjoint gate still to be applied to mu (from the previous gate of the walk)
  const double2* pend = nullptr;
  int pend_t = 0;
  for (int n = n_hi - 1; n >= n_lo; --n) {
    for (int j = R.r - 1; j >= 0; --j) {
      for (int q = len - 1; q >= 0; --q) {
        const int t = q < K ? q : 2 * K - 1 - q;   // local term of this gate
        const bool single = t < R.M;
        const double2* gi;
        const double2* ga;
        int s0, s1;
        if (single) {
          const size_t b = ((size_t)n * R.r + j) * R.M + t;
          gi = sg_inv + b * dd;
          ga = sg_adj + b * dd;
          s0 = R.stride[t];
          s1 = 0;
        } else {
          const size_t b = (size_t)j * R.E + (t - R.M);
          gi = pg_inv + b * dd * dd;
          ga = pg_adj + b * dd * dd;
          s0 = R.stride[R.ci[t - R.M]];
          s1 = R.stride[R.cj[t - R.M]];
        }
        // phase A: psi <- G^-1 psi; mu <- (previous gate)^dag mu, through one
        // copy of the code (separately inlined copies were scheduled very
        // differently, one with a full wait after nearly every gate read)
#pragma unroll 1
        for (int v = 0; v < 2; ++v) {
          const bool isp = v == 0;
          if (!isp && pend == nullptr) break;
          const int pe = pend_t < R.M ? 0 : pend_t - R.M;   // pending pair gate's coupling
          const bool one = isp ? single : pend_t < R.M;
          const int sa = isp ? s0 : (one ? R.stride[pend_t] : R.stride[R.ci[pe]]);
          const int sb = isp ? s1 : (one ? 0 : R.stride[R.cj[pe]]);
          double2* Lv = isp ? L : Lm;
          const double2* Gv = isp ? gi : pend;
          if (one)
            lc_apply1<d>(Lv, R.D, sa, Gv);
          else
            lc_apply2<d>(Lv, R.D, sa, sb, Gv);
        }
        __syncthreads();
        // phase B: the gate's local reduced matrix M_AB = sum conj(mu[A]) phi[B]
        {
          const int nloc = single ? d : dd;
          const int ent = nloc * nloc;
          const int ch = ent >= TR_THREADS ? 1 : TR_THREADS / ent;
          const int nf = R.D / nloc;
          int sp = 0, sq = 0, w = 0;
          double isq = 0.0, iw = 0.0, is0 = 1.0 / s0;
          if (!single) {
            sp = s0 > s1 ? s0 : s1;
            sq = s0 > s1 ? s1 : s0;
            w = sp / (sq * d);
            isq = 1.0 / sq;
            iw = 1.0 / w;
          }
          double2* Mdst = single
              ? Ms + ((((size_t)(n - n_lo) * R.r + j) * R.M + t) * R.S + col) * dd
              : Mp + col * np_col + ((size_t)j * R.E + (t - R.M)) * dd * dd;
          for (int wi = threadIdx.x; wi < ent * ch; wi += blockDim.x) {
            const int e = wi / ch, c = wi - e * ch;
            const int A = e / nloc, B = e - A * nloc;
            const int oa = single ? A * s0 : (A / d) * s0 + (A % d) * s1;
            const int ob = single ? B * s0 : (B / d) * s0 + (B % d) * s1;
            double re = 0.0, im = 0.0;
            for (int f = c; f < nf; f += ch) {
              const int base = single ? fibre1<d>(f, s0, is0) : fibre2<d>(f, sp, sq, w, isq, iw);
              const double2 u = Lm[base + oa], v = L[base + ob];
              re = fma(u.x, v.x, re);
              re = fma(u.y, v.y, re);
              im = fma(u.x, v.y, im);
              im = fma(-u.y, v.x, im);
            }
            if (ch == 1) {
              const double2 o = Mdst[e];
              Mdst[e] = make_double2(o.x + re, o.y + im);
            } else {
              scr[wi] = make_double2(re, im);
            }
          }
          if (ch > 1) {
            __syncthreads();
            for (int e = threadIdx.x; e < ent; e += blockDim.x) {
              double re = 0.0, im = 0.0;
              for (int c = 0; c < ch; ++c) {
                re += scr[e * ch + c].x;
                im += scr[e * ch + c].y;
              }
              const double2 o = Mdst[e];
              Mdst[e] = make_double2(o.x + re, o.y + im);
            }
          }
        }
        __syncthreads();
        pend = ga;
        pend_t = t;
      }
    }
  }
  if (pend != nullptr) {
    if (pend_t < R.M)
      lc_apply1<d>(Lm, R.D, R.stride[pend_t], pend);
    else
      lc_apply2<d>(Lm, R.D, R.stride[R.ci[pend_t - R.M]], R.stride[R.cj[pend_t - R.M]], pend);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R.D; i += blockDim.x) {
    psi_st[off + i] = L[i];
    mu_st[off + i] = Lm[i];
  }
}

// Split walk, for columns small enough that LDS holds two buffers each of psi
// and mu, two slots each of inverse and adjoint gate tables, two slots of
// partial sums and three of fibre offsets (see lc_split_lds).  The in-place
// walk above keeps only D / d^2 threads busy on a pair gate and needs three
// barriers per gate; here a work item computes d output rows of one fibre
// from one buffer into the other, and the interval between two barriers holds
//   A. psi' = G_g^-1 psi and mu' = G_{g-1}^dag mu (g: position in the walk),
//   B. the reduced matrix of gate g-1 from psi and mu (the state before that
//      gate and the costate after it, the same buffers A reads), its fibres
//      split over ch items whose partial sums go to an LDS slot when ch > 1,
//   C. the sum of those partial sums for gate g-2, in a fixed order,
//   D. the tables A needs in the next interval (G_{g+1}^-1, G_g^dag), read
//      from memory during the interval before, are stored to the free LDS
//      slots at the start of the interval, and the fibre offsets of gate g+1
//      at its end,
// so one barrier per gate.  The items of psi's A, mu's A, B and C each start
// on a wave boundary: a wave that mixed two of them would run both codes one
// after the other.  A single-mode gate's reduced matrix of one visit is
// stored once (its own slot); a pair gate's is added to the column's sum,
// whose old value is loaded at the start of the interval by the thread that
// adds to it.  Every sum is in a fixed order: bitwise reproducible.
// On the 4-fluxonium chain (d = 5, D = 625) the intervals with a pair gate
// dominate, bound by the LDS reads of A's gate rows and fibres.
constexpr int LC_THREADS = 512;   // split-walk workgroup (2 waves per SIMD)

struct LcGate {
  const double2* gi;   // G^-1 (memory)
  const double2* ga;   // G^dag
  double2* m;          // this column's reduced matrix of the gate (Ms slot or Mp block)
  int s0, s1;          // strides of the gate's digits (s1 = 0: single-mode gate)
};

// Position of a gate in the walk over steps [n_lo, n_hi): steps backward,
// pieces backward, the len = nvis K local terms of a piece backward (a
// symmetric piece visits every term twice: visit 0 in the first half of the
// piece, visit 1 in the second).  Advanced by one gate at a time (no
// divisions in the loop).
struct LcPos {
  int n, j, q;
};
__device__ __forceinline__ void lc_advance(LcPos& p, int r, int len) {
  if (--p.q < 0) {
    p.q = len - 1;
    if (--p.j < 0) {
      p.j = r - 1;
      --p.n;
    }
  }
}

// the gate at position p
__device__ __forceinline__ LcGate lc_gate(const LcRun& R, const LcPos& p, int n_lo, int col,
                                          const double2* sgi, const double2* sga,
                                          const double2* pgi, const double2* pga, double2* Ms,
                                          double2* Mp, int dd) {
  const int K = R.M + R.E, nvis = R.H == 2 ? 2 : 1;
  const int n = p.n, j = p.j, q = p.q;
  const int t = q < K ? q : 2 * K - 1 - q, vis = q < K ? 0 : 1;
  LcGate G;
  if (t < R.M) {
    const size_t b = ((size_t)n * R.r + j) * R.M + t;
    G.gi = sgi + b * dd;
    G.ga = sga + b * dd;
    G.m = Ms + (((((size_t)(n - n_lo) * R.r + j) * R.M + t) * nvis + vis) * R.S + col) * dd;
    G.s0 = R.stride[t];
    G.s1 = 0;
  } else {
    const size_t b = (size_t)j * R.E + (t - R.M);
    G.gi = pgi + b * dd * dd;
    G.ga = pga + b * dd * dd;
    G.m = Mp + ((size_t)col * R.r * R.E + b) * dd * dd;
    G.s0 = R.stride[R.ci[t - R.M]];
    G.s1 = R.stride[R.cj[t - R.M]];
  }
  return G;
}

// partial sums per entry of a reduced matrix with ent entries over nf fibres
__device__ __forceinline__ int lc_chunks(int ent, int nf) {
  const int c = ent >= LC_THREADS ? 1 : LC_THREADS / ent;
  return c < nf ? (c < 16 ? c : 16) : nf;
}

// first item of this thread in a loop whose items follow `off` earlier ones
// (so consecutive loops of one interval fill the block in turn)
__device__ __forceinline__ int lc_first(int off) {
  return (int)((threadIdx.x + LC_THREADS - (unsigned)off % LC_THREADS) % LC_THREADS);
}

// fibre offsets of gate G (D/d of a single-mode gate, D/d^2 of a pair gate)
template <int d>
__device__ __forceinline__ void lc_fibres(const LcGate& G, int D, int* tab) {
  if (G.s1 == 0) {
    const double is = 1.0 / G.s0;
    for (int f = threadIdx.x; f < D / d; f += LC_THREADS) tab[f] = fibre1<d>(f, G.s0, is);
  } else {
    const int sp = G.s0 > G.s1 ? G.s0 : G.s1, sq = G.s0 > G.s1 ? G.s1 : G.s0;
    const int wd = sp / (sq * d);
    const double isq = 1.0 / sq, iw = 1.0 / wd;
    for (int f = threadIdx.x; f < D / (d * d); f += LC_THREADS)
      tab[f] = fibre2<d>(f, sp, sq, wd, isq, iw);
  }
}

// A: out = Gt in (Gt and the fibre offsets in LDS), from the item w0 on;
// D/d items: the d rows of a fibre of a single-mode gate, or the rows
// (a, 0..d-1) of a pair fibre
template <int d>
__device__ __forceinline__ void lc_split_apply(const double2* in, double2* out, const LcGate& G,
                                               const double2* Gt, const int* tab, int D, int w0) {
  constexpr int dd = d * d;
  if (G.s1 == 0) {
    const int s = G.s0;
    for (int w = w0; w < D / d; w += LC_THREADS) {
      const int base = tab[w];
      double2 x[d], y[d];
#pragma unroll
      for (int a = 0; a < d; ++a) x[a] = in[base + a * s];
#pragma unroll
      for (int r = 0; r < d; ++r) y[r] = crow<d>(Gt + r * d, x);
#pragma unroll
      for (int r = 0; r < d; ++r) out[base + r * s] = y[r];
    }
  } else {
    const int si = G.s0, sj = G.s1, nf = D / dd;
    for (int w = w0; w < d * nf; w += LC_THREADS) {
      const int a = w / nf, base = tab[w - a * nf];
      double2 x[dd], y[d];
#pragma unroll
      for (int u = 0; u < d; ++u)
#pragma unroll
        for (int v = 0; v < d; ++v) x[u * d + v] = in[base + u * si + v * sj];
#pragma unroll
      for (int k = 0; k < d; ++k) y[k] = crow<dd>(Gt + (a * d + k) * dd, x);
#pragma unroll
      for (int k = 0; k < d; ++k) out[base + a * si + k * sj] = y[k];
    }
  }
}

__device__ __forceinline__ void lc_copy(const double2* in, double2* out, int D, int w0) {
  for (int i = w0; i < D; i += LC_THREADS) out[i] = in[i];
}

// One B item of a gate of NL local levels, wi = c ent + e: the sum over the
// fibres f = c mod ch of conj(mu[A]) psi[B] for the entry e = (A, B).  ch = 1:
// it adds o (the entry's earlier sum, which this thread loaded) and stores;
// else the partial sum goes to scr[e ch + c].
template <int d, int NL>
__device__ __forceinline__ void lc_split_item(const double2* mu, const double2* psi,
                                              const LcGate& G, const int* tab, int nf, int ch,
                                              double2* scr, double2 o, int wi) {
  constexpr int ent = NL * NL, U = 4;   // U fibres in flight, each its own partial sum
  const int c = wi / ent, e = wi - c * ent;
  const int A = e / NL, B = e - A * NL;
  const int oa = NL == d ? A * G.s0 : (A / d) * G.s0 + (A % d) * G.s1;
  const int ob = NL == d ? B * G.s0 : (B / d) * G.s0 + (B % d) * G.s1;
  double re[U], im[U];
#pragma unroll
  for (int k = 0; k < U; ++k) re[k] = im[k] = 0.0;
  int f = c;
  for (; f + (U - 1) * ch < nf; f += U * ch) {
    int b[U];
#pragma unroll
    for (int k = 0; k < U; ++k) b[k] = tab[f + k * ch];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const double2 u = mu[b[k] + oa], v = psi[b[k] + ob];
      re[k] = fma(u.x, v.x, re[k]);
      re[k] = fma(u.y, v.y, re[k]);
      im[k] = fma(u.x, v.y, im[k]);
      im[k] = fma(-u.y, v.x, im[k]);
    }
  }
  for (; f < nf; f += ch) {
    const int base = tab[f];
    const double2 u = mu[base + oa], v = psi[base + ob];
    re[0] = fma(u.x, v.x, re[0]);
    re[0] = fma(u.y, v.y, re[0]);
    im[0] = fma(u.x, v.y, im[0]);
    im[0] = fma(-u.y, v.x, im[0]);
  }
  const double sr = (re[0] + re[1]) + (re[2] + re[3]), si = (im[0] + im[1]) + (im[2] + im[3]);
  if (ch == 1)
    G.m[e] = make_double2(o.x + sr, o.y + si);
  else
    scr[e * ch + c] = make_double2(sr, si);
}

// B for a gate of NL local levels: M_AB = sum over fibres of conj(mu[A]) psi[B];
// item wi = c ent + e (w0 and w0 + T for this thread: ent ch <= d^4 <= 2 T)
// sums the fibres f = c mod ch.  ch = 1: it adds old[0] or old[1] (the earlier
// sums this thread loaded) and stores; else the partial sum goes to
// scr[e ch + c].  Straight-line code, no item loop: a loop that stores to
// memory and uses values loaded before it makes the compiler wait for every
// load in flight (the prefetched tables) at its entry.
template <int d, int NL>
__device__ __forceinline__ void lc_split_reduce_n(const double2* mu, const double2* psi,
                                                  const LcGate& G, const int* tab, int nf, int ch,
                                                  double2* scr, const double2* old, int w0) {
  constexpr int ent = NL * NL;
  static_assert(ent <= 2 * LC_THREADS, "at most two B items per thread");
  if (w0 < ent * ch) lc_split_item<d, NL>(mu, psi, G, tab, nf, ch, scr, old[0], w0);
  if (w0 + LC_THREADS < ent * ch)
    lc_split_item<d, NL>(mu, psi, G, tab, nf, ch, scr, old[1], w0 + LC_THREADS);
}

// C: the partial sums of B for gate G, in the order c = 0, 1, ...; entry e
// (< T here) is this thread's, which adds old[0] for a pair gate
template <int d>
__device__ __forceinline__ void lc_split_fold(const LcGate& G, int ch, const double2* scr,
                                              const double2* old, int e) {
  const bool single = G.s1 == 0;
  const int ent = single ? d * d : d * d * d * d;
  if (ch == 1 || e >= ent) return;
  double re = 0.0, im = 0.0;
#pragma unroll 4
  for (int c = 0; c < ch; ++c) {
    re += scr[e * ch + c].x;
    im += scr[e * ch + c].y;
  }
  if (single) {
    G.m[e] = make_double2(re, im);
  } else {
    G.m[e] = make_double2(old[0].x + re, old[0].y + im);
  }
}

template <int d>
__global__ void __launch_bounds__(LC_THREADS)
lc_walk_split_kernel(LcRun R, int n_hi, int n_lo, int first, const double2* __restrict__ psiT,
                     const double2* __restrict__ lamT, double2* __restrict__ psi_st,
                     double2* __restrict__ mu_st, const double2* __restrict__ sg_inv,
                     const double2* __restrict__ sg_adj, const double2* __restrict__ pg_inv,
                     const double2* __restrict__ pg_adj, double2* __restrict__ Ms,
                     double2* __restrict__ Mp) {
  extern __shared__ double2 lds[];
  constexpr int dd = d * d, NN = dd * dd;
  static_assert(NN <= 2 * LC_THREADS, "a gate table is prefetched as two entries per thread");
  const int col = blockIdx.x, D = R.D, tid = threadIdx.x, nft = D / d;
  const size_t off = (size_t)col * D;
  double2* P = lds;                  // psi: two buffers of D
  double2* U = lds + 2 * D;          // mu: two buffers of D
  double2* Gi = lds + 4 * D;         // inverse gates: two slots of NN
  double2* Ga = Gi + 2 * NN;         // adjoint gates: two slots of NN
  double2* scr = Ga + 2 * NN;        // partial sums: two slots of LC_THREADS
  int* tab = reinterpret_cast<int*>(scr + 2 * LC_THREADS);   // fibre offsets: three slots of D/d
  const size_t np_col = (size_t)R.r * R.E * NN;
  const int K = R.M + R.E, len = R.H == 2 ? 2 * K : K;
  const int ng = (n_hi - n_lo) * R.r * len;   // gates of this launch
  // launch constants of the two gate kinds: fibres and partial sums per entry
  const int nf1 = D / d, nf2 = D / dd;
  const int ch1 = lc_chunks(dd, nf1), ch2 = lc_chunks(NN, nf2);
  auto gate = [&](const LcPos& p) {
    return lc_gate(R, p, n_lo, col, sg_inv, sg_adj, pg_inv, pg_adj, Ms, Mp, dd);
  };
  auto nn_of = [&](const LcGate& G) { return G.s1 ? NN : dd; };
  auto chunks_of = [&](const LcGate& G) { return G.s1 ? ch2 : ch1; };
  if (first) {
    for (int i = tid; i < D; i += LC_THREADS) {
      P[i] = unrotate(R, d, i, psiT[off + i]);
      U[i] = unrotate(R, d, i, lamT[off + i]);
    }
    for (size_t e = tid; e < np_col; e += LC_THREADS) Mp[col * np_col + e] = make_double2(0, 0);
  } else {
    for (int i = tid; i < D; i += LC_THREADS) {
      P[i] = psi_st[off + i];
      U[i] = mu_st[off + i];
    }
  }
  auto ent_of = [&](const LcGate& G) { return G.s1 ? NN : dd; };
  LcPos pos{n_hi - 1, R.r - 1, len - 1};   // gate 0
  LcGate gc = gate(pos), gp = gc, gpp = gc;
  lc_advance(pos, R.r, len);               // gate 1
  LcGate gn = ng > 1 ? gate(pos) : gc;
  lc_advance(pos, R.r, len);               // gate 2: gate g + 2 in interval g
  for (int e = tid; e < nn_of(gc); e += LC_THREADS) Gi[e] = gc.gi[e];
  lc_fibres<d>(gc, D, tab);
  // tables stored at the start of interval g (G_{g+1}^-1, G_g^dag), read from
  // memory during the interval before (every gate pointer here is a valid
  // table, so the reads are unconditional, with clamped indices)
  // (entries tid and tid + T of each table: named registers, not arrays, which
  // the compiler would index in scratch memory)
  const int e0 = tid, e1 = tid + LC_THREADS;
  auto clampi = [](int e, int n) { return e < n ? e : n - 1; };
  double2 ri0 = gn.gi[clampi(e0, nn_of(gn))], ri1 = gn.gi[clampi(e1, nn_of(gn))];
  double2 ra0 = gc.ga[clampi(e0, nn_of(gc))], ra1 = gc.ga[clampi(e1, nn_of(gc))];
  __syncthreads();
  for (int g = 0; g <= ng + 1; ++g) {
    const int cur = g & 1, nxt = cur ^ 1;
    const bool hasC = g < ng, hasP = g >= 1 && g <= ng, hasPP = g >= 2;
    const bool hasN = g + 1 < ng, hasN2 = g + 2 < ng;
    const LcGate gn2 = hasN2 ? gate(pos) : gn;
    lc_advance(pos, R.r, len);
    // work items of this interval, each kind from a wave boundary on, so that
    // no wave mixes the code of two gates: psi's (A), mu's (A), B's, C's
    const int nAp = hasC ? D / d : (g == ng ? D : 0);
    const int nAm = hasP ? D / d : (g == 0 ? D : 0);
    const int nB = hasP ? ent_of(gp) * chunks_of(gp) : 0;
    const int oAm = (nAp + 63) & ~63, oB = oAm + ((nAm + 63) & ~63), oF = oB + ((nB + 63) & ~63);
    const int wB = lc_first(oB), eF = lc_first(oF);
    // D: the tables read during the interval before into their free slots
    // (the slots of gates g - 1 and g - 2, which the last interval read);
    // then the old sums this thread adds to, and the tables of the next
    // interval into the same registers (no register copies, which would wait
    // for the reads in flight)
    if (hasN) {
      if (e0 < nn_of(gn)) Gi[((g + 1) & 1) * NN + e0] = ri0;
      if (e1 < nn_of(gn)) Gi[((g + 1) & 1) * NN + e1] = ri1;
    }
    if (hasC) {
      if (e0 < nn_of(gc)) Ga[(g & 1) * NN + e0] = ra0;
      if (e1 < nn_of(gc)) Ga[(g & 1) * NN + e1] = ra1;
    }
    double2 old[2];
    const bool addP = hasP && gp.s1 != 0 && chunks_of(gp) == 1;
    const bool addPP = hasPP && gpp.s1 != 0 && chunks_of(gpp) > 1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int eb = wB + k * LC_THREADS;
      old[k] = addP && eb < NN ? gp.m[eb]
                               : (addPP && k == 0 && eF < NN ? gpp.m[eF] : make_double2(0, 0));
    }
    ri0 = gn2.gi[clampi(e0, nn_of(gn2))];
    ri1 = gn2.gi[clampi(e1, nn_of(gn2))];
    ra0 = gn.ga[clampi(e0, nn_of(gn))];
    ra1 = gn.ga[clampi(e1, nn_of(gn))];
    const double2 *Pc = P + cur * D, *Uc = U + cur * D;
    double2 *Pn = P + nxt * D, *Un = U + nxt * D;
    const int* tc = tab + (g % 3) * nft;          // gate g
    const int* tp = tab + ((g + 2) % 3) * nft;    // gate g - 1
    // A: psi' = G_g^-1 psi, then mu' = G_{g-1}^dag mu, through one copy of the
    // code (a second inlined copy was scheduled with a wait after every LDS
    // read of its gate rows)
#pragma unroll 1
    for (int v = 0; v < 2; ++v) {
      const bool isp = v == 0;
      const LcGate G = isp ? gc : gp;
      const double2* in = isp ? Pc : Uc;
      double2* out = isp ? Pn : Un;
      const double2* Gt = isp ? Gi + (g & 1) * NN : Ga + ((g + 1) & 1) * NN;   // (g-1) & 1
      const int w0 = isp ? tid : lc_first(oAm);
      if (isp ? hasC : hasP)
        lc_split_apply<d>(in, out, G, Gt, isp ? tc : tp, D, w0);
      else if (isp ? g == ng : g == 0)
        lc_copy(in, out, D, w0);
    }
    // B
    if (hasP) {
      double2* sp = scr + ((g - 1) & 1) * LC_THREADS;
      if (gp.s1 == 0)
        lc_split_reduce_n<d, d>(Uc, Pc, gp, tp, nf1, ch1, sp, old, wB);
      else
        lc_split_reduce_n<d, dd>(Uc, Pc, gp, tp, nf2, ch2, sp, old, wB);
    }
    // C
    if (hasPP) lc_split_fold<d>(gpp, chunks_of(gpp), scr + (g & 1) * LC_THREADS, old, eF);
    if (g == ng + 1) {
      for (int i = tid; i < D; i += LC_THREADS) {
        psi_st[off + i] = Pc[i];
        mu_st[off + i] = Uc[i];
      }
    }
    if (hasN) lc_fibres<d>(gn, D, tab + ((g + 1) % 3) * nft);
    __syncthreads();
    gpp = gp;
    gp = gc;
    gc = gn;
    gn = gn2;
  }
}

// Tr(K P) for n x n K (row stride ks) and P given by a functor p(row, col)
template <typename F>
__device__ __forceinline__ double2 trace_kp(const double2* K, int ks, int n, F p) {
  double re = 0.0, im = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const double2 k = K[a * ks + b], v = p(b, a);
      re += k.x * v.x - k.y * v.y;
      im += k.x * v.y + k.y * v.x;
    }
  return make_double2(re, im);
}

// Single-mode gates of steps [n_lo, n_lo + nsteps): block b = (nl r + j) M + m.
// The sum of M over the nvis visits and the columns (visit-major, a fixed
// order), K = L(X, M^T) with X = -i a tau h(t), then the traces
// z = (Tr K n, Tr K phi, Tr K dh/dEJ, Tr K dh/dEC, Tr K dh/dEL) into
// z[(step r + j) M + m][5].
__global__ void __launch_bounds__(64)
lc_single_kernel(TrGen G, int n_lo, int S, int nvis, const double* __restrict__ eps,
                 const double2* __restrict__ ops, const double* __restrict__ par,
                 const double* __restrict__ deps, const double2* __restrict__ dops,
                 const double2* __restrict__ Ms, double2* __restrict__ z) {
  extern __shared__ double2 sh[];
  const int d = G.d, dd = d * d, n2 = 2 * d, nn = n2 * n2;
  double2 *X = sh, *E = sh + nn, *T = sh + 2 * nn, *W = sh + 3 * nn;
  double* ck = reinterpret_cast<double*>(sh + 4 * nn);
  const int b = blockIdx.x, m = b % G.M, q = b / G.M, j = q % G.r, nl = q / G.r;
  const long step = n_lo + nl;
  const double t = step * G.dt + G.mid[j];
  for (int k = threadIdx.x; k < G.ndrives; k += blockDim.x) {
    const TrDrive Rd = G.dr[k];
    double v = 0.0;
    if (Rd.mode == m) {
      for (int i = 0; i < Rd.npar; ++i)
        v += par[Rd.par0 + i] * envelope_basis(Rd.env, i, Rd.npar, step, G.N, t, G.T, Rd.sigma);
      v *= cos(wrap_2pi(Rd.omega * t + Rd.phase));
    }
    ck[k] = v;
  }
  __syncthreads();
  const double2 w = gate_factor(G, j, 1.0);
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
    const int row = idx / n2, cc = idx % n2;
    double2 v = make_double2(0.0, 0.0);
    if ((row < d) == (cc < d)) {              // the diagonal blocks: X
      const int r0 = row % d, c0 = cc % d;
      double2 h = make_double2(r0 == c0 ? eps[m * d + r0] : 0.0, 0.0);
      for (int k = 0; k < G.ndrives; ++k) {
        if (G.dr[k].mode != m) continue;
        const double2 o = ops[(size_t)(m * 2 + G.dr[k].op) * dd + r0 * d + c0];
        h.x += ck[k] * o.x;
        h.y += ck[k] * o.y;
      }
      v = cmul(w, h);
    } else if (row < d) {                     // upper right: M^T, summed over columns
      const int r0 = row, c0 = cc - d;
      const double2* src = Ms + (((size_t)nl * G.r + j) * G.M + m) * nvis * S * dd + (size_t)c0 * d + r0;
      double re = 0.0, im = 0.0;
      for (int c = 0; c < nvis * S; ++c) {
        re += src[(size_t)c * dd].x;
        im += src[(size_t)c * dd].y;
      }
      v = make_double2(re, im);
    }
    X[idx] = v;
  }
  __syncthreads();
  expm_taylor(n2, X, E, T, W);
  if (threadIdx.x < 5) {
    const double2* Kp = E + d;   // rows 0..d-1, columns d..2d-1
    const int k5 = threadIdx.x;
    double2 out;
    if (k5 < 2) {
      const double2* O = ops + (size_t)(m * 2 + k5) * dd;
      out = trace_kp(Kp, n2, d, [&](int r0, int c0) { return O[r0 * d + c0]; });
    } else {
      const int th = k5 - 2;
      out = trace_kp(Kp, n2, d, [&](int r0, int c0) {
        double2 v = make_double2(r0 == c0 ? deps[(m * 3 + th) * d + r0] : 0.0, 0.0);
        for (int k = 0; k < G.ndrives; ++k) {
          if (G.dr[k].mode != m) continue;
          const double2 o = dops[((size_t)(m * 3 + th) * 2 + G.dr[k].op) * dd + r0 * d + c0];
          v.x += ck[k] * o.x;
          v.y += ck[k] * o.y;
        }
        return v;
      });
    }
    z[((size_t)step * G.r + j) * G.M * 5 + (size_t)m * 5 + k5] = out;
  }
}

// Pair gates: block b = j E + e.  The sum of M over columns (steps and passes
// already summed per column), K = L(X, M^T), X = -i a tau g A (x) B, and the
// traces (Tr K A(x)B, Tr K dA(x)B for EJ, EC, EL of mode i, Tr K A(x)dB for
// those of mode j) into zp[b][7].
__global__ void __launch_bounds__(256)
lc_pair_kernel(TrGen G, int S, const double2* __restrict__ ops, const double2* __restrict__ dops,
               const double2* __restrict__ Mp, double2* __restrict__ zp) {
  extern __shared__ double2 sh[];
  const int d = G.d, dd = d * d, n = dd, n2 = 2 * n, nn = n2 * n2;
  double2 *X = sh, *E = sh + nn, *T = sh + 2 * nn, *W = sh + 3 * nn;
  const int b = blockIdx.x, j = b / G.E, e = b % G.E;
  const double2 w = gate_factor(G, j, G.g[e]);
  const double2* A = ops + (size_t)(G.ci[e] * 2 + G.coi[e]) * dd;
  const double2* B = ops + (size_t)(G.cj[e] * 2 + G.coj[e]) * dd;
  const size_t np_col = (size_t)G.r * G.E * n * n;
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
    const int row = idx / n2, cc = idx % n2;
    double2 v = make_double2(0.0, 0.0);
    if ((row < n) == (cc < n)) {
      const int r0 = row % n, c0 = cc % n;
      v = cmul(w, cmul(A[(r0 / d) * d + c0 / d], B[(r0 % d) * d + c0 % d]));
    } else if (row < n) {
      const int r0 = row, c0 = cc - n;
      const double2* src = Mp + (size_t)b * n * n + (size_t)c0 * n + r0;
      double re = 0.0, im = 0.0;
      for (int c = 0; c < S; ++c) {
        re += src[(size_t)c * np_col].x;
        im += src[(size_t)c * np_col].y;
      }
      v = make_double2(re, im);
    }
    X[idx] = v;
  }
  __syncthreads();
  expm_taylor(n2, X, E, T, W);
  if (threadIdx.x < 7) {
    const double2* Kp = E + n;
    const int k7 = threadIdx.x;
    const double2* dA = k7 >= 1 && k7 <= 3 ? dops + ((size_t)(G.ci[e] * 3 + (k7 - 1)) * 2 + G.coi[e]) * dd : A;
    const double2* dB = k7 >= 4 ? dops + ((size_t)(G.cj[e] * 3 + (k7 - 4)) * 2 + G.coj[e]) * dd : B;
    const double2 out = trace_kp(Kp, n2, n, [&](int r0, int c0) {
      return cmul(dA[(r0 / d) * d + c0 / d], dB[(r0 % d) * d + c0 % d]);
    });
    zp[(size_t)b * 7 + k7] = out;
  }
}

// LDS of the split walk: two buffers each of psi and mu, two slots each of
// inverse and adjoint gates (d^4 entries), two slots of partial sums
inline size_t lc_split_lds(int64_t D, int d) {
  const int64_t nn = (int64_t)d * d * d * d;
  return (size_t)(4 * D + 4 * nn + 2 * LC_THREADS) * sizeof(double2) +
         (size_t)3 * (D / d) * sizeof(int);
}
inline bool lc_split_fits(int64_t D, int d) { return lc_split_lds(D, d) <= (size_t)TR_MAXLDS; }

template <int d>
hipError_t run_lc_walk(const LcRun& R, int n_hi, int n_lo, int first, const double2* psiT,
                       const double2* lamT, double2* psi_st, double2* mu_st, const double2* sgi,
                       const double2* sga, const double2* pgi, const double2* pga, double2* Ms,
                       double2* Mp, hipStream_t st) {
  if (lc_split_fits(R.D, d)) {
    const size_t sh = lc_split_lds(R.D, d);
    hipError_t e = hipFuncSetAttribute((const void*)lc_walk_split_kernel<d>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lc_walk_split_kernel<d>, dim3(R.S), dim3(LC_THREADS), sh, st, R, n_hi, n_lo,
                       first, psiT, lamT, psi_st, mu_st, sgi, sga, pgi, pga, Ms, Mp);
    return hipGetLastError();
  }
  const size_t sh = ((size_t)2 * R.D + TR_THREADS) * sizeof(double2);
  hipError_t e = hipFuncSetAttribute((const void*)lc_walk_kernel<d>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lc_walk_kernel<d>, dim3(R.S), dim3(TR_THREADS), sh, st, R, n_hi, n_lo, first,
                     psiT, lamT, psi_st, mu_st, sgi, sga, pgi, pga, Ms, Mp);
  return hipGetLastError();
}

struct LcLayout {
  TrLayout F;              // the forward's layout (its tables are reused)
  size_t psiT, psi_st, mu_st, sgi, sga, pgi, pga, ms, mp, z, zp, deps, dops, total;
  int chunk;
};

LcLayout lc_layout(const scp_system* sys, int order, int S) {
  LcLayout L{};
  L.F = tr_layout(sys, order);
  const size_t d = sys->d, dd = d * d, M = sys->n_modes, E = std::max<size_t>(1, sys->coup.size());
  const size_t N = sys->n_steps, r = L.F.r, D = sys->D;
  L.chunk = (int)std::min<size_t>(N, LC_CHUNK);
  size_t o = L.F.total;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.psiT = take((size_t)S * D * sizeof(double2));
  L.psi_st = take((size_t)S * D * sizeof(double2));
  L.mu_st = take((size_t)S * D * sizeof(double2));
  L.sgi = take(N * r * M * dd * sizeof(double2));
  L.sga = take(N * r * M * dd * sizeof(double2));
  L.pgi = take(r * E * dd * dd * sizeof(double2));
  L.pga = take(r * E * dd * dd * sizeof(double2));
  L.ms = take((size_t)L.chunk * r * M * (L.F.H == 2 ? 2 : 1) * S * dd * sizeof(double2));
  L.mp = take((size_t)S * r * E * dd * dd * sizeof(double2));
  L.z = take(N * r * M * 5 * sizeof(double2));
  L.zp = take(r * E * 7 * sizeof(double2));
  L.deps = take(M * 3 * d * sizeof(double));
  L.dops = take(M * 3 * 2 * dd * sizeof(double2));
  L.total = o;
  return L;
}

}  // namespace

scp_status trotter_adjoint_check(const scp_system* sys, int order) {
  scp_status chk = trotter_check(sys, order);
  if (chk != SCP_OK) return chk;
  if (((int64_t)2 * sys->D + TR_THREADS) * (int64_t)sizeof(double2) > TR_MAXLDS)
    return fail(SCP_EINVAL, "the product-formula adjoint keeps a column and its costate in LDS: "
                            "16 (2 D + 512) bytes must be <= 160 KiB (D <= 4864)");
  return SCP_OK;
}

size_t trotter_adjoint_workspace_bytes(const scp_system* sys, int order, int S) {
  return lc_layout(sys, order, S).total;
}

// psi0 given: the forward runs first (its final state into the workspace);
// else psiT_in is that final state and only the gate tables are built
static scp_status lc_adjoint(scp_system* sys, int order, int S, void* ws, const double2* psi0,
                             const double2* psiT_in, const double2* cot, double* grad,
                             hipStream_t st) {
  scp_status chk = trotter_adjoint_check(sys, order);
  if (chk != SCP_OK) return chk;
  const LcLayout Y = lc_layout(sys, order, S);
  const TrLayout& W = Y.F;
  const int d = sys->d, dd = d * d, M = sys->n_modes, E = (int)sys->coup.size(), N = sys->n_steps;
  char* base = static_cast<char*>(ws);
  // the forward: only its final state is kept (its gate tables are reused)
  const double2* psiT = psi0 ? reinterpret_cast<double2*>(base + Y.psiT) : psiT_in;
  scp_status s = launch_trotter(sys, order, S, ws, psi0, const_cast<double2*>(psiT), st);
  if (s != SCP_OK) return s;
  // operator derivatives of every mode (FP64)
  std::vector<double> hdeps((size_t)M * 3 * d);
  std::vector<double2> hdops((size_t)M * 3 * 2 * dd);
  for (int m = 0; m < M; ++m)
    for (int th = 0; th < 3; ++th) {
      for (int a = 0; a < d; ++a) hdeps[((size_t)m * 3 + th) * d + a] = sys->modes[m].deps[th][a];
      for (int op = 0; op < 2; ++op)
        for (int i = 0; i < dd; ++i) {
          const cplx v = sys->modes[m].dops[th][op][i];
          hdops[(((size_t)m * 3 + th) * 2 + op) * dd + i] = make_double2(v.real(), v.imag());
        }
    }
  std::vector<double> ipar(std::max<size_t>(1, W.npar));
  TrGen G = make_gen(sys, order, W, ipar.data());
  HIPCHK(hipMemcpyAsync(base + Y.deps, hdeps.data(), hdeps.size() * sizeof(double),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(base + Y.dops, hdops.data(), hdops.size() * sizeof(double2),
                        hipMemcpyHostToDevice, st));
  const double* deps = reinterpret_cast<const double*>(base + W.eps);
  const double2* dops = reinterpret_cast<const double2*>(base + W.ops);
  const double* dpar = reinterpret_cast<const double*>(base + W.par);
  const double2* pg = reinterpret_cast<const double2*>(base + W.pg);
  const double2* sg = reinterpret_cast<const double2*>(base + W.sg);
  double2* sgi = reinterpret_cast<double2*>(base + Y.sgi);
  double2* sga = reinterpret_cast<double2*>(base + Y.sga);
  double2* pgi = reinterpret_cast<double2*>(base + Y.pgi);
  double2* pga = reinterpret_cast<double2*>(base + Y.pga);
  // inverse gates exp(-X): the same generators with the piece coefficients negated
  TrGen Gi = G;
  for (int j = 0; j < W.r; ++j) {
    Gi.a_re[j] = -G.a_re[j];
    Gi.a_im[j] = -G.a_im[j];
  }
  if (E > 0) {
    hipLaunchKernelGGL(tr_pair_gate_kernel, dim3(W.r * E), dim3(256), 4 * dd * dd * sizeof(double2),
                       st, Gi, dops, pgi);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(lc_adjoint_table_kernel, dim3(std::max(1, W.r * E)), dim3(256), 0, st, pg, pga,
                       dd, (size_t)W.r * E);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(tr_single_gate_kernel, dim3((unsigned)((size_t)N * W.r * M)), dim3(64),
                     4 * dd * sizeof(double2) + TR_MAXDRV * sizeof(double), st, Gi, deps, dops, dpar,
                     sgi);
  HIPCHK(hipGetLastError());
  {
    const size_t count = (size_t)N * W.r * M;
    const int blocks = (int)std::min<size_t>((count * dd + 255) / 256, 65535);
    hipLaunchKernelGGL(lc_adjoint_table_kernel, dim3(blocks), dim3(256), 0, st, sg, sga, d, count);
    HIPCHK(hipGetLastError());
  }
  LcRun R{};
  R.M = M;
  R.E = E;
  R.N = N;
  R.r = W.r;
  R.H = W.H;
  R.D = (int)sys->D;
  R.S = S;
  {
    int sd = 1;
    for (int m = M - 1; m >= 0; --m) {
      R.stride[m] = sd;
      sd *= d;
    }
  }
  for (int e = 0; e < E; ++e) {
    R.ci[e] = sys->coup[e].i;
    R.cj[e] = sys->coup[e].j;
  }
  const double twopi = 6.283185307179586476925286766559;
  for (int m = 0; m < M; ++m)
    for (int a = 0; a < d; ++a) R.fT[m][a] = std::remainder(sys->modes[m].frame[a] * N * sys->h, twopi);
  double2* psi_st = reinterpret_cast<double2*>(base + Y.psi_st);
  double2* mu_st = reinterpret_cast<double2*>(base + Y.mu_st);
  double2* Ms = reinterpret_cast<double2*>(base + Y.ms);
  double2* Mp = reinterpret_cast<double2*>(base + Y.mp);
  double2* z = reinterpret_cast<double2*>(base + Y.z);
  double2* zp = reinterpret_cast<double2*>(base + Y.zp);
  const double* ddeps = reinterpret_cast<const double*>(base + Y.deps);
  const double2* ddops = reinterpret_cast<const double2*>(base + Y.dops);
  // the split walk stores each visit of a single-mode gate in its own slot,
  // the in-place walk adds the visits of a step into one
  const int nvis = lc_split_fits(R.D, d) && W.H == 2 ? 2 : 1;
  for (int n_hi = N; n_hi > 0; n_hi -= Y.chunk) {
    const int n_lo = std::max(0, n_hi - Y.chunk);
    const int first = n_hi == N ? 1 : 0;
    hipError_t e;
    switch (d) {
      case 2: e = run_lc_walk<2>(R, n_hi, n_lo, first, psiT, cot, psi_st, mu_st, sgi, sga, pgi, pga, Ms, Mp, st); break;
      case 3: e = run_lc_walk<3>(R, n_hi, n_lo, first, psiT, cot, psi_st, mu_st, sgi, sga, pgi, pga, Ms, Mp, st); break;
      case 4: e = run_lc_walk<4>(R, n_hi, n_lo, first, psiT, cot, psi_st, mu_st, sgi, sga, pgi, pga, Ms, Mp, st); break;
      default: e = run_lc_walk<5>(R, n_hi, n_lo, first, psiT, cot, psi_st, mu_st, sgi, sga, pgi, pga, Ms, Mp, st); break;
    }
    HIPCHK(e);
    const int nb = (n_hi - n_lo) * W.r * M;
    hipLaunchKernelGGL(lc_single_kernel, dim3(nb), dim3(64),
                       4 * 4 * dd * sizeof(double2) + TR_MAXDRV * sizeof(double), st, G, n_lo, S,
                       nvis, deps,
                       dops, dpar, ddeps, ddops, Ms, z);
    HIPCHK(hipGetLastError());
  }
  if (E > 0) {
    const size_t sh = 4 * (size_t)(2 * dd) * (2 * dd) * sizeof(double2);
    HIPCHK(hipFuncSetAttribute((const void*)lc_pair_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sh));
    hipLaunchKernelGGL(lc_pair_kernel, dim3(W.r * E), dim3(256), sh, st, G, S, dops, ddops, Mp, zp);
    HIPCHK(hipGetLastError());
  }
  std::vector<double2> hz((size_t)N * W.r * M * 5), hzp((size_t)std::max(1, W.r * E) * 7);
  HIPCHK(hipMemcpyAsync(hz.data(), z, hz.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
  if (E > 0)
    HIPCHK(hipMemcpyAsync(hzp.data(), zp, (size_t)W.r * E * 7 * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // dL/dtheta = sum 2 Re(w_j Tr(K dh/dtheta)), w_j = -i a_j tau (FP64, fixed order)
  const int npulse = sys->n_pulse;
  std::vector<double> g((size_t)sys->n_params, 0.0);
  auto re2 = [](cplx w, double2 v) { return 2.0 * (w * cplx(v.x, v.y)).real(); };
  for (int n = 0; n < N; ++n)
    for (int j = 0; j < W.r; ++j) {
      const cplx wj = cplx(0.0, -1.0) * cplx(G.a_re[j], G.a_im[j]) * G.tau;
      const double t = n * G.dt + G.mid[j];
      const double2* zz = hz.data() + ((size_t)n * W.r + j) * M * 5;
      int p0 = 0;
      for (int k = 0; k < (int)sys->drives.size(); ++k) {
        const Drive& Rd = sys->drives[k];
        const double cr = std::cos(Rd.omega * t + Rd.phase);
        const double2 zo = zz[Rd.mode * 5 + Rd.op];
        for (int p = 0; p < (int)Rd.par.size(); ++p) {
          const double b = envelope_basis(Rd.env, p, (int)Rd.par.size(), n, N, t, sys->T, Rd.sigma);
          g[p0 + p] += re2(wj * (b * cr), zo);
        }
        p0 += (int)Rd.par.size();
      }
      for (int m = 0; m < M; ++m)
        for (int th = 0; th < 3; ++th) g[npulse + 3 * m + th] += re2(wj, zz[m * 5 + 2 + th]);
    }
  for (int j = 0; j < W.r; ++j) {
    const cplx wj = cplx(0.0, -1.0) * cplx(G.a_re[j], G.a_im[j]) * G.tau;
    for (int e = 0; e < E; ++e) {
      const Coupling& c = sys->coup[e];
      const double2* zz = hzp.data() + ((size_t)j * E + e) * 7;
      g[npulse + 3 * M + e] += re2(wj, zz[0]);
      for (int th = 0; th < 3; ++th) {
        g[npulse + 3 * c.i + th] += re2(wj * c.g, zz[1 + th]);
        g[npulse + 3 * c.j + th] += re2(wj * c.g, zz[4 + th]);
      }
    }
  }
  bool finite = true;
  for (int i = 0; i < sys->n_params; ++i) {
    grad[i] = g[i];
    finite &= std::isfinite(g[i]);
  }
  if (!finite) return fail(SCP_ENONFINITE, "gradient is not finite");
  return SCP_OK;
}

scp_status launch_trotter_adjoint(scp_system* sys, int order, int S, void* ws, const double2* psi0,
                                  const double2* cot, double* grad, hipStream_t st) {
  return lc_adjoint(sys, order, S, ws, psi0, nullptr, cot, grad, st);
}

scp_status launch_trotter_adjoint_final(scp_system* sys, int order, int S, void* ws,
                                        const double2* psiT, const double2* cot, double* grad,
                                        hipStream_t st) {
  return lc_adjoint(sys, order, S, ws, nullptr, psiT, cot, grad, st);
}

}  // namespace scp
