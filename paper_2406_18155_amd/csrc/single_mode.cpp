// Host-side FP64 single-mode builders and dressed truncation.
//
// Transmon (charge basis |n| <= ncut): H = 4 EC (n - ng)^2 - EJ cos(phi),
// cos(phi) hopping n -> n +- 1 with amplitude 1/2; operator n = diag(n - ng).
// Fluxonium (Sec. 3.1, single fluxonium Hamiltonian; external flux taken in
// the Josephson term): H = sqrt(8 EC EL) (k + 1/2) on the harmonic-oscillator
// states k < K, minus EJ cos(phi - phiext) from the exact displacement
// operator elements <m| exp(i phi) |n> (generalised Laguerre form);
// phi = phi_osc (a + a^dag)/sqrt2, n = i (a^dag - a)/(sqrt2 phi_osc),
// phi_osc = (8 EC / EL)^(1/4).
// Dressed truncation (App. D step 1): lowest d eigenvectors, energies
// referenced to the ground level, operators V_d^T O V_d; each eigenvector's
// largest-magnitude entry made positive (ties within 1e-12 relative to the
// lowest basis index).  Parameter derivatives by first-order perturbation
// theory over the full basis.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace scp {

namespace {
constexpr double kSignTie = 1e-12;
constexpr double kDegenerate = 1e-9;

// L_n^{(k)}(x) for n = 0..nmax-1 (three-term recurrence in n).
void laguerre_row(int k, double x, int nmax, std::vector<double>& out) {
  out.assign(nmax, 0.0);
  if (nmax == 0) return;
  out[0] = 1.0;
  if (nmax == 1) return;
  out[1] = 1.0 + k - x;
  for (int n = 1; n + 1 < nmax; ++n)
    out[n + 1] = ((2.0 * n + 1.0 + k - x) * out[n] - (n + k) * out[n - 1]) / (n + 1.0);
}

// <m| exp(alpha a^dag - conj(alpha) a) |n> for alpha = i r (r real), m < rows, n < cols.
// For this alpha, -conj(alpha) = alpha, so the element is
// sqrt(min!/max!) alpha^|m-n| e^{-r^2/2} L_min^{(|m-n|)}(r^2).
std::vector<cplx> displacement(double r, int rows, int cols) {
  std::vector<cplx> D((size_t)rows * cols);
  const double x = r * r;
  const int nmax = std::max(rows, cols);
  std::vector<std::vector<double>> lag(nmax + 1);
  for (int k = 0; k <= nmax; ++k) laguerre_row(k, x, nmax, lag[k]);
  const cplx ipow[4] = {cplx(1, 0), cplx(0, 1), cplx(-1, 0), cplx(0, -1)};
  for (int m = 0; m < rows; ++m)
    for (int n = 0; n < cols; ++n) {
      int lo = std::min(m, n), hi = std::max(m, n), k = hi - lo;
      double logmag = 0.5 * (std::lgamma(lo + 1.0) - std::lgamma(hi + 1.0)) - 0.5 * x;
      double mag = (k > 0 ? std::pow(r, k) : 1.0) * std::exp(logmag) * lag[k][lo];
      D[(size_t)m * cols + n] = mag * ipow[k & 3];
    }
  return D;
}
}  // namespace

void build_transmon(ModeData& m) {
  const int K = m.K, ncut = K / 2;
  m.H.assign((size_t)K * K, 0.0);
  for (int p = 0; p < 3; ++p) m.dH[p].assign((size_t)K * K, 0.0);
  m.opB[0].assign((size_t)K * K, 0.0);
  m.opB[1].assign((size_t)K * K, 0.0);
  for (int p = 0; p < 3; ++p)
    for (int o = 0; o < 2; ++o) m.dopB[p][o].assign((size_t)K * K, 0.0);
  for (int i = 0; i < K; ++i) {
    double n = (double)(i - ncut) - m.ng;
    m.H[(size_t)i * K + i] = 4.0 * m.EC * n * n;
    m.dH[1][(size_t)i * K + i] = 4.0 * n * n;
    m.opB[0][(size_t)i * K + i] = n;
    if (i + 1 < K) {
      m.H[(size_t)i * K + i + 1] = m.H[(size_t)(i + 1) * K + i] = -0.5 * m.EJ;
      m.dH[0][(size_t)i * K + i + 1] = m.dH[0][(size_t)(i + 1) * K + i] = -0.5;
    }
  }
  m.has_phi = false;
}

void build_fluxonium(ModeData& m) {
  const int K = m.K;
  const double phi_osc = std::pow(8.0 * m.EC / m.EL, 0.25);
  const double wp = std::sqrt(8.0 * m.EC * m.EL);
  const double s2 = std::sqrt(2.0);
  std::vector<cplx> Dext = displacement(phi_osc / s2, K + 1, K);   // one extra row
  const cplx eph = std::exp(cplx(0.0, -m.phiext));
  std::vector<double> C((size_t)K * K), dC((size_t)K * K);
  // dD/dphi_osc = (i/sqrt2) X D with X = a + a^dag (needs row K of D)
  for (int r = 0; r < K; ++r)
    for (int c = 0; c < K; ++c) {
      cplx Drc = Dext[(size_t)r * K + c], Dcr = Dext[(size_t)c * K + r];
      C[(size_t)r * K + c] = (0.5 * (eph * Drc + std::conj(eph) * std::conj(Dcr))).real();
    }
  auto XD = [&](int r, int c) {   // (X D)_{rc}
    cplx v = 0;
    v += std::sqrt((double)(r + 1)) * Dext[(size_t)(r + 1) * K + c];
    if (r > 0) v += std::sqrt((double)r) * Dext[(size_t)(r - 1) * K + c];
    return v;
  };
  for (int r = 0; r < K; ++r)
    for (int c = 0; c < K; ++c) {
      cplx dDrc = cplx(0, 1.0 / s2) * XD(r, c);
      cplx dDcr = cplx(0, 1.0 / s2) * XD(c, r);
      dC[(size_t)r * K + c] = (0.5 * (eph * dDrc + std::conj(eph) * std::conj(dDcr))).real();
    }
  const double dphi[3] = {0.0, phi_osc / (4.0 * m.EC), -phi_osc / (4.0 * m.EL)};
  const double dwp[3] = {0.0, wp / (2.0 * m.EC), wp / (2.0 * m.EL)};
  m.H.assign((size_t)K * K, 0.0);
  for (int p = 0; p < 3; ++p) m.dH[p].assign((size_t)K * K, 0.0);
  for (int r = 0; r < K; ++r)
    for (int c = 0; c < K; ++c) {
      size_t ix = (size_t)r * K + c;
      double diag = (r == c) ? (r + 0.5) : 0.0;
      m.H[ix] = wp * diag - m.EJ * C[ix];
      for (int p = 0; p < 3; ++p) m.dH[p][ix] = dwp[p] * diag - m.EJ * dC[ix] * dphi[p];
      m.dH[0][ix] -= C[ix];
    }
  m.opB[0].assign((size_t)K * K, 0.0);
  m.opB[1].assign((size_t)K * K, 0.0);
  for (int r = 0; r + 1 < K; ++r) {
    double s = std::sqrt((double)(r + 1));          // a_{r, r+1}
    // phi = phi_osc/sqrt2 (a + a^dag)
    m.opB[1][(size_t)r * K + r + 1] = m.opB[1][(size_t)(r + 1) * K + r] = phi_osc / s2 * s;
    // n = i/(sqrt2 phi_osc) (a^dag - a): (a^dag)_{r+1, r} = s, a_{r, r+1} = s
    m.opB[0][(size_t)(r + 1) * K + r] = cplx(0, 1.0 / (s2 * phi_osc)) * s;
    m.opB[0][(size_t)r * K + r + 1] = cplx(0, -1.0 / (s2 * phi_osc)) * s;
  }
  for (int p = 0; p < 3; ++p) {
    m.dopB[p][0].resize((size_t)K * K);
    m.dopB[p][1].resize((size_t)K * K);
    for (size_t ix = 0; ix < (size_t)K * K; ++ix) {
      m.dopB[p][0][ix] = -m.opB[0][ix] / phi_osc * dphi[p];
      m.dopB[p][1][ix] = m.opB[1][ix] / phi_osc * dphi[p];
    }
  }
  m.has_phi = true;
}

scp_status finish_mode(ModeData& m) {
  const int K = m.K, d = m.d;
  // sort ascending (stable on index)
  std::vector<int> ord(K);
  for (int i = 0; i < K; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return m.w[a] < m.w[b]; });
  std::vector<double> w(K), V((size_t)K * K);
  for (int a = 0; a < K; ++a) {
    w[a] = m.w[ord[a]];
    for (int k = 0; k < K; ++k) V[(size_t)k * K + a] = m.V[(size_t)k * K + ord[a]];
  }
  // sign convention
  for (int a = 0; a < K; ++a) {
    double mx = 0;
    for (int k = 0; k < K; ++k) mx = std::max(mx, std::fabs(V[(size_t)k * K + a]));
    double thr = mx * (1.0 - kSignTie);
    for (int k = 0; k < K; ++k) {
      double v = V[(size_t)k * K + a];
      if (std::fabs(v) >= thr) {
        if (v < 0)
          for (int q = 0; q < K; ++q) V[(size_t)q * K + a] = -V[(size_t)q * K + a];
        break;
      }
    }
  }
  m.w = w;
  m.V = V;
  double scale = 1e-300;
  for (int a = 0; a <= std::min(d, K - 1); ++a) scale = std::max(scale, std::fabs(w[a]));
  for (int a = 0; a < d; ++a)
    for (int c = 0; c < K; ++c)
      if (c != a && std::fabs(w[a] - w[c]) < kDegenerate * scale)
        return fail(SCP_EDEGENERATE, "level " + std::to_string(a) + " degenerate with level " +
                                         std::to_string(c));
  for (int a = 0; a < d; ++a) m.eps[a] = w[a] - w[0];
  auto VT_op_V = [&](const std::vector<cplx>& op, const std::vector<double>& Vl,
                     const std::vector<double>& Vr, cplx* out) {
    // out[a*d+b] = sum_kl Vl[k, a] op[k, l] Vr[l, b]   (Vl, Vr: K x d column a at [k*d + a])
    std::vector<cplx> tmp((size_t)K * d);
    for (int k = 0; k < K; ++k)
      for (int b = 0; b < d; ++b) {
        cplx s = 0;
        for (int l = 0; l < K; ++l) s += op[(size_t)k * K + l] * Vr[(size_t)l * d + b];
        tmp[(size_t)k * d + b] = s;
      }
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        cplx s = 0;
        for (int k = 0; k < K; ++k) s += Vl[(size_t)k * d + a] * tmp[(size_t)k * d + b];
        out[a * d + b] = s;
      }
  };
  std::vector<double> Vd((size_t)K * d);
  for (int k = 0; k < K; ++k)
    for (int a = 0; a < d; ++a) Vd[(size_t)k * d + a] = V[(size_t)k * K + a];
  const int nops = m.has_phi ? 2 : 1;
  for (int o = 0; o < 2; ++o)
    for (int i = 0; i < d * d; ++i) m.ops[o][i] = 0;
  for (int o = 0; o < nops; ++o) VT_op_V(m.opB[o], Vd, Vd, m.ops[o]);
  // derivatives
  std::vector<double> M((size_t)K * K), tmp((size_t)K * K), dV((size_t)K * d);
  for (int p = 0; p < 3; ++p) {
    // M = V^T dH V
    for (int k = 0; k < K; ++k)
      for (int b = 0; b < K; ++b) {
        double s = 0;
        for (int l = 0; l < K; ++l) s += m.dH[p][(size_t)k * K + l] * V[(size_t)l * K + b];
        tmp[(size_t)k * K + b] = s;
      }
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b) {
        double s = 0;
        for (int k = 0; k < K; ++k) s += V[(size_t)k * K + a] * tmp[(size_t)k * K + b];
        M[(size_t)a * K + b] = s;
      }
    for (int a = 0; a < d; ++a) m.deps[p][a] = M[(size_t)a * K + a] - M[0];
    std::fill(dV.begin(), dV.end(), 0.0);
    for (int a = 0; a < d; ++a)
      for (int c = 0; c < K; ++c) {
        if (c == a) continue;
        double f = M[(size_t)c * K + a] / (w[a] - w[c]);
        for (int k = 0; k < K; ++k) dV[(size_t)k * d + a] += V[(size_t)k * K + c] * f;
      }
    for (int o = 0; o < 2; ++o)
      for (int i = 0; i < d * d; ++i) m.dops[p][o][i] = 0;
    for (int o = 0; o < nops; ++o) {
      cplx t1[SCP_MAX_TRUNC * SCP_MAX_TRUNC], t2[SCP_MAX_TRUNC * SCP_MAX_TRUNC],
          t3[SCP_MAX_TRUNC * SCP_MAX_TRUNC];
      VT_op_V(m.opB[o], dV, Vd, t1);
      VT_op_V(m.opB[o], Vd, dV, t2);
      VT_op_V(m.dopB[p][o], Vd, Vd, t3);
      for (int i = 0; i < d * d; ++i) m.dops[p][o][i] = t1[i] + t2[i] + t3[i];
    }
  }
  return SCP_OK;
}

}  // namespace scp
