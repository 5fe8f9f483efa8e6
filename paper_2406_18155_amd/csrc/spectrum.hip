// Static spectrum of the composite system: bare-labelled dressed energies
// and the static longitudinal (ZZ) coupling of a qubit pair (Sec. 3.2).
//
// H0 = sum_m diag(eps_m) + sum_e g_e A_i (x) B_j in the dressed single-mode
// bases (the generator's static part, drives excluded) is assembled on the
// host in FP64 and diagonalised by FP64 cyclic Jacobi on the device (one
// workgroup with the matrix in LDS for D <= 96, the device-memory variant for
// 96 < D <= 2048).  Every bare product state k is labelled with the
// eigenvector of largest overlap |<k|v>|^2 (ties to the lowest eigenvector
// index); zeta = E(0) + E(1_i 1_j) - E(1_i) - E(1_j) with every other mode in
// its ground state, and d zeta / d theta = sum of the signed <v| dH0 |v>
// (Hellmann-Feynman, non-degenerate levels) with dH0 from the single-mode
// derivatives of the dressed energies and operators.
#include <cmath>
#include <vector>

#include "internal.h"

namespace scp {

namespace {

constexpr int SPEC_MAXD_LDS = 96;   // the one-workgroup Jacobi kernel's largest matrix
constexpr int SPEC_MAXD = 2048;     // the device-memory Jacobi beyond it

struct DevBuf2 {
  void* p = nullptr;
  ~DevBuf2() {
    if (p) (void)hipFree(p);
  }
};

// digits of bare index k, mode 0 most significant
void digits(int64_t k, int n, int d, int* a) {
  for (int m = n - 1; m >= 0; --m) {
    a[m] = (int)(k % d);
    k /= d;
  }
}

// sum over the (i, j) entries of the two-body term c * A (on mode mi) (x) B
// (on mode mj), added into the real matrix M (D x D); returns false if an
// entry has an imaginary part
bool add_two_body(std::vector<double>& M, int64_t D, int n, int d, int mi, int mj,
                  const cplx* A, const cplx* B, double c) {
  std::vector<int> r(n), s(n);
  bool real = true;
  for (int64_t row = 0; row < D; ++row) {
    digits(row, n, d, r.data());
    for (int64_t col = 0; col < D; ++col) {
      digits(col, n, d, s.data());
      bool same = true;
      for (int m = 0; m < n; ++m)
        if (m != mi && m != mj && r[m] != s[m]) same = false;
      if (!same) continue;
      const cplx v = c * A[r[mi] * d + s[mi]] * B[r[mj] * d + s[mj]];
      if (v.imag() != 0.0) real = false;
      M[(size_t)row * D + col] += v.real();
    }
  }
  return real;
}

// one-body diagonal term diag(e) on mode m
void add_diag(std::vector<double>& M, int64_t D, int n, int d, int m, const double* e) {
  std::vector<int> r(n);
  for (int64_t k = 0; k < D; ++k) {
    digits(k, n, d, r.data());
    M[(size_t)k * D + k] += e[r[m]];
  }
}

// two-body term with the identity on the partner, d(A) (x) B etc.
const cplx* op_of(const scp_system* sys, int m, int op) { return sys->modes[m].ops[op]; }

scp_status spectrum(const scp_system* sys, hipStream_t st, std::vector<double>& w,
                    std::vector<double>& V) {
  const int n = sys->n_modes, d = sys->d;
  const int64_t D = sys->D;
  if (D > SPEC_MAXD) return fail(SCP_EINVAL, "static spectrum: D > 2048");
  std::vector<double> H((size_t)D * D, 0.0);
  for (int m = 0; m < n; ++m) add_diag(H, D, n, d, m, sys->modes[m].eps);
  for (const Coupling& c : sys->coup)
    if (!add_two_body(H, D, n, d, c.i, c.j, op_of(sys, c.i, c.op_i), op_of(sys, c.j, c.op_j), c.g))
      return fail(SCP_EINVAL, "static spectrum: the static Hamiltonian is not real");
  if (D > SPEC_MAXD_LDS) {
    // device-memory Jacobi on the matrix padded to even order
    const int Dp = (int)(D + (D & 1));
    std::vector<double> Hp((size_t)Dp * Dp, 0.0);
    for (int64_t r = 0; r < D; ++r)
      for (int64_t c = 0; c < D; ++c) Hp[(size_t)r * Dp + c] = H[(size_t)r * D + c];
    DevBuf2 bA, bV, bw;
    HIPCHK(hipMalloc(&bA.p, Hp.size() * sizeof(double)));
    HIPCHK(hipMalloc(&bV.p, Hp.size() * sizeof(double)));
    HIPCHK(hipMalloc(&bw.p, 16 * (size_t)Dp + 64));
    HIPCHK(hipMemcpyAsync(bA.p, Hp.data(), Hp.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(launch_jacobi_big((double*)bA.p, (double*)bV.p, Dp, bw.p, st));
    std::vector<double> Vp(Hp.size());
    HIPCHK(hipMemcpyAsync(Vp.data(), bV.p, Vp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(Hp.data(), bA.p, Hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    V.assign((size_t)D * D, 0.0);
    w.assign((size_t)D, 0.0);
    for (int64_t a = 0; a < D; ++a) {
      w[a] = Hp[(size_t)a * Dp + a];
      for (int64_t k = 0; k < D; ++k) V[(size_t)k * D + a] = Vp[(size_t)k * Dp + a];
    }
    for (double x : w)
      if (!std::isfinite(x)) return fail(SCP_ENONFINITE, "static spectrum is not finite");
    return SCP_OK;
  }
  DevBuf2 bA, bV, bw, bK, bo;
  const int K = (int)D;
  const int64_t off = 0;
  HIPCHK(hipMalloc(&bA.p, H.size() * sizeof(double)));
  HIPCHK(hipMalloc(&bV.p, H.size() * sizeof(double)));
  HIPCHK(hipMalloc(&bw.p, H.size() * sizeof(double)));
  HIPCHK(hipMalloc(&bK.p, sizeof(int)));
  HIPCHK(hipMalloc(&bo.p, sizeof(int64_t)));
  HIPCHK(hipMemcpyAsync(bA.p, H.data(), H.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bK.p, &K, sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bo.p, &off, sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(launch_jacobi((double*)bA.p, (double*)bV.p, (double*)bw.p, (const int*)bK.p,
                       (const int64_t*)bo.p, 1, st));
  V.assign((size_t)D * D, 0.0);
  std::vector<double> wall((size_t)D * D);
  HIPCHK(hipMemcpyAsync(V.data(), bV.p, V.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(wall.data(), bw.p, wall.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  w.assign(wall.begin(), wall.begin() + D);
  for (double x : w)
    if (!std::isfinite(x)) return fail(SCP_ENONFINITE, "static spectrum is not finite");
  return SCP_OK;
}

// eigenvector (column) of largest overlap with bare state k
int label(const std::vector<double>& V, int64_t D, int64_t k) {
  int best = 0;
  double bv = -1.0;
  for (int v = 0; v < (int)D; ++v) {
    const double x = V[(size_t)k * D + v] * V[(size_t)k * D + v];
    if (x > bv) {
      bv = x;
      best = v;
    }
  }
  return best;
}

int64_t bare(const scp_system* sys, const std::vector<int>& lv) {
  int64_t k = 0;
  for (int m = 0; m < sys->n_modes; ++m) k = k * sys->d + lv[m];
  return k;
}

}  // namespace

}  // namespace scp

using namespace scp;

extern "C" {

scp_status scp_eigenbasis_states(const scp_system* sys, int32_t n, const int64_t* labels,
                                 const double* target, double T, int32_t precision,
                                 void* psi0_out, void* phi_out, void* W_out, double* E_out,
                                 void* stream) {
  set_error("");
  if (!sys || !labels || !psi0_out || n < 1 || (precision != 0 && precision != 1))
    return fail(SCP_EINVAL, "bad argument");
  if (phi_out && !target) return fail(SCP_EINVAL, "phi_out needs the target");
  const int64_t D = sys->D;
  for (int j = 0; j < n; ++j)
    if (labels[j] < 0 || labels[j] >= D) return fail(SCP_EINVAL, "label out of range");
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> w, V;
  scp_status s = spectrum(sys, st, w, V);
  if (s != SCP_OK) return s;
  const int nm = sys->n_modes, d = sys->d;
  // H_f on the product basis
  std::vector<double> f((size_t)D, 0.0);
  {
    std::vector<int> a(nm);
    for (int64_t k = 0; k < D; ++k) {
      digits(k, nm, d, a.data());
      for (int m = 0; m < nm; ++m) f[k] += sys->modes[m].frame[a[m]];
    }
  }
  // dressed state of each label: the eigenvector of largest overlap, <k|v> > 0
  std::vector<cplx> Vc((size_t)D * n), Wc((size_t)D * n);
  std::vector<double> Ec(n);
  for (int j = 0; j < n; ++j) {
    const int v = label(V, D, labels[j]);
    const double sgn = V[(size_t)labels[j] * D + v] < 0.0 ? -1.0 : 1.0;
    Ec[j] = w[v];
    for (int64_t k = 0; k < D; ++k) {
      const double x = sgn * V[(size_t)k * D + v];
      Vc[(size_t)j * D + k] = x;
      Wc[(size_t)j * D + k] = std::polar(x, (f[k] - Ec[j]) * T);
    }
  }
  if (E_out)
    for (int j = 0; j < n; ++j) E_out[j] = Ec[j];
  if (precision == 0) {
    std::vector<float2> h((size_t)D * n);
    for (size_t i = 0; i < h.size(); ++i) h[i] = make_float2((float)Vc[i].real(), 0.f);
    HIPCHK(hipMemcpyAsync(psi0_out, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  } else {
    HIPCHK(hipMemcpyAsync(psi0_out, Vc.data(), Vc.size() * sizeof(cplx), hipMemcpyHostToDevice, st));
  }
  if (W_out)
    HIPCHK(hipMemcpyAsync(W_out, Wc.data(), Wc.size() * sizeof(cplx), hipMemcpyHostToDevice, st));
  std::vector<cplx> phi;
  if (phi_out) {
    // phi_j = sum_i T_ij w_i (target row-major, (re, im) pairs)
    phi.assign((size_t)D * n, 0.0);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const cplx t(target[2 * ((size_t)i * n + j)], target[2 * ((size_t)i * n + j) + 1]);
        for (int64_t k = 0; k < D; ++k) phi[(size_t)j * D + k] += t * Wc[(size_t)i * D + k];
      }
    HIPCHK(hipMemcpyAsync(phi_out, phi.data(), phi.size() * sizeof(cplx), hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return SCP_OK;
}

scp_status scp_energy_tensor(const scp_system* sys, double* E_out, void* stream) {
  set_error("");
  if (!sys || !E_out) return fail(SCP_EINVAL, "null argument");
  std::vector<double> w, V;
  scp_status s = spectrum(sys, (hipStream_t)stream, w, V);
  if (s != SCP_OK) return s;
  for (int64_t k = 0; k < sys->D; ++k) E_out[k] = w[label(V, sys->D, k)];
  return SCP_OK;
}

scp_status scp_static_zz(const scp_system* sys, int32_t qi, int32_t qj, double* zeta_out,
                         double* grad_out, void* stream) {
  set_error("");
  if (!sys || !zeta_out) return fail(SCP_EINVAL, "null argument");
  const int n = sys->n_modes, d = sys->d;
  if (qi < 0 || qj < 0 || qi >= n || qj >= n || qi == qj || d < 2)
    return fail(SCP_EINVAL, "static_zz: bad mode pair");
  std::vector<double> w, V;
  scp_status s = spectrum(sys, (hipStream_t)stream, w, V);
  if (s != SCP_OK) return s;
  const int64_t D = sys->D;
  std::vector<int> z(n, 0), s11 = z, s10 = z, s01 = z;
  s11[qi] = s11[qj] = 1;
  s10[qi] = 1;
  s01[qj] = 1;
  const int64_t ks[4] = {bare(sys, z), bare(sys, s11), bare(sys, s10), bare(sys, s01)};
  const double sg[4] = {1.0, 1.0, -1.0, -1.0};
  int vs[4];
  double zeta = 0.0;
  for (int t = 0; t < 4; ++t) {
    vs[t] = label(V, D, ks[t]);
    zeta += sg[t] * w[vs[t]];
  }
  *zeta_out = zeta;
  if (!grad_out) return SCP_OK;
  // signed sum over the four levels of <v| dH0 |v> for a real symmetric dH0
  auto expect = [&](const std::vector<double>& dH) {
    double acc = 0.0;
    for (int t = 0; t < 4; ++t) {
      double e = 0.0;
      for (int64_t a = 0; a < D; ++a) {
        double row = 0.0;
        for (int64_t b = 0; b < D; ++b) row += dH[(size_t)a * D + b] * V[(size_t)b * D + vs[t]];
        e += V[(size_t)a * D + vs[t]] * row;
      }
      acc += sg[t] * e;
    }
    return acc;
  };
  int idx = 0;
  for (size_t k = 0; k < sys->drives.size(); ++k)
    for (size_t p = 0; p < sys->drives[k].par.size(); ++p) grad_out[idx++] = 0.0;
  std::vector<double> dH((size_t)D * D);
  for (int m = 0; m < n; ++m) {
    const ModeData& md = sys->modes[m];
    for (int th = 0; th < 3; ++th) {
      std::fill(dH.begin(), dH.end(), 0.0);
      add_diag(dH, D, n, d, m, md.deps[th]);
      bool real = true;
      for (const Coupling& c : sys->coup) {
        if (c.i == m) real &= add_two_body(dH, D, n, d, c.i, c.j, md.dops[th][c.op_i],
                                           op_of(sys, c.j, c.op_j), c.g);
        if (c.j == m) real &= add_two_body(dH, D, n, d, c.i, c.j, op_of(sys, c.i, c.op_i),
                                           md.dops[th][c.op_j], c.g);
      }
      if (!real) return fail(SCP_EINVAL, "static spectrum: a derivative is not real");
      grad_out[idx++] = expect(dH);
    }
  }
  for (const Coupling& c : sys->coup) {
    std::fill(dH.begin(), dH.end(), 0.0);
    add_two_body(dH, D, n, d, c.i, c.j, op_of(sys, c.i, c.op_i), op_of(sys, c.j, c.op_j), 1.0);
    grad_out[idx++] = expect(dH);
  }
  for (int i = 0; i < idx; ++i)
    if (!std::isfinite(grad_out[i])) return fail(SCP_ENONFINITE, "static ZZ gradient is not finite");
  return SCP_OK;
}

}  // extern "C"
